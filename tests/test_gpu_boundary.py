"""The C-ABI conventions on the GPU: stepping one call at a time, the growth
trip of QHP_EUNSTABLE, a batch holding its contexts, and the caller
allocator hook (MI355X only)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _wave(f0, diameter):
    from workloads import waves
    return waves.Wave((0.0, 0.0, -1.0), (1.0, 0.0, 0.0), 1.0, waves.mod_gauss_t0(f0, diameter), 0, 0.0, f0, f0)


@pytest.fixture(scope="module")
def ico1():
    """Level-1 icosphere (120 edges), c dt = 0.15 m, 200 steps: the oracle's march."""
    from oracle import excitation as E, mot, operators as O
    from workloads import meshes
    xyz, tri = meshes.icosphere(1)
    dt, n = 0.15, 200
    _say("[ico1] oracle assembly and march")
    asm = O.Assembly(xyz, tri, dt)
    asm.build()
    w = _wave(0.1, asm.D)
    y = mot.march(asm.T, E.rhs(asm, w, n))
    j = mot.currents(asm.proj.PLH, asm.proj.PS, asm.dtn, y)
    return dict(xyz=xyz, tri=tri, dt=dt, n=n, w=w, j=j, ne=asm.topo.ne)


def _solver(d, precision="f64", solver="lu", **kw):
    import paper_2312_06367_amd as qhp
    s = qhp.Solver(d["dt"], precision="f64", solver=solver, **kw)
    s.mesh(d["xyz"], d["tri"])
    s.assemble()
    if precision != "f64":
        s.set_precision(precision)
    return s


def test_step_by_step_march_equals_the_oracle(ico1):
    """qhp_step, one call per step (Sec. IV-B update and eq. post_processing),
    against the oracle's march: FP64 within 1e-10 of the peak current."""
    s = _solver(ico1)
    n, ne = ico1["n"], ico1["ne"]
    s.set_incident([ico1["w"]], n)
    j = torch.zeros((n, ne, 1), dtype=torch.float64, device="cuda")
    for i in range(n):
        s.step(j[i])
    assert s.info()["step"] == n
    from paper_2312_06367_amd import QhpError
    with pytest.raises(QhpError) as e:  # no right-hand side left
        s.step(j[0])
    assert e.value.code == -3
    s.close()
    jj = j[:, :, 0].cpu().numpy()
    err = float(np.linalg.norm(jj - ico1["j"], axis=1).max() / np.linalg.norm(ico1["j"], axis=1).max())
    _say("[ico1] qhp_step march vs oracle: %.3e" % err)
    assert err < 1e-10


def test_growth_trip(ico1):
    """QHP_EUNSTABLE from the growth trip: a limit no march can meet stops
    the run and the context refuses further steps until qhp_set_incident; the
    default limit and a disabled check let the whole march through with the
    same result."""
    from paper_2312_06367_amd import QhpError
    s = _solver(ico1)
    n, ne = ico1["n"], ico1["ne"]
    jh = torch.zeros((n, ne, 1), dtype=torch.float64, device="cuda")
    s.set_incident([ico1["w"]], n)
    s.run(n, jh)  # default limit
    ref = jh.clone()
    s.set_growth_limit(1e-3)
    s.set_incident([ico1["w"]], n)
    with pytest.raises(QhpError) as e:
        s.run(n, jh)
    assert e.value.code == -8 and "growth" in str(e.value)
    with pytest.raises(QhpError) as e:
        s.step(None)
    assert e.value.code == -3
    s.set_growth_limit(0.0)
    s.set_incident([ico1["w"]], n)
    s.run(n, jh)
    # each qhp_set_incident re-times the history kernel's split count, which
    # regroups the FP64 sums: equal up to rounding
    assert float((jh - ref).abs().max() / ref.abs().max()) < 1e-12
    with pytest.raises(QhpError) as e:
        s.set_growth_limit(-1.0)
    assert e.value.code == -1
    s.close()


def test_batch_holds_its_contexts_and_resumes_their_marches():
    """FP32 blocks with FP64 y and sums, 4 waves, on a torus with two global
    loops: 30 steps alone, 30 in a batch, 30 alone, 30 in the batch again give
    the 120-step march of a context alone (the batch works on the context's
    own transposed ring and picks up its steps); while the batch exists the
    context refuses qhp_set_incident and qhp_set_precision.  The contexts
    solve with the FP64 inverse of T_0, as the batch does; the batch's kernels
    sum in other orders than the context's, and this torus march amplifies
    those roundings to ~1e-10 (the bound of the other batch-against-eager
    tests, 1e-9); a ring left behind by either side would be off by O(1)."""
    import paper_2312_06367_amd as qhp
    from workloads import meshes, waves
    xyz, tri = meshes.torus(1.0, 0.4, 12, 6)
    dt, n = 0.12, 120
    d = dict(xyz=xyz, tri=tri, dt=dt)
    ws = waves.batched_waves(2, 5, 0.1, 0.1, 2.8)
    ref_s = _solver(d, "f32a", solver="inv")
    ne = ref_s.info()["ne"]
    ref_s.set_incident(ws, n)
    ref = torch.zeros((n, ne, 4), dtype=torch.float64, device="cuda")
    ref_s.run(n, ref)
    ref_s.close()
    s = _solver(d, "f32a", solver="inv")
    s.set_incident(ws, n)
    j = torch.zeros((n, ne, 4), dtype=torch.float64, device="cuda")
    s.run(30, j[0:30])
    b = qhp.Batch([s])
    b.run(30, [j[30:60]])
    with pytest.raises(qhp.QhpError) as e:
        s.set_incident(ws, n)
    assert e.value.code == -3
    with pytest.raises(qhp.QhpError) as e:
        s.set_precision("f32")
    assert e.value.code == -3
    s.run(30, j[60:90])
    b.run(30, [j[90:120]])
    assert s.info()["step"] == 120
    b.close()
    s.set_incident(ws, n)  # allowed again once the batch is gone
    s.close()
    err = float((j - ref).abs().max() / ref.abs().max())
    _say("[torus f32a x4] alone / batch / alone / batch vs alone: %.3e" % err)
    assert err < 1e-9


def test_torch_allocator_hook(ico1):
    """qhp_params.dev_alloc / dev_free backed by PyTorch's caching allocator:
    every device buffer of the context comes from it and goes back to it at
    qhp_destroy, and the march is the oracle's (FP64 within 1e-10)."""
    s = _solver(ico1, allocator="torch")
    al = s.allocator
    n, ne = ico1["n"], ico1["ne"]
    s.set_incident([ico1["w"]], n)
    j = torch.zeros((n, ne, 1), dtype=torch.float64, device="cuda")
    s.run(n, j)
    held = al.bytes_held()
    _say("[ico1] torch allocator: %d allocations, %d frees, %.1f MB held before destroy"
         % (al.calls["alloc"], al.calls["free"], held / 1e6))
    assert al.calls["alloc"] > 20 and held > 0
    s.close()
    assert al.bytes_held() == 0 and al.calls["free"] == al.calls["alloc"]
    jj = j[:, :, 0].cpu().numpy()
    err = float(np.linalg.norm(jj - ico1["j"], axis=1).max() / np.linalg.norm(ico1["j"], axis=1).max())
    _say("[ico1] march with the torch allocator vs oracle: %.3e" % err)
    assert err < 1e-10
