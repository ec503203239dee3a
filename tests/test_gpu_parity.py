"""Parity of the HIP path with the CPU FP64 oracle (MI355X only).

Every comparison is relative to the largest magnitude of the oracle's
result: FP64 path <= 1e-10, FP32 slabs <= 1e-5, BF16 slabs <= 5e-2 on the
current (the bound for each form is stated in its test)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _wave(f0, diameter):
    from workloads import waves
    return waves.Wave((0.0, 0.0, -1.0), (1.0, 0.0, 0.0), 1.0, waves.mod_gauss_t0(f0, diameter), 0, 0.0, f0, f0)


@pytest.fixture(scope="module")
def small():
    """Level-1 icosphere (120 edges), c dt = 0.15 m: oracle and GPU."""
    from oracle import operators as O, excitation as E, mot
    from workloads import meshes
    import paper_2312_06367_amd as qhp
    xyz, tri = meshes.icosphere(1)
    dt = 0.15
    _say("[small] oracle assembly")
    asm = O.Assembly(xyz, tri, dt)
    asm.build()
    w = _wave(0.1, asm.D)
    n_steps = 300
    r = E.rhs(asm, w, n_steps)
    y = mot.march(asm.T, r)
    j = mot.currents(asm.proj.PLH, asm.proj.PS, asm.dtn, y)
    _say("[small] GPU assembly")
    s = qhp.Solver(dt, precision="f64", solver="lu")
    s.mesh(xyz, tri)
    s.keep_raw(True)
    s.assemble()
    return dict(asm=asm, w=w, n_steps=n_steps, r=r, y=y, j=j, s=s, xyz=xyz, tri=tri, dt=dt)


def test_topology_numbering(small):
    e, c = small["s"].edges()
    t = small["asm"].topo
    assert np.array_equal(e, t.edges.astype(np.int32))
    assert np.array_equal(c, t.cells.astype(np.int32))
    inf = small["s"].info()
    assert inf["K"] == small["asm"].K and inf["n_harmonic"] == 0


@pytest.mark.parametrize("name,attr", [
    ("gram", "G"), ("zs", "Zs"), ("zh", "Zh"), ("m", "M"), ("pe", "PE"), ("pm", "PM"),
])
def test_static_operator_parity(small, name, attr):
    got = small["s"].get_matrix(name)
    ref = getattr(small["asm"], attr)
    err = _rel(got, ref)
    _say("[small] %s rel err %.3e" % (name, err))
    assert err < 1e-10


def test_projector_parity(small):
    p = small["asm"].proj
    assert _rel(small["s"].get_matrix("psigma"), p.PS) < 1e-12
    assert _rel(small["s"].get_matrix("plambda"), p.PPL) < 1e-12


def test_raw_lag_and_slab_parity(small):
    asm, s = small["asm"], small["s"]
    worst = 0.0
    for k in range(asm.K + 1):
        for name, ref in (("a", asm.A[k]), ("b", asm.B[k]), ("c", asm.C[k])):
            got = s.get_matrix(name, k)
            scale = max(np.abs(ref).max(), 1e-300)
            worst = max(worst, float(np.abs(got - ref).max() / scale) if np.abs(ref).max() > 0 else np.abs(got).max())
        got = s.get_matrix("slab", k)
        e = _rel(got, asm.T[k])
        worst = max(worst, e)
    _say("[small] lag/slab worst rel err %.3e" % worst)
    assert worst < 1e-10


def test_march_parity_f64(small):
    s = small["s"]
    n = small["n_steps"]
    ne = small["asm"].topo.ne
    s.set_incident([small["w"]], n)
    jh = torch.zeros((n, ne, 1), dtype=torch.float64, device="cuda")
    yh = torch.zeros((n, ne, 1), dtype=torch.float64, device="cuda")
    s.run(n, jh, yh)
    j = jh[:, :, 0].cpu().numpy()
    y = yh[:, :, 0].cpu().numpy()
    ej = float(np.linalg.norm(j - small["j"], axis=1).max() / np.linalg.norm(small["j"], axis=1).max())
    ey = float(np.linalg.norm(y - small["y"], axis=1).max() / np.linalg.norm(small["y"], axis=1).max())
    _say("[small] march f64: current err %.3e, y err %.3e" % (ej, ey))
    assert ej < 1e-10 and ey < 1e-10
