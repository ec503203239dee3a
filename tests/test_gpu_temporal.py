"""Quadratic temporal basis pairs on the GPU (Remark of Sec. IV-B): the
shifted quadratic Lagrange interpolators h_i with q_i' = (h_i - h_{i+1})/dt,
assembled from x-weighted shell moments.  Against the oracle (120-edge
sphere, c dt = 0.15 m, an oblique pulse at 0.5 per metre, about 13 steps a
period): the raw lag matrices A_k, B_k, C_k and the blocks T_k (to 1e-10 of
each matrix's largest entry), the FP64 march (1e-10 of the peak current),
FP32 blocks with FP64 sums (1e-7) and the factored history in FP64 (1e-10)
(MI355X only)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def quad2():
    from oracle import operators as O, excitation as E, mot
    from workloads import meshes, waves
    xyz, tri = meshes.icosphere(1)
    dt, n, f0 = 0.15, 300, 0.5
    _say("[order 2] oracle assembly")
    asm = O.Assembly(xyz, tri, dt, order=2)
    asm.build()
    w = waves.Wave((0.3, 0.2, -0.93), (1.0, 0.0, 0.3), 1.0, waves.mod_gauss_t0(f0, asm.D), 0, 0.0, f0, f0)
    r = E.rhs(asm, w, n)
    j = mot.currents(asm.proj.PLH, asm.proj.PS, asm.dtn, mot.march(asm.T, r))
    return dict(asm=asm, w=w, n=n, j=j, xyz=xyz, tri=tri, dt=dt)


def _march(c, precision, solver="lu"):
    import paper_2312_06367_amd as qhp
    s = qhp.Solver(c["dt"], precision="fac64" if precision.startswith("fac") else "f64", solver=solver, order=2)
    s.mesh(c["xyz"], c["tri"])
    s.assemble()
    if precision != s.precision:
        s.set_precision(precision)
    assert s.info()["K"] == c["asm"].K
    ne = s.info()["ne"]
    s.set_incident([c["w"]], c["n"])
    jh = torch.zeros((c["n"], ne, 1), dtype=torch.float64, device="cuda")
    s.run(c["n"], jh)
    s.close()
    j = jh[:, :, 0].cpu().numpy()
    return float(np.linalg.norm(j - c["j"], axis=1).max() / np.linalg.norm(c["j"], axis=1).max())


def test_order2_lag_matrices_against_the_oracle(quad2):
    import paper_2312_06367_amd as qhp
    asm = quad2["asm"]
    s = qhp.Solver(quad2["dt"], precision="f64", solver="lu", order=2)
    s.mesh(quad2["xyz"], quad2["tri"])
    s.keep_raw(True)
    s.assemble()
    assert s.info()["K"] == asm.K
    worst = 0.0
    for k in range(asm.K + 1):
        for name, ref in (("a", asm.A[k]), ("b", asm.B[k]), ("c", asm.C[k]), ("slab", asm.T[k])):
            got = s.get_matrix(name, k)
            scale = np.abs(ref).max()
            worst = max(worst, float(np.abs(got - ref).max() / scale) if scale > 0 else float(np.abs(got).max()))
    s.close()
    _say("[order 2] raw lag matrices and blocks: worst %.3e of the largest entry (K = %d)" % (worst, asm.K))
    assert worst < 1e-10


@pytest.mark.parametrize("form,bound", [("f64", 1e-10), ("f32a", 1e-7), ("fac64", 1e-10)])
def test_order2_march_against_the_oracle(quad2, form, bound):
    err = _march(quad2, form, "lu" if form == "f64" else "inv")
    _say("[order 2] %s march: current err vs oracle %.3e (bound %.0e)" % (form, err, bound))
    assert err < bound
