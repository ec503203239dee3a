"""The factored history (QHP_FAC64, QHP_FAC32): the raw lag matrices stored
lag-banded and applied to the histories of the current and of the cell
charges, P_E and P_M once per step (Sec. IV-A, T_k = P_E W^E_k + P_M W^M_k,
with the difference quotients moved onto the history by summation by
parts).  The march is the same method as the dense blocks': FP64 against the
oracle within 1e-10 of the peak current (MI355X only)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _err(j, jref):
    return float(np.linalg.norm(j - jref, axis=1).max() / np.linalg.norm(jref, axis=1).max())


def _oracle(xyz, tri, dt, waves_, n):
    from oracle import excitation as E, mot, operators as O
    asm = O.Assembly(xyz, tri, dt)
    asm.build()
    r = np.stack([E.rhs(asm, w, n) for w in waves_], axis=-1)
    return mot.currents(asm.proj.PLH, asm.proj.PS, asm.dtn, mot.march(asm.T, r))


def _march(xyz, tri, dt, waves_, n, precision, solver="lu"):
    import paper_2312_06367_amd as qhp
    s = qhp.Solver(dt, precision="fac64" if precision.startswith("fac") else "f64", solver=solver)
    s.mesh(xyz, tri)
    s.assemble()
    if precision != s.precision:
        s.set_precision(precision)
    ne = s.info()["ne"]
    s.set_incident(waves_, n)
    jh = torch.zeros((n, ne, len(waves_)), dtype=torch.float64, device="cuda")
    s.run(n, jh)
    out = jh.cpu().numpy()
    inf = s.info()
    s.close()
    return out, inf


# stated bound of the FP32 band values (carried rounding)
FAC32_BOUND = {"sphere120": 1e-6, "sphere480": 1e-6, "torus": 5e-6}


@pytest.mark.parametrize("case", ["sphere120", "sphere480", "torus"])
def test_factored_march_against_the_oracle(case):
    from workloads import meshes, waves
    if case == "sphere120":
        xyz, tri = meshes.icosphere(1)
        dt, n = 0.15, 300
        ws = [waves.Wave((0.0, 0.0, -1.0), (1.0, 0.0, 0.0), 1.0, waves.mod_gauss_t0(0.1, 2.0), 0, 0.0, 0.1, 0.1)]
    elif case == "sphere480":
        cfg = waves.sphere_small()
        (xyz, tri), dt, n, ws = cfg.mesh, cfg.dt, cfg.n_steps, cfg.waves
    else:
        xyz, tri = meshes.torus(1.0, 0.4, 12, 6)
        dt, n = 0.12, 150
        ws = waves.batched_waves(1, 5, 0.1, 0.1, 2.8)[:1]
    _say("[%s] oracle" % case)
    jref = _oracle(xyz, tri, dt, ws, n)[:, :, 0]
    for prec in ("fac64", "fac32"):
        # LU back-solves, and the inverse folded into the [P_E P_M] product
        for solver in ("lu", "inv"):
            j, inf = _march(xyz, tri, dt, ws, n, prec, solver)
            err = _err(j[:, :, 0], jref)
            _say("[%s] %s %s: current err vs oracle %.3e (ne=%d K=%d, %d band bytes)"
                 % (case, prec, solver, err, inf["ne"], inf["K"], inf["slab_bytes"]))
            assert err < (1e-10 if prec == "fac64" else FAC32_BOUND[case])


def test_factored_equals_dense_blocks_at_101_lags():
    """1920-edge sphere at c dt = 0.02 m (K = 101, the 7680-edge workload's
    lag count), 600 steps: the factored FP64 march equals the dense FP64
    blocks' march (the dense march is pinned to the oracle elsewhere)."""
    from workloads import meshes, waves
    xyz, tri = meshes.icosphere(3)
    dt, n = 0.02, 600
    f0 = waves.hz_to_per_m(150e6)
    ws = [waves.Wave((0.0, 0.0, -1.0), (1.0, 0.0, 0.0), 1.0, waves.mod_gauss_t0(f0, 2.0), 0, 0.0, f0, f0)]
    jd, infd = _march(xyz, tri, dt, ws, n, "f64")
    jf, inff = _march(xyz, tri, dt, ws, n, "fac64")
    j32, _ = _march(xyz, tri, dt, ws, n, "fac32")
    assert infd["K"] == 101
    e64, e32 = _err(jf[:, :, 0], jd[:, :, 0]), _err(j32[:, :, 0], jd[:, :, 0])
    _say("[sphere1920 K=101] fac64 vs dense f64 %.3e, fac32 %.3e; bytes dense %d, factored %d"
         % (e64, e32, infd["slab_bytes"], inff["slab_bytes"]))
    assert e64 < 1e-10 and e32 < 1e-6


def test_factored_refusals():
    """Host checks of the factored form: one right-hand side, no conversion to
    or from dense storage, no dense blocks to read back, no batches."""
    import paper_2312_06367_amd as qhp
    from workloads import meshes, waves
    xyz, tri = meshes.icosphere(0)
    s = qhp.Solver(0.3, precision="fac64", solver="lu")
    s.mesh(xyz, tri)
    s.assemble()
    ws = waves.batched_waves(1, 0, 0.1, 0.1, 2.0)
    for call, code in ((lambda: s.set_incident(ws, 10), -1), (lambda: s.set_precision("f32"), -1),
                       (lambda: s.get_matrix("slab", 1), -3)):
        with pytest.raises(qhp.QhpError) as e:
            call()
        assert e.value.code == code
    assert np.isfinite(s.get_matrix("slab", 0)).all()
    s.set_precision("fac32")
    s.set_incident(ws[:1], 10)
    with pytest.raises(qhp.QhpError) as e:
        qhp.Batch([s])
    assert e.value.code == -1
    s.close()


@pytest.mark.parametrize("precision", ["fac64", "fac32"])
def test_factored_passes_in_pieces(precision):
    """The far lags are applied in passes of band_block steps, each pass
    within one qhp_run / qhp_step call: a march in pieces whose lengths are
    not multiples of the pass (7, 5, then single steps) equals one run of the
    same steps to rounding (Sec. IV-B march; the sums are the same, grouped
    differently)."""
    # K = 15 on this mesh: several passes of band_block steps in 24 steps
    import paper_2312_06367_amd as qhp
    from workloads import meshes, waves
    xyz, tri = meshes.icosphere(1)
    ws = waves.batched_waves(1, 0, 0.1, 0.1, 2.0)
    n = 24

    def solver():
        s = qhp.Solver(0.15, precision="fac64", solver="lu")
        s.mesh(xyz, tri)
        s.assemble()
        if precision != "fac64":
            s.set_precision(precision)
        s.set_incident(ws[:1], n)
        return s

    s = solver()
    inf = s.info()
    assert inf["band_block"] > 1 and inf["K"] > inf["band_block"]
    ne = inf["ne"]
    one = torch.zeros((n, ne, 1), dtype=torch.float64, device="cuda")
    s.run(n, one)
    s.close()
    s = solver()
    parts = torch.zeros_like(one)
    s.run(7, parts[:7])
    s.run(5, parts[7:12])
    for t in range(12, n):
        s.step(parts[t])
    s.close()
    a, b = one.cpu().numpy(), parts.cpu().numpy()
    err = float(np.abs(a - b).max() / np.abs(a).max())
    _say("[pieces] %s: 7 + 5 + 12 single steps vs one run of 24: %.3e" % (precision, err))
    assert err < 1e-12


@pytest.mark.parametrize("dt", [4.0, 1.0, 0.7, 0.6])
def test_factored_few_lags_against_the_oracle(dt):
    """Lag counts K = 2 .. 5 on the 120-edge sphere (c dt from 0.6 to 4 m,
    the large-time-step regime included): no far band (K < 4), a far band of
    one lag (K = 4, where A_K = C_K = 0 leave only Sq_4) and of two; the
    FP64 march equals the oracle's within 1e-10 of the peak current."""
    from workloads import meshes, waves
    xyz, tri = meshes.icosphere(1)
    f = 1.0 / (64.0 * dt) if dt > 1.0 else 0.05
    ws = waves.batched_waves(1, 0, f, f, 2.0)[:1]
    n = 120
    j, inf = _march(xyz, tri, dt, ws, n, "fac64")
    jref = _oracle(xyz, tri, dt, ws, n)
    err = _err(j[:, :, 0], jref[:, :, 0])
    _say("[few lags] c dt %.2f: K = %d, band_block %d: fac64 vs oracle %.3e" % (dt, inf["K"], inf["band_block"], err))
    assert err < 1e-10


@pytest.mark.parametrize("precision", ["fac64", "fac32"])
def test_factored_solver_switch_mid_march(precision):
    """A factored context changes solver between calls: the inverse solve
    (y_i = T_0^{-1} r_i - T_0^{-1} [P_E P_M] [E; M], both factors formed
    ahead) and the LU back-solves of r_i - [P_E P_M] [E; M] (Sec. IV-B, the
    one solve per step) alternate over 10 + 9 + 11 steps and equal one LU
    run of the 30 steps to rounding."""
    import paper_2312_06367_amd as qhp
    from workloads import meshes, waves
    xyz, tri = meshes.icosphere(1)
    ws = waves.batched_waves(1, 0, 0.1, 0.1, 2.0)
    n = 30

    def solver():
        s = qhp.Solver(0.15, precision="fac64", solver="lu")
        s.mesh(xyz, tri)
        s.assemble()
        if precision != "fac64":
            s.set_precision(precision)
        s.set_incident(ws[:1], n)
        return s

    s = solver()
    ne = s.info()["ne"]
    one = torch.zeros((n, ne, 1), dtype=torch.float64, device="cuda")
    s.run(n, one)
    s.close()
    s = solver()
    mixed = torch.zeros_like(one)
    s.set_solver("inv")
    s.run(10, mixed[:10])
    s.set_solver("lu")
    s.run(9, mixed[10:19])
    s.set_solver("inv")
    s.run(11, mixed[19:])
    s.close()
    a, b = one.cpu().numpy(), mixed.cpu().numpy()
    err = float(np.abs(a - b).max() / np.abs(a).max())
    _say("[solver switch] %s: inv 10 + lu 9 + inv 11 vs one lu run of 30: %.3e" % (precision, err))
    # the two solves differ by the rounding order of FP64 sums (3e-13 over a
    # whole 7680-edge march)
    assert err < 1e-11
