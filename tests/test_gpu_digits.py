"""Int8 digit storage and the int8 matrix-core history sum (QHP_I8X4) against
the numpy model of the storage and the plain FP64 definition (MI355X only)."""
import sys

import numpy as np
import pytest

from tests import digits_model as dm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("nrhs", [2, 3, 70, 130])
@pytest.mark.parametrize("variant", [-1, 0, 1, 2])
def test_history_sum_i8x4_ragged(nrhs, variant):
    """b = r - sum_k T_k y_{i-k} through qhp_history_sum with digit-stored
    blocks and ring slots: ragged rows (1003, not a multiple of 16 or 128),
    right-hand sides not a multiple of 16 or 64, a circular ring with a head
    offset, rows of very different magnitudes, one all-zero row; every
    kernel variant the autotuner chooses from."""
    import paper_2312_06367_amd as qhp
    if variant >= qhp.history_variants("i8x4", nrhs):
        pytest.skip("no such variant")
    rng = np.random.default_rng(5 + nrhs)
    ne, ld, kmax, n_slots, head = 1003, 1024, 5, 7, 3
    T = rng.standard_normal((kmax, ne, ne)) * np.logspace(-3, 2, ne)[None, :, None]
    T[:, 17, :] = 0.0
    S, Q = dm.quantise_blocks(T)
    slabs = np.stack([dm.block_bytes(S[k], Q[k], ld) for k in range(kmax)])
    ys = [dm.quantise_columns(rng.standard_normal((ne, nrhs)) * rng.uniform(0.1, 10, (1, nrhs)))
          for _ in range(n_slots)]
    ring = np.stack([dm.slot_bytes(sy, qy, ld) for sy, qy in ys])
    r = rng.standard_normal((ne, nrhs))
    dev = "cuda"
    rt = torch.from_numpy(r).to(dev)
    b = torch.zeros_like(rt)
    qhp.history_sum("i8x4", torch.from_numpy(slabs.view(np.int8)).to(dev), None,
                    torch.from_numpy(ring.view(np.int8)).to(dev), head, rt, b, kmax=kmax, variant=variant)
    torch.cuda.synchronize()
    got = b.cpu().numpy()
    model = r.copy()
    exact = r.copy()
    bound = np.zeros_like(r)
    for k in range(1, kmax + 1):
        sy, qy = ys[(head + k - 1) % n_slots]
        model -= dm.product(S[k - 1], Q[k - 1], sy, qy)
        exact -= dm.value(S[k - 1][:, None], Q[k - 1]) @ dm.value(sy[None, :], qy)
        bound += dm.dropped_bound(S[k - 1], sy, ne)
    scale = np.abs(exact).max()
    e_model = float(np.abs(got - model).max() / scale)
    e_exact = float(np.abs(got - exact).max() / scale)
    _say("[history_sum i8x4 nrhs=%d variant %d] vs model %.2e, vs FP64 of the stored values %.2e"
         % (nrhs, variant, e_model, e_exact))
    assert e_model < 1e-13
    assert np.all(np.abs(got - exact) <= bound + 1e-13 * scale)


def test_quantise_i8x4_bit_exact():
    """Blocks re-stored from FP64 as digits: the GPU's stored values equal the
    model's lag-carried digit rounding of the same FP64 blocks bit for bit."""
    import paper_2312_06367_amd as qhp
    from workloads import meshes
    xyz, tri = meshes.icosphere(1)
    s = qhp.Solver(0.15, precision="f64")
    s.mesh(xyz, tri)
    s.assemble()
    K = s.info()["K"]
    T = np.stack([s.get_matrix("slab", k) for k in range(1, K + 1)])
    s.set_precision("i8x4")
    got = np.stack([s.get_matrix("slab", k) for k in range(1, K + 1)])
    s.close()
    S, Q = dm.quantise_blocks(T)
    want = np.stack([dm.value(S[k][:, None], Q[k]) for k in range(K)])
    diff = int(np.count_nonzero(got != want))
    _say("[quantise i8x4] %d of %d stored values differ; max |T - stored| / max |T| %.2e"
         % (diff, got.size, np.abs(got - T).max() / np.abs(T).max()))
    if diff:
        per_lag = [int(np.count_nonzero(got[k] != want[k])) for k in range(K)]
        k0 = int(np.nonzero(per_lag)[0][0])
        i0, j0 = np.argwhere(got[k0] != want[k0])[0]
        quanta = np.abs(got - want) / (S[:, :, None] * 2.0 ** -21 + 1e-300)
        _say("  per lag: %s" % per_lag)
        _say("  first at lag %d (%d, %d): got %r want %r T %r; max diff in quanta %.3g"
             % (k0 + 1, i0, j0, got[k0, i0, j0], want[k0, i0, j0], T[k0, i0, j0], quanta.max()))
    assert diff == 0


def test_batched_march_i8x4():
    """Three waves on the torus with two global loops (150 steps): the GPU
    digit march against the FP64 oracle march and against the model of the
    digit march.  The model differs from the GPU only in the order of the FP64
    sums over lags, which moves a few digit decisions of y by one quantum; the
    march amplifies those like any rounding, so the two agree to about the
    scheme's own error (measured 1.0e-7 and 2.7e-7)."""
    import paper_2312_06367_amd as qhp
    from oracle import operators as O, excitation as E, mot
    from workloads import meshes, waves
    from tests.test_digits import march_digits
    xyz, tri = meshes.torus(1.0, 0.4, 12, 6)
    dt, n = 0.12, 150
    asm = O.Assembly(xyz, tri, dt)
    asm.build()
    ws = waves.batched_waves(2, 5, 0.1, 0.1, asm.D)[:3]
    r = np.stack([E.rhs(asm, w, n) for w in ws], axis=-1)
    jref = mot.currents(asm.proj.PLH, asm.proj.PS, asm.dtn, mot.march(asm.T, r))
    jmod = mot.currents(asm.proj.PLH, asm.proj.PS, asm.dtn, march_digits(asm.T, r))
    s = qhp.Solver(dt, precision="f64")
    s.mesh(xyz, tri)
    s.assemble()
    s.set_precision("i8x4")
    ne = s.info()["ne"]
    s.set_incident(ws, n)
    jh = torch.zeros((n, ne, len(ws)), dtype=torch.float64, device="cuda")
    s.run(n, jh)
    j = jh.cpu().numpy()
    s.close()
    peak = np.abs(jref).max()
    err, err_model = float(np.abs(j - jref).max() / peak), float(np.abs(j - jmod).max() / peak)
    _say("[torus batched] i8x4: current err %.3e vs FP64, %.3e vs the digit model" % (err, err_model))
    assert err < 2e-6
    assert err_model < 1e-6


def test_history_sum_i8x4_full_size_sampled():
    """The int8 history kernel at the shape of the batched torus workload
    (6000 edges, K = 88 digit blocks of 6000 x 6144 x 4 bytes, 128
    right-hand sides), in the launch configuration the march uses, on random
    digits and scales: 32 sampled rows against the model's digit products."""
    import paper_2312_06367_amd as qhp
    ne, K, nrhs, ld, head = 6000, 88, 128, 6144, 29
    R, P, nkc = 6000, 128, ld // 64
    g = torch.Generator(device="cuda")
    g.manual_seed(4)

    def random_blocks(n_blk, rows):
        buf = torch.empty((n_blk, rows * ld * 4 + rows * 8), dtype=torch.int8, device="cuda")
        dig = buf[:, :rows * ld * 4].view(n_blk, rows // 16, nkc, 4, 1024)
        dig[:, :, :, 0] = torch.randint(-127, 128, dig[:, :, :, 0].shape, generator=g, device="cuda",
                                        dtype=torch.int8)
        dig[:, :, :, 1:] = torch.randint(-64, 65, dig[:, :, :, 1:].shape, generator=g, device="cuda",
                                         dtype=torch.int8)
        dig[:, :, ne // 64 + 1:] = 0         # columns 6016.. (whole 64-column chunks past ne)
        dig[:, :, ne // 64, :, 768:] = 0     # columns 6000..6015 (lanes 48..63 of the last chunk)
        sc = torch.rand((n_blk, rows), generator=g, device="cuda", dtype=torch.float64)
        buf[:, rows * ld * 4:].view(torch.float64).copy_((0.5 + sc) * 10.0 ** (3 * sc - 2))
        return buf

    slabs = random_blocks(K, R)
    ring = random_blocks(K, P)
    r = torch.randn((ne, nrhs), dtype=torch.float64, device="cuda", generator=g)
    outs = []
    for variant in range(qhp.history_variants("i8x4", nrhs)):
        b = torch.zeros_like(r)
        qhp.history_sum("i8x4", slabs, None, ring, head, r, b, variant=variant)
        torch.cuda.synchronize()
        outs.append(b.cpu().numpy())
    rows = np.sort(np.random.default_rng(1).choice(ne, 32, replace=False))

    def digits(buf, n_rows, sel):
        """[n_blk][4][len(sel)][ld] int8 digits of the selected rows, and their scales"""
        nb = buf.shape[0]
        d = buf[:, :n_rows * ld * 4].view(nb, n_rows // 16, nkc, 4, 4, 16, 16)  # blk, rt, kc, a, g, r, e
        tiles = np.unique(sel // 16)
        dd = d.index_select(1, torch.from_numpy(tiles).cuda()).cpu().numpy()
        dd = dd.transpose(0, 3, 1, 5, 2, 4, 6).reshape(nb, 4, len(tiles) * 16, ld)
        pos = {int(t_): q for q, t_ in enumerate(tiles)}
        out = dd[:, :, [pos[int(i) // 16] * 16 + int(i) % 16 for i in sel], :]
        scales = buf[:, n_rows * ld * 4:].view(torch.float64).cpu().numpy()[:, sel]
        return out, scales

    t, sr = digits(slabs, R, rows)
    u, sc = digits(ring, P, np.arange(P))
    ref = r.cpu().numpy()[rows].copy()
    for k in range(1, K + 1):
        s_ = (head + k - 1) % K
        G = [np.zeros((len(rows), P)) for _ in range(5)]
        for a_, b_ in dm.PAIRS:
            G[a_ + b_] += t[k - 1, a_].astype(np.float64) @ u[s_, b_].astype(np.float64).T
        gsum = G[4]
        for w in (3, 2, 1, 0):
            gsum = gsum * 2.0 ** -7 + G[w]
        ref -= sr[k - 1][:, None] * sc[s_][None, :] * gsum
    errs = [float(np.abs(o[rows] - ref).max() / np.abs(ref).max()) for o in outs]
    _say("[history_sum i8x4 full size] sampled-row err per variant %s" % " ".join("%.2e" % e for e in errs))
    del slabs, ring
    torch.cuda.empty_cache()
    assert max(errs) < 1e-12


def test_torus_i8x4_2000_steps_and_dc_10k():
    """The batched torus workload (6000 edges, c dt = 0.03 m, K = 88) with 8
    of its waves: the digit march against the FP64 march over the full 2000
    steps (bound 1e-5 relative to the peak current), then 10^4 steps of the
    digit march: the current decays after the pulse and never grows."""
    import paper_2312_06367_amd as qhp
    from workloads import waves
    cfg = waves.torus_batched(4)
    xyz, tri = cfg.mesh
    s = qhp.Solver(cfg.dt, precision="f64", solver="inv")
    s.mesh(xyz, tri)
    s.assemble()
    ne, nw = s.info()["ne"], len(cfg.waves)
    n_ref = 2000
    s.set_incident(cfg.waves, n_ref)
    ref = torch.zeros((n_ref, ne, nw), dtype=torch.float64, device="cuda")
    s.run(n_ref, ref)
    s.set_precision("i8x4")
    n = 10000
    s.set_incident(cfg.waves, n)
    jh = torch.zeros((1000, ne, nw), dtype=torch.float64, device="cuda")
    norms, err = [], 0.0
    peak = torch.linalg.vector_norm(ref, dim=1).max().item()
    for c in range(0, n, 1000):
        s.run(1000, jh)
        if c < n_ref:
            err = max(err, torch.linalg.vector_norm(jh - ref[c:c + 1000], dim=1).max().item() / peak)
        norms.append(torch.linalg.vector_norm(jh, dim=1).max(dim=1).values.cpu().numpy())
    s.close()
    nj = np.concatenate(norms)
    blocks = nj.reshape(-1, 500).max(1) / nj.max()
    _say("[torus i8x4] 2000-step current err %.3e; dc 10k block maxima / peak: %s"
         % (err, " ".join("%.1e" % v for v in blocks)))
    assert err < 1e-5
    assert nj[-1000:].max() < 1e-3 * nj.max()
    assert blocks[-1] <= 10 * blocks[len(blocks) // 2] + 1e-12  # no late growth
