"""The history sum that allocates nothing (qhp_history_sum_noalloc) against
the one that allocates its partial sums per call (qhp_history_sum_variant):
the same kernels and split counts, so the results are bit-identical, on two
calls in a row, the second smaller, for each arithmetic form tried."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _case(precision, ne, ld, nrhs, kmax, n_slots, head, seed):
    rng = np.random.default_rng(seed)
    dt_ = {"f64": torch.float64, "f32": torch.float32, "f32a": torch.float32}[precision]
    ydt = torch.float64 if precision in ("f64", "f32a") else torch.float32
    T = rng.standard_normal((kmax, ne, ld))
    T[:, :, ne:] = 1e6  # padding the kernels must ignore
    Y = rng.standard_normal((n_slots, ld, nrhs))
    Y[:, ne:, :] = 1e6
    slabs = torch.from_numpy(T).to(dt_).cuda()
    ring = torch.from_numpy(Y).to(ydt).cuda()
    r = torch.from_numpy(rng.standard_normal((ne, nrhs))).cuda()
    return slabs, ring, r


@pytest.mark.parametrize("precision,nrhs,variant", [("f32a", 1, 10), ("f32a", 1, -1), ("f64", 1, -1),
                                                     ("f32", 8, -1), ("f64", 3, -1)])
def test_noalloc_matches_the_allocating_entry_point(precision, nrhs, variant):
    import paper_2312_06367_amd as qhp
    # first call: several tiles and a ragged tail; second: smaller, so that
    # stale partial sums of the first call would show
    for ne, ld, kmax, n_slots, head, seed in ((3001, 3072, 12, 14, 5, 1), (1003, 1024, 5, 7, 3, 2)):
        _say("[noalloc] %s nrhs=%d variant=%d ne=%d kmax=%d" % (precision, nrhs, variant, ne, kmax))
        slabs, ring, r = _case(precision, ne, ld, nrhs, kmax, n_slots, head, seed)
        b_alloc = torch.full_like(r, float("nan"))
        b_none = torch.full_like(r, float("nan"))
        qhp.history_sum(precision, slabs, None, ring, head, r, b_alloc, kmax=kmax, variant=variant)
        qhp.history_sum_noalloc(precision, slabs, None, ring, head, r, b_none, kmax=kmax, variant=variant)
        torch.cuda.synchronize()
        assert torch.equal(b_none, b_alloc)
        ref = r.cpu().numpy().copy()
        Ts = slabs.double().cpu().numpy()
        Ys = ring.double().cpu().numpy()
        for k in range(1, kmax + 1):
            ref -= Ts[k - 1][:, :ne] @ Ys[(head + k - 1) % n_slots][:ne]
        err = float(np.abs(b_none.cpu().numpy() - ref).max() / np.abs(ref).max())
        _say("[noalloc] identical to qhp_history_sum_variant; vs FP64 of the stored values %.2e" % err)
        assert err < (1e-13 if precision in ("f64", "f32a") else 2e-5)
