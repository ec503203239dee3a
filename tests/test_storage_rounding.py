"""Why reduced-precision lag blocks are stored with lag-carried rounding.

The retarded history sum of the rescaled, preconditioned formulation cancels
strongly across lags (the blocks carry difference quotients in time from the
projector rescaling of Sec. III and the derivative combinations of Sec. IV-A),
so rounding each T_k independently perturbs the march by far more than one
rounding.  Carrying each block's rounding into the next lag makes the
perturbation act only on differences y_{i-k-1} - y_{i-k}.  These tests march
the oracle's FP64 blocks after numpy rounding, plain and carried, on the
multiply connected torus used by the GPU batched-march test."""
import numpy as np
import pytest


def _round_bf16(a):
    a32 = np.ascontiguousarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _round_f32(a):
    return a.astype(np.float32).astype(np.float64)


def _store(T, rnd, carried, per_block_scale):
    out = T.copy()
    c = np.zeros_like(T[0])
    for k in range(1, T.shape[0]):
        v = T[k] + c if carried else T[k]
        sc = np.abs(v).max() if per_block_scale else 1.0
        out[k] = rnd(v / sc) * sc
        c = v - out[k]
    return out


@pytest.fixture(scope="module")
def torus():
    from oracle import excitation as E, mot, operators as O
    from workloads import meshes, waves
    xyz, tri = meshes.torus(1.0, 0.4, 12, 6)
    dt, n = 0.12, 150
    asm = O.Assembly(xyz, tri, dt)
    asm.build()
    ws = waves.batched_waves(2, 5, 0.1, 0.1, asm.D)[:3]
    r = np.stack([E.rhs(asm, w, n) for w in ws], axis=-1)
    y = mot.march(asm.T, r)
    j = mot.currents(asm.proj.PLH, asm.proj.PS, asm.dtn, y)
    return asm, r, j


def _err(torus, T):
    from oracle import mot
    asm, r, j = torus
    jq = mot.currents(asm.proj.PLH, asm.proj.PS, asm.dtn, mot.march(T, r))
    return float(np.abs(jq - j).max() / np.abs(j).max())


def test_history_cancels_across_lags(torus):
    """sum_k |T_k||y_{i-k}| exceeds |sum_k T_k y_{i-k}| by more than an order
    of magnitude at the peak of the response."""
    from oracle import mot
    asm, r, _ = torus
    y = mot.march(asm.T, r)[:, :, 0]
    i = int(np.argmax(np.linalg.norm(y, axis=1))) + 1
    K = asm.K
    h = sum(asm.T[k] @ y[i - k - 1] for k in range(1, min(i - 1, K) + 1))
    ha = sum(np.abs(asm.T[k]) @ np.abs(y[i - k - 1]) for k in range(1, min(i - 1, K) + 1))
    assert np.linalg.norm(ha) > 10 * np.linalg.norm(h)


def test_carried_rounding_bf16(torus):
    plain = _err(torus, _store(torus[0].T, _round_bf16, False, True))
    carried = _err(torus, _store(torus[0].T, _round_bf16, True, True))
    assert plain > 0.3  # independent BF16 rounding loses the solution
    assert carried < 0.06
    assert carried < plain / 10


def test_carried_rounding_f32(torus):
    plain = _err(torus, _store(torus[0].T, _round_f32, False, False))
    carried = _err(torus, _store(torus[0].T, _round_f32, True, False))
    assert carried < plain / 5
    assert carried < 1e-5
