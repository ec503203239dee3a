"""Numpy model of the int8 digit storage of the lag blocks and history
vectors (QHP_I8X4), for the tests only.

A row of a lag block (or a column of y) with scale s = max |v| / 127 is held
as q = rint(v 2^21 / s), |q| <= 127 2^21, written with balanced base-128
digits q = t0 2^21 + t1 2^14 + t2 2^7 + t3 (t0 in [-127, 127], t1..t3 in
[-64, 64]); the stored value is s q 2^-21.  Blocks are rounded lag by lag
with the rounding carried into the next lag.  The history product keeps the
digit products t_a u_b with a + b <= 4, summed exactly per weight 2^-7(a+b),
then scaled by s_row s_col in FP64.  Every floating-point step that decides
a digit is taken in FP64 in the same order as the library does it."""
import numpy as np

Q21 = 2.0 ** 21
LIM = 127.0 * Q21
PAIRS = [(a, b) for a in range(4) for b in range(4) if a + b <= 4]  # 13 products


def fixed(v, s):
    """q = clip(rint(v * (2^21 / s))) with s broadcast against v (0 where s = 0)."""
    s = np.asarray(s, dtype=np.float64)
    f = np.where(s > 0.0, Q21 / np.where(s > 0.0, s, 1.0), 0.0)
    return np.clip(np.rint(v * f), -LIM, LIM).astype(np.int64)


def split4(q):
    """balanced base-128 digits of q (int64 array) -> [t0, t1, t2, t3]"""
    t0 = (q + (1 << 20)) >> 21
    r = q - (t0 << 21)
    t1 = (r + (1 << 13)) >> 14
    r = r - (t1 << 14)
    t2 = (r + (1 << 6)) >> 7
    t3 = r - (t2 << 7)
    return [t0, t1, t2, t3]


def value(s, q):
    """stored value s (q 2^-21), s broadcast against q"""
    return s * (q.astype(np.float64) * 2.0 ** -21)


def quantise_blocks(T):
    """T [K, n, m] FP64 -> (row scales [K, n], q [K, n, m]) with lag-carried rounding."""
    K, n, m = T.shape
    S = np.zeros((K, n))
    Q = np.zeros((K, n, m), dtype=np.int64)
    c = np.zeros((n, m))
    for k in range(K):
        v = T[k] + c
        S[k] = np.abs(v).max(axis=1) / 127.0
        Q[k] = fixed(v, S[k][:, None])
        c = v - value(S[k][:, None], Q[k])
    return S, Q


def quantise_columns(Y):
    """Y [n, nrhs] -> (column scales [nrhs], q [n, nrhs]); no carry."""
    s = np.abs(Y).max(axis=0) / 127.0
    return s, fixed(Y, s[None, :])


def pack(q, ld):
    """q [rows, cols] int64 (cols <= ld, ld a multiple of 64) -> digit planes in
    matrix-core operand order, rows padded to 16: byte
    ((i / 16 * ld / 64 + j / 64) * 4 + a) * 1024 + (i % 16 + 16 (j % 64 / 16)) * 16 + j % 16."""
    rows, cols = q.shape
    R = (rows + 15) // 16 * 16
    full = np.zeros((R, ld), dtype=np.int64)
    full[:rows, :cols] = q
    d = np.stack(split4(full)).astype(np.int8)                   # a, i, j
    d = d.reshape(4, R // 16, 16, ld // 64, 4, 16)                # a, rt, r, kc, g, e
    return np.ascontiguousarray(d.transpose(1, 3, 0, 4, 2, 5)).reshape(-1)


def block_bytes(scales, q, ld):
    """one stored block: digit planes then FP64 scales padded to 16 rows"""
    R = (q.shape[0] + 15) // 16 * 16
    sc = np.zeros(R)
    sc[:len(scales)] = scales
    return np.concatenate([pack(q, ld).view(np.uint8), sc.view(np.uint8)])


def slot_bytes(y_scales, yq, ld):
    """one ring slot from y digits [n, nrhs]: y^T digit planes then column scales"""
    return block_bytes(y_scales, np.ascontiguousarray(yq.T), ld)


def product(s_row, q_rows, s_col, q_cols):
    """sum_j T(i, j) y(j, n) as the matrix cores form it: exact digit products
    with a + b <= 4 grouped by weight, FP64 scaling."""
    t = [d.astype(np.float64) for d in split4(q_rows)]  # digit sums stay integers below 2^53
    u = [d.astype(np.float64) for d in split4(q_cols)]
    G = [np.zeros((q_rows.shape[0], q_cols.shape[1])) for _ in range(5)]
    for a, b in PAIRS:
        G[a + b] += t[a] @ u[b]
    g = G[4]
    for w in (3, 2, 1, 0):
        g = g * 2.0 ** -7 + G[w]
    return s_row[:, None] * s_col[None, :] * g


def dropped_bound(s_row, s_col, n):
    """bound on the digit products left out (a + b > 4): per entry
    n (2 * 64 * 64 * 2^-35 + 64 * 64 * 2^-42) s_row s_col"""
    return n * (2 * 4096 * 2.0 ** -35 + 4096 * 2.0 ** -42) * np.abs(s_row)[:, None] * np.abs(s_col)[None, :]
