"""Marching-on-in-time and post-processing (oracle; test infrastructure).

Sec. IV-B: y_i = T_0^{-1} (r_i - sum_{k=1}^{i-1} T_k y_{i-k}), with T_k = 0 for
k > K; this is block forward substitution of the lower-triangular Toeplitz
system eq. dis_TD_CFIE.  T_0^{-1} is applied through an LU factorisation with
partial pivoting (the paper does not say how T_0 is inverted).
Eq. post_processing: j_i = P^{LH} y_i + dt~^-1 P^Sigma (y_i - y_{i-1}), y_0 = 0.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def march(T: np.ndarray, r: np.ndarray) -> np.ndarray:
    """T [K+1, n, n], r [n_steps, n] (or [n_steps, n, B]) -> y [n_steps, ...]
    (y[i-1] holds y_i)."""
    K = T.shape[0] - 1
    lu = sla.lu_factor(T[0])
    y = np.zeros_like(r)
    for i in range(1, r.shape[0] + 1):
        b = r[i - 1].copy()
        for k in range(1, min(i - 1, K) + 1):
            b -= T[k] @ y[i - k - 1]
        y[i - 1] = sla.lu_solve(lu, b)
    return y


def history_sum(T: np.ndarray, ring: list, i: int) -> np.ndarray:
    """sum_{k=1}^{min(i-1,K)} T_k y_{i-k} with ring[k-1] = y_{i-k}."""
    K = T.shape[0] - 1
    acc = np.zeros(T.shape[1:2] + np.shape(ring[0])[1:])
    for k in range(1, min(i - 1, K) + 1):
        acc = acc + T[k] @ ring[k - 1]
    return acc


def history_sum_factored(A, B, C, PLH, PS, dtn, PE, PM, ring: list) -> np.ndarray:
    """sum_{k=1}^{K} T_k y_{i-k} from the raw lag matrices A_k, B_k, C_k
    (k = 0..K) and the preconditioners, without forming T_k (Sec. IV-A:
    T_k = P_E W^E_k + P_M W^M_k, W^E_k = A_k P^{LH} + (A_k - A_{k-1})/dt~ P^Sigma
    + B_k, W^M_k = C_k P^{LH} + (C_k - C_{k-1})/dt~ P^Sigma).  The difference
    of consecutive lag matrices is moved onto the history by summation by
    parts: with u_j = P^{LH} y_j, v_j = P^Sigma y_j, d_j = v_j - v_{j-1},
      sum_k (A_k - A_{k-1}) v_{i-k} = sum_k A_k d_{i-k} + A_K v_{i-K-1} - A_0 v_{i-1},
    so that
      E = sum_k [A_k (u_{i-k} + d_{i-k}/dt~) + B_k y_{i-k}] + (A_K v_{i-K-1} - A_0 v_{i-1})/dt~
      M = sum_k C_k (u_{i-k} + d_{i-k}/dt~) + (C_K v_{i-K-1} - C_0 v_{i-1})/dt~
    and the sum is P_E E + P_M M.  ring[k-1] = y_{i-k} for k = 1..K+1 (zero
    vectors before the first step)."""
    K = len(A) - 1
    if len(ring) < K + 1:
        raise ValueError("the factored history needs y_{i-1} .. y_{i-K-1}")
    u = [PLH @ y for y in ring[:K + 1]]
    v = [PS @ y for y in ring[:K + 1]]
    E = np.zeros(A[0].shape[:1] + np.shape(ring[0])[1:])
    M = np.zeros_like(E)
    for k in range(1, K + 1):
        w = u[k - 1] + (v[k - 1] - v[k]) / dtn
        E = E + A[k] @ w + B[k] @ ring[k - 1]
        M = M + C[k] @ w
    E = E + (A[K] @ v[K] - A[0] @ v[0]) / dtn
    M = M + (C[K] @ v[K] - C[0] @ v[0]) / dtn
    return PE @ E + PM @ M


def companion_radius(T: np.ndarray) -> float:
    """Spectral radius of the block companion matrix of the march
    y_i = -T_0^{-1} sum_{k=1}^{K} T_k y_{i-k} (Sec. IV-B with r = 0): the
    largest |lambda| with det(sum_k lambda^{K-k} T_k) = 0.  Dense eigenvalues;
    small meshes only."""
    K, n = T.shape[0] - 1, T.shape[1]
    T0i = np.linalg.inv(T[0])
    comp = np.zeros((K * n, K * n))
    for k in range(1, K + 1):
        comp[:n, (k - 1) * n:k * n] = -T0i @ T[k]
    comp[n:, :-n] = np.eye((K - 1) * n)
    return float(np.abs(np.linalg.eigvals(comp)).max())


def condition_1(A: np.ndarray) -> float:
    """1-norm condition number |A|_1 |A^{-1}|_1 (largest absolute column sum)."""
    return float(np.abs(A).sum(axis=0).max() * np.abs(np.linalg.inv(A)).sum(axis=0).max())


def condition_2(A: np.ndarray) -> float:
    """2-norm condition number sigma_max / sigma_min (singular values by SVD)."""
    sv = np.linalg.svd(A, compute_uv=False)
    return float(sv[0] / sv[-1])


def block_solve(T: np.ndarray, r: np.ndarray) -> np.ndarray:
    """Direct dense solve of the full block lower-triangular system."""
    K = T.shape[0] - 1
    n = T.shape[1]
    N = r.shape[0]
    big = np.zeros((N * n, N * n))
    for i in range(N):
        for k in range(0, min(i, K) + 1):
            big[i * n:(i + 1) * n, (i - k) * n:(i - k + 1) * n] = T[k]
    return np.linalg.solve(big, r.reshape(N * n, -1)).reshape(r.shape)


def currents(PLH: np.ndarray, PS: np.ndarray, dtn: float, y: np.ndarray) -> np.ndarray:
    prev = np.concatenate([np.zeros_like(y[:1]), y[:-1]], axis=0)
    return np.einsum("mn,in...->im...", PLH, y) + np.einsum("mn,in...->im...", PS, y - prev) / dtn
