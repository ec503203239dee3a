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
