"""Learned warm start of the per-step T_0 solve (oracle; test infrastructure).

This is not part of the paper's method: the paper only writes the step as
T_0^{-1} applied to the history-corrected right-hand side (Sec. IV-B).  The
warm start guesses y_i from the four previous solutions before an iterative
solve refines it; whatever the guess, the refined y_i is the plain solve.

Features: the coefficients of y in the loop/star/harmonic decomposition of
the RWG span (Sec. II-D: a current in the span is Lambda l + Sigma s + H h).
Readings fixed here, identically on the GPU side:
  * s = (Sigma^T Sigma)^+ Sigma^T y and l = (Lambda^T Lambda)^+ Lambda^T y,
    the minimum-norm (zero-mean) coefficients, so Sigma s = P^Sigma y and
    Lambda l = P^Lambda y;
  * h = H^T y for an orthonormal basis H of the range of
    P^H = I - P^Sigma - P^Lambda (N_H = 2 x genus columns).  H is fixed only up
    to a rotation, so comparisons go through H h = P^H y;
  * feature vector f = [l (N_V), s (N_C), h (N_H)], N_V + N_C + N_H = N_E + 2.
Network (a 3-layer perceptron, tanh hidden units) on backward differences
of the features, each block scaled by its own rms:
  d0 = f_{i-1}, d1 = d0 - f_{i-2}, d2 = d1 - (f_{i-2} - f_{i-3}),
  d3 = f_{i-1} - 3 f_{i-2} + 3 f_{i-3} - f_{i-4},  rho_j = rms(d_j),
  x = [d0 / rho0, d1 / rho1, d2 / rho2, d3 / rho3]   (a zero block stays 0),
  a1 = tanh(W1 x + b1),  a2 = tanh(W2 a1 + b2),  o = W3 a2 + b3,
  guess  f_i ~ 3 f_{i-1} - 3 f_{i-2} + f_{i-3} + rho3 o   (a correction to
  quadratic extrapolation; o = 0 is plain quadratic extrapolation),
  loss = mean over samples and outputs of (o - t)^2 with
  t = (f_i - 3 f_{i-1} + 3 f_{i-2} - f_{i-3}) / rho3.
Optimiser: Adam with bias correction (Kingma and Ba, ICLR 2015).
"""
from __future__ import annotations

import numpy as np

from .operators import Projectors
from .topology import Topology


# ------------------------------------------------------------ loop/star coordinates
class LoopStar:
    """Loop/star/harmonic coordinates of vectors in the RWG span, FP64."""

    def __init__(self, topo: Topology, proj: Projectors | None = None):
        self.topo = topo
        self.proj = proj if proj is not None else Projectors(topo)
        self.S = topo.Sigma.toarray()
        self.L = topo.Lambda.toarray()
        PH = np.eye(topo.ne) - self.proj.PS - self.proj.PPL
        w, v = np.linalg.eigh(0.5 * (PH + PH.T))
        self.H = v[:, w > 0.5]  # eigenvalues of a projector are 0 or 1
        self.nv, self.nc, self.nh = topo.nv, topo.nc, self.H.shape[1]
        self.nf = self.nv + self.nc + self.nh

    def features(self, Y: np.ndarray) -> np.ndarray:
        """Y [n, N_E] -> F [n, N_V + N_C + N_H]."""
        Y = np.atleast_2d(Y)
        l = Y @ self.L @ self.proj.LL_pinv.T
        s = Y @ self.S @ self.proj.LS_pinv.T
        h = Y @ self.H
        return np.concatenate([l, s, h], axis=1)

    def reconstruct(self, F: np.ndarray) -> np.ndarray:
        F = np.atleast_2d(F)
        l, s, h = F[:, :self.nv], F[:, self.nv:self.nv + self.nc], F[:, self.nv + self.nc:]
        return l @ self.L.T + s @ self.S.T + h @ self.H.T


# ------------------------------------------------------------ training windows
def _rms(v: np.ndarray) -> float:
    return float(np.sqrt(np.mean(v * v)))


def window(F: np.ndarray, i: int):
    """Sample for step i (0-based row of F, i >= 4): x, t, rho3."""
    f1, f2, f3, f4 = F[i - 1], F[i - 2], F[i - 3], F[i - 4]
    d = [f1, f1 - f2, f1 - 2.0 * f2 + f3, f1 - 3.0 * f2 + 3.0 * f3 - f4]
    rho = [_rms(v) for v in d]
    x = np.concatenate([v / r if r > 0.0 else np.zeros_like(v) for v, r in zip(d, rho)])
    t = (F[i] - 3.0 * f1 + 3.0 * f2 - f3) / rho[3]
    return x, t, rho[3]


def guess(params, F: np.ndarray, i: int) -> np.ndarray:
    """Warm-start guess of the features of step i from rows i-1..i-4."""
    x, _, rho3 = window(F, i)
    o = forward(params, x[None, :])[0][0]
    return 3.0 * F[i - 1] - 3.0 * F[i - 2] + F[i - 3] + rho3 * o


# ------------------------------------------------------------ network
def init_params(n_in: int, hidden: int, n_out: int, rng: np.random.Generator, out_scale: float = 0.01):
    def glorot(o, i, scale=1.0):
        a = np.sqrt(6.0 / (i + o)) * scale
        return rng.uniform(-a, a, size=(o, i))
    return {"W1": glorot(hidden, n_in), "b1": np.zeros(hidden),
            "W2": glorot(hidden, hidden), "b2": np.zeros(hidden),
            "W3": glorot(n_out, hidden, out_scale), "b3": np.zeros(n_out)}


def forward(p, X: np.ndarray):
    """X [B, n_in] -> (o [B, n_out], cache)."""
    a1 = np.tanh(X @ p["W1"].T + p["b1"])
    a2 = np.tanh(a1 @ p["W2"].T + p["b2"])
    o = a2 @ p["W3"].T + p["b3"]
    return o, (X, a1, a2)


def loss_grad(p, X: np.ndarray, T: np.ndarray):
    """Mean squared error over samples and outputs, and its gradient."""
    o, (X, a1, a2) = forward(p, X)
    n = o.size
    e = o - T
    loss = float(np.sum(e * e) / n)
    do = 2.0 * e / n
    g = {"W3": do.T @ a2, "b3": do.sum(0)}
    dz2 = (do @ p["W3"]) * (1.0 - a2 * a2)
    g["W2"] = dz2.T @ a1
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ p["W2"]) * (1.0 - a1 * a1)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(0)
    return loss, g


def adam_step(p, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (step t >= 1) of every array in p, in place."""
    for k in p:
        m[k] = b1 * m[k] + (1.0 - b1) * g[k]
        v[k] = b2 * v[k] + (1.0 - b2) * g[k] * g[k]
        mh = m[k] / (1.0 - b1 ** t)
        vh = v[k] / (1.0 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
