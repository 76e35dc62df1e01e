"""Chebyshev interpolation and Tucker factors (test infrastructure).

Sec. 3.1 of the paper:

* 1D Chebyshev points of the first kind on [a, b]:
  xi_t = (b-a)/2 * cos((2t-1) pi / (2p)) + (b+a)/2,  t = 1..p.
* Lagrange basis L_t(x) = prod_{j != t} (x - xi_j) / (xi_t - xi_j).  The
  printed formula has the roles of t and j exchanged in the factors; this
  module uses the standard basis, the only reading with L_t(xi_s) = delta_ts.
* Factor matrices U_l(i, t) = L_t(x_{l;i}) and the core
  G(t, s) = k(xi_t, eta_s) over tensor Chebyshev points, multi-indices with
  the first component fastest (eq. 3.4).

Parity: pinned in tests/test_oracle_basics.py (points are the roots of T_p,
L_t(xi_s) = delta_ts, rows of U sum to one, exact reproduction of
polynomials of degree < p, interpolation error decaying in p as Thm. 3.4
predicts).
"""
from __future__ import annotations

import numpy as np

from . import kernels


def chebyshev_points(a: float, b: float, p: int) -> np.ndarray:
    t = np.arange(1, p + 1)
    return 0.5 * (b - a) * np.cos((2 * t - 1) * np.pi / (2 * p)) + 0.5 * (b + a)


def lagrange_matrix(x: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """L[i, t] = L_t(x_i) for the nodes xi."""
    x = np.asarray(x, dtype=np.float64)
    p = len(xi)
    L = np.ones((len(x), p))
    for t in range(p):
        for j in range(p):
            if j != t:
                L[:, t] *= (x - xi[j]) / (xi[t] - xi[j])
    return L


def tensor_points(node_lists) -> np.ndarray:
    """All tensor-product points of per-dimension node lists, shape (p^d, d),
    first index fastest."""
    mesh = np.meshgrid(*node_lists, indexing="ij")
    return np.stack([m.reshape(-1, order="F") for m in mesh], axis=1)


def core(kernel: str, xi_lists, eta_lists, p_kernel: int) -> np.ndarray:
    """G(t, s) = k(xi_t, eta_s), a p^d x p^d matrix (eq. 3.4)."""
    Xi = tensor_points(xi_lists)
    Eta = tensor_points(eta_lists)
    return kernels.evaluate(kernel, Xi[:, None, :], Eta[None, :, :], p_kernel)
