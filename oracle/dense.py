"""O1: dense brute-force Nystrom product (test infrastructure).

Computes eq. (1.3) row by row, in its quasi-uniform form (Sec. 3.3):

    f_i = a_i u_i + sum_j K_ij |Omega_j| u_j,
    K_ij = k(x_i, x_j) for j != i,   K_ii |Omega_i| = D_i (eq. 1.4),

with D_i from ``geometry.diagonal``.  No approximation: this is the operator
HTLR approximates.

Parity: pinned in tests/test_oracle_htlr.py (against closed forms for k = 1,
symmetry, and against a fully assembled matrix on tiny grids).
"""
from __future__ import annotations

import numpy as np

from . import geometry, kernels


def matvec(grid, kernel: str, p: int, a: np.ndarray, u: np.ndarray, rows=None,
           gl_order: int = 0, chunk: int = 16) -> np.ndarray:
    """Rows ``rows`` (default all) of A u, A the dense Nystrom matrix.

    u has shape (N,) or (N, nrhs); the result has shape (len(rows),) or
    (len(rows), nrhs).
    """
    rows = np.arange(grid.N) if rows is None else np.asarray(rows)
    U = u.reshape(grid.N, -1)
    X = grid.points()
    w = grid.weights()
    wu = w[:, None] * U
    D = geometry.diagonal(grid, kernel, p, gl_order, lin=rows)
    out = np.empty((len(rows), U.shape[1]))
    for c0 in range(0, len(rows), chunk):
        r = rows[c0:c0 + chunk]
        with np.errstate(divide="ignore", invalid="ignore"):
            K = kernels.evaluate(kernel, X[r][:, None, :], X[None, :, :], p)
        K[np.arange(len(r)), r] = 0.0                    # diagonal handled below
        out[c0:c0 + chunk] = K @ wu
    out += (a[rows] + D)[:, None] * U[rows]
    return out.reshape((len(rows),) + u.shape[1:])


def assemble(grid, kernel: str, p: int, a: np.ndarray, gl_order: int = 0) -> np.ndarray:
    """The full N x N matrix (tiny grids only)."""
    X = grid.points()
    w = grid.weights()
    with np.errstate(divide="ignore", invalid="ignore"):
        K = kernels.evaluate(kernel, X[:, None, :], X[None, :, :], p) * w[None, :]
    D = geometry.diagonal(grid, kernel, p, gl_order)
    K[np.diag_indices(grid.N)] = D + a
    return K
