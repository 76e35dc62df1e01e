"""O3: reference solvers for A u = f (test infrastructure).

The paper covers only construction and products; solving A u = f is the
"backward evaluation" of Sec. 1 (eq. 1.2).  The references here are:

* ``direct``: numpy.linalg.solve on an assembled matrix (tiny grids);
* ``gmres``: textbook restarted GMRES(m) (Saad & Schultz), x0 = 0, modified
  Gram-Schmidt Arnoldi and Givens rotations, stopping on the true relative
  residual ||f - A x|| / ||f||.

Parity: ``gmres`` is pinned against ``direct`` on tiny grids in
tests/test_oracle_htlr.py.
"""
from __future__ import annotations

import numpy as np


def direct(A: np.ndarray, f: np.ndarray) -> np.ndarray:
    return np.linalg.solve(A, f)


def gmres(matvec, f: np.ndarray, restart: int = 30, tol: float = 1e-10,
          max_restarts: int = 100):
    """Returns (x, relative residual, total inner iterations)."""
    N = f.shape[0]
    x = np.zeros(N)
    fn = np.linalg.norm(f)
    if fn == 0.0:
        return x, 0.0, 0
    iters = 0
    for _ in range(max_restarts):
        r = f - matvec(x)
        beta = np.linalg.norm(r)
        if beta / fn <= tol:
            return x, beta / fn, iters
        V = np.zeros((N, restart + 1))
        Hm = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[:, 0] = r / beta
        k_used = 0
        for k in range(restart):
            w = matvec(V[:, k])
            for j in range(k + 1):
                Hm[j, k] = V[:, j] @ w
                w = w - Hm[j, k] * V[:, j]
            Hm[k + 1, k] = np.linalg.norm(w)
            if Hm[k + 1, k] > 0:
                V[:, k + 1] = w / Hm[k + 1, k]
            for j in range(k):
                t = cs[j] * Hm[j, k] + sn[j] * Hm[j + 1, k]
                Hm[j + 1, k] = -sn[j] * Hm[j, k] + cs[j] * Hm[j + 1, k]
                Hm[j, k] = t
            den = np.hypot(Hm[k, k], Hm[k + 1, k])
            cs[k], sn[k] = Hm[k, k] / den, Hm[k + 1, k] / den
            Hm[k, k] = den
            Hm[k + 1, k] = 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k] * g[k]
            iters += 1
            k_used = k + 1
            if abs(g[k + 1]) / fn <= tol:
                break
        y = np.linalg.solve(np.triu(Hm[:k_used, :k_used]), g[:k_used])
        x = x + V[:, :k_used] @ y
    r = f - matvec(x)
    return x, np.linalg.norm(r) / fn, iters
