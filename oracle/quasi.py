"""The HTLR product on a quasi-uniform grid through a uniform one (test
infrastructure).

Sec. 3.3 approximates the Nystrom matrix A of a quasi-uniform grid by
T Ahat S (eq. 3.9): S interpolates a vector from the quasi-uniform cells
Omega_i to the cells Omega_t of a uniform grid of M = m^d cells, Ahat is
the uniform-grid matrix (applied as an HTLR matrix), and T interpolates back.
Reading a vector as a piecewise-constant function and projecting (Galerkin)
gives the overlap matrices

    S[t, i] = |Omega_t^uni  cap Omega_i^quasi| / |Omega_t^uni|,
    T[i, t] = |Omega_i^quasi cap Omega_t^uni|  / |Omega_i^quasi|.

On a tensor grid the cells are products of 1D intervals, so S and T are
Kronecker products of 1D overlap matrices (one per dimension).

Reading: the term a(x_i) u_i is applied on the quasi-uniform grid itself (a
is given at its points and needs no interpolation); T Ahat S approximates the
integral part, so Ahat is the uniform matrix with a = 0 (its diagonal
integrals D included):

    f = a o u + T Khat S u.

Parity: pinned in tests/test_oracle_quasi.py (rows of S and T sum to 1,
both conserve the integral sum_i |Omega_i| u_i, coincident grids reproduce
the uniform product exactly, the error against the dense quasi-uniform
product falls as m grows).
"""
from __future__ import annotations

import numpy as np

from . import dense, geometry, htlr


def overlap_1d(e_quasi: np.ndarray, e_uni: np.ndarray) -> np.ndarray:
    """O[t, i] = length of [e_uni[t], e_uni[t+1]] cap [e_quasi[i], e_quasi[i+1]]."""
    lo = np.maximum(e_uni[:-1, None], e_quasi[None, :-1])
    hi = np.minimum(e_uni[1:, None], e_quasi[None, 1:])
    return np.maximum(hi - lo, 0.0)


def s_1d(e_quasi, e_uni) -> np.ndarray:
    """1D factor of S (m x n): overlaps divided by the uniform cell lengths."""
    return overlap_1d(e_quasi, e_uni) / np.diff(e_uni)[:, None]


def t_1d(e_quasi, e_uni) -> np.ndarray:
    """1D factor of T (n x m): overlaps divided by the quasi-uniform cell lengths."""
    return overlap_1d(e_quasi, e_uni).T / np.diff(e_quasi)[:, None]


def _kron_apply(mats, x: np.ndarray, n_in) -> np.ndarray:
    """Apply per-dimension matrices to a vector in natural order (first index
    fastest): returns (mats[d-1] x ... x mats[0]) x, column by column for an
    (N, nrhs) array."""
    cols = x.shape[1:]
    X = x.reshape(tuple(n_in) + cols, order="F")
    for l, Mt in enumerate(mats):
        X = np.moveaxis(np.tensordot(Mt, X, axes=([1], [l])), 0, l)
    return X.reshape((-1,) + cols, order="F")


def s_apply(gq: geometry.Grid, m: int, u: np.ndarray) -> np.ndarray:
    eu = np.arange(m + 1) / m
    return _kron_apply([s_1d(gq.edges[l], eu) for l in range(gq.d)], u, gq.n)


def t_apply(gq: geometry.Grid, m: int, v: np.ndarray) -> np.ndarray:
    eu = np.arange(m + 1) / m
    return _kron_apply([t_1d(gq.edges[l], eu) for l in range(gq.d)], v, [m] * gq.d)


def matvec(gq: geometry.Grid, m: int, kernel: str, p: int, leaf: int, a: np.ndarray, u: np.ndarray,
           khat: str = "htlr", **htlr_kw) -> np.ndarray:
    """f = a o u + T Khat S u, Khat on the uniform m^d grid (a = 0): the HTLR
    oracle O2 (khat="htlr") or the dense product O1 (khat="dense").  u has
    shape (N,) or (N, nrhs)."""
    gu = geometry.uniform_grid(gq.d, m)
    uh = s_apply(gq, m, u)
    zero = np.zeros(gu.N)
    if khat == "dense":
        fh = dense.matvec(gu, kernel, p, zero, uh)
    else:
        fh = htlr.HTLR(gu, kernel, p, leaf, zero, **htlr_kw).matvec(uh)
    return a.reshape((-1,) + (1,) * (u.ndim - 1)) * u + t_apply(gq, m, fh)
