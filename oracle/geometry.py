"""Tensor grids, cells, weights and diagonal integrals (test infrastructure).

Follows the discretisation of Sec. 1 (eqs. 1.3-1.4) and its quasi-uniform
form (Sec. 3.3):

* Every point x_i owns a cell Omega_i; the cells do not overlap and cover
  [0,1]^d (Sec. 2.2, cells from Voronoi regions).  On a tensor grid the
  Voronoi cell of x_i is the product of 1D cells bounded by the midpoints
  between neighbouring nodes, with 0 and 1 at the ends.  On a uniform
  cell-centred grid (Example 2.2) these are exactly [(k-1)h, kh].
* The weight of x_j is |Omega_j| (h^d on a uniform grid, eq. 1.3).
* The diagonal entry K_ii * |Omega_i| is the integral of k(x_i, .) over
  Omega_i (eq. 1.4), "computed numerically": here by a tensor Gauss-Legendre
  rule mapped onto Omega_i (order 16 per dimension in 2D, 8 in 3D by
  default).  Gauss-Legendre of even order never samples the singular point.

Uniform grids also carry exact integer cell edges (in units of h) so that
admissibility ties (dist == diam) are decided exactly.

Parity: pinned in tests/test_oracle_basics.py (Example 2.2 cells, weights sum
to 1, k = 1 gives |Omega_i|, polynomial integrands exact, singular integrals
converge to library cubature values).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial.legendre import leggauss

from . import kernels


class Grid:
    """A tensor grid in [0,1]^d with per-dimension nodes and cell edges."""

    def __init__(self, nodes, uniform: bool, edges=None):
        self.d = len(nodes)
        self.nodes = [np.asarray(x, dtype=np.float64) for x in nodes]
        self.n = [len(x) for x in self.nodes]
        self.N = int(np.prod(self.n))
        self.uniform = uniform
        if uniform:
            # exact edges k/n, represented as integers k with denominator n
            self.int_edges = [np.arange(m + 1) for m in self.n]
            self.edges = [np.arange(m + 1) / m for m in self.n]
        elif edges is not None:
            # cells given by the caller: Omega_i is the product of the 1D
            # intervals [e_{l;k}, e_{l;k+1}] that hold the nodes (eq. 1.3)
            self.int_edges = None
            self.edges = [np.asarray(e, dtype=np.float64) for e in edges]
            for x, e in zip(self.nodes, self.edges):
                assert len(e) == len(x) + 1 and np.all(np.diff(e) > 0)
                assert np.all(e[:-1] <= x) and np.all(x <= e[1:])
        else:
            self.int_edges = None
            self.edges = []
            for x in self.nodes:
                e = np.empty(len(x) + 1)
                e[0], e[-1] = 0.0, 1.0
                e[1:-1] = 0.5 * (x[:-1] + x[1:])
                self.edges.append(e)
        self.cell_len = [np.diff(e) for e in self.edges]

    # natural order: i_1 fastest
    def multi_index(self, lin):
        lin = np.asarray(lin)
        idx = []
        for m in self.n:
            idx.append(lin % m)
            lin = lin // m
        return idx

    def linear_index(self, idx):
        lin = np.zeros_like(np.asarray(idx[0]))
        stride = 1
        for l in range(self.d):
            lin = lin + np.asarray(idx[l]) * stride
            stride *= self.n[l]
        return lin

    def points(self, lin=None) -> np.ndarray:
        lin = np.arange(self.N) if lin is None else np.asarray(lin)
        idx = self.multi_index(lin)
        return np.stack([self.nodes[l][idx[l]] for l in range(self.d)], axis=-1)

    def weights(self, lin=None) -> np.ndarray:
        """|Omega_j| = product of the 1D cell lengths."""
        lin = np.arange(self.N) if lin is None else np.asarray(lin)
        idx = self.multi_index(lin)
        w = np.ones(lin.shape)
        for l in range(self.d):
            w = w * self.cell_len[l][idx[l]]
        return w


def uniform_grid(d: int, n: int) -> Grid:
    x = (np.arange(n) + 0.5) / n
    return Grid([x] * d, uniform=True)


def tensor_grid(nodes, edges=None) -> Grid:
    """Tensor grid of the given nodes; cells from ``edges`` (one array of
    n_l + 1 increasing values per dimension) or, by default, the 1D Voronoi
    cells (midpoints between neighbouring nodes, 0 and 1 at the ends)."""
    return Grid(nodes, uniform=False, edges=edges)


def default_gl_order(d: int) -> int:
    return 16 if d == 2 else 8


def diagonal(grid: Grid, kernel: str, p: int, order: int = 0, lin=None) -> np.ndarray:
    """D_i = integral over Omega_i of k(x_i, y) dy by tensor Gauss-Legendre.

    This is K_ii * |Omega_i| in eq. (1.4) and its quasi-uniform form.
    """
    order = order or default_gl_order(grid.d)
    g, gw = leggauss(order)                       # nodes/weights on [-1, 1]
    lin = np.arange(grid.N) if lin is None else np.asarray(lin)
    idx = grid.multi_index(lin)
    X = grid.points(lin)
    out = np.empty(len(lin))
    # quadrature nodes per dimension, per point: y = lo + (g+1)/2 * len
    # tensor rule, first quadrature index fastest
    qidx = np.meshgrid(*([np.arange(order)] * grid.d), indexing="ij")
    qidx = [q.reshape(-1, order="F") for q in qidx]
    qw = np.ones(order ** grid.d)
    for l in range(grid.d):
        qw = qw * gw[qidx[l]]
    chunk = 4096
    for c0 in range(0, len(lin), chunk):
        sl = slice(c0, c0 + chunk)
        Y = np.empty((X[sl].shape[0], order ** grid.d, grid.d))
        jac = np.ones(X[sl].shape[0])
        for l in range(grid.d):
            lo = grid.edges[l][idx[l][sl]]
            ln = grid.cell_len[l][idx[l][sl]]
            Y[:, :, l] = lo[:, None] + 0.5 * (g[qidx[l]][None, :] + 1.0) * ln[:, None]
            jac = jac * 0.5 * ln
        vals = kernels.evaluate(kernel, X[sl][:, None, :], Y, p)
        out[sl] = jac * (vals @ qw)
    return out
