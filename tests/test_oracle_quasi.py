"""Pins for the quasi-uniform oracle (T Khat S of Sec. 3.3, eq. 3.9)."""
import numpy as np
import pytest
from numpy.polynomial.legendre import leggauss

import htlr_workloads as W
from oracle import dense, geometry, kernels, quasi


def _skewed(n, c):
    """Quasi-uniform nodes t + c (cos(2 pi t) - 1), t the cell centres: unlike
    a sine warp, not symmetric about 1/2, so a reversed or shifted index fails."""
    t = W.uniform_nodes(n)
    return t + c * (np.cos(2 * np.pi * t) - 1)


def _warped(d, n):
    return geometry.tensor_grid([_skewed(n, 0.03)] * d)


def _aniso():
    """A 12 x 10 grid warped differently in each dimension."""
    return geometry.tensor_grid([_skewed(12, 0.03), _skewed(10, -0.025)])


@pytest.mark.parametrize("n,m", [(12, 16), (20, 8), (16, 16)])
def test_rows_sum_to_one(n, m):
    """The cells of each grid tile [0, 1], so every row of S and of T is a
    partition of its cell's length: the rows sum to 1."""
    eq = _warped(1, n).edges[0]
    eu = np.arange(m + 1) / m
    assert np.allclose(quasi.s_1d(eq, eu).sum(axis=1), 1.0, atol=1e-15)
    assert np.allclose(quasi.t_1d(eq, eu).sum(axis=1), 1.0, atol=1e-15)


@pytest.mark.parametrize("d,n,m", [(2, 12, 16), (3, 6, 8), (2, 20, 8), (2, 0, 16)])
def test_integral_is_conserved(d, n, m):
    """S and T preserve the integral of the piecewise-constant function:
    sum_t |Omega_t| (S u)_t = sum_i |Omega_i| u_i, and the same for T
    (n = 0: the anisotropic 12 x 10 grid)."""
    gq = _warped(d, n) if n else _aniso()
    gu = geometry.uniform_grid(d, m)
    rng = np.random.default_rng(0)
    u = rng.standard_normal(gq.N)
    v = rng.standard_normal(gu.N)
    assert abs(gu.weights() @ quasi.s_apply(gq, m, u) - gq.weights() @ u) < 1e-13
    assert abs(gq.weights() @ quasi.t_apply(gq, m, v) - gu.weights() @ v) < 1e-13


def test_coincident_grids_reproduce_the_uniform_product():
    """A quasi-uniform grid that is the uniform grid itself: S = T = I, so the
    scheme is the uniform product exactly (against the dense O1)."""
    d, n = 2, 16
    g = geometry.uniform_grid(d, n)
    gq = geometry.tensor_grid(g.nodes)                 # same nodes, edges from midpoints
    eu = np.arange(n + 1) / n
    assert np.allclose(quasi.s_1d(gq.edges[0], eu), np.eye(n), atol=1e-15)
    a = 1.0 + 0.5 * g.points()[:, 0]
    u = np.random.default_rng(1).standard_normal(g.N)
    f = quasi.matvec(gq, n, "neg_log", 6, 4, a, u, khat="dense")
    ref = dense.matvec(g, "neg_log", 6, a, u)
    assert np.linalg.norm(f - ref) / np.linalg.norm(ref) < 1e-13


def _galerkin(gq, kernel, p, u, q=4):
    """The m -> infinity limit of T Khat S u, computed independently: the
    Galerkin operator (G u)_i = |Omega_i|^-1 int_{Omega_i} int k(x, y) u(y) dy dx,
    u piecewise constant on the quasi-uniform cells; tensor Gauss-Legendre
    with q points per dimension in every cell (smooth kernels only)."""
    t, w = leggauss(q)
    idx = gq.multi_index(np.arange(gq.N))
    pts, wts, owner = [], [], []
    for c in range(gq.N):
        lo = [gq.edges[l][idx[l][c]] for l in range(gq.d)]
        hi = [gq.edges[l][idx[l][c] + 1] for l in range(gq.d)]
        xs = [0.5 * (lo[l] + hi[l]) + 0.5 * (hi[l] - lo[l]) * t for l in range(gq.d)]
        ws = [0.5 * (hi[l] - lo[l]) * w for l in range(gq.d)]
        pts.append(np.stack(np.meshgrid(*xs, indexing="ij"), -1).reshape(-1, gq.d))
        wts.append(np.prod(np.stack(np.meshgrid(*ws, indexing="ij"), -1).reshape(-1, gq.d), axis=1))
        owner.append(np.full(q ** gq.d, c))
    pts, wts, owner = np.concatenate(pts), np.concatenate(wts), np.concatenate(owner)
    g = kernels.evaluate(kernel, pts[:, None], pts[None], p) @ (wts * u[owner])
    return np.bincount(owner, weights=wts * g) / gq.weights()


def test_converges_to_the_galerkin_operator():
    """As the uniform grid is refined, S u resolves the piecewise-constant u,
    Khat S u samples its integral at the uniform centres and T averages that
    over each quasi-uniform cell: T Khat S u tends to the Galerkin cell-average
    operator.  Anisotropic grid (different n and warp per dimension) and a
    non-symmetric u, so a swapped mode or a transposed factor fails."""
    gq = _aniso()
    X = gq.points()
    u = 1 + 0.5 * np.exp(-(X[:, 0] - 0.3) ** 2 - (X[:, 1] - 0.6) ** 2) + np.sin(5 * X[:, 0] * X[:, 1])
    ref = _galerkin(gq, "gauss", 6, u)
    errs = [np.linalg.norm(quasi.matvec(gq, m, "gauss", 6, 4, np.zeros(gq.N), u, khat="dense") - ref)
            / np.linalg.norm(ref) for m in (8, 16, 32, 64)]
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[3] < errs[0] / 20
    # and not to the Nystrom product at the quasi-uniform points themselves
    # (the nodes are not the centres of their cells)
    nys = dense.matvec(gq, "gauss", 6, np.zeros(gq.N), u)
    assert np.linalg.norm(nys - ref) / np.linalg.norm(ref) > 10 * errs[3]


def test_htlr_khat_matches_dense_khat():
    """With an exact (polynomial) kernel the HTLR Khat equals the dense one,
    so the two forms of the oracle agree to rounding."""
    d, n, m, p = 2, 12, 16, 4
    gq = _warped(d, n)
    a = np.linspace(0.5, 1.5, gq.N)
    u = np.random.default_rng(2).standard_normal(gq.N)
    f1 = quasi.matvec(gq, m, "poly_test", p, 4, a, u, khat="htlr")
    f2 = quasi.matvec(gq, m, "poly_test", p, 4, a, u, khat="dense")
    assert np.linalg.norm(f1 - f2) / np.linalg.norm(f2) < 1e-12


def test_columns_are_independent():
    """Several right-hand sides: each column is transformed as if alone (up
    to the rounding of a matrix-matrix against a matrix-vector product)."""
    gq = _aniso()
    U = np.asfortranarray(np.random.default_rng(3).standard_normal((gq.N, 3)))
    a = np.linspace(0.5, 1.5, gq.N)
    F = quasi.matvec(gq, 16, "exp", 4, 4, a, U, khat="dense")
    for r in range(3):
        f = quasi.matvec(gq, 16, "exp", 4, 4, a, U[:, r].copy(), khat="dense")
        assert np.linalg.norm(F[:, r] - f) <= 1e-14 * np.linalg.norm(f)
