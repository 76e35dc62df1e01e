"""Pins for the oracle's interpolation, kernels, grids and diagonal quadrature.

Everything here is checked against closed forms, library routines or the
paper's statements, never against the oracle itself.
"""
import math

import numpy as np
import pytest
from numpy.polynomial import chebyshev as C
from scipy import integrate

from oracle import geometry, interp, kernels


@pytest.mark.parametrize("p", [1, 2, 5, 8, 13])
def test_chebyshev_points_are_roots_of_Tp(p):
    xi = interp.chebyshev_points(-1.0, 1.0, p)
    Tp = C.Chebyshev.basis(p)
    assert np.max(np.abs(Tp(xi))) < 1e-12
    assert len(np.unique(np.round(xi, 14))) == p
    # mapped to [a, b]: affine image
    a, b = 0.25, 0.75
    assert np.allclose(interp.chebyshev_points(a, b, p), a + (xi + 1) * (b - a) / 2)


@pytest.mark.parametrize("p", [2, 4, 6, 8])
def test_lagrange_delta_and_partition_of_unity(p):
    xi = interp.chebyshev_points(0.0, 1.0, p)
    L = interp.lagrange_matrix(xi, xi)
    assert np.allclose(L, np.eye(p), atol=1e-13)
    x = np.linspace(-0.2, 1.2, 57)
    assert np.allclose(interp.lagrange_matrix(x, xi).sum(axis=1), 1.0, atol=1e-12)


@pytest.mark.parametrize("p", [3, 6, 8])
def test_polynomial_reproduction_degree_below_p(p):
    rng = np.random.default_rng(p)
    coef = rng.standard_normal(p)            # degree p-1
    xi = interp.chebyshev_points(0.3, 0.9, p)
    x = rng.uniform(0.3, 0.9, 40)
    approx = interp.lagrange_matrix(x, xi) @ np.polyval(coef, xi)
    assert np.allclose(approx, np.polyval(coef, x), rtol=0, atol=1e-12 * np.abs(coef).sum())
    # degree p is generally not reproduced
    coef2 = np.concatenate([[1.0], coef])
    approx2 = interp.lagrange_matrix(x, xi) @ np.polyval(coef2, xi)
    assert np.max(np.abs(approx2 - np.polyval(coef2, x))) > 1e-8


@pytest.mark.parametrize("p", [2, 4, 6, 8, 10])
def test_lemma_3_1_bound_1d(p):
    """Lemma 3.1 with d = 1.  The lemma is printed for p+1 interpolation points
    (degree p); with the p Chebyshev points of Sec. 3.1 the interpolant has
    degree p-1 and the bound reads 2 ((b-a)/4)^p ||f^(p)|| / p!."""
    a, b = 0.0, 1.5
    f = np.exp                                   # all derivatives equal exp
    xi = interp.chebyshev_points(a, b, p)
    x = np.linspace(a, b, 2001)
    err = np.max(np.abs(interp.lagrange_matrix(x, xi) @ f(xi) - f(x)))
    bound = 2 * ((b - a) / 4) ** p * math.exp(b) / math.factorial(p)
    assert err > 0.05 * bound             # and the bound is not vacuous
    assert err <= bound


def test_thm_3_4_error_decays_with_p():
    """Interpolated 1/r between two well separated 3D boxes: the error of
    the tensor interpolation of eq. (3.2) falls nearly exponentially in p."""
    errs = []
    for p in (2, 4, 6, 8):
        bt = [(0.0, 0.25)] * 3
        bs = [(0.5, 0.75), (0.0, 0.25), (0.5, 0.75)]
        xi = [interp.chebyshev_points(a, b, p) for a, b in bt]
        eta = [interp.chebyshev_points(a, b, p) for a, b in bs]
        G = interp.core("inv_r", xi, eta, p)
        rng = np.random.default_rng(0)
        X = rng.uniform(0, 0.25, (50, 3))
        Y = rng.uniform(0, 0.25, (50, 3)) + np.array([0.5, 0.0, 0.5])
        Lx = np.ones((50, p ** 3))
        Ly = np.ones((50, p ** 3))
        tp = interp.tensor_points([np.arange(p)] * 3).astype(int)
        for l in range(3):
            Lx *= interp.lagrange_matrix(X[:, l], xi[l])[:, tp[:, l]]
            Ly *= interp.lagrange_matrix(Y[:, l], eta[l])[:, tp[:, l]]
        approx = Lx @ G @ Ly.T
        exact = kernels.evaluate("inv_r", X[:, None, :], Y[None, :, :], p)
        errs.append(np.max(np.abs(approx - exact)) / np.max(np.abs(exact)))
    assert all(e2 < e1 / 5 for e1, e2 in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-6


def test_kernel_values_closed_form():
    x = np.array([0.1, 0.2, 0.3])
    y = np.array([0.4, 0.6, 0.3])                # |x-y| = 0.5
    assert kernels.evaluate("inv_r", x, y, 4) == pytest.approx(2.0, rel=1e-15)
    assert kernels.evaluate("neg_log", x, y, 4) == pytest.approx(math.log(2.0), rel=1e-15)
    assert kernels.evaluate("exp", x, y, 4) == pytest.approx(math.exp(-0.5), rel=1e-15)
    assert kernels.evaluate("gauss", x, y, 4) == pytest.approx(math.exp(-0.25 / 6), rel=1e-15)
    # p = 1 makes the polynomial test kernel the constant 1
    assert kernels.evaluate("poly_test", x, y, 1) == 1.0
    # factorisation over dimensions, degree p-1 in each variable
    v = kernels.evaluate("poly_test", x, y, 3)
    manual = (1 - 0.5 * 0.3) ** 2 * (1 - 0.3 * 0.4) ** 2 * 1.0
    assert v == pytest.approx(manual, rel=1e-14)
    # non-symmetric on purpose
    assert kernels.evaluate("poly_test", x, y, 3) != pytest.approx(kernels.evaluate("poly_test", y, x, 3))


def test_example_2_2_uniform_cells():
    n = 16
    g = geometry.uniform_grid(2, n)
    h = 1.0 / n
    i1, i2 = 5, 11                          # 1-based as in Example 2.2
    lin = (i1 - 1) + n * (i2 - 1)
    assert np.allclose(g.points([lin])[0], [(i1 - 1) * h + h / 2, (i2 - 1) * h + h / 2])
    assert g.edges[0][i1 - 1] == pytest.approx((i1 - 1) * h) and g.edges[0][i1] == pytest.approx(i1 * h)
    assert np.allclose(g.weights(), h * h)
    assert g.weights().sum() == pytest.approx(1.0)


def test_warped_cells_cover_and_contain_nodes():
    t = (np.arange(24) + 0.5) / 24
    x = t + 0.08 * np.sin(2 * np.pi * t) / (2 * np.pi)
    g = geometry.tensor_grid([x, x, x])
    e = g.edges[0]
    assert e[0] == 0.0 and e[-1] == 1.0 and np.all(np.diff(e) > 0)
    assert np.all((e[:-1] < x) & (x < e[1:]))
    assert g.weights().sum() == pytest.approx(1.0, rel=1e-13)


def test_diagonal_constant_kernel_is_cell_volume():
    x = np.sort(np.random.default_rng(3).uniform(0, 1, 10))
    g = geometry.tensor_grid([x, x ** 1.5])
    D = geometry.diagonal(g, "poly_test", 1)
    assert np.allclose(D, g.weights(), rtol=1e-14)


def test_diagonal_polynomial_exact():
    """poly_test with p = 3 is quadratic in each y_l: Gauss-Legendre of order 2
    already integrates it exactly; compare with the antiderivative
    -(1 + A (x - y))^3 / (3 A)."""
    t = (np.arange(7) + 0.5) / 7
    x = t + 0.05 * np.sin(2 * np.pi * t)
    g = geometry.tensor_grid([x, x, x])
    lin = np.arange(0, g.N, 17)
    for order in (2, 8):
        D = geometry.diagonal(g, "poly_test", 3, order=order, lin=lin)
        P = g.points(lin)
        idx = g.multi_index(lin)
        exact = np.ones(len(lin))
        for l in range(3):
            A = kernels.POLY_A[l]
            lo, hi = g.edges[l][idx[l]], g.edges[l][idx[l] + 1]
            F = lambda y: -(1 + A * (P[:, l] - y)) ** 3 / (3 * A)
            exact *= F(hi) - F(lo)
        assert np.allclose(D, exact, rtol=1e-13)


def _unit_cube_inv_r():
    # sum over the 6 faces of the pyramid integral a/(2|y|) over the face (a = 1/2)
    val, _ = integrate.dblquad(lambda s, t: 1.0 / math.sqrt(0.25 + s * s + t * t),
                               -0.5, 0.5, -0.5, 0.5, epsabs=1e-14, epsrel=1e-14)
    return 6 * 0.25 * val


def _unit_square_neg_log():
    # sum over the 4 edges of a*(1/4 - log|y|/2) integrated along the edge (a = 1/2)
    val, _ = integrate.quad(lambda s: 0.5 * (0.25 - 0.5 * math.log(math.sqrt(0.25 + s * s))),
                            -0.5, 0.5, epsabs=1e-15, epsrel=1e-15)
    return 4 * val


def test_cell_integral_constants(golden):
    ref = golden["cell_integrals"]
    assert _unit_cube_inv_r() == pytest.approx(ref["inv_r_unit_cube"], abs=1e-9)
    assert _unit_square_neg_log() == pytest.approx(ref["neg_log_unit_square"], abs=1e-9)


def test_diagonal_singular_converges(golden):
    ref = golden["cell_integrals"]
    h = 1.0 / 64
    g3 = geometry.uniform_grid(3, 64)
    exact3 = h * h * ref["inv_r_unit_cube"]
    errs3 = [abs(geometry.diagonal(g3, "inv_r", 6, order=o, lin=[777])[0] - exact3) / exact3
             for o in (4, 8, 16, 32)]
    g2 = geometry.uniform_grid(2, 64)
    exact2 = h * h * (ref["neg_log_unit_square"] - math.log(h))
    errs2 = [abs(geometry.diagonal(g2, "neg_log", 6, order=o, lin=[777])[0] - exact2) / exact2
             for o in (4, 8, 16, 32)]
    for errs in (errs3, errs2):
        assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert 5e-3 < errs3[1] < 3e-2          # the configured 8^3 rule
    assert errs2[2] < 1e-2                 # the configured 16^2 rule


def test_caller_cells():
    """Cells given as edges: Voronoi edges written out reproduce the default
    grid; the uniform edges with uniform nodes give weights h^d; any edges
    spanning [0, 1] give weights summing to 1; k = 1 gives |Omega_i| on every
    skewed cell; a polynomial integrand over skewed cells matches its
    antiderivative on those cells (and differs from the Voronoi cells' value)."""
    import htlr_workloads as W
    x = W.warped_nodes(10)
    g0 = geometry.tensor_grid([x, x])
    g1 = geometry.tensor_grid([x, x], edges=[W.split_edges(x, 0.5)] * 2)
    assert np.allclose(g0.weights(), g1.weights(), rtol=1e-13, atol=0)
    u = W.uniform_nodes(8)
    gu = geometry.tensor_grid([u, u, u], edges=[np.arange(9) / 8.0] * 3)
    assert np.allclose(gu.weights(), 8.0 ** -3, rtol=1e-15, atol=0)
    e1, e2 = W.split_edges(x, 0.3), W.split_edges(x, 0.8)
    gs = geometry.tensor_grid([x, x], edges=[e1, e2])
    assert abs(gs.weights().sum() - 1.0) < 1e-14
    assert not np.allclose(gs.weights(), g0.weights())
    assert np.allclose(geometry.diagonal(gs, "poly_test", 1), gs.weights(), rtol=1e-14, atol=0)
    lin = np.arange(gs.N)
    D = geometry.diagonal(gs, "poly_test", 3, lin=lin)
    P = gs.points(lin)
    idx = gs.multi_index(lin)
    exact = np.ones(len(lin))
    for l, e in enumerate((e1, e2)):
        A = kernels.POLY_A[l]
        F = lambda y: -(1 + A * (P[:, l] - y)) ** 3 / (3 * A)
        exact *= F(e[idx[l] + 1]) - F(e[idx[l]])
    assert np.allclose(D, exact, rtol=1e-13)
    assert not np.allclose(D, geometry.diagonal(g0, "poly_test", 3, lin=lin), rtol=1e-3)
