"""Plant plausible mistakes in the oracle (on the CPU) and check that at
least one pin catches each.  This shows the pins constrain the oracle, not
just that the oracle agrees with itself."""
import numpy as np
import pytest

from oracle import geometry, htlr, interp, tree
import test_oracle_basics as B
import test_oracle_htlr as H
import test_oracle_tree as T


def _fails(fn, *args, **kw):
    try:
        fn(*args, **kw)
    except AssertionError:
        return True
    return False


def test_transposed_core_is_caught(monkeypatch):
    orig = interp.core
    monkeypatch.setattr(interp, "core", lambda *a: orig(*a).T.copy())
    assert _fails(H.test_polynomial_kernel_is_exact, 2, 32, 4, 5, "uniform")


def test_swapped_modes_are_caught(monkeypatch):
    orig = htlr.HTLR.tlr_block

    def swapped(self, tau, sigma):
        U, V, G = orig(self, tau, sigma)
        return U, V[::-1], G
    monkeypatch.setattr(htlr.HTLR, "tlr_block", swapped)
    assert _fails(H.test_polynomial_kernel_is_exact, 2, 24, 3, 4, "warped")


def test_dropped_weight_is_caught(monkeypatch):
    orig = geometry.Grid.weights

    def weights(self, lin=None):
        w = orig(self, lin)
        return np.ones_like(w)
    monkeypatch.setattr(geometry.Grid, "weights", weights)
    assert _fails(H.test_constant_kernel_closed_form)


def test_wrong_diagonal_is_caught(monkeypatch):
    orig = geometry.diagonal
    monkeypatch.setattr(geometry, "diagonal", lambda *a, **k: 0.5 * orig(*a, **k))
    assert _fails(B.test_diagonal_constant_kernel_is_cell_volume)


def test_strict_admissibility_is_caught(monkeypatch, golden):
    def strict(self, tau, sigma):
        bt, bs = self.tree.box(tau), self.tree.box(sigma)
        return max(tree.diam2(bt), tree.diam2(bs)) < self.eta2 * tree.dist2(bt, bs)
    monkeypatch.setattr(tree.Admissibility, "__call__", strict)
    assert _fails(T.test_ties_are_admissible_exactly)


def test_garbled_lagrange_formula_is_caught(monkeypatch):
    """The basis as printed in Sec. 3.1 (t and j exchanged) is not a basis."""
    def printed(x, xi):
        x = np.asarray(x, dtype=np.float64)
        p = len(xi)
        L = np.ones((len(x), p))
        for t in range(p):
            for j in range(p):
                if j != t:
                    L[:, t] *= (x - xi[t]) / (xi[j] - xi[t])
        return L
    monkeypatch.setattr(interp, "lagrange_matrix", printed)
    assert _fails(B.test_lagrange_delta_and_partition_of_unity, 4)
    assert _fails(H.test_polynomial_kernel_is_exact, 2, 32, 4, 5, "uniform")


def test_wrong_chebyshev_points_are_caught(monkeypatch):
    def wrong(a, b, p):
        t = np.arange(1, p + 1)
        return 0.5 * (b - a) * np.cos(t * np.pi / (p + 1)) + 0.5 * (b + a)
    monkeypatch.setattr(interp, "chebyshev_points", wrong)
    assert _fails(B.test_chebyshev_points_are_roots_of_Tp, 5)
