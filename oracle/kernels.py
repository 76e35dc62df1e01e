"""Kernel functions k(x, y) (test infrastructure, see oracle/__init__.py).

The paper's experiments (Sec. 5) use a Gaussian kernel with bandwidth sqrt(d)
and single-layer-potential kernels (-log r in 2D, 1/r in 3D).  The workloads
use the unnormalised forms 1/r, -log r and exp(-r).  ``poly_test`` is
prod_l (1 + A_l (x_l - y_l))^(p-1), a polynomial of degree p-1 in every
coordinate of x and of y; Chebyshev interpolation with p points per
dimension reproduces it exactly (Lemma 3.1: the error bound vanishes), which
pins the whole far field.  It is deliberately anisotropic and non-symmetric
so that swapped modes or a transposed core change the result.

Parity: pinned by closed-form values in tests/test_oracle_basics.py.
"""
import numpy as np

# Coefficients of the polynomial test kernel, per dimension.
POLY_A = (0.50, 0.30, 0.20)


def evaluate(name: str, X: np.ndarray, Y: np.ndarray, p: int) -> np.ndarray:
    """k(X, Y) for broadcastable point arrays X, Y of shape (..., d)."""
    diff = X - Y
    if name in ("inv_r", "neg_log", "exp", "gauss"):
        r2 = np.sum(diff * diff, axis=-1)
        if name == "inv_r":
            return 1.0 / np.sqrt(r2)
        if name == "neg_log":
            return -0.5 * np.log(r2)
        if name == "exp":
            return np.exp(-np.sqrt(r2))
        d = X.shape[-1]
        return np.exp(-r2 / (2.0 * d))          # sigma^2 = d
    if name == "poly_test":
        d = X.shape[-1]
        out = 1.0
        for l in range(d):
            out = out * (1.0 + POLY_A[l] * diff[..., l]) ** (p - 1)
        return out
    raise ValueError(f"unknown kernel {name}")
