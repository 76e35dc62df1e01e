"""Comparison of a reduced-precision product with the FP64 product: the
relative 2-norm over all entries, and per right-hand side both the relative
2-norm and the relative max-norm, so that one wrong leaf or column cannot
hide inside a global norm."""
import numpy as np


def reduced_errors(f, ref):
    """(all entries, worst column 2-norm, worst column max-norm), relative."""
    f = np.asarray(f, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    f2 = f.reshape(f.shape[0], -1)
    r2 = ref.reshape(ref.shape[0], -1)
    d = f2 - r2
    tot = float(np.linalg.norm(d) / np.linalg.norm(r2))
    col2 = np.linalg.norm(d, axis=0) / np.linalg.norm(r2, axis=0)
    colinf = np.abs(d).max(axis=0) / np.abs(r2).max(axis=0)
    return tot, float(col2.max()), float(colinf.max())


def assert_reduced_close(f, ref, tol):
    tot, c2, cinf = reduced_errors(f, ref)
    assert np.isfinite(tot) and np.isfinite(c2) and np.isfinite(cinf)
    assert tot <= tol, (tot, tol)
    assert c2 <= tol, (c2, tol)
    assert cinf <= tol, (cinf, tol)
