"""htlr_matvec_noalloc: the product with its work buffers in the library's
fixed device scratch, checked against htlr_matvec (which allocates its own)
on two calls in a row, the second with a smaller input, and against the
FP64 HTLR oracle on the small one; sizes beyond the scratch are refused."""
import sys

import numpy as np
import pytest

from oracle import geometry, htlr

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _cols(torch, u):
    """(N, nrhs) host array -> column-major CUDA tensor."""
    return torch.tensor(u.T.copy(), device="cuda").t()


def _rel_cols(a, b):
    a = np.asarray(a).reshape(a.shape[0], -1)
    b = np.asarray(b).reshape(b.shape[0], -1)
    return max(np.linalg.norm(a[:, c] - b[:, c]) / np.linalg.norm(b[:, c]) for c in range(b.shape[1]))


def test_noalloc_matches_matvec_two_calls(torch):
    import paper_2508_05958_amd as H
    # first call: 3D n = 32, p = 6, leaves of 8^3, four right-hand sides
    d, n, p, leaf, nrhs = 3, 32, 6, 8, 4
    g = geometry.uniform_grid(d, n)
    a = 1.0 + 0.5 * g.points()[:, 0]
    u = np.random.default_rng(11).standard_normal((g.N, nrhs))
    _say(f"[gpu] noalloc call 1: d={d} n={n} p={p} nrhs={nrhs} fp64 + fp32")
    M = H.htlr_build(None, "inv_r", d, n, p, leaf, a=a)
    u64 = _cols(torch, u)
    want = M.matvec(u64, prec="fp64")
    got = torch.full_like(want, float("nan"))
    M.matvec_noalloc(u64, got, prec="fp64")
    u32 = u64.float().t().contiguous().t()
    want32 = M.matvec(u32, prec="fp32")
    got32 = torch.full_like(want32, float("nan"))
    M.matvec_noalloc(u32, got32, prec="fp32")
    torch.cuda.synchronize()
    w, gg = want.cpu().numpy(), got.cpu().numpy()
    rel = _rel_cols(gg, w)
    rel32 = _rel_cols(got32.double().cpu().numpy(), w)
    rel32m = _rel_cols(want32.double().cpu().numpy(), w)
    _say(f"[gpu]   fp64 noalloc vs matvec {rel:.2e}; fp32 noalloc vs fp64 {rel32:.2e} (matvec fp32 {rel32m:.2e})")
    assert np.isfinite(gg).all()
    assert rel <= 1e-12
    assert rel32 <= 1e-5
    M.free()

    # second call right after: a smaller input (2D n = 32, one right-hand side)
    d, n, p, leaf = 2, 32, 5, 4
    g = geometry.uniform_grid(d, n)
    a = 1.0 + 0.5 * g.points()[:, 0]
    u = np.random.default_rng(12).standard_normal(g.N)
    _say(f"[gpu] noalloc call 2: d={d} n={n} p={p} nrhs=1 fp64")
    M = H.htlr_build(None, "neg_log", d, n, p, leaf, a=a)
    ut = torch.tensor(u, device="cuda")
    want = M.matvec(ut, prec="fp64")
    got = torch.full_like(want, float("nan"))
    M.matvec_noalloc(ut, got, prec="fp64")
    torch.cuda.synchronize()
    w, gg = want.cpu().numpy(), got.cpu().numpy()
    fo = htlr.HTLR(g, "neg_log", p, leaf, a).matvec(u)
    rel = np.linalg.norm(gg - w) / np.linalg.norm(w)
    relo = np.linalg.norm(gg - fo) / np.linalg.norm(fo)
    _say(f"[gpu]   noalloc vs matvec {rel:.2e}, vs oracle {relo:.2e}")
    assert np.isfinite(gg).all()
    assert rel <= 1e-12
    assert relo <= 1e-12
    M.free()


def test_noalloc_refuses_work_beyond_scratch(torch):
    import paper_2508_05958_amd as H
    # 64^3, p = 6, 64 right-hand sides: the level-3 source and output tensors
    # alone take 2 x 512 x 64 x 216 x 8 bytes = 113 MB > 64 MiB
    _say("[gpu] noalloc: 64^3 x 64 right-hand sides is refused")
    M = H.htlr_build(None, "inv_r", 3, 64, 6, 8)
    u = torch.zeros((64, M.N), dtype=torch.float64, device="cuda").t()
    f = torch.zeros_like(u)
    with pytest.raises(H.HTLRError, match="exceed the fixed scratch"):
        M.matvec_noalloc(u, f, prec="fp64")
    M.free()
