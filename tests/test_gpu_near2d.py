"""The 2D uniform-grid near field with row reuse (leaves of 8 or 16 points
per side, radial kernels) against the generic uniform-grid kernel, forced
through the tuner's cache file, and against the O2 oracle."""
import sys

import numpy as np
import pytest

import htlr_workloads as W
from oracle import geometry, htlr

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _product(torch, M, u, prec):
    dt = torch.float64 if prec == "fp64" else torch.float32
    ut = torch.tensor(u.T.copy(), dtype=dt, device="cuda").t() if u.ndim == 2 else torch.tensor(u, dtype=dt,
                                                                                                  device="cuda")
    f = M.matvec(ut, prec=prec)
    torch.cuda.synchronize()
    return f.double().cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("n,leaf,p,kernel,adm,eta2,nrhs", [
    (64, 16, 8, "neg_log", "strong", 2.0, 1),     # the 2D tables' leaf and rank
    (64, 16, 6, "gauss", "weak", 1.0, 3),
    (64, 8, 6, "inv_r", "strong", 1.0, 5),
    (128, 16, 8, "exp", "strong", 2.0, 2)])
def test_rows2d_matches_generic_and_oracle(torch, tmp_path, monkeypatch, prec, n, leaf, p, kernel, adm, eta2, nrhs):
    import paper_2508_05958_amd as H
    _say(f"[gpu] 2D near rows n={n} leaf={leaf} {kernel} {adm} nrhs={nrhs} {prec}")
    g = geometry.uniform_grid(2, n)
    a = 1.0 + 0.5 * g.points()[:, 0]
    rng = np.random.default_rng(31)
    u = rng.standard_normal(g.N) if nrhs == 1 else rng.standard_normal((g.N, nrhs))
    M = H.htlr_build(None, kernel, 2, n, p, leaf, a=a, eta2=eta2, admissibility=adm)
    f_rows = _product(torch, M, u, prec)
    # the generic kernel, forced through the cache
    pid = {"fp64": 0, "fp32": 1, "bf16": 2}[prec]
    kid = W.KERNEL_IDS[kernel]
    cache = tmp_path / "tune.txt"
    key = f"d2_n{n}_p{p}_leaf{leaf}_k{kid}_uniform_eta{eta2:g}_adm{0 if adm == 'strong' else 1}_nrhs{nrhs}_prec{pid}"
    cache.write_text(f"{key} 2048 3 0 0 0 0 0 0 0 1.0 1.0\n")
    monkeypatch.setenv("HTLR_TUNE_CACHE", str(cache))
    M2 = H.htlr_build(None, kernel, 2, n, p, leaf, a=a, eta2=eta2, admissibility=adm)
    assert M2.autotune(nrhs, prec)["candidates"] == 0
    f_gen = _product(torch, M2, u, prec)
    assert _rel(f_rows, f_gen) <= (1e-14 if prec == "fp64" else 1e-5)
    if prec == "fp64":
        O = htlr.HTLR(g, kernel, p, leaf, a, adm_kind=adm, eta2=eta2)
        leaves = O.tree.leaves()
        pick = [leaves[i] for i in W.sample_leaves(n, len(leaves), 4)]
        assert _rel(f_rows[O.leaf_rows(pick)], O.matvec(u, pick)) <= 1e-12
