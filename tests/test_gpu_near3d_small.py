"""The 3D uniform-grid near field for leaves of 4 x 4 x 4 points (radial
kernels; the paper's 3D shapes) against the row kernel it replaces, forced
through the tuner's cache file, and against the O2 oracle on sampled leaves."""
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
@pytest.mark.parametrize("n,p,kernel,adm,eta2,nrhs", [
    (32, 4, "inv_r", "strong", 3.0, 1),       # Table 5.4's kernel, rank, leaf and eta
    (32, 4, "gauss", "weak", 1.0, 3),         # Table 5.3's
    (16, 5, "exp", "strong", 1.0, 5),
    (32, 4, "inv_r", "strong", 1.0, 9)])
def test_rows3d_matches_row_kernel_and_oracle(torch, tmp_path, monkeypatch, prec, n, p, kernel, adm, eta2, nrhs):
    import paper_2508_05958_amd as H
    leaf = 5                                   # 32 -> 16 -> 8 -> 4: leaves of 4^3 points
    _say(f"[gpu] 3D small-leaf near n={n} {kernel} {adm} nrhs={nrhs} {prec}")
    g = geometry.uniform_grid(3, n)
    a = 1.0 + 0.5 * g.points()[:, 0]
    rng = np.random.default_rng(41)
    u = rng.standard_normal(g.N) if nrhs == 1 else rng.standard_normal((g.N, nrhs))
    M = H.htlr_build(None, kernel, 3, n, p, leaf, a=a, eta2=eta2, admissibility=adm)
    assert M.info()["leaf_side"] == 4
    f_new = _product(torch, M, u, prec)
    pid = {"fp64": 0, "fp32": 1, "bf16": 2}[prec]
    cache = tmp_path / "tune.txt"
    key = f"d3_n{n}_p{p}_leaf{leaf}_k{W.KERNEL_IDS[kernel]}_uniform_eta{eta2:g}_adm{0 if adm == 'strong' else 1}" \
          f"_nrhs{nrhs}_prec{pid}"
    cache.write_text(f"{key} 2048 3 0 0 0 0 0 0 0 1.0 1.0\n")
    monkeypatch.setenv("HTLR_TUNE_CACHE", str(cache))
    M2 = H.htlr_build(None, kernel, 3, n, p, leaf, a=a, eta2=eta2, admissibility=adm)
    assert M2.autotune(nrhs, prec)["candidates"] == 0
    f_old = _product(torch, M2, u, prec)
    assert _rel(f_new, f_old) <= (1e-14 if prec == "fp64" else 1e-5)
    if prec == "fp64":
        O = htlr.HTLR(g, kernel, p, leaf, a, adm_kind=adm, eta2=eta2)
        leaves = O.tree.leaves()
        pick = [leaves[i] for i in W.sample_leaves(n + nrhs, len(leaves), 3)]
        assert _rel(f_new[O.leaf_rows(pick)], O.matvec(u, pick)) <= 1e-12
