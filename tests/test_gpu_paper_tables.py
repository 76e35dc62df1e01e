"""The GPU product at the shapes of the paper's Tables 5.1-5.4 (a = 0).

Against the dense product O1 on sampled rows, the relative error must lie
within a factor 5 of the printed e_apply;rand (the paper states neither u's
distribution nor eta; eta^2 = d for strong admissibility, as in Prop. 3.9).
On sampled leaves the GPU product must also match the HTLR oracle O2 to
1e-12 (the first row of each table, and the 256^3 row of Table 5.3).
"""
import sys

import numpy as np
import pytest

from oracle import dense, geometry, htlr

pytestmark = pytest.mark.gpu

# (key, compare with the printed error, compare with O2 on sampled leaves)
CASES = [("table_5_1_gauss_weak_2d", True, True), ("table_5_1_gauss_weak_2d_n512", True, False),
         ("table_5_2_slp_strong_2d", True, True), ("table_5_2_slp_strong_2d_n512", True, False),
         ("table_5_3_gauss_weak_3d", True, True), ("table_5_3_gauss_weak_3d_n64", True, False),
         ("table_5_4_slp_strong_3d", True, True), ("table_5_4_slp_strong_3d_n64", True, False),
         # level-1 boxes of 128^3 points (slices staged in row chunks).  Here the
         # HTLR error with u ~ N(0, 1) is ~1.3e-4 in O2 as on the GPU, ten times
         # the printed 1.2e-5, so only parity with O2 is asserted
         ("table_5_3_gauss_weak_3d_n256", False, True)]


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("key,vs_paper,vs_o2", CASES)
def test_paper_table_error(torch, golden, key, vs_paper, vs_o2):
    import paper_2508_05958_amd as H
    e = golden[key]
    d, n, p, leaf, kern, adm = e["d"], e["n"], e["p"], e["leaf"], e["kernel"], e["adm"]
    eta2 = float(d) if adm == "strong" else 1.0
    print(f"[gpu] paper shape {key}: d={d} n={n} p={p} leaf={leaf} {kern} {adm}", flush=True)
    sys.stdout.flush()
    g = geometry.uniform_grid(d, n)
    a = np.zeros(g.N)
    u = np.random.default_rng(0).standard_normal(g.N)
    M = H.htlr_build(None, kern, d, n, p, leaf, a=a, eta2=eta2, admissibility=adm, precisions=["fp64"])
    f = M.matvec(torch.tensor(u, dtype=torch.float64, device="cuda"), prec="fp64").cpu().numpy()
    if vs_paper:
        rows = np.sort(np.random.default_rng(1).choice(g.N, 256, replace=False))
        err = _rel(f[rows], dense.matvec(g, kern, p, a, u, rows=rows, chunk=4))
        assert e["e_apply"] / 5 < err < e["e_apply"] * 5, (err, e["e_apply"])
    if vs_o2:
        O = htlr.HTLR(g, kern, p, leaf, a, adm_kind=adm, eta2=eta2)
        leaves = O.tree.leaves()
        pick = [leaves[i] for i in np.random.default_rng(2).choice(len(leaves), 3, replace=False)]
        assert _rel(f[O.leaf_rows(pick)], O.matvec(u, pick)) <= 1e-12
