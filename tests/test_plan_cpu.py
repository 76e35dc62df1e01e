"""Host-side checks of the library (no GPU): the C ABI loads and exports
every declared entry point, the C++ planner's block lists equal the
oracle's independent block cluster tree, and argument errors come back as
status codes."""
import os
import re

import numpy as np
import pytest

import htlr_workloads as W
import paper_2508_05958_amd as H
from oracle import geometry
from oracle.tree import Admissibility, ClusterTree, block_leaves

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    text = open(os.path.join(ROOT, "include", "htlr.h")).read()
    names = set(re.findall(r"^(?:htlr_status|void|const char\*)\s+(htlr_\w+)\s*\(", text, re.M))
    assert len(names) >= 10
    L = H.lib()
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert not missing, missing


def _oracle_pairs(grid, leaf, eta2, kind, level):
    t = ClusterTree(grid, leaf)
    adm = Admissibility(t, kind, eta2)
    out = []
    for k, tau, sigma in block_leaves(t, adm):
        if (level >= 0 and k == "A" and tau.level == level) or (level < 0 and k == "N"):
            B = grid.n[0] // (tau.hi[0] - tau.lo[0])
            m = tau.hi[0] - tau.lo[0]

            def lin(nd):
                return sum((nd.lo[l] // m) * B ** l for l in range(grid.d))
            out.append((lin(tau), lin(sigma)))
    return sorted(out)


@pytest.mark.parametrize("d,n,leaf,eta2,kind,grid", [
    (2, 64, 8, 1.0, "strong", "uniform"), (3, 32, 4, 1.0, "strong", "uniform"),
    (3, 32, 4, 3.0, "strong", "uniform"), (2, 32, 4, 1.0, "weak", "uniform"),
    (2, 48, 6, 1.0, "strong", "warped"), (3, 24, 3, 1.0, "strong", "warped"),
])
def test_planner_pairs_equal_oracle_tree(d, n, leaf, eta2, kind, grid):
    if grid == "uniform":
        g = geometry.uniform_grid(d, n)
        pts = None
    else:
        x = W.warped_nodes(n)
        g = geometry.tensor_grid([x] * d)
        pts = np.concatenate([x] * d)
    L, adm, near = H.htlr_plan_counts(pts, d, n, leaf, eta2, kind)
    for level in list(range(L + 1)) + [-1]:
        tau, sig = H.htlr_plan_pairs(pts, d, n, leaf, level, eta2, kind)
        mine = sorted(zip(tau.tolist(), sig.tolist()))
        assert mine == _oracle_pairs(g, leaf, eta2, kind, level), level


def test_planner_counts_match_derived(golden):
    for case in golden["derived_block_counts"]["cases"]:
        L, adm, near = H.htlr_plan_counts(None, case["d"], case["n"], case["leaf"])
        got = {str(l): c for l, c in enumerate(adm) if c}
        assert got == case["adm_per_level"]
        assert near == case["near"]


def test_planner_large_config_counts():
    L, adm, near = H.htlr_plan_counts(None, 3, 128, 8)
    assert L == 4
    assert adm[2:] == [1416, 133944, 2021592]
    assert near == 383272


def test_footprint_without_gpu():
    b = H.htlr_footprint(None, "inv_r", 3, 32, 6, 8, precisions=["fp64"])
    assert b > 0


@pytest.mark.parametrize("args,status", [
    (dict(d=4, n=16, leaf=4), -2), (dict(d=3, n=100, leaf=8), -2), (dict(d=2, n=0, leaf=4), -1),
])
def test_invalid_arguments_return_status(args, status):
    with pytest.raises(H.HTLRError) as e:
        H.htlr_plan_counts(None, args["d"], args["n"], args["leaf"])
    assert e.value.status == status


def test_nodes_must_increase():
    x = W.uniform_nodes(16)[::-1].copy()
    with pytest.raises(H.HTLRError) as e:
        H.htlr_plan_counts(np.concatenate([x, x]), 2, 16, 4)
    assert e.value.status == -1


def test_footprint_follows_the_qr_rank():
    """The dry build runs the host QR(CP) of the shared factors.  Where every
    level's factor has rank m < p (n = 16, leaf 2: boxes of 4 and 2 points,
    p = 8) the stored rank is 4 and the cores shrink from (8^2)^2 to (4^2)^2
    per offset; with p at most the box side everywhere the size is unchanged."""
    full = H.htlr_footprint(None, "inv_r", 2, 16, 8, 2)
    qr = H.htlr_footprint(None, "inv_r", 2, 16, 8, 2, orthonormalize="qr")
    qrcp = H.htlr_footprint(None, "inv_r", 2, 16, 8, 2, orthonormalize="qrcp")
    assert qr == qrcp and qr < full / 8
    assert H.htlr_footprint(None, "inv_r", 2, 64, 6, 8, orthonormalize="qr") == H.htlr_footprint(None, "inv_r", 2, 64, 6, 8)
    # a loose pivot tolerance truncates full-rank factors too (rank 4 of 6)
    assert H.htlr_footprint(None, "inv_r", 2, 32, 6, 4, orthonormalize="qrcp", rank_tol=0.3) < \
        H.htlr_footprint(None, "inv_r", 2, 32, 6, 4) / 4


def test_orthonormalize_and_quasi_arguments_are_checked():
    with pytest.raises(H.HTLRError) as e:
        H.htlr_footprint(None, "inv_r", 2, 16, 8, 2, orthonormalize=3)
    assert e.value.status == -1
    x = W.warped_nodes(16)
    with pytest.raises(H.HTLRError) as e:
        H.htlr_footprint(np.concatenate([x] * 2), "inv_r", 2, 16, 4, 4, orthonormalize="qr")
    assert e.value.status == -2
    with pytest.raises(H.HTLRError) as e:
        H.htlr_build_quasi(None, "inv_r", 3, 12, 0, 4, 4)
    assert e.value.status == -1
    bad = np.concatenate([W.warped_nodes(12)] * 3)
    bad[3] = bad[2]
    with pytest.raises(H.HTLRError) as e:
        H.htlr_build_quasi(bad, "inv_r", 3, 12, 16, 4, 4)
    assert e.value.status == -1
