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


@pytest.mark.parametrize("d,n,leaf,grid,t", [(2, 32, 4, "uniform", 0.3), (3, 16, 2, "uniform", 0.7),
                                            (2, 24, 3, "warped", 0.7), (3, 12, 3, "warped", 0.35)])
def test_planner_with_cell_edges_equals_oracle_tree(d, n, leaf, grid, t):
    """Cells given by the caller (htlr_build_opts.edges): the boxes Omega_tau
    are unions of those cells, so the block cluster tree follows them.  Each
    case's pairs differ from those of the default (Voronoi) cells, so an
    ignored edges argument fails."""
    x = W.uniform_nodes(n) if grid == "uniform" else W.warped_nodes(n)
    e = W.split_edges(x, t)
    g = geometry.tensor_grid([x] * d, edges=[e] * d)
    pts = None if grid == "uniform" else np.concatenate([x] * d)
    edges = np.concatenate([e] * d)
    L, adm, near = H.htlr_plan_counts(pts, d, n, leaf, 1.0, "strong", edges=edges)
    differs = False
    for level in list(range(L + 1)) + [-1]:
        tau, sig = H.htlr_plan_pairs(pts, d, n, leaf, level, 1.0, "strong", edges=edges)
        mine = sorted(zip(tau.tolist(), sig.tolist()))
        assert mine == _oracle_pairs(g, leaf, 1.0, "strong", level), level
        t0, s0 = H.htlr_plan_pairs(pts, d, n, leaf, level, 1.0, "strong")
        differs |= mine != sorted(zip(t0.tolist(), s0.tolist()))
    assert differs


def test_cell_edges_are_checked():
    x = W.uniform_nodes(8)
    e = W.split_edges(x, 0.5)
    with pytest.raises(H.HTLRError) as ex:
        H.htlr_plan_counts(None, 2, 8, 2, edges=np.concatenate([e, e[::-1]]))     # not increasing
    assert ex.value.status == -1
    bad = e.copy()
    bad[3] = x[3] + 1e-3                                                        # node 3 left of its cell
    with pytest.raises(H.HTLRError) as ex:
        H.htlr_plan_counts(None, 2, 8, 2, edges=np.concatenate([e, bad]))
    assert ex.value.status == -1
    with pytest.raises(H.HTLRError) as ex:
        H.htlr_plan_counts(None, 2, 8, 2, edges=np.concatenate([e, e[:-1]]))    # wrong count
    assert ex.value.status == -1
    # the uniform edges k/n on the uniform nodes are the uniform grid
    u = np.arange(9) / 8.0
    assert H.htlr_plan_counts(None, 2, 8, 2, edges=np.concatenate([u, u])) == H.htlr_plan_counts(None, 2, 8, 2)


@pytest.mark.slow
def test_planner_equals_oracle_tree_on_warped_96():
    """The warped 96^3 grid of the solve workload, pair for pair against the
    oracle's block cluster tree (counts 1352 / 136312 / 2110448 admissible
    leaves at levels 2-4 and 405008 near pairs)."""
    x = W.warped_nodes(96)
    g = geometry.tensor_grid([x] * 3)
    pts = np.concatenate([x] * 3)
    t = ClusterTree(g, 8)
    adm = Admissibility(t, "strong", 1.0)
    want = {}
    for k, tau, sigma in block_leaves(t, adm):
        m = tau.hi[0] - tau.lo[0]
        B = 96 // m
        lin = lambda nd: sum((nd.lo[l] // m) * B ** l for l in range(3))
        want.setdefault(tau.level if k == "A" else -1, []).append((lin(tau), lin(sigma)))
    L, cnt, near = H.htlr_plan_counts(pts, 3, 96, 8)
    assert cnt[2:] == [1352, 136312, 2110448] and near == 405008
    for level in (2, 3, 4, -1):
        tau, sig = H.htlr_plan_pairs(pts, 3, 96, 8, level)
        assert sorted(zip(tau.tolist(), sig.tolist())) == sorted(want[level]), level


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
