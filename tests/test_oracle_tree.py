"""Pins for the oracle's cluster tree, admissibility and block cluster tree."""
from collections import Counter, defaultdict
from fractions import Fraction
import itertools

import numpy as np
import pytest

from oracle import geometry
from oracle.tree import Admissibility, ClusterTree, block_leaves, node_indices


def _tree(d, n, leaf, kind="strong", eta2=1):
    g = geometry.uniform_grid(d, n)
    t = ClusterTree(g, leaf)
    return g, t, Admissibility(t, kind, eta2)


def test_example_2_2_leaves(golden):
    ex = golden["example_2_2_leaves"]
    g, t, _ = _tree(ex["d"], ex["n"], ex["leaf"])
    leaves = t.leaves()
    assert len(leaves) == ex["num_leaves"]
    assert all(nd.size == ex["leaf_size"] for nd in leaves)
    cover = np.concatenate([node_indices(t, nd).ravel() for nd in leaves])
    assert np.array_equal(np.sort(cover), np.arange(g.N))


def _dense_per_row(t, adm):
    per_row = defaultdict(lambda: Counter())
    for kind, tau, sigma in block_leaves(t, adm):
        per_row[tau.index][kind] += 1
    return per_row


def test_fig_2_3_dense_blocks_per_row(golden):
    ex = golden["fig_2_3_dense_blocks_per_row"]
    _, t, weak = _tree(ex["d"], ex["n"], ex["leaf"], "weak")
    rows = _dense_per_row(t, weak)
    leaf_rows = [rows[nd.index]["N"] for nd in t.leaves()]
    assert all(c == ex["weak_exact"] for c in leaf_rows)
    _, t, strong = _tree(ex["d"], ex["n"], ex["leaf"], "strong", ex["strong_eta2"])
    rows = _dense_per_row(t, strong)
    leaf_rows = [rows[nd.index]["N"] for nd in t.leaves()]
    assert max(leaf_rows) == ex["strong_max"]


@pytest.mark.parametrize("d,n,leaf", [(2, 64, 4), (3, 32, 4)])
def test_prop_3_9_bounds(golden, d, n, leaf):
    ref = golden["prop_3_9_bounds"]
    _, t, adm = _tree(d, n, leaf, "strong", d)          # eta = sqrt(d)
    rows = _dense_per_row(t, adm)
    assert max(c["N"] for c in rows.values()) <= ref["inadmissible_max"][str(d)]
    assert max(c["A"] for c in rows.values()) <= ref["admissible_max"][str(d)]


@pytest.mark.parametrize("d,n,leaf,kind,eta2", [(2, 16, 2, "strong", 1), (2, 12, 3, "strong", 2),
                                                 (3, 8, 2, "strong", 1), (2, 16, 4, "weak", 1),
                                                 (2, 10, 3, "strong", 1)])
def test_block_leaves_partition_I_x_I(d, n, leaf, kind, eta2):
    g, t, adm = _tree(d, n, leaf, kind, eta2)
    cover = np.zeros((g.N, g.N), dtype=np.int32)
    for _, tau, sigma in block_leaves(t, adm):
        it = node_indices(t, tau).ravel()
        js = node_indices(t, sigma).ravel()
        cover[np.ix_(it, js)] += 1
    assert np.all(cover == 1)


def test_admissible_blocks_are_well_separated_and_parents_are_not():
    g, t, adm = _tree(3, 32, 4)
    for kind, tau, sigma in block_leaves(t, adm):
        if kind == "A":
            assert adm(tau, sigma)
            assert tau.parent is not None and not adm(tau.parent, sigma.parent)
        else:
            assert not adm(tau, sigma)
            assert not tau.children or not sigma.children


@pytest.mark.parametrize("d", [2, 3])
def test_interior_near_counts(golden, d):
    """Interior leaves have the closed-form number of dense partners."""
    expected = golden["near_field_interior_counts"][str(d)]
    # brute force over offsets with real-valued box geometry (unit boxes)
    count = 0
    for off in itertools.product(range(-3, 4), repeat=d):
        gap2 = sum(max(abs(o) - 1, 0) ** 2 for o in off)
        if not d <= gap2:
            count += 1
    assert count == expected
    n, leaf = (64, 4) if d == 2 else (32, 4)
    _, t, adm = _tree(d, n, leaf)
    rows = _dense_per_row(t, adm)
    B = n // leaf
    for nd in t.leaves():
        box = [lo // leaf for lo in nd.lo]
        if all(3 <= b < B - 3 for b in box):
            assert rows[nd.index]["N"] == expected


def test_ties_are_admissible_exactly():
    """Offset (2,2,2) between leaves: dist == diam exactly; admissible (<=)."""
    _, t, adm = _tree(3, 16, 2)
    leaves = {tuple(lo // 2 for lo in nd.lo): nd for nd in t.leaves()}
    a, b = leaves[(0, 0, 0)], leaves[(2, 2, 2)]
    assert adm(a, b)
    assert not adm(leaves[(0, 0, 0)], leaves[(2, 2, 1)])


def test_derived_block_counts(golden):
    for case in golden["derived_block_counts"]["cases"]:
        _, t, adm = _tree(case["d"], case["n"], case["leaf"])
        cnt = Counter()
        near = 0
        for kind, tau, sigma in block_leaves(t, adm):
            if kind == "A":
                cnt[str(tau.level)] += 1
            else:
                near += 1
        assert dict(cnt) == case["adm_per_level"]
        assert near == case["near"]


def test_warped_grid_tree_is_valid_partition():
    x = (np.arange(12) + 0.5) / 12
    x = x + 0.08 * np.sin(2 * np.pi * x) / (2 * np.pi)
    g = geometry.tensor_grid([x, x])
    t = ClusterTree(g, 3)
    adm = Admissibility(t, "strong", 1.0)
    cover = np.zeros((g.N, g.N), dtype=np.int32)
    for _, tau, sigma in block_leaves(t, adm):
        cover[np.ix_(node_indices(t, tau).ravel(), node_indices(t, sigma).ravel())] += 1
    assert np.all(cover == 1)
