"""Property the tiled near field rests on, pinned on the oracle: on a uniform
grid the inadmissible block between two leaves (eq. 4.1 with the weights of
Sec. 3, and the diagonal term of eq. 1.4 on the self block) depends only on
the leaf offset sigma - tau, and each entry depends only on the squared
index distance |I - J|^2 (radial kernel).  So one block per near offset,
filled from a table indexed by |I - J|^2, reproduces every near block."""
import numpy as np
import pytest

from oracle import geometry, htlr, tree as T


@pytest.mark.parametrize("kernel", ["inv_r", "exp"])
def test_near_blocks_depend_only_on_the_offset_and_distance(kernel):
    n = 32
    g = geometry.uniform_grid(3, n)
    O = htlr.HTLR(g, kernel, 4, 8, np.zeros(g.N))
    leaves = O.tree.leaves()
    # inadmissible leaf pairs of the block cluster tree (Def. 2.4)
    adm = T.Admissibility(O.tree, "strong", 1)
    near = [(t, s) for k, t, s in T.block_leaves(O.tree, adm) if k == "N"]
    assert near
    by_off = {}
    for t, s in near:
        off = tuple((b - a) // 8 for a, b in zip(t.lo, s.lo))
        by_off.setdefault(off, []).append((t, s))
    # points of a leaf in x-fastest order, as the GPU's blocks are laid out
    loc = np.array([(i & 7, (i >> 3) & 7, i >> 6) for i in range(512)])
    checked = 0
    for off, pairs in sorted(by_off.items()):
        if len(pairs) < 2:
            continue
        (t0, s0), (t1, s1) = pairs[0], pairs[-1]
        B0, B1 = O.dense_block(t0, s0), O.dense_block(t1, s1)
        scale = np.abs(B0).max()
        # same offset, same block
        assert np.abs(B0 - B1).max() <= 1e-13 * scale, off
        # entries equal wherever |I - J|^2 is equal (a table by squared distance)
        d2 = ((loc[:, None, :] - (loc[None, :, :] + 8 * np.array(off))) ** 2).sum(-1)
        tab = {}
        for v, k in zip(B0.ravel(), d2.ravel()):
            ref = tab.setdefault(int(k), v)
            assert abs(v - ref) <= 1e-13 * scale
        checked += 1
    assert checked >= 20
