"""Cluster tree, admissibility and block cluster tree (test infrastructure).

* Cluster tree (Def. 2.1) built by the recursive 2^d partition of Sec. 2.2:
  a node is a tensor product of index ranges tau_1 x ... x tau_d (Def. 3.5);
  it is a leaf when |tau| <= N_0 = leaf^d, otherwise every dimension of
  length > 1 is split into a first half of ceil(len/2) indices and the rest.
  Children are listed with the first dimension's half varying fastest.
* Omega_tau is the union of the cells of tau, i.e. the box
  prod_l [e_{l; lo_l}, e_{l; hi_l}].
* Strong admissibility (Def. 2.3): max(diam tau, diam sigma) <= eta * dist,
  diam the Euclidean diameter of the box, dist the distance between the
  closed boxes.  Squares are compared: max(diam^2) <= eta^2 * dist^2.  On a
  uniform grid the edges are integers in units of h, so the comparison is
  exact (ties dist == diam are admissible).
* Weak admissibility (Def. 2.2): the boxes do not overlap (zero-volume
  intersection).
* Block cluster tree (Def. 2.4, Def. 3.6): from (root, root), an admissible
  pair is an admissible leaf; otherwise, if either node is a leaf, the pair
  is an inadmissible leaf; otherwise recurse into children x children.

Parity: pinned in tests/test_oracle_tree.py (Example 2.2 / Fig. 2.1 leaves,
Fig. 2.3 dense-block counts, Prop. 3.9 bounds, partition of I x I, interior
near-field counts from the closed form).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from fractions import Fraction

import numpy as np


@dataclass(eq=False)
class Node:
    lo: tuple
    hi: tuple
    level: int
    children: list = field(default_factory=list)
    parent: "Node | None" = None
    index: int = -1

    @property
    def size(self) -> int:
        return int(np.prod([h - l for l, h in zip(self.lo, self.hi)]))

    def contains_index(self, midx) -> bool:
        return all(l <= i < h for l, i, h in zip(self.lo, midx, self.hi))


class ClusterTree:
    def __init__(self, grid, leaf: int):
        self.grid = grid
        self.d = grid.d
        self.N0 = leaf ** grid.d
        self.nodes = []
        self.root = self._build(tuple([0] * grid.d), tuple(grid.n), 0, None)

    def _build(self, lo, hi, level, parent):
        node = Node(lo, hi, level, parent=parent)
        node.index = len(self.nodes)
        self.nodes.append(node)
        if node.size <= self.N0:
            return node
        halves = []
        for l in range(self.d):
            ln = hi[l] - lo[l]
            if ln > 1:
                mid = lo[l] + (ln + 1) // 2
                halves.append([(lo[l], mid), (mid, hi[l])])
            else:
                halves.append([(lo[l], hi[l])])
        # first dimension's half varies fastest
        combos = [[]]
        for l in range(self.d):
            combos = [c + [hv] for hv in halves[l] for c in combos]
        for c in combos:
            clo = tuple(x[0] for x in c)
            chi = tuple(x[1] for x in c)
            node.children.append(self._build(clo, chi, level + 1, node))
        return node

    def leaves(self):
        return [nd for nd in self.nodes if not nd.children]

    # ---- box geometry -------------------------------------------------
    def box(self, node):
        """(lo, hi) edge coordinates per dimension: exact ints (units of h) on
        uniform grids, floats otherwise."""
        g = self.grid
        if g.uniform:
            return ([int(g.int_edges[l][node.lo[l]]) for l in range(self.d)],
                    [int(g.int_edges[l][node.hi[l]]) for l in range(self.d)])
        return ([float(g.edges[l][node.lo[l]]) for l in range(self.d)],
                [float(g.edges[l][node.hi[l]]) for l in range(self.d)])


def diam2(box):
    lo, hi = box
    return sum((h - l) ** 2 for l, h in zip(lo, hi))


def dist2(b1, b2):
    (lo1, hi1), (lo2, hi2) = b1, b2
    s = 0
    for l in range(len(lo1)):
        gap = max(0, lo2[l] - hi1[l], lo1[l] - hi2[l])
        s += gap * gap
    return s


def overlap_volume(b1, b2):
    (lo1, hi1), (lo2, hi2) = b1, b2
    v = 1
    for l in range(len(lo1)):
        v *= max(0, min(hi1[l], hi2[l]) - max(lo1[l], lo2[l]))
    return v


class Admissibility:
    """Strong (Def. 2.3, with eta^2 given exactly) or weak (Def. 2.2)."""

    def __init__(self, tree: ClusterTree, kind: str = "strong", eta2=1):
        self.tree = tree
        self.kind = kind
        if tree.grid.uniform and not isinstance(eta2, Fraction):
            eta2 = Fraction(eta2).limit_denominator(10 ** 6)
        self.eta2 = eta2

    def __call__(self, tau: Node, sigma: Node) -> bool:
        bt, bs = self.tree.box(tau), self.tree.box(sigma)
        if self.kind == "weak":
            return overlap_volume(bt, bs) == 0
        return max(diam2(bt), diam2(bs)) <= self.eta2 * dist2(bt, bs)


def block_leaves(tree: ClusterTree, adm: Admissibility, tau_filter=None):
    """Leaves of the block cluster tree (Def. 2.4) as (kind, tau, sigma),
    kind 'A' (admissible) or 'N' (inadmissible).  ``tau_filter(node)`` may
    prune target nodes whose rows are not wanted."""
    out = []
    stack = [(tree.root, tree.root)]
    while stack:
        tau, sigma = stack.pop()
        if tau_filter is not None and not tau_filter(tau):
            continue
        if adm(tau, sigma):
            out.append(("A", tau, sigma))
        elif not tau.children or not sigma.children:
            out.append(("N", tau, sigma))
        else:
            for tc in tau.children:
                for sc in sigma.children:
                    stack.append((tc, sc))
    return out


def node_indices(tree: ClusterTree, node: Node) -> np.ndarray:
    """Linear indices of the points of a node, as a d-way tensor (first index
    fastest when flattened in Fortran order)."""
    rng = [np.arange(node.lo[l], node.hi[l]) for l in range(tree.d)]
    mesh = np.meshgrid(*rng, indexing="ij")
    return tree.grid.linear_index(mesh)
