"""Test helper: the per-level Tucker ranks the O2 oracle's QR step keeps."""
from oracle import htlr
from oracle.tree import block_leaves


def oracle_level_ranks(O, levels, under=None):
    """Per level, the rank O2's QR step keeps for one admissible block of
    that level (every block of a level has the same factors on a uniform
    grid); 0 where the level has no admissible block.  With a leaf `under`,
    only blocks whose target holds that leaf are visited."""
    out = [0] * (levels + 1)
    keep = None if under is None else (lambda nd: htlr.HTLR._is_under(under, nd))
    for kind, tau, sigma in block_leaves(O.tree, O.adm, keep):
        if kind == "A" and out[tau.level] == 0:
            U, V, G = O.tlr_block(tau, sigma)
            assert len({x.shape[1] for x in U + V}) == 1
            out[tau.level] = U[0].shape[1]
    return out
