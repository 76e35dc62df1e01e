"""Near field on the matrix-core core apply (eq. 4.1 restricted to near leaf
pairs, plus the diagonal term of eq. 1.4): on a uniform grid with 8^3-point
leaves each near pair's block depends only on the leaf offset, so the near
field runs as class tiles of precomputed 512 x 512 blocks.  Checked against
the oracle on sampled leaves, against the near-field kernel that evaluates
the table on the fly, and for FP32 against the FP64 product."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def _build(H, monkeypatch, tmp_path, n, p, nrhs, near_kind, tag):
    """Matrix whose products of this shape take near-field kernel near_kind
    (-1: the automatic choice), through the tuner's cache file."""
    cache = tmp_path / f"tune_{tag}.txt"
    lines = []
    if near_kind >= 0:
        for pid in (0, 1):
            key = f"d3_n{n}_p{p}_leaf8_k0_uniform_eta1_adm0_nrhs{nrhs}_prec{pid}"
            lines.append(f"{key} 2048 {near_kind} 0 0 0 0 0 0 0 1.0 1.0\n")
    cache.write_text("".join(lines))
    monkeypatch.setenv("HTLR_TUNE_CACHE", str(cache))
    from oracle import geometry
    g = geometry.uniform_grid(3, n)
    a = 1.0 + 0.5 * g.points()[:, 0]
    M = H.htlr_build(None, "inv_r", 3, n, p, 8, a=a)
    if near_kind >= 0:
        for pr in ("fp64", "fp32"):
            assert M.autotune(nrhs, pr)["candidates"] == 0   # read from the cache file
    return M, g, a


# 32^3: 4^3 leaves (every leaf touches the boundary); 64^3: 8^3 leaves;
# 20 right-hand sides: tiles of 4 leaves x 20 columns, the rest of the 128 empty;
# 2 and 5: tiles of 64 and 16 leaves
@pytest.mark.parametrize("n,p,nrhs", [(32, 4, 16), (64, 4, 16), (64, 4, 20), (64, 4, 2), (32, 4, 5)])
def test_near_tiles_match_oracle_and_table_kernel(torch, tmp_path, monkeypatch, n, p, nrhs):
    import paper_2508_05958_amd as H
    from oracle import htlr
    _say(f"[gpu] near field on the core apply n={n} p={p} nrhs={nrhs}")
    rng = np.random.default_rng(n + nrhs)
    u = rng.standard_normal((n ** 3, nrhs))
    u64 = torch.tensor(u.T.copy(), dtype=torch.float64, device="cuda").t()
    u32 = torch.tensor(u.T.copy(), dtype=torch.float32, device="cuda").t()
    out = {}
    for kind in (4, 1, -1):
        M, g, a = _build(H, monkeypatch, tmp_path, n, p, nrhs, kind, str(kind))
        out[kind] = (M.matvec(u64, prec="fp64").cpu().numpy(), M.matvec(u32, prec="fp32").double().cpu().numpy())
        M.free()
    f4, f4s = out[4]
    f1, _ = out[1]
    # the automatic choice at two or more right-hand sides is the tiled near field
    assert np.array_equal(out[-1][0], f4) and np.array_equal(out[-1][1], f4s)
    # same sums as the on-the-fly kernel, in another order
    assert np.linalg.norm(f4 - f1) / np.linalg.norm(f1) <= 1e-13
    assert np.abs(f4 - f1).max() / np.abs(f1).max() <= 1e-13
    # FP32 against FP64, per column and elementwise
    for c in range(nrhs):
        assert np.linalg.norm(f4s[:, c] - f4[:, c]) / np.linalg.norm(f4[:, c]) <= 1e-5
    assert np.abs(f4s - f4).max() / np.abs(f4).max() <= 1e-5
    # oracle on sampled leaves (O2, eq. 4.1 + Alg. 4.2), all right-hand sides
    O = htlr.HTLR(g, "inv_r", p, 8, a)
    leaves = O.tree.leaves()
    pick = [leaves[i] for i in sorted({0, len(leaves) // 3, len(leaves) // 2, len(leaves) - 1})]
    fo = O.matvec(u, pick)
    assert np.linalg.norm(f4[O.leaf_rows(pick)] - fo) / np.linalg.norm(fo) <= 1e-12
