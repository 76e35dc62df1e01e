"""Autotuner: tuning changes speed, not results; the cache file is reused."""
import os
import sys

import numpy as np
import pytest
from precision_checks import assert_reduced_close

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.mark.parametrize("prec,nrhs,tol", [("fp64", 1, 1e-13), ("fp32", 16, 1e-6), ("bf16", 4, 1e-6)])
def test_tuning_keeps_results(torch, prec, nrhs, tol):
    import paper_2508_05958_amd as H
    _say(f"[gpu] autotune {prec} nrhs={nrhs}")
    n = 32
    M = H.htlr_build(None, "inv_r", 3, n, 6, 8, a=np.ones(n ** 3))
    dt = torch.float64 if prec == "fp64" else torch.float32
    u = torch.randn(nrhs, n ** 3, dtype=dt, device="cuda").t() if nrhs > 1 else torch.randn(n ** 3, dtype=dt,
                                                                                              device="cuda")
    f0 = M.matvec(u, prec=prec).double().cpu().numpy()
    r = M.autotune(nrhs, prec)
    assert r["candidates"] >= 2 and r["ms_best"] <= r["ms_default"] * 1.0001
    f1 = M.matvec(u, prec=prec).double().cpu().numpy()
    assert np.linalg.norm(f1 - f0) / np.linalg.norm(f0) <= tol


def test_tune_cache_file(torch, tmp_path, monkeypatch):
    import paper_2508_05958_amd as H
    _say("[gpu] autotune cache")
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("HTLR_TUNE_CACHE", str(cache))
    M = H.htlr_build(None, "exp", 3, 16, 4, 4, a=np.ones(16 ** 3))
    r1 = M.autotune(2, "fp64")
    assert r1["candidates"] > 0 and cache.exists()
    M2 = H.htlr_build(None, "exp", 3, 16, 4, 4, a=np.ones(16 ** 3))
    r2 = M2.autotune(2, "fp64")
    assert r2["candidates"] == 0 and r2["ks_target"] == r1["ks_target"]


def test_server_with_autotune(torch):
    import paper_2508_05958_amd as H
    import test_gpu_serve as TS
    _say("[gpu] server with autotune")
    reqs = TS._requests(4)
    outs = []
    for tune in (False, True):
        S = H.Server(max_batch=4, inner_prec="fp32", autotune=tune)
        ids = [S.submit(**r) for r in reqs]
        res = TS._drain(S, list(ids))
        outs.append([res[i][0] for i in ids])
        S.close()
    for a, b in zip(*outs):
        assert np.linalg.norm(a - b) / np.linalg.norm(b) <= 10 * TS.TOL


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("tile", [1, 2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("mode,order", [(1, 0), (1, 1), (1, 2), (2, 0)])
def test_every_tile_variant_matches(torch, tmp_path, monkeypatch, prec, tile, mode, order):
    """Force each matrix-core tile shape (128x128, 128x64, 256x128, 224x64, 256x256, 64x128, 64x64) through
    the tuner's cache file, in class-tile mode with each work-item order
    (row block major, tile major, tile major with the longest lists first) and
    in offset-major mode, and compare with the oracle (FP64) or with the GPU
    FP64 product (FP32, BF16)."""
    import paper_2508_05958_amd as H
    from oracle import geometry, htlr
    _say(f"[gpu] forced tile {tile} mode {mode} order {order} {prec}")
    n, p, leaf, nrhs = 32, 6, 8, 3
    pid = {"fp64": 0, "fp32": 1, "bf16": 2}[prec]
    cache = tmp_path / "tune.txt"
    key = f"d3_n{n}_p{p}_leaf{leaf}_k0_uniform_eta1_adm0_nrhs{nrhs}_prec{pid}"
    cache.write_text(f"{key} 2048 -1 0 {tile} {mode} 0 0 0 0 1.0 1.0 {order}\n")
    monkeypatch.setenv("HTLR_TUNE_CACHE", str(cache))
    g = geometry.uniform_grid(3, n)
    a = 1.0 + 0.5 * g.points()[:, 0]
    u = np.random.default_rng(tile).standard_normal((g.N, nrhs))
    M = H.htlr_build(None, "inv_r", 3, n, p, leaf, a=a)
    ref_t = torch.tensor(u.T.copy(), dtype=torch.float64, device="cuda").t()
    f_ref = M.matvec(ref_t, prec="fp64").cpu().numpy()
    r = M.autotune(nrhs, prec)
    assert r["candidates"] == 0
    dt = torch.float64 if prec == "fp64" else torch.float32
    ut = torch.tensor(u.T.copy(), dtype=dt, device="cuda").t()
    f = M.matvec(ut, prec=prec).double().cpu().numpy()
    if prec == "fp64":
        O = htlr.HTLR(g, "inv_r", p, leaf, a)
        leaves = O.tree.leaves()
        pick = [leaves[i] for i in (0, 21, 42, 63)]
        fo = O.matvec(u, pick)
        assert np.linalg.norm(f[O.leaf_rows(pick)] - fo) / np.linalg.norm(fo) <= 1e-12
    tol = {"fp64": 1e-13, "fp32": 1e-5, "bf16": 5e-3}[prec]
    assert_reduced_close(f, f_ref, tol)


_NEAR_REF = {}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nrhs", [1, 5])
@pytest.mark.parametrize("near_kind,nw,ks,tpw,ct", [(1, 0, 0, 0, 0), (0, 1, 0, 0, 0), (0, 8, 0, 0, 0), (2, 0, 1, 8, 1),
                                                    (2, 0, 4, 4, 1), (2, 0, 32, 8, 1), (2, 0, 1, 8, 2),
                                                    (2, 0, 8, 4, 2)])
def test_every_near_variant_matches(torch, tmp_path, monkeypatch, prec, nrhs, near_kind, nw, ks, tpw, ct):
    """Force the near-field variant through the tuner's cache file and compare
    with the oracle: matrix cores with right-hand sides as columns (1), VALU
    rows with 1 or 8 waves per leaf (0), matrix cores with target leaves as
    columns (2) at several K splits, row tiles and column tiles per wave."""
    import paper_2508_05958_amd as H
    from oracle import geometry, htlr
    _say(f"[gpu] forced near kind={near_kind} nw={nw} ks={ks} tpw={tpw} ct={ct} {prec} nrhs={nrhs}")
    n, p, leaf = 32, 4, 8
    pid = {"fp64": 0, "fp32": 1}[prec]
    cache = tmp_path / "tune.txt"
    key = f"d3_n{n}_p{p}_leaf{leaf}_k1_uniform_eta1_adm0_nrhs{nrhs}_prec{pid}"
    cache.write_text(f"{key} 2048 {near_kind} {nw} 0 0 {ks} {tpw} {ct} 0 1.0 1.0\n")
    monkeypatch.setenv("HTLR_TUNE_CACHE", str(cache))
    g = geometry.uniform_grid(3, n)
    a = 1.0 + 0.5 * g.points()[:, 0]
    u = np.random.default_rng(nrhs).standard_normal((g.N, nrhs))
    if nrhs not in _NEAR_REF:
        _NEAR_REF[nrhs] = htlr.HTLR(g, "neg_log", p, leaf, a).matvec(u)
    fo = _NEAR_REF[nrhs]
    M = H.htlr_build(None, "neg_log", 3, n, p, leaf, a=a)
    assert M.autotune(nrhs, prec)["candidates"] == 0
    dt = torch.float64 if prec == "fp64" else torch.float32
    ut = torch.tensor(u.T.copy(), dtype=dt, device="cuda").t()
    f = M.matvec(ut, prec=prec).double().cpu().numpy()
    tol = 1e-12 if prec == "fp64" else 1e-5
    assert np.linalg.norm(f - fo) / np.linalg.norm(fo) <= tol


@pytest.mark.parametrize("prec,nrhs", [("fp64", 1), ("fp32", 3)])
def test_level_concurrency_is_bitwise_serial(torch, tmp_path, monkeypatch, prec, nrhs):
    """Levels run on side streams concurrently with the near field; the down
    expansions add into f in level order on the caller's stream, so the
    product equals the all-serial launch order bit for bit."""
    import paper_2508_05958_amd as H
    _say(f"[gpu] level concurrency vs serial {prec} nrhs={nrhs}")
    n, p, leaf = 64, 4, 8
    pid = {"fp64": 0, "fp32": 1}[prec]
    dt = torch.float64 if prec == "fp64" else torch.float32
    u = torch.randn(nrhs, n ** 3, dtype=dt, generator=torch.Generator().manual_seed(7)).to("cuda").t()
    outs = []
    for serial in (2, 1):   # forced concurrent, then serial
        cache = tmp_path / f"tune{serial}.txt"
        key = f"d3_n{n}_p{p}_leaf{leaf}_k0_uniform_eta1_adm0_nrhs{nrhs}_prec{pid}"
        cache.write_text(f"{key} 2048 -1 0 0 0 0 0 0 {serial} 1.0 1.0\n")
        monkeypatch.setenv("HTLR_TUNE_CACHE", str(cache))
        M = H.htlr_build(None, "inv_r", 3, n, p, leaf, a=np.ones(n ** 3))
        assert sum(1 for x in M.info()["adm_pairs"] if x) >= 2
        assert M.autotune(nrhs, prec)["candidates"] == 0
        outs.append([M.matvec(u, prec=prec).cpu().numpy() for _ in range(2)])
        M.free()
    assert np.array_equal(outs[0][0], outs[0][1])
    assert np.array_equal(outs[0][0], outs[1][0])
