"""Autotuner: tuning changes speed, not results; the cache file is reused."""
import os
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
