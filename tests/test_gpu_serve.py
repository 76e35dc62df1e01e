"""Request server: continuous batching of solves through the C ABI.

Each request's answer must be the same alone and in a mix (within the
solve tolerance), fused products and graph replays must not change results,
and admission must respect the memory budget.
"""
import sys

import numpy as np
import pytest

import htlr_workloads as W

pytestmark = pytest.mark.gpu

STRUCTS = [("inv_r", 2, 32, 6, 8), ("neg_log", 2, 64, 6, 8), ("exp", 3, 16, 4, 4)]
TOL = 1e-8


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def _requests(count=8):
    out = []
    for rid in range(count):
        kern, d, n, p, leaf = STRUCTS[rid % len(STRUCTS)]
        pts = W.grid_points([W.uniform_nodes(n)] * d)
        a = 1.0 + 0.5 * pts[:, 0]
        f = np.random.default_rng([4, rid]).standard_normal(n ** d)
        out.append(dict(f=f, kernel=kern, d=d, n=n, p=p, leaf=leaf, a=a, tol=TOL))
    return out


def _drain(S, ids, max_ticks=5000):
    res = {}
    for _ in range(max_ticks):
        S.step()
        for rid in list(ids):
            u, info = S.result(rid)
            if u is not None or info["state"] >= 2:
                res[rid] = (u, info)
                ids.remove(rid)
        if not ids:
            return res
    raise AssertionError("server did not finish")


def _residual(torch, H, req, u):
    M = H.htlr_build(None, req["kernel"], req["d"], req["n"], req["p"], req["leaf"], a=req["a"])
    Au = M.matvec(torch.tensor(u, device="cuda"), prec="fp64").cpu().numpy()
    M.free()
    return np.linalg.norm(req["f"] - Au) / np.linalg.norm(req["f"])


def test_alone_equals_mixed(torch):
    import paper_2508_05958_amd as H
    _say("[gpu] server: alone vs mixed")
    reqs = _requests(8)
    S = H.Server(max_batch=8, inner_prec="fp32", use_graphs=True)
    alone = []
    for r in reqs:
        rid = S.submit(**r)
        alone.append(_drain(S, [rid])[rid])
    alone_products = S.stats()["fused_products"]
    S.close()
    S = H.Server(max_batch=8, inner_prec="fp32", use_graphs=True)
    ids = [S.submit(**r) for r in reqs[:3]]
    S.step()
    S.step()
    ids += [S.submit(**r) for r in reqs[3:6]]
    S.step()
    ids += [S.submit(**r) for r in reqs[6:]]
    mixed = _drain(S, list(ids))
    st = S.stats()
    S.close()
    assert st["fused_products"] < alone_products          # products were shared
    assert st["graph_launches"] > 0
    for k, rid in enumerate(ids):
        u_m, info = mixed[rid]
        u_a, _ = alone[k]
        assert info["status"] == 0 and info["rel_residual"] <= TOL
        assert np.linalg.norm(u_m - u_a) / np.linalg.norm(u_a) <= 10 * TOL
        assert _residual(torch, H, reqs[k], u_m) <= TOL


def test_graph_replay_equals_eager(torch):
    import paper_2508_05958_amd as H
    _say("[gpu] server: graphs vs eager")
    reqs = _requests(6)
    outs = []
    for g in (False, True):
        S = H.Server(max_batch=4, inner_prec="fp32", use_graphs=g)
        ids = [S.submit(**r) for r in reqs]
        res = _drain(S, list(ids))
        outs.append([res[i][0] for i in ids])
        if g:
            assert S.stats()["graph_launches"] > 0
        S.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_admission_by_footprint(torch):
    import paper_2508_05958_amd as H
    _say("[gpu] server: admission under a small budget")
    reqs = _requests(6)
    sizes = []
    for r in reqs[:3]:                    # resident bytes of each structure as the server counts them
        P = H.Server(max_batch=4, inner_prec="fp32")
        rid = P.submit(**r)
        _drain(P, [rid])
        sizes.append(P.stats()["resident_bytes"])
        P.close()
    state = 64 * 64 * 8 * 40              # request state of the largest grid, generous
    budget = max(max(sizes) + 2 * state, int(0.6 * sum(sizes)))
    assert budget < sum(sizes)
    S = H.Server(memory_budget=budget, max_batch=4, inner_prec="fp32")
    ids = [S.submit(**r) for r in reqs]
    res = _drain(S, list(ids))
    st = S.stats()
    S.close()
    assert st["evictions"] >= 1
    assert all(res[i][1]["status"] == 0 for i in ids)


def test_request_that_cannot_fit(torch):
    import paper_2508_05958_amd as H
    _say("[gpu] server: request larger than the budget")
    r = _requests(1)[0]
    S = H.Server(memory_budget=64 << 10, max_batch=2)
    rid = S.submit(**r)
    res = _drain(S, [rid])
    S.close()
    assert res[rid][1]["state"] == 3 and res[rid][1]["status"] == -3
