"""Request server: continuous batching of solves through the C ABI.

Each request's answer must be the same alone and in a mix (within the
solve tolerance), fused products and graph replays must not change results,
and admission must respect the memory budget.  Served answers are checked
against the CPU oracles: the residual ||f - A u|| / ||f|| is recomputed with
the FP64 HTLR oracle (O2, Alg. 4.2) on the whole grid, and on the smallest
grid u is compared with numpy.linalg.solve on the assembled O2 operator.
"""
import sys

import numpy as np
import pytest

import htlr_workloads as W
from oracle import geometry, gmres, htlr

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


_ORACLES = {}


def _oracle(req):
    key = (req["kernel"], req["d"], req["n"], req["p"], req["leaf"])
    if key not in _ORACLES:
        g = geometry.uniform_grid(req["d"], req["n"])
        _ORACLES[key] = htlr.HTLR(g, req["kernel"], req["p"], req["leaf"], req["a"])
    return _ORACLES[key]


def _residual(req, u):
    """||f - A u|| / ||f|| with A applied by the CPU oracle O2."""
    Au = _oracle(req).matvec(u)
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
        # recomputed by the oracle: a little above the server's own FP64
        # residual, by rounding in a different summation order
        assert _residual(reqs[k], u_m) <= 2 * TOL


# structures that share their factors (same d, n, p, leaf; different kernels)
GROUPED = [("inv_r", 2, 64, 6, 8), ("neg_log", 2, 64, 6, 8), ("exp", 2, 64, 6, 8),
           ("inv_r", 3, 16, 4, 4), ("exp", 3, 16, 4, 4)]


def _grouped_requests(count=10):
    out = []
    for rid in range(count):
        kern, d, n, p, leaf = GROUPED[rid % len(GROUPED)]
        a = 1.0 + 0.5 * W.grid_points([W.uniform_nodes(n)] * d)[:, 0]
        f = np.random.default_rng([4, 100 + rid]).standard_normal(n ** d)
        out.append(dict(f=f, kernel=kern, d=d, n=n, p=p, leaf=leaf, a=a, tol=TOL))
    return out


def test_cross_structure_fusion(torch):
    """Requests on structures that differ only in the kernel: with fusion
    their products of a tick run as one grouped product whose up
    contractions and down expansions cover all of them in one launch per
    level.  The answers equal those without fusion bit for bit (each column
    takes the same kernels either way), and they solve the oracle's system."""
    import paper_2508_05958_amd as H
    _say("[gpu] server: cross-structure fusion on vs off")
    reqs = _grouped_requests(10)
    outs, stats = [], []
    # unfused (graphs), fused eager, fused with grouped products replayed from graphs
    for fuse, graphs in ((False, True), (True, False), (True, True)):
        S = H.Server(max_batch=4, inner_prec="fp32", use_graphs=graphs, group_fusion=fuse)
        ids = [S.submit(**r) for r in reqs]
        res = _drain(S, list(ids))
        stats.append(S.stats())
        outs.append([res[i] for i in ids])
        S.close()
    _say(f"[gpu]   fused: {stats[2]['group_products']} grouped products, {stats[2]['grouped_launches']} shared "
         f"launches, {stats[2]['graph_launches']} graph launches; unfused: {stats[0]['fused_products']} products")
    assert stats[0]["group_products"] == 0
    assert stats[1]["group_products"] > 0 and stats[1]["grouped_launches"] > 0
    assert stats[1]["graph_launches"] == 0
    assert stats[2]["group_products"] > 0 and stats[2]["graph_launches"] > 0
    assert stats[2]["grouped_launches"] == stats[1]["grouped_launches"]
    for (u0, i0), (u1, i1), (u2, i2) in zip(*outs):
        assert i0["status"] == 0 and i1["status"] == 0 and i2["status"] == 0
        assert np.array_equal(u0, u1)
        assert np.array_equal(u1, u2)
    for k in (0, 1, 3):
        assert _residual(reqs[k], outs[1][k][0]) <= 2 * TOL


def test_served_answer_equals_direct_solve(torch):
    """The smallest structure (2D n = 32, N = 1024): served answers against
    numpy.linalg.solve on the densely assembled O2 operator, within
    cond(A) * tol, alone and in a mix with other structures."""
    import paper_2508_05958_amd as H
    _say("[gpu] server: served u vs direct solve of the assembled oracle")
    reqs = [r for r in _requests(9) if r["n"] == 32]
    O = _oracle(reqs[0])
    A = O.assemble()
    kappa = np.linalg.cond(A)
    S = H.Server(max_batch=8, inner_prec="fp32", use_graphs=True)
    ids = [S.submit(**r) for r in _requests(9)]
    res = _drain(S, list(ids))
    S.close()
    checked = 0
    for rid, r in zip(ids, _requests(9)):
        if r["n"] != 32:
            continue
        u, info = res[rid]
        x = gmres.direct(A, r["f"])
        err = np.linalg.norm(u - x) / np.linalg.norm(x)
        _say(f"[gpu]   request {rid}: |u - x|/|x| {err:.2e}, cond {kappa:.1f}")
        assert info["status"] == 0
        assert err <= kappa * TOL
        checked += 1
    assert checked == 3


def test_bf16_core_inner_products(torch):
    """Inner products with bfloat16 cores, refined in FP64: every request
    reaches the FP64 tolerance (recomputed by O2), agrees with its FP32-inner
    answer to the tolerance, and, with the default inner target 1e-4, takes
    at most four refinement steps (the bfloat16-core product is far more
    accurate than bfloat16 itself: factors and near field stay FP32)."""
    import paper_2508_05958_amd as H
    _say("[gpu] server: bfloat16-core inner products")
    reqs = _requests(6)
    outs = {}
    for inner in ("fp32", "bf16"):
        S = H.Server(max_batch=4, inner_prec=inner, use_graphs=True)
        ids = [S.submit(**r) for r in reqs]
        res = _drain(S, list(ids))
        S.close()
        outs[inner] = [res[i] for i in ids]
    for k, ((u32, i32), (u16, i16)) in enumerate(zip(outs["fp32"], outs["bf16"])):
        _say(f"[gpu]   request {k}: outer {i16['outer_iters']}, inner {i16['inner_iters']}, "
             f"residual {i16['rel_residual']:.2e}")
        assert i16["status"] == 0 and i16["rel_residual"] <= TOL
        assert i16["outer_iters"] <= 4
        assert np.linalg.norm(u16 - u32) / np.linalg.norm(u32) <= 10 * TOL
        assert _residual(reqs[k], u16) <= 2 * TOL


def test_bf16_server_with_a_warped_grid(torch):
    """A bfloat16-inner server also serves a request on a warped tensor grid
    (given points, no bfloat16 cores there): that structure takes FP32 inner
    products, its answer solves O2's system to the tolerance, and the
    uniform-grid requests beside it still converge."""
    import paper_2508_05958_amd as H
    _say("[gpu] server: bfloat16 inner products with a warped-grid request")
    d, n, p, leaf = 2, 32, 6, 8
    x = W.warped_nodes(n)
    g = geometry.tensor_grid([x] * d)
    a = 1.0 + 0.5 * g.points()[:, 0]
    f = np.random.default_rng([4, 500]).standard_normal(g.N)
    warped = dict(f=f, kernel="exp", d=d, n=n, p=p, leaf=leaf, a=a, tol=TOL, points=np.concatenate([x] * d))
    reqs = _requests(3)
    S = H.Server(max_batch=4, inner_prec="bf16", use_graphs=True)
    ids = [S.submit(**r) for r in reqs] + [S.submit(**warped)]
    res = _drain(S, list(ids))
    S.close()
    for rid in ids:
        assert res[rid][1]["status"] == 0 and res[rid][1]["rel_residual"] <= TOL
    u = res[ids[-1]][0]
    O = htlr.HTLR(g, "exp", p, leaf, a)
    rel = np.linalg.norm(f - O.matvec(u)) / np.linalg.norm(f)
    _say(f"[gpu]   warped request: O2 residual {rel:.2e}")
    assert rel <= 2 * TOL


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
