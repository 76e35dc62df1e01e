"""GPU parity of the quasi-uniform transfer form (htlr_build_quasi,
Sec. 3.3, eq. 3.9) against the oracle O5 (oracle/quasi.py).

FP64 products must match O5 with Ahat by the HTLR oracle O2 to 1e-12
relative; FP32 and bfloat16-core products are compared with the GPU FP64
product at 1e-5 and 5e-3.  The full-size workload (2D, n = 512, m = 1024)
is checked on the quasi-uniform points whose transfer rows fall inside
sampled uniform-grid leaves, whose rows O2 computes one leaf at a time.
"""
import sys

import numpy as np
import pytest

import htlr_workloads as W
from precision_checks import assert_reduced_close
from oracle import geometry, htlr, quasi

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 1e-5
BF16_TOL = 5e-3


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _gpu_matvec(torch, M, u, prec="fp64"):
    dt = torch.float64 if prec == "fp64" else torch.float32
    ut = torch.tensor(np.asfortranarray(u), dtype=dt, device="cuda")
    if u.ndim == 2:
        ut = ut.t().contiguous().t()          # column-major
    f = M.matvec(ut, prec=prec)
    torch.cuda.synchronize()
    return f.cpu().numpy().astype(np.float64)


def _nodes(d, n, kind):
    if kind == "skewed":
        return [W.skewed_nodes(n, 0.03 if l % 2 == 0 else -0.025) for l in range(d)]
    if kind == "warped":
        return [W.warped_nodes(n)] * d
    return [W.uniform_nodes(n)] * d


def _u(g, nrhs, seed):
    rng = np.random.default_rng(seed)
    if nrhs == 1:
        return rng.standard_normal(g.N)
    return np.asfortranarray(rng.standard_normal((g.N, nrhs)))


CASES = [
    # d, n, m, leaf, p, kernel, adm, eta2, nodes, nrhs
    (2, 24, 32, 4, 5, "neg_log", "strong", 1.0, "skewed", 1),    # rho > 1
    (2, 40, 32, 4, 4, "gauss", "weak", 1.0, "warped", 2),        # rho < 1
    (2, 33, 64, 8, 6, "inv_r", "strong", 2.0, "skewed", 1),      # odd n
    (3, 12, 16, 4, 4, "inv_r", "strong", 1.0, "skewed", 1),
    (3, 10, 8, 4, 3, "exp", "strong", 1.0, "warped", 3),
    (2, 20, 16, 4, 4, "poly_test", "strong", 1.0, "skewed", 1),  # exact far field
]


@pytest.mark.parametrize("d,n,m,leaf,p,kernel,adm,eta2,nodes,nrhs", CASES)
def test_fp64_matches_oracle(torch, d, n, m, leaf, p, kernel, adm, eta2, nodes, nrhs):
    import paper_2508_05958_amd as H
    _say(f"[gpu] quasi fp64 d={d} n={n} m={m} {kernel} {adm} {nodes} nrhs={nrhs}")
    nd = _nodes(d, n, nodes)
    gq = geometry.tensor_grid(nd)
    a = 1.0 + 0.5 * gq.points()[:, 0]
    u = _u(gq, nrhs, 11)
    M = H.htlr_build_quasi(np.concatenate(nd), kernel, d, n, m, p, leaf, a=a, eta2=eta2, admissibility=adm)
    ref = quasi.matvec(gq, m, kernel, p, leaf, a, u, khat="htlr", adm_kind=adm, eta2=eta2)
    assert _rel(_gpu_matvec(torch, M, u), ref) <= FP64_TOL


def test_caller_cells_match_oracle(torch):
    """Quasi-uniform cells given by the caller (htlr_build_opts.edges): S and
    T follow them (cell-overlap matrices of Sec. 3.3)."""
    import paper_2508_05958_amd as H
    _say("[gpu] quasi with caller cells")
    d, n, m, leaf, p = 2, 24, 32, 4, 5
    nd = _nodes(d, n, "skewed")
    ed = [W.split_edges(x, 0.3 if l == 0 else 0.65) for l, x in enumerate(nd)]
    gq = geometry.tensor_grid(nd, edges=ed)
    a = 1.0 + 0.5 * gq.points()[:, 0]
    u = _u(gq, 2, 13)
    M = H.htlr_build_quasi(np.concatenate(nd), "neg_log", d, n, m, p, leaf, a=a, edges=np.concatenate(ed))
    ref = quasi.matvec(gq, m, "neg_log", p, leaf, a, u, khat="htlr")
    assert _rel(_gpu_matvec(torch, M, u), ref) <= FP64_TOL
    ref0 = quasi.matvec(geometry.tensor_grid(nd), m, "neg_log", p, leaf, a, u, khat="htlr")
    assert _rel(ref, ref0) > 1e-6          # the cells matter


def test_coincident_grid_equals_uniform_product(torch):
    """n = m on the uniform grid: S = T = I, the transfer form equals the
    uniform handle's product."""
    import paper_2508_05958_amd as H
    _say("[gpu] quasi coincident grid")
    d, n = 3, 16
    g = geometry.uniform_grid(d, n)
    a = 1.0 + 0.5 * g.points()[:, 0]
    u = _u(g, 2, 12)
    Mq = H.htlr_build_quasi(None, "inv_r", d, n, n, 4, 4, a=a)
    Mu = H.htlr_build(None, "inv_r", d, n, 4, 4, a=a)
    assert _rel(_gpu_matvec(torch, Mq, u), _gpu_matvec(torch, Mu, u)) <= 1e-14


@pytest.mark.parametrize("d,n,m,leaf,p,kernel,nrhs", [(3, 24, 32, 8, 6, "inv_r", 4), (2, 96, 128, 8, 6, "neg_log", 3),
                                                      (3, 20, 16, 4, 4, "exp", 1)])
def test_reduced_precision_vs_fp64(torch, d, n, m, leaf, p, kernel, nrhs):
    import paper_2508_05958_amd as H
    _say(f"[gpu] quasi fp32/bf16 vs fp64 d={d} n={n} m={m} nrhs={nrhs}")
    nd = _nodes(d, n, "warped")
    gq = geometry.tensor_grid(nd)
    u = _u(gq, nrhs, 13)
    M = H.htlr_build_quasi(np.concatenate(nd), kernel, d, n, m, p, leaf, a=np.ones(gq.N))
    f64 = _gpu_matvec(torch, M, u, "fp64")
    assert_reduced_close(_gpu_matvec(torch, M, u, "fp32"), f64, FP32_TOL)
    assert_reduced_close(_gpu_matvec(torch, M, u, "bf16"), f64, BF16_TOL)


def test_full_size_sampled(torch):
    """The 2D quasi-uniform workload at full size (N = 512^2, M = 1024^2),
    in the launch configuration of the benchmark: quasi-uniform points whose
    transfer rows lie inside sampled uniform leaves, against O5 with Ahat by O2."""
    import paper_2508_05958_amd as H
    w = W.WORKLOADS["wq2d_log_n512_m1024"]
    _say(f"[gpu] {w.name} full size, sampled")
    nd = w.nodes()
    gq = geometry.tensor_grid(nd)
    a, u = w.a(), w.rhs()
    M = H.htlr_build_quasi(np.concatenate(nd), w.kernel, 2, w.n, w.m, w.p, w.leaf, a=a, eta2=w.eta2)
    fg = _gpu_matvec(torch, M, u)
    gu = geometry.uniform_grid(2, w.m)
    O = htlr.HTLR(gu, w.kernel, w.p, w.leaf, np.zeros(gu.N), eta2=w.eta2)
    leaves = O.tree.leaves()
    pick = [leaves[i] for i in W.sample_leaves(w.seed, len(leaves), 3)]
    rows = O.leaf_rows(pick)
    fh = np.zeros(gu.N)
    have = np.zeros(gu.N, dtype=bool)
    fh[rows] = O.matvec(quasi.s_apply(gq, w.m, u), pick)
    have[rows] = True
    eu = np.arange(w.m + 1) / w.m
    T = [quasi.t_1d(gq.edges[l], eu) for l in range(2)]
    runs = [[np.nonzero(T[l][i])[0] for i in range(w.n)] for l in range(2)]
    got, ref = [], []
    for leaf in pick:
        # quasi-uniform points whose overlapping uniform cells all lie in this leaf
        inside = [[i for i in range(w.n) if runs[l][i][0] >= leaf.lo[l] and runs[l][i][-1] < leaf.hi[l]]
                  for l in range(2)]
        for i2 in inside[1]:
            t2 = runs[1][i2]
            for i1 in inside[0]:
                t1 = runs[0][i1]
                cells = t1[:, None] + w.m * t2[None, :]
                assert have[cells].all()
                i = i1 + w.n * i2
                got.append(fg[i])
                ref.append(a[i] * u[i] + T[0][i1, t1] @ fh[cells] @ T[1][i2, t2])
    assert len(got) >= 50
    assert _rel(got, ref) <= FP64_TOL


def test_solve_on_quasi_handle(torch):
    """GMRES with FP64 refinement on the transfer form: the FP64 residual
    reaches the tolerance and the solution reproduces f through O5."""
    import paper_2508_05958_amd as H
    _say("[gpu] quasi solve")
    d, n, m = 2, 48, 64
    nd = _nodes(d, n, "skewed")
    gq = geometry.tensor_grid(nd)
    a = 1.0 + 0.5 * gq.points()[:, 0]
    M = H.htlr_build_quasi(np.concatenate(nd), "neg_log", d, n, m, 6, 8, a=a)
    xs = W.smooth_u(gq.points())
    f = torch.tensor(quasi.matvec(gq, m, "neg_log", 6, 8, a, xs, khat="htlr"), device="cuda")
    x, info, st = M.solve(f, tol=1e-11, inner_prec="fp32")
    torch.cuda.synchronize()
    assert st == 0 and info.rel_residual <= 1e-11
    xh = x.cpu().numpy()
    fr = quasi.matvec(gq, m, "neg_log", 6, 8, a, xh, khat="htlr")
    assert _rel(fr, f.cpu().numpy()) <= 1e-10
    assert _rel(xh, xs) <= 1e-8


def test_info_profile_and_errors(torch):
    import paper_2508_05958_amd as H
    _say("[gpu] quasi info, profile, error paths")
    nd = _nodes(3, 12, "warped")
    M = H.htlr_build_quasi(np.concatenate(nd), "inv_r", 3, 12, 16, 4, 4)
    Mu = H.htlr_build(None, "inv_r", 3, 16, 4, 4)
    i, iu = M.info(), Mu.info()
    assert (i["d"], i["n"], i["uniform_m"], iu["uniform_m"]) == (3, 12, 16, 0)
    assert i["adm_pairs"] == iu["adm_pairs"] and i["near_pairs"] == iu["near_pairs"]
    assert i["device_bytes"] > iu["device_bytes"]
    assert M.workspace_bytes(2, "fp64") == Mu.workspace_bytes(2, "fp64") + 2 * 16 ** 3 * 2 * 8
    M.profile(True)
    _gpu_matvec(torch, M, np.ones(12 ** 3))
    names = M.profile_read()
    M.profile(False)
    assert {"quasi_s", "quasi_t"} <= set(names) and any(k.startswith("core") or k.startswith("near") for k in names)
    with pytest.raises(H.HTLRError) as e:
        H.htlr_build_quasi(np.concatenate(nd), "inv_r", 3, 12, 20, 4, 4)    # 20 -> 10 -> 5 does not halve to 4
    assert e.value.status in (-1, -2)
    with pytest.raises(H.HTLRError) as e:
        H.htlr_build_quasi(np.concatenate(nd), "inv_r", 3, 12, 0, 4, 4)
    assert e.value.status == -1
    bad = np.concatenate(nd)
    bad[3] = bad[2]
    with pytest.raises(H.HTLRError) as e:
        H.htlr_build_quasi(bad, "inv_r", 3, 12, 16, 4, 4)
    assert e.value.status == -1
    u = torch.zeros(12 ** 3, dtype=torch.float32, device="cuda")
    with pytest.raises(H.HTLRError):
        M.matvec(u, prec="fp64")


def test_autotune_and_qr_form_on_quasi_handle(torch):
    """htlr_autotune on a transfer-form handle tunes Ahat's products and keeps
    the result; the build options (here Alg. 4.1's QR step) reach Ahat."""
    import paper_2508_05958_amd as H
    _say("[gpu] quasi autotune and QR form")
    d, n, m = 3, 20, 32
    nd = _nodes(d, n, "skewed")
    gq = geometry.tensor_grid(nd)
    a = 1.0 + 0.5 * gq.points()[:, 0]
    u = _u(gq, 2, 14)
    M = H.htlr_build_quasi(np.concatenate(nd), "inv_r", d, n, m, 6, 8, a=a)
    f0 = _gpu_matvec(torch, M, u)
    r = M.autotune(2, "fp64")
    assert r["candidates"] >= 2 and r["ms_best"] <= r["ms_default"] * 1.0001
    assert _rel(_gpu_matvec(torch, M, u), f0) <= 1e-13
    Mq = H.htlr_build_quasi(np.concatenate(nd), "inv_r", d, n, m, 6, 8, a=a, orthonormalize="qr")
    assert Mq.info()["rank"] == 6
    assert _rel(_gpu_matvec(torch, Mq, u), f0) <= 1e-13
