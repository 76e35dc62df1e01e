"""O2: straightforward HTLR construction and matrix-vector product
(test infrastructure, see oracle/__init__.py).

Construction follows Alg. 4.1 leaf by leaf of the block cluster tree:

* admissible leaf (tau, sigma): Chebyshev points on every side of the boxes
  Omega_tau and Omega_sigma, factors U_l, V_l and core G by interpolation
  (eq. 3.4); optionally a thin QR of every factor, U_l = W_l R_l,
  V_l = Q_l T_l, and G <- G x_1 R_1 ... x_d R_d x_{d+1} T_1 ... x_{2d} T_d;
  or the same with QR with column pivoting truncated at a relative pivot
  tolerance, which lowers the Tucker rank where a factor is rank deficient
  (Sec. 2.1: more points per dimension than the box has, p > m);
* inadmissible leaf: the dense block a_i delta_ij + K_ij |Omega_j| (eq. 4.1),
  with K_ii |Omega_i| = D_i.

The quadrature weight multiplies the source vector (u~ = |Omega| o u) instead
of the core.  On a uniform grid this equals the paper's (h^d G); on a
quasi-uniform tensor grid the weight differs per point and cannot sit in G.

The product follows Alg. 4.2 / eq. (4.3): for an admissible leaf, reshape
u~_sigma into a d-way tensor (first index fastest), W = U x_1 V_1^T ...
x_d V_d^T, H = G x_{[d+1..2d],[1..d]} W, F = H x_1 U_1 ... x_d U_d, and
f_tau += vec(F); for an inadmissible leaf, f_tau += A_tau,sigma u_sigma.
Blocks are built when visited and discarded after use, so memory stays
small; nothing is batched, shared between blocks or reordered.

``rows_of_leaves`` restricts the product to the rows of chosen leaf boxes
(the walk prunes target nodes that contain none of them), which is how
large workloads are checked on sampled outputs.

Parity: pinned in tests/test_oracle_htlr.py (HTLR == dense when no block is
admissible; HTLR == dense to rounding for the polynomial kernel; error
decays with p; symmetry; QR and raw forms agree; worked-example counts).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import geometry, interp
from .tree import Admissibility, ClusterTree, block_leaves, node_indices


def mode_product(T: np.ndarray, M: np.ndarray, mode: int) -> np.ndarray:
    """(T x_mode M)[..., i, ...] = sum_t M[i, t] T[..., t, ...]."""
    return np.moveaxis(np.tensordot(M, T, axes=([1], [mode])), 0, mode)


class HTLR:
    def __init__(self, grid, kernel: str, p: int, leaf: int, a: np.ndarray,
                 adm_kind: str = "strong", eta2=1, gl_order: int = 0,
                 orthonormalize=False, rank_tol: float = 1e-13):
        self.grid = grid
        self.kernel = kernel
        self.p = p
        self.a = np.asarray(a, dtype=np.float64)
        self.gl_order = gl_order
        self.orthonormalize = orthonormalize    # False, True (QR) or "qrcp"
        self.rank_tol = rank_tol
        self.tree = ClusterTree(grid, leaf)
        self.adm = Admissibility(self.tree, adm_kind, eta2)

    # ---- construction of one leaf block (Alg. 4.1) --------------------
    def box_edges(self, node):
        g = self.grid
        return [(g.edges[l][node.lo[l]], g.edges[l][node.hi[l]]) for l in range(g.d)]

    def tlr_block(self, tau, sigma):
        g, p = self.grid, self.p
        bt, bs = self.box_edges(tau), self.box_edges(sigma)
        xi = [interp.chebyshev_points(a, b, p) for a, b in bt]
        eta = [interp.chebyshev_points(a, b, p) for a, b in bs]
        U = [interp.lagrange_matrix(g.nodes[l][tau.lo[l]:tau.hi[l]], xi[l]) for l in range(g.d)]
        V = [interp.lagrange_matrix(g.nodes[l][sigma.lo[l]:sigma.hi[l]], eta[l]) for l in range(g.d)]
        G = interp.core(self.kernel, xi, eta, p)
        if self.orthonormalize:
            Gt = G.reshape([p] * (2 * g.d), order="F")
            for l in range(g.d):
                Wq, R = self._orth(U[l])
                Qq, T = self._orth(V[l])
                U[l], V[l] = Wq, Qq
                Gt = mode_product(Gt, R, l)
                Gt = mode_product(Gt, T, g.d + l)
            rt = [U[l].shape[1] for l in range(g.d)]
            rs = [V[l].shape[1] for l in range(g.d)]
            G = Gt.reshape(int(np.prod(rt)), int(np.prod(rs)), order="F")
        return U, V, G

    def _orth(self, F):
        """F = Q R with orthonormal Q (Alg. 4.1's QR step).  With
        orthonormalize="qrcp", QR with column pivoting (Sec. 2.1) F P = Q R,
        truncated to the pivots with |R_kk| > rank_tol |R_00|; R's columns are
        put back in F's order, so that F ~ Q R."""
        if self.orthonormalize != "qrcp":
            return np.linalg.qr(F, mode="reduced")
        Q, R, piv = scipy.linalg.qr(F, mode="economic", pivoting=True)
        diag = np.abs(np.diag(R))
        r = max(1, int(np.count_nonzero(diag > self.rank_tol * diag[0])))
        Rf = np.empty((r, F.shape[1]))
        Rf[:, piv] = R[:r]
        return Q[:, :r], Rf

    def dense_block(self, tau, sigma, rows=None):
        g = self.grid
        it = node_indices(self.tree, tau).reshape(-1, order="F")
        js = node_indices(self.tree, sigma).reshape(-1, order="F")
        if rows is not None:
            it = it[rows]
        X, Y = g.points(it), g.points(js)
        from . import kernels
        with np.errstate(divide="ignore", invalid="ignore"):
            K = kernels.evaluate(self.kernel, X[:, None, :], Y[None, :, :], self.p)
        K = K * g.weights(js)[None, :]
        same = it[:, None] == js[None, :]
        if same.any():
            ii = np.nonzero(same)
            D = geometry.diagonal(g, self.kernel, self.p, self.gl_order, lin=it[ii[0]])
            K[ii] = D + self.a[it[ii[0]]]
        return K

    # ---- product (Alg. 4.2) -------------------------------------------
    def matvec(self, u: np.ndarray, leaves=None) -> np.ndarray:
        """f = A^HTLR u.  With ``leaves`` (a list of leaf nodes), only the rows
        of those leaves are computed; the result then has one row per point
        of those leaves, in leaf order, each leaf's points in natural order."""
        g = self.grid
        U2 = u.reshape(g.N, -1)
        nrhs = U2.shape[1]
        wu = g.weights()[:, None] * U2
        if leaves is None:
            want = None
            f = np.zeros((g.N, nrhs))
        else:
            want = set(id(nd) for nd in leaves)
            anc = set()
            for nd in leaves:
                x = nd
                while x is not None:
                    anc.add(id(x))
                    x = x.parent
            f = {id(nd): np.zeros((nd.size, nrhs)) for nd in leaves}
        tau_filter = None if want is None else (lambda nd: id(nd) in anc)
        for kind, tau, sigma in block_leaves(self.tree, self.adm, tau_filter):
            it = node_indices(self.tree, tau)              # d-way tensor of indices
            js = node_indices(self.tree, sigma)
            if kind == "A":
                Uf, Vf, G = self.tlr_block(tau, sigma)
                T = wu[js.reshape(-1, order="F")].reshape(js.shape + (nrhs,), order="F")
                for l in range(g.d):
                    T = mode_product(T, Vf[l].T, l)
                w = T.reshape(-1, nrhs, order="F")
                h = G @ w
                shape_h = tuple(Uf[l].shape[1] for l in range(g.d)) + (nrhs,)
                F = h.reshape(shape_h, order="F")
                targets = [tau] if want is None else self._wanted_under(tau, leaves, want)
                for tgt in targets:
                    Ft = F
                    for l in range(g.d):
                        off = tgt.lo[l] - tau.lo[l] if want is not None else 0
                        ln = (tgt.hi[l] - tgt.lo[l]) if want is not None else (tau.hi[l] - tau.lo[l])
                        Ft = mode_product(Ft, Uf[l][off:off + ln], l)
                    self._accumulate(f, tgt, Ft.reshape(-1, nrhs, order="F"), want)
            else:
                u_s = U2[js.reshape(-1, order="F")]
                targets = [tau] if want is None else self._wanted_under(tau, leaves, want)
                for tgt in targets:
                    rows = None
                    if want is not None:
                        rows = self._rows_within(tau, tgt)
                    A = self.dense_block(tau, sigma, rows)
                    self._accumulate(f, tgt, A @ u_s, want)
        if want is None:
            return f.reshape(u.shape)
        out = np.concatenate([f[id(nd)] for nd in leaves], axis=0)
        return out if u.ndim > 1 else out[:, 0]

    def _wanted_under(self, tau, leaves, want):
        return [nd for nd in leaves if self._is_under(nd, tau)]

    @staticmethod
    def _is_under(nd, tau):
        x = nd
        while x is not None:
            if x is tau:
                return True
            x = x.parent
        return False

    def _rows_within(self, tau, tgt):
        """Positions (Fortran order within tau) of the points of leaf tgt."""
        d = self.grid.d
        rng = [np.arange(tgt.lo[l], tgt.hi[l]) - tau.lo[l] for l in range(d)]
        mesh = np.meshgrid(*rng, indexing="ij")
        lin = np.zeros_like(mesh[0])
        stride = 1
        for l in range(d):
            lin = lin + mesh[l] * stride
            stride *= tau.hi[l] - tau.lo[l]
        return lin.reshape(-1, order="F")

    def _accumulate(self, f, tgt, vals, want):
        if want is None:
            it = node_indices(self.tree, tgt).reshape(-1, order="F")
            f[it] += vals
        else:
            f[id(tgt)] += vals

    # ---- helpers ------------------------------------------------------
    def leaf_rows(self, leaves) -> np.ndarray:
        """Linear indices of the rows ``matvec(u, leaves)`` returns."""
        return np.concatenate([node_indices(self.tree, nd).reshape(-1, order="F")
                               for nd in leaves])

    def assemble(self) -> np.ndarray:
        """Dense N x N form of the HTLR operator (tiny grids only)."""
        g = self.grid
        A = np.zeros((g.N, g.N))
        for kind, tau, sigma in block_leaves(self.tree, self.adm):
            it = node_indices(self.tree, tau).reshape(-1, order="F")
            js = node_indices(self.tree, sigma).reshape(-1, order="F")
            if kind == "A":
                Uf, Vf, G = self.tlr_block(tau, sigma)
                Ub, Vb = Uf[0], Vf[0]
                for l in range(1, g.d):          # U_d (x) ... (x) U_1, eq. (3.5)
                    Ub = np.kron(Uf[l], Ub)
                    Vb = np.kron(Vf[l], Vb)
                A[np.ix_(it, js)] = (Ub @ G @ Vb.T) * g.weights(js)[None, :]
            else:
                A[np.ix_(it, js)] = self.dense_block(tau, sigma)
        return A
