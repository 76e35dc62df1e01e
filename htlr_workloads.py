"""Seeded synthetic inputs for the HTLR workloads.

This module is shared by the oracle and by the GPU path's tests and
benchmark.  It holds only input recipes (grid nodes, a(x) samples, random
vectors, sampled row / leaf indices, request streams); none of the HTLR
method's arithmetic lives here.

Vectors follow the natural ordering of the tensor grid: multi-index
(i_1, ..., i_d) maps to i_1 + n*i_2 + n^2*i_3 (first index fastest, 0-based),
and several right-hand sides are stored column-major (each RHS contiguous).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Kernel enumeration shared with the C ABI (include/htlr.h).
KERNEL_IDS = {"inv_r": 0, "neg_log": 1, "exp": 2, "gauss": 3, "poly_test": 100}


def uniform_nodes(n: int) -> np.ndarray:
    """Cell-centred uniform nodes (k + 1/2)/n, k = 0..n-1 (paper Example 2.2)."""
    return (np.arange(n, dtype=np.float64) + 0.5) / n


def warped_nodes(n: int, amp: float = 0.08) -> np.ndarray:
    """Quasi-uniform nodes x_k = t_k + amp*sin(2 pi t_k)/(2 pi), t_k cell centres."""
    t = uniform_nodes(n)
    return t + amp * np.sin(2.0 * np.pi * t) / (2.0 * np.pi)


def skewed_nodes(n: int, c: float = 0.03) -> np.ndarray:
    """Quasi-uniform nodes t_k + c (cos(2 pi t_k) - 1), t_k cell centres; not
    symmetric about 1/2 (increasing for |c| < 1/(2 pi))."""
    t = uniform_nodes(n)
    return t + c * (np.cos(2.0 * np.pi * t) - 1.0)


def smooth_u(points: np.ndarray) -> np.ndarray:
    """u(x) = 1 + 0.5 exp(-(x1-0.3)^2 - (x2-0.6)^2) + sin(5 x1 x2), the input
    function of the paper's quasi-uniform experiment (Sec. 5.4)."""
    x1, x2 = points[:, 0], points[:, 1]
    return 1.0 + 0.5 * np.exp(-(x1 - 0.3) ** 2 - (x2 - 0.6) ** 2) + np.sin(5.0 * x1 * x2)


def split_edges(nodes: np.ndarray, t: float) -> np.ndarray:
    """Cell edges 0, x_0 + t (x_1 - x_0), ..., x_{n-2} + t (x_{n-1} - x_{n-2}), 1:
    each interior edge splits the gap between neighbouring nodes at fraction
    t (t = 1/2 gives the Voronoi cells)."""
    x = np.asarray(nodes, dtype=np.float64)
    e = np.empty(len(x) + 1)
    e[0], e[-1] = 0.0, 1.0
    e[1:-1] = x[:-1] + t * (x[1:] - x[:-1])
    return e


def grid_points(nodes_per_dim) -> np.ndarray:
    """All tensor-grid points, shape (N, d), natural order (first index fastest)."""
    d = len(nodes_per_dim)
    mesh = np.meshgrid(*nodes_per_dim, indexing="ij")
    return np.stack([m.reshape(-1, order="F") for m in mesh], axis=1).reshape(-1, d)


def a_values(spec: str, points: np.ndarray) -> np.ndarray:
    """Samples of a(x) at the grid points for the recipes used by the workloads."""
    if spec == "zero":
        return np.zeros(points.shape[0])
    if spec == "one":
        return np.ones(points.shape[0])
    if spec == "two_plus_x1":
        return 2.0 + points[:, 0]
    if spec == "one_plus_half_x1":
        return 1.0 + 0.5 * points[:, 0]
    raise ValueError(spec)


@dataclass
class Workload:
    name: str
    d: int
    n: int
    kernel: str
    p: int
    leaf: int
    a_spec: str
    seed: int
    nrhs: int = 1
    dist: str = "normal"          # "uniform" -> U[-1,1], "normal" -> N(0,1), "smooth" -> smooth_u
    grid: str = "uniform"         # "uniform" or "warped"
    eta2: float = 1.0             # eta^2 of the strong admissibility test
    gl_order: int = 0             # 0 -> 16 in 2D, 8 in 3D
    m: int = 0                    # > 0: transfer to the uniform grid of m cells per dimension
    sample_rows: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.n ** self.d

    def nodes(self):
        f = uniform_nodes if self.grid == "uniform" else warped_nodes
        return [f(self.n) for _ in range(self.d)]

    def points(self) -> np.ndarray:
        return grid_points(self.nodes())

    def a(self) -> np.ndarray:
        return a_values(self.a_spec, self.points())

    def rhs(self) -> np.ndarray:
        """Right-hand side(s), shape (N,) for one RHS else (N, nrhs) column-major."""
        rng = np.random.default_rng(self.seed)
        if self.dist == "smooth":
            u = smooth_u(self.points())
        elif self.dist == "uniform":
            u = rng.uniform(-1.0, 1.0, self.N)
        elif self.nrhs == 1:
            u = rng.standard_normal(self.N)
        else:
            u = np.asfortranarray(rng.standard_normal((self.nrhs, self.N)).T)
        return u

    def rows(self, size: int | None = None) -> np.ndarray:
        size = size or self.sample_rows
        rng = np.random.default_rng([self.seed, 1])
        return np.sort(rng.choice(self.N, size=size, replace=False))


# The five workloads: 2D log kernel (small, full dense check); 3D 1/r FP64;
# 3D 1/r mixed precision with 16 right-hand sides; warped-grid GMRES solve;
# serving stream (see request_stream).
WORKLOADS = {
    "w2d_log_n64": Workload("w2d_log_n64", 2, 64, "neg_log", 6, 8, "one", 0, dist="uniform"),
    "w3d_invr_n64": Workload("w3d_invr_n64", 3, 64, "inv_r", 6, 8, "one", 1, sample_rows=2048),
    "w3d_invr_n128_r16": Workload("w3d_invr_n128_r16", 3, 128, "inv_r", 8, 8, "one", 2, nrhs=16,
                                  sample_rows=2048),
    "w3d_exp_warp_n96": Workload("w3d_exp_warp_n96", 3, 96, "exp", 6, 8, "two_plus_x1", 3,
                                 grid="warped"),
    # quasi-uniform 2D grid through the uniform grid of m = 2n cells (rho = 2),
    # the SLP kernel with strong admissibility, p and leaf of the 2D tables
    "wq2d_log_n512_m1024": Workload("wq2d_log_n512_m1024", 2, 512, "neg_log", 8, 16, "one", 5, dist="smooth",
                                    grid="warped", eta2=2.0, m=1024),
}


def solve_target(points: np.ndarray) -> np.ndarray:
    """u*(x) = sin(2 pi x1) cos(pi x2) x3 for the warped-grid solve workload."""
    return np.sin(2 * np.pi * points[:, 0]) * np.cos(np.pi * points[:, 1]) * points[:, 2]


def sample_leaves(seed: int, nleaves: int, count: int) -> np.ndarray:
    rng = np.random.default_rng([seed, 2])
    return np.sort(rng.choice(nleaves, size=min(count, nleaves), replace=False))


@dataclass
class Request:
    rid: int
    arrival: float
    d: int
    n: int
    kernel: str
    p: int

    def rhs(self) -> np.ndarray:
        return np.random.default_rng([4, self.rid]).standard_normal(self.n ** self.d)


def request_stream(count: int = 512, rate: float = 1.0, seed: int = 4,
                   n3=(32, 48, 64, 96, 128), n2=(128, 256, 512, 1024),
                   kernels=("inv_r", "neg_log", "exp"), ps=(6, 8)) -> list[Request]:
    """Poisson arrivals (exponential gaps of mean 1/rate) with random problem shapes."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(count):
        t += rng.exponential(1.0 / rate)
        d = int(rng.choice([2, 3]))
        n = int(rng.choice(n3 if d == 3 else n2))
        k = str(rng.choice(kernels))
        p = int(rng.choice(ps))
        out.append(Request(rid, t, d, n, k, p))
    return out
