// Internal declarations shared by the host planner, construction and the
// product/solver drivers of the HTLR library.
#pragma once

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "htlr.h"

namespace htlr {

struct Error : std::runtime_error {
  htlr_status code;
  Error(htlr_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(htlr_status c, const std::string& m) { throw Error(c, m); }

constexpr int kMaxLevels = 16;
constexpr int kMaxP = 12;

// Tensor grid in [0,1]^d: nodes, Voronoi cell edges and cell lengths per
// dimension (Sec. 2.2; quasi-uniform weights of Sec. 3.3).
struct Grid {
  int d = 0, n = 0;
  bool uniform = false;           // cell-centred uniform grid (Example 2.2)
  std::vector<double> x;          // d*n nodes, x[l*n + k]
  std::vector<double> e;          // d*(n+1) edges, e[l*(n+1) + k]
  std::vector<double> w;          // d*n cell lengths, w[l*n + k]
};

// The tensor grid of the nodes (NULL: uniform cell centres) and its cells:
// the caller's edges (d*(n+1), dimension-major) or, with NULL, the 1D Voronoi
// cells (midpoints, 0 and 1 at the ends).  Uniform when nodes and cells equal
// the uniform ones to 1e-14.
Grid make_grid(const double* points, int d, int n, const double* edges = nullptr);

// Per-level block lists in CSR form over target boxes: the leaves of the
// block cluster tree (Def. 2.4) at one level of the cluster tree.
struct Csr {
  std::vector<int64_t> ptr;       // B^d + 1
  std::vector<int32_t> src;       // source boxes (linear index), sorted per row
  int64_t nnz() const { return src.empty() ? 0 : (int64_t)src.size(); }
};

struct Plan {
  int d = 0, n = 0, L = 0;        // L = depth of the cluster tree
  std::vector<int> m;             // points per box side at level l (0..L)
  std::vector<int> B;             // boxes per dimension at level l
  std::vector<Csr> adm;           // admissible leaves per level (0..L)
  Csr near;                       // inadmissible leaves (all at level L)
};

// Depth and box sides for n points per side and leaf threshold leaf^d;
// throws HTLR_ERR_UNSUPPORTED when n does not halve exactly.
void tree_shape(int d, int n, int leaf, int* L, std::vector<int>* m);

Plan make_plan(const Grid& g, int leaf, double eta2, int adm_kind);

// Interpolation on one interval (Sec. 3.1).
void chebyshev_points(double a, double b, int p, double* out);
// L[i*p + t] = L_t(x_i) for the p nodes xi.
void lagrange_matrix(const double* x, int m, const double* xi, int p, double* L);

// Kernel k evaluated at the difference vector dx = x - y (host, double).
double kernel_host(int kid, int d, int p, const double* dx);
bool kernel_known(int kid);

// Diagonal integral of eq. 1.4: int over the cell [lo, hi] of k(x - y) dy by
// tensor Gauss-Legendre of the given order (host, double).
double cell_integral(int kid, int d, int p, const double* x, const double* lo, const double* hi,
                     int order);
void gauss_legendre(int order, std::vector<double>* nodes, std::vector<double>* weights);

}  // namespace htlr
