// Host planner: tensor grid, cluster tree shape, block cluster tree lists,
// Chebyshev/Lagrange interpolation and Gauss-Legendre diagonal integrals.
//
// Cluster tree: the recursive 2^d partition of Sec. 2.2 (Def. 2.1, 3.5); on
// the grids this library accepts every box at level l has m_l = n / 2^l
// points per side, and a box is a leaf when m_l^d <= leaf^d.
//
// Block cluster tree (Def. 2.4): built level by level.  A pair (tau, sigma)
// at level l is visited iff its parent pair was visited and inadmissible;
// a visited pair is an admissible leaf if admissible, an inadmissible leaf
// if l = L (both nodes are leaves), and is refined otherwise.
//
// Admissibility: strong (Def. 2.3), max(diam^2) <= eta2 * dist^2 with
// equality admissible, or weak (Def. 2.2), zero-volume overlap.  On uniform
// grids box edges are integers in units of h, so the test is exact.

#include <algorithm>
#include <cmath>
#include <cstring>

#include "htlr_internal.h"

namespace htlr {

Grid make_grid(const double* points, int d, int n, const double* edges) {
  if (d != 2 && d != 3) fail(HTLR_ERR_UNSUPPORTED, "d must be 2 or 3");
  if (n < 1 || n > (1 << 15)) fail(HTLR_ERR_INVALID, "n out of range");
  Grid g;
  g.d = d;
  g.n = n;
  g.x.resize((size_t)d * n);
  g.e.resize((size_t)d * (n + 1));
  g.w.resize((size_t)d * n);
  bool uniform = true;
  for (int l = 0; l < d; ++l) {
    for (int k = 0; k < n; ++k) {
      double xu = (k + 0.5) / n;
      double v = points ? points[(size_t)l * n + k] : xu;
      if (!std::isfinite(v) || v <= 0.0 || v >= 1.0) fail(HTLR_ERR_INVALID, "node outside (0,1)");
      if (k > 0 && !(v > g.x[(size_t)l * n + k - 1])) fail(HTLR_ERR_INVALID, "nodes not increasing");
      if (std::fabs(v - xu) > 1e-14) uniform = false;
      g.x[(size_t)l * n + k] = v;
    }
  }
  if (edges) {
    // caller's cells: every node inside its cell, cells increasing within [0, 1]
    for (int l = 0; l < d; ++l) {
      const double* e = edges + (size_t)l * (n + 1);
      for (int k = 0; k <= n; ++k) {
        if (!std::isfinite(e[k]) || e[k] < 0.0 || e[k] > 1.0) fail(HTLR_ERR_INVALID, "cell edge outside [0,1]");
        if (k > 0 && !(e[k] > e[k - 1])) fail(HTLR_ERR_INVALID, "cell edges not increasing");
        if (std::fabs(e[k] - (double)k / n) > 1e-14) uniform = false;
      }
      for (int k = 0; k < n; ++k) {
        const double x = g.x[(size_t)l * n + k];
        if (x < e[k] || x > e[k + 1]) fail(HTLR_ERR_INVALID, "node outside its cell");
      }
    }
  }
  g.uniform = uniform;
  for (int l = 0; l < d; ++l) {
    double* e = &g.e[(size_t)l * (n + 1)];
    const double* x = &g.x[(size_t)l * n];
    if (uniform) {
      for (int k = 0; k <= n; ++k) e[k] = (double)k / n;
      for (int k = 0; k < n; ++k) g.x[(size_t)l * n + k] = (k + 0.5) / n;
    } else if (edges) {
      for (int k = 0; k <= n; ++k) e[k] = edges[(size_t)l * (n + 1) + k];
    } else {
      e[0] = 0.0;
      e[n] = 1.0;
      for (int k = 1; k < n; ++k) e[k] = 0.5 * (x[k - 1] + x[k]);
    }
    for (int k = 0; k < n; ++k) g.w[(size_t)l * n + k] = e[k + 1] - e[k];
  }
  return g;
}

void tree_shape(int d, int n, int leaf, int* L, std::vector<int>* m) {
  if (leaf < 1) fail(HTLR_ERR_INVALID, "leaf must be >= 1");
  m->clear();
  int side = n;
  m->push_back(side);
  // a cluster is a leaf when it has at most leaf^d points
  while (side > leaf) {
    if (side % 2) fail(HTLR_ERR_UNSUPPORTED, "n does not halve exactly down to the leaf level");
    side /= 2;
    m->push_back(side);
  }
  *L = (int)m->size() - 1;
  if (*L >= kMaxLevels) fail(HTLR_ERR_UNSUPPORTED, "tree too deep");
  (void)d;
}

namespace {

struct BoxGeom {
  const Grid* g;
  bool integer;
  int L;
  const std::vector<int>* m;
  // edge coordinate of index k in dimension l (units of h when integer)
  double edge(int l, int64_t k) const {
    if (integer) return (double)k;
    return g->e[(size_t)l * (g->n + 1) + k];
  }
  void box(int level, const int* b, double* lo, double* hi) const {
    int ml = (*m)[level];
    for (int l = 0; l < g->d; ++l) {
      lo[l] = edge(l, (int64_t)b[l] * ml);
      hi[l] = edge(l, (int64_t)(b[l] + 1) * ml);
    }
  }
};

inline void unrank(int64_t lin, int B, int d, int* b) {
  for (int l = 0; l < d; ++l) {
    b[l] = (int)(lin % B);
    lin /= B;
  }
}

inline int64_t rank(const int* b, int B, int d) {
  int64_t lin = 0, s = 1;
  for (int l = 0; l < d; ++l) {
    lin += (int64_t)b[l] * s;
    s *= B;
  }
  return lin;
}

}  // namespace

Plan make_plan(const Grid& g, int leaf, double eta2, int adm_kind) {
  if (adm_kind != HTLR_ADM_STRONG && adm_kind != HTLR_ADM_WEAK)
    fail(HTLR_ERR_INVALID, "unknown admissibility");
  if (!(eta2 > 0.0)) eta2 = 1.0;
  Plan P;
  P.d = g.d;
  P.n = g.n;
  tree_shape(g.d, g.n, leaf, &P.L, &P.m);
  const int d = g.d;
  for (int l = 0; l <= P.L; ++l) P.B.push_back(g.n / P.m[l]);
  BoxGeom geo{&g, g.uniform, P.L, &P.m};

  auto admissible = [&](int level, const int* bt, const int* bs) -> bool {
    double lo1[3], hi1[3], lo2[3], hi2[3];
    geo.box(level, bt, lo1, hi1);
    geo.box(level, bs, lo2, hi2);
    if (adm_kind == HTLR_ADM_WEAK) {
      double v = 1.0;
      for (int l = 0; l < d; ++l) v *= std::max(0.0, std::min(hi1[l], hi2[l]) - std::max(lo1[l], lo2[l]));
      return v == 0.0;
    }
    double dm1 = 0, dm2 = 0, ds = 0;
    for (int l = 0; l < d; ++l) {
      dm1 += (hi1[l] - lo1[l]) * (hi1[l] - lo1[l]);
      dm2 += (hi2[l] - lo2[l]) * (hi2[l] - lo2[l]);
      double gap = std::max(0.0, std::max(lo2[l] - hi1[l], lo1[l] - hi2[l]));
      ds += gap * gap;
    }
    return std::max(dm1, dm2) <= eta2 * ds;
  };

  P.adm.resize(P.L + 1);
  // inadmissible visited pairs at the current level (CSR over target boxes)
  Csr inad;
  inad.ptr = {0, 0};
  {
    int b0[3] = {0, 0, 0};
    P.adm[0].ptr = {0, 0};
    if (admissible(0, b0, b0)) {
      P.adm[0].src.push_back(0);
      P.adm[0].ptr[1] = 1;
    } else {
      inad.src.push_back(0);
      inad.ptr[1] = 1;
    }
  }
  for (int l = 1; l <= P.L; ++l) {
    const int B = P.B[l], Bp = P.B[l - 1];
    int64_t nb = 1;
    for (int k = 0; k < d; ++k) nb *= B;
    Csr A, I;
    A.ptr.assign(nb + 1, 0);
    I.ptr.assign(nb + 1, 0);
    std::vector<int32_t> rowA, rowI;
    const int nchild = 1 << d;
    for (int64_t t = 0; t < nb; ++t) {
      int bt[3] = {0, 0, 0}, pt[3] = {0, 0, 0};
      unrank(t, B, d, bt);
      for (int k = 0; k < d; ++k) pt[k] = bt[k] / 2;
      int64_t tp = rank(pt, Bp, d);
      rowA.clear();
      rowI.clear();
      for (int64_t q = inad.ptr[tp]; q < inad.ptr[tp + 1]; ++q) {
        int ps[3] = {0, 0, 0};
        unrank(inad.src[q], Bp, d, ps);
        for (int c = 0; c < nchild; ++c) {
          int bs[3] = {0, 0, 0};
          for (int k = 0; k < d; ++k) bs[k] = 2 * ps[k] + ((c >> k) & 1);
          int32_t s = (int32_t)rank(bs, B, d);
          if (admissible(l, bt, bs)) rowA.push_back(s);
          else rowI.push_back(s);
        }
      }
      std::sort(rowA.begin(), rowA.end());
      std::sort(rowI.begin(), rowI.end());
      A.src.insert(A.src.end(), rowA.begin(), rowA.end());
      I.src.insert(I.src.end(), rowI.begin(), rowI.end());
      A.ptr[t + 1] = (int64_t)A.src.size();
      I.ptr[t + 1] = (int64_t)I.src.size();
    }
    P.adm[l] = std::move(A);
    inad = std::move(I);
  }
  P.near = std::move(inad);
  return P;
}

// ---------------------------------------------------------------------------
// Interpolation (Sec. 3.1)

void chebyshev_points(double a, double b, int p, double* out) {
  for (int t = 1; t <= p; ++t)
    out[t - 1] = 0.5 * (b - a) * std::cos((2.0 * t - 1.0) * M_PI / (2.0 * p)) + 0.5 * (b + a);
}

void lagrange_matrix(const double* x, int m, const double* xi, int p, double* L) {
  for (int i = 0; i < m; ++i)
    for (int t = 0; t < p; ++t) {
      double v = 1.0;
      for (int j = 0; j < p; ++j)
        if (j != t) v *= (x[i] - xi[j]) / (xi[t] - xi[j]);
      L[(size_t)i * p + t] = v;
    }
}

// ---------------------------------------------------------------------------
// Kernels (host copies; the device versions live with the kernels)

static const double kPolyA[3] = {0.50, 0.30, 0.20};

bool kernel_known(int kid) {
  return kid == HTLR_K_INV_R || kid == HTLR_K_NEG_LOG || kid == HTLR_K_EXP || kid == HTLR_K_GAUSS ||
         kid == HTLR_K_POLY_TEST;
}

double kernel_host(int kid, int d, int p, const double* dx) {
  double r2 = 0;
  for (int l = 0; l < d; ++l) r2 += dx[l] * dx[l];
  switch (kid) {
    case HTLR_K_INV_R: return 1.0 / std::sqrt(r2);
    case HTLR_K_NEG_LOG: return -0.5 * std::log(r2);
    case HTLR_K_EXP: return std::exp(-std::sqrt(r2));
    case HTLR_K_GAUSS: return std::exp(-r2 / (2.0 * d));
    case HTLR_K_POLY_TEST: {
      double v = 1.0;
      for (int l = 0; l < d; ++l) v *= std::pow(1.0 + kPolyA[l] * dx[l], p - 1);
      return v;
    }
  }
  fail(HTLR_ERR_INVALID, "unknown kernel");
}

// Gauss-Legendre rule on [-1, 1]: Newton's method on P_order using the
// three-term recurrence, started from the asymptotic root estimates.
void gauss_legendre(int order, std::vector<double>* nodes, std::vector<double>* weights) {
  nodes->assign(order, 0.0);
  weights->assign(order, 0.0);
  for (int i = 0; i < (order + 1) / 2; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (order + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= order; ++k) {
        double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      dp = order * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    {
      // re-evaluate the derivative at the converged root
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= order; ++k) {
        double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      dp = order * (z * p1 - p0) / (z * z - 1.0);
    }
    (*nodes)[i] = -z;
    (*nodes)[order - 1 - i] = z;
    double wgt = 2.0 / ((1.0 - z * z) * dp * dp);
    (*weights)[i] = wgt;
    (*weights)[order - 1 - i] = wgt;
  }
}

double cell_integral(int kid, int d, int p, const double* x, const double* lo, const double* hi,
                     int order) {
  std::vector<double> gn, gw;
  gauss_legendre(order, &gn, &gw);
  double total = 0.0;
  int npts = 1;
  for (int l = 0; l < d; ++l) npts *= order;
  for (int q = 0; q < npts; ++q) {
    int r = q;
    double wt = 1.0, dx[3] = {0, 0, 0};
    for (int l = 0; l < d; ++l) {
      int k = r % order;
      r /= order;
      double half = 0.5 * (hi[l] - lo[l]);
      double y = lo[l] + (gn[k] + 1.0) * half;
      dx[l] = x[l] - y;
      wt *= gw[k] * half;
    }
    total += wt * kernel_host(kid, d, p, dx);
  }
  return total;
}

}  // namespace htlr
