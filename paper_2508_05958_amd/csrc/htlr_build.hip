// HTLR construction (Alg. 4.1) on the GPU, and the ABI entry points that
// create, inspect and release a matrix.
//
// What is built (all resident in HBM inside the handle):
// * geometry: nodes and cell lengths per dimension, a(x_i);
// * diagonal integrals D_i = int_Omega_i k(x_i, y) dy (eq. 1.4) by tensor
//   Gauss-Legendre: one value on a uniform grid (every cell is the same),
//   one per point otherwise (FP64 kernel);
// * inadmissible leaves (eq. 4.1) are NOT stored as dense blocks: the
//   product evaluates them on the fly.  Uniform grids with a radial kernel
//   keep a table of h^d k(h sqrt(s)) indexed by the integer squared distance
//   s (entry 0 holds D);
// * per level with admissible leaves: the CSR list of leaves, the Lagrange
//   factors U (targets) and V (sources, with the cell lengths folded into
//   the rows, so that W = (|Omega| o u) x_l V_l^T), and the cores
//   G(t, s) = k(xi_t - eta_s) of eq. 3.4.  On a uniform grid with a kernel
//   of x - y, G depends only on the offset between the two boxes, so one
//   core per (level, offset) is built (FP64, then rounded copies in FP32
//   and bfloat16); on other grids cores are generated inside the product.
//
// The orthonormalisation step of Alg. 4.1 (QR of every factor, core updated
// by the R factors) changes the representation but not the operator; the
// GPU keeps the interpolation form (raw Lagrange factors), which needs no
// per-pair core update and lets one core serve every pair with the same
// offset.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>

#include "htlr_device.h"
#include "htlr_handle.h"

namespace htlr {

thread_local std::string g_last_error;

htlr_status record(const Error& e) {
  g_last_error = e.what();
  return e.code;
}

template <class F>
htlr_status guarded(F&& f) {
  try {
    g_last_error.clear();
    f();
    return HTLR_OK;
  } catch (const Error& e) {
    return record(e);
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return HTLR_ERR_OOM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return HTLR_ERR_INVALID;
  }
}

// ---------------------------------------------------------------------------
// Construction kernels

// One core per offset: G[c][t][s] (s fastest).
template <int KID>
__global__ void k_core_build(const int* __restrict__ offs, const double* __restrict__ crel, double side,
                             int d, int p, int P, int pm1, double* __restrict__ G) {
  const int c = blockIdx.y;
  const int64_t PP = (int64_t)P * P;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < PP;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int t = (int)(idx / P), s = (int)(idx % P);
    double dx[3] = {0.0, 0.0, 0.0};
    int tt = t, ss = s;
    for (int l = 0; l < d; ++l) {
      int tl = tt % p, sl = ss % p;
      tt /= p;
      ss /= p;
      dx[l] = (crel[tl] - crel[sl]) - offs[3 * c + l] * side;
    }
    G[c * PP + idx] = kvec<KID, double>(dx[0], dx[1], dx[2], d, pm1);
  }
}

__global__ void k_downcast(const double* __restrict__ in, int64_t n, float* __restrict__ o32,
                           uint16_t* __restrict__ o16) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    float f = (float)in[i];
    if (o32) o32[i] = f;
    if (o16) o16[i] = f2bf(f);
  }
}

// Alg. 4.1's core update on a batch of cores: one mode product
// out = in x_axis M (M: r x dims[axis], row-major), the axes in memory order
// (fastest first: s_1..s_d, then t_1..t_d).  Grid: (blocks, cores).
struct CoreDims { int n[6]; };

__global__ void k_core_mode(const double* __restrict__ in, double* __restrict__ out, CoreDims dims, int axis,
                            const double* __restrict__ M, int r, int64_t in_per_core, int64_t out_per_core) {
  int64_t stride = 1;
  for (int k = 0; k < axis; ++k) stride *= dims.n[k];
  const int na = dims.n[axis];
  const double* src = in + (int64_t)blockIdx.y * in_per_core;
  double* dst = out + (int64_t)blockIdx.y * out_per_core;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < out_per_core;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t pre = idx % stride, rest = idx / stride;
    const int j = (int)(rest % r);
    const int64_t post = rest / r;
    const double* x = src + pre + stride * na * post;
    double acc = 0.0;
    for (int k = 0; k < na; ++k) acc += M[(int64_t)j * na + k] * x[stride * k];
    dst[idx] = acc;
  }
}

// Per-point diagonal integrals on a tensor grid (tensor Gauss-Legendre on
// the cell of each point, eq. 1.4).
template <int KID>
__global__ void k_diag(const double* __restrict__ x, const double* __restrict__ e, int n, int d, int pm1,
                       const double* __restrict__ gn, const double* __restrict__ gw, int order,
                       double* __restrict__ D, int64_t N) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * blockDim.x) {
    int idx[3] = {0, 0, 0};
    int64_t r = i;
    for (int l = 0; l < d; ++l) { idx[l] = (int)(r % n); r /= n; }
    double xi[3] = {0, 0, 0}, lo[3] = {0, 0, 0}, half[3] = {0, 0, 0};
    for (int l = 0; l < d; ++l) {
      xi[l] = x[l * n + idx[l]];
      lo[l] = e[l * (n + 1) + idx[l]];
      half[l] = 0.5 * (e[l * (n + 1) + idx[l] + 1] - lo[l]);
    }
    double tot = 0.0;
    int npts = (d == 3) ? order * order * order : order * order;
    for (int q = 0; q < npts; ++q) {
      int qq = q;
      double wt = 1.0, dx[3] = {0, 0, 0};
      for (int l = 0; l < d; ++l) {
        int k = qq % order;
        qq /= order;
        dx[l] = xi[l] - (lo[l] + (gn[k] + 1.0) * half[l]);
        wt *= gw[k] * half[l];
      }
      tot += wt * kvec<KID, double>(dx[0], dx[1], dx[2], d, pm1);
    }
    D[i] = tot;
  }
}

#define HTLR_DISPATCH_KID(kid, ...)                                              \
  switch (kid) {                                                                 \
    case HTLR_K_INV_R: { constexpr int KID = HTLR_K_INV_R; __VA_ARGS__; break; } \
    case HTLR_K_NEG_LOG: { constexpr int KID = HTLR_K_NEG_LOG; __VA_ARGS__; break; } \
    case HTLR_K_EXP: { constexpr int KID = HTLR_K_EXP; __VA_ARGS__; break; }     \
    case HTLR_K_GAUSS: { constexpr int KID = HTLR_K_GAUSS; __VA_ARGS__; break; } \
    case HTLR_K_POLY_TEST: { constexpr int KID = HTLR_K_POLY_TEST; __VA_ARGS__; break; } \
    default: fail(HTLR_ERR_INVALID, "unknown kernel");                          \
  }

// ---------------------------------------------------------------------------
// Allocation with a dry-run mode (htlr_footprint shares the build code).

struct Builder {
  htlr_matrix_impl* A;
  bool dry;
  size_t total = 0;

  void alloc(DevBuf& b, size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    total += bytes;
    if (!dry) b.alloc(bytes);
  }
  template <class T>
  void upload(DevBuf& b, const T* src, size_t count) {
    alloc(b, count * sizeof(T));
    if (!dry && count) HTLR_HIP(hipMemcpy(b.ptr, src, count * sizeof(T), hipMemcpyHostToDevice));
  }
  template <class T>
  void upload(DevBuf& b, const std::vector<T>& v) { upload(b, v.data(), v.size()); }
  template <class T>
  void upload_f32(DevBuf& b, const std::vector<T>& v) {
    std::vector<float> f(v.begin(), v.end());
    upload(b, f);
  }
};

// Alg. 4.1's QR step for one factor F (m x p, row-major): F = W R, W (m x r)
// with orthonormal columns, R (r x p), by Householder reflections.  With
// pivot, the column of largest remaining norm goes first and the
// factorisation stops at the first pivot with |R_kk| <= tol |R_00| (QR with
// column pivoting, truncated; the pivots' magnitudes do not increase).  R's
// columns come back in F's order, so F ~ W R.  Returns r.
static int orth_factor(const std::vector<double>& F, int m, int p, bool pivot, double tol, std::vector<double>* W,
                       std::vector<double>* R) {
  std::vector<double> A((size_t)m * p);                // column-major working copy
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < p; ++j) A[i + (size_t)m * j] = F[(size_t)i * p + j];
  std::vector<int> perm(p);
  for (int j = 0; j < p; ++j) perm[j] = j;
  const int kmax = std::min(m, p);
  std::vector<std::vector<double>> vs;
  std::vector<double> vvs;
  int r = kmax;
  double r00 = 0.0;
  for (int k = 0; k < kmax; ++k) {
    if (pivot) {
      int best = k;
      double bn = -1.0;
      for (int j = k; j < p; ++j) {
        double sq = 0.0;
        for (int i = k; i < m; ++i) sq += A[i + (size_t)m * j] * A[i + (size_t)m * j];
        if (sq > bn) { bn = sq; best = j; }
      }
      if (best != k) {
        for (int i = 0; i < m; ++i) std::swap(A[i + (size_t)m * k], A[i + (size_t)m * best]);
        std::swap(perm[k], perm[best]);
      }
    }
    double nrm = 0.0;
    for (int i = k; i < m; ++i) nrm += A[i + (size_t)m * k] * A[i + (size_t)m * k];
    nrm = std::sqrt(nrm);
    const double alpha = A[k + (size_t)m * k] >= 0.0 ? -nrm : nrm;
    std::vector<double> v(m - k);
    for (int i = k; i < m; ++i) v[i - k] = A[i + (size_t)m * k];
    v[0] -= alpha;
    double vv = 0.0;
    for (double x : v) vv += x * x;
    if (vv > 0.0)
      for (int j = k; j < p; ++j) {
        double dot = 0.0;
        for (int i = k; i < m; ++i) dot += v[i - k] * A[i + (size_t)m * j];
        const double f = 2.0 * dot / vv;
        for (int i = k; i < m; ++i) A[i + (size_t)m * j] -= f * v[i - k];
      }
    vs.push_back(std::move(v));
    vvs.push_back(vv);
    const double rkk = std::fabs(A[k + (size_t)m * k]);
    if (k == 0) r00 = rkk;
    if (pivot && rkk <= tol * r00) { r = k; break; }
  }
  r = std::max(r, 1);
  // W = first r columns of H_0 ... H_{r-1}
  W->assign((size_t)m * r, 0.0);
  std::vector<double> e(m);
  for (int j = 0; j < r; ++j) {
    std::fill(e.begin(), e.end(), 0.0);
    e[j] = 1.0;
    for (int k = std::min(r, (int)vs.size()) - 1; k >= 0; --k) {
      if (vvs[k] <= 0.0) continue;
      double dot = 0.0;
      for (int i = k; i < m; ++i) dot += vs[k][i - k] * e[i];
      const double f = 2.0 * dot / vvs[k];
      for (int i = k; i < m; ++i) e[i] -= f * vs[k][i - k];
    }
    for (int i = 0; i < m; ++i) (*W)[(size_t)i * r + j] = e[i];
  }
  R->assign((size_t)r * p, 0.0);
  for (int i = 0; i < r; ++i)
    for (int j = i; j < p; ++j) (*R)[(size_t)i * p + perm[j]] = A[i + (size_t)m * j];
  return r;
}

static bool translation_invariant(const htlr_matrix_impl& A) {
  // every kernel of the enumeration is a function of x - y; the grid decides
  return A.uniform;
}

static void build_impl(htlr_matrix_impl& A, Builder& bd, const double* a_host) {
  const int d = A.d, p = A.p, P = A.P;
  const Grid& g = A.grid;
  const Plan& pl = A.plan;
  const int pm1 = p - 1;
  const bool ti = translation_invariant(A);

  // geometry
  bd.upload(A.x64, g.x);
  bd.upload_f32(A.x32, g.x);
  bd.upload(A.w64, g.w);
  bd.upload_f32(A.w32, g.w);
  {
    std::vector<double> a(A.N, 0.0);
    if (a_host && !bd.dry) std::copy(a_host, a_host + A.N, a.begin());
    bd.upload(A.a64, a);
    bd.upload_f32(A.a32, a);
  }

  // diagonal integrals (eq. 1.4)
  if (A.uniform) {
    double x0[3] = {0, 0, 0}, lo[3], hi[3];
    for (int l = 0; l < d; ++l) { lo[l] = -0.5 * A.h; hi[l] = 0.5 * A.h; }
    A.D0 = cell_integral(A.kid, d, p, x0, lo, hi, A.gl_order);
  } else {
    bd.alloc(A.D64, A.N * sizeof(double));
    bd.alloc(A.D32, A.N * sizeof(float));
    if (!bd.dry) {
      std::vector<double> gn, gw;
      gauss_legendre(A.gl_order, &gn, &gw);
      DevBuf dgn, dgw, de;
      Builder tmp{&A, false};
      tmp.upload(dgn, gn);
      tmp.upload(dgw, gw);
      tmp.upload(de, g.e);
      int blocks = (int)std::min<int64_t>((A.N + 255) / 256, 65535);
      HTLR_DISPATCH_KID(A.kid, hipLaunchKernelGGL(k_diag<KID>, dim3(blocks), dim3(256), 0, 0,
                                                  A.x64.as<double>(), de.as<double>(), A.n, d, pm1,
                                                  dgn.as<double>(), dgw.as<double>(), A.gl_order,
                                                  A.D64.as<double>(), A.N));
      HTLR_HIP(hipGetLastError());
      hipLaunchKernelGGL(k_downcast, dim3(blocks), dim3(256), 0, 0, A.D64.as<double>(), A.N,
                         A.D32.as<float>(), (uint16_t*)nullptr);
      HTLR_HIP(hipDeviceSynchronize());
      std::vector<double> d0(1);
      HTLR_HIP(hipMemcpy(d0.data(), A.D64.ptr, sizeof(double), hipMemcpyDeviceToHost));
      A.D0 = d0[0];
    }
  }

  // inadmissible leaves (level L)
  bd.upload(A.near_ptr, pl.near.ptr);
  bd.upload(A.near_src, pl.near.src);
  if (A.uniform && A.kid != HTLR_K_POLY_TEST) {
    // largest |offset| between near boxes, then the largest squared index distance
    const int B = pl.B[A.L], m = pl.m[A.L];
    int maxoff = 0;
    for (int64_t t = 0; t + 1 < (int64_t)pl.near.ptr.size(); ++t)
      for (int64_t q = pl.near.ptr[t]; q < pl.near.ptr[t + 1]; ++q) {
        int64_t a = t, b = pl.near.src[q];
        for (int l = 0; l < d; ++l) {
          maxoff = std::max(maxoff, (int)std::abs((int)(a % B) - (int)(b % B)));
          a /= B;
          b /= B;
        }
      }
    int64_t dmax = (int64_t)maxoff * m + m - 1;
    A.Tsize = (int)(d * dmax * dmax + 1);
    std::vector<double> T(A.Tsize);
    T[0] = A.D0;
    for (int s = 1; s < A.Tsize; ++s) {
      double dx[3] = {A.h * std::sqrt((double)s), 0.0, 0.0};
      T[s] = A.w0 * kernel_host(A.kid, d, p, dx);
    }
    bd.upload(A.T64, T);
    bd.upload_f32(A.T32, T);
  }

  // Alg. 4.1's QR step (uniform grids: one factor per level).  Each level
  // keeps its own rank: QRCP truncates a level's factor to its numerical
  // rank, and that level's cores become rank^d x rank^d.
  std::vector<std::vector<double>> orthW(A.L + 1), orthR(A.L + 1);
  std::vector<int> rl(A.L + 1, p);
  if (A.orth) {
    std::vector<double> ch(p);
    for (int l = 0; l <= A.L; ++l) {
      if (pl.adm[l].nnz() == 0) continue;
      const int m = pl.m[l];
      chebyshev_points(0.0, m * A.h, p, ch.data());
      std::vector<double> xs(m), U((size_t)m * p);
      for (int i = 0; i < m; ++i) xs[i] = (i + 0.5) * A.h;
      lagrange_matrix(xs.data(), m, ch.data(), p, U.data());
      rl[l] = orth_factor(U, m, p, A.orth == 2, A.rank_tol, &orthW[l], &orthR[l]);
    }
  }
  int rank_max = 0, P_max = 0;

  // admissible leaves, factors and cores per level
  A.levels.clear();
  A.levels.resize(A.L + 1);
  std::vector<double> cheb(p), Lm;
  for (int l = 0; l <= A.L; ++l) {
    LevelData& lv = A.levels[l];
    lv.level = l;
    lv.B = pl.B[l];
    lv.m = pl.m[l];
    lv.rank = rl[l];
    lv.P = 1;
    for (int k = 0; k < d; ++k) lv.P *= lv.rank;
    lv.nbox = 1;
    for (int k = 0; k < d; ++k) lv.nbox *= lv.B;
    lv.npairs = pl.adm[l].nnz();
    if (lv.npairs == 0) continue;
    rank_max = std::max(rank_max, lv.rank);
    P_max = std::max(P_max, lv.P);
    const int m = lv.m, B = lv.B, rank = lv.rank, Pr = lv.P;
    bd.upload(lv.ptr, pl.adm[l].ptr);
    bd.upload(lv.src, pl.adm[l].src);
    if (A.uniform) {
      // one factor for every box and dimension: nodes (i + 1/2) h on [0, m h]
      chebyshev_points(0.0, m * A.h, p, cheb.data());
      std::vector<double> xs(m);
      for (int i = 0; i < m; ++i) xs[i] = (i + 0.5) * A.h;
      std::vector<double> U((size_t)m * p), V;
      lagrange_matrix(xs.data(), m, cheb.data(), p, U.data());
      if (A.orth) U = orthW[l];            // U = W R: store W (m x rank), R goes into the cores
      V.resize(U.size());
      for (size_t i = 0; i < U.size(); ++i) V[i] = A.h * U[i];
      bd.upload(lv.U64, U);
      bd.upload(lv.V64, V);
      bd.upload_f32(lv.U32, U);
      bd.upload_f32(lv.V32, V);
    } else {
      std::vector<double> U((size_t)d * B * m * p), V(U.size()), ch((size_t)d * B * p);
      for (int k = 0; k < d; ++k)
        for (int b = 0; b < B; ++b) {
          const double* e = &g.e[(size_t)k * (g.n + 1)];
          chebyshev_points(e[(size_t)b * m], e[(size_t)(b + 1) * m], p, &ch[((size_t)k * B + b) * p]);
          double* Ub = &U[(((size_t)k * B + b) * m) * p];
          lagrange_matrix(&g.x[(size_t)k * g.n + (size_t)b * m], m, &ch[((size_t)k * B + b) * p], p, Ub);
          for (int i = 0; i < m; ++i)
            for (int t = 0; t < p; ++t)
              V[(((size_t)k * B + b) * m + i) * p + t] = g.w[(size_t)k * g.n + (size_t)b * m + i] * Ub[(size_t)i * p + t];
        }
      bd.upload(lv.U64, U);
      bd.upload(lv.V64, V);
      bd.upload_f32(lv.U32, U);
      bd.upload_f32(lv.V32, V);
      bd.upload(lv.cheb64, ch);
      bd.upload_f32(lv.cheb32, ch);
    }
    if (ti) {
      // one core per offset sigma - tau
      const int span = 2 * B - 1;
      std::vector<int> lut((size_t)span * span * (d == 3 ? span : 1), -1);
      std::vector<int32_t> cid(lv.npairs);
      lv.offsets.clear();
      const Csr& cs = pl.adm[l];
      for (int64_t t = 0; t < lv.nbox; ++t)
        for (int64_t q = cs.ptr[t]; q < cs.ptr[t + 1]; ++q) {
          int64_t a = t, b = cs.src[q];
          int off[3] = {0, 0, 0};
          int64_t key = 0, stride = 1;
          for (int k = 0; k < d; ++k) {
            off[k] = (int)(b % B) - (int)(a % B);
            a /= B;
            b /= B;
            key += (off[k] + B - 1) * stride;
            stride *= span;
          }
          if (lut[key] < 0) {
            lut[key] = (int)(lv.offsets.size() / 3);
            lv.offsets.insert(lv.offsets.end(), {off[0], off[1], off[2]});
          }
          cid[q] = lut[key];
        }
      lv.ncore = (int)(lv.offsets.size() / 3);
      bd.upload(lv.cid, cid);
      const size_t csz = (size_t)lv.ncore * Pr * Pr;      // stored cores, rank^d x rank^d each
      const bool want64 = A.precisions & (1 << HTLR_FP64);
      const bool want32 = A.precisions & (1 << HTLR_FP32);
      const bool want16 = A.precisions & (1 << HTLR_BF16_CORE);
      DevBuf tmp64;
      DevBuf& G64 = want64 ? lv.Gm64 : tmp64;
      if (want64) bd.alloc(lv.Gm64, csz * sizeof(double));
      if (want32) bd.alloc(lv.Gm32, csz * sizeof(float));
      if (want16) bd.alloc(lv.Gm16, csz * sizeof(uint16_t));
      if (!bd.dry) {
        if (!want64) tmp64.alloc(csz * sizeof(double));
        DevBuf doff, dcrel;
        Builder t2{&A, false};
        t2.upload(doff, lv.offsets);
        std::vector<double> crel(cheb.begin(), cheb.end());
        chebyshev_points(0.0, m * A.h, p, crel.data());
        t2.upload(dcrel, crel);
        const int64_t PP = (int64_t)P * P;
        // interpolation cores (eq. 3.4); with the QR step, into a work buffer
        DevBuf raw, work, dR;
        if (A.orth) {
          raw.alloc((size_t)lv.ncore * PP * sizeof(double));
          work.alloc((size_t)lv.ncore * PP * sizeof(double));
          t2.upload(dR, orthR[l]);
        }
        double* Gbuild = A.orth ? raw.as<double>() : G64.as<double>();
        int bx = (int)std::min<int64_t>((PP + 255) / 256, 1024);
        HTLR_DISPATCH_KID(A.kid, hipLaunchKernelGGL(k_core_build<KID>, dim3(bx, lv.ncore), dim3(256), 0, 0,
                                                    doff.as<int>(), dcrel.as<double>(), m * A.h, d, p, P,
                                                    pm1, Gbuild));
        HTLR_HIP(hipGetLastError());
        if (A.orth) {
          // G <- G x_1 R ... x_d R x_{d+1} R ... x_{2d} R (U = W R and V = h W R),
          // one mode product per axis, the last one into the stored cores
          CoreDims dims{};
          for (int k = 0; k < 2 * d; ++k) dims.n[k] = p;
          double* bufs[2] = {raw.as<double>(), work.as<double>()};
          int cur = 0;
          int64_t in_per = PP;
          for (int ax = 0; ax < 2 * d; ++ax) {
            int64_t out_per = in_per / p * rank;
            double* dst = ax == 2 * d - 1 ? G64.as<double>() : bufs[cur ^ 1];
            int bm = (int)std::min<int64_t>((out_per + 255) / 256, 1024);
            hipLaunchKernelGGL(k_core_mode, dim3(bm, lv.ncore), dim3(256), 0, 0, bufs[cur], dst, dims, ax,
                               dR.as<double>(), rank, in_per, out_per);
            HTLR_HIP(hipGetLastError());
            dims.n[ax] = rank;
            in_per = out_per;
            cur ^= 1;
          }
        }
        int nb = (int)std::min<int64_t>(((int64_t)csz + 255) / 256, 65535);
        if (want32 || want16)
          hipLaunchKernelGGL(k_downcast, dim3(nb), dim3(256), 0, 0, G64.as<double>(), (int64_t)csz,
                             want32 ? lv.Gm32.as<float>() : (float*)nullptr,
                             want16 ? lv.Gm16.as<uint16_t>() : (uint16_t*)nullptr);
        HTLR_HIP(hipGetLastError());
        HTLR_HIP(hipDeviceSynchronize());
      }
    }
  }
  // the handle's rank and P: the largest over the levels with admissible leaves
  if (rank_max == 0) {
    rank_max = p;
    P_max = P;
  }
  A.rank = rank_max;
  A.P = P_max;
}

static void init_handle(htlr_matrix_impl& A, const double* points, int kernel, int d, int n, int p,
                        int leaf, const htlr_build_opts* opts) {
  if (!kernel_known(kernel)) fail(HTLR_ERR_INVALID, "unknown kernel");
  if (p < 1 || p > kMaxP) fail(HTLR_ERR_INVALID, "p out of range (1..12)");
  A.grid = make_grid(points, d, n, opts ? opts->edges : nullptr);
  A.d = d;
  A.n = n;
  A.p = p;
  A.leaf = leaf;
  A.kid = kernel;
  A.N = 1;
  A.P = 1;
  for (int l = 0; l < d; ++l) { A.N *= n; A.P *= p; }
  A.uniform = A.grid.uniform;
  A.eta2 = (opts && opts->eta2 > 0) ? opts->eta2 : 1.0;
  A.adm_kind = opts ? opts->admissibility : HTLR_ADM_STRONG;
  A.gl_order = (opts && opts->gl_order > 0) ? opts->gl_order : (d == 2 ? 16 : 8);
  if (A.gl_order > 64) fail(HTLR_ERR_INVALID, "gl_order too large");
  A.precisions = (opts && opts->precisions) ? (opts->precisions & 7) : 7;
  if (!A.precisions) fail(HTLR_ERR_INVALID, "precisions mask selects nothing");
  A.orth = opts ? opts->orthonormalize : 0;
  if (A.orth < 0 || A.orth > 2) fail(HTLR_ERR_INVALID, "orthonormalize must be 0, 1 or 2");
  A.rank_tol = (opts && opts->rank_tol > 0) ? opts->rank_tol : 1e-13;
  A.rank = p;
  A.h = 1.0 / n;
  A.w0 = std::pow(A.h, d);
  A.plan = make_plan(A.grid, leaf, A.eta2, A.adm_kind);
  A.L = A.plan.L;
  if (A.orth && !A.grid.uniform)
    fail(HTLR_ERR_UNSUPPORTED, "orthonormal factors need a uniform grid (cores are shared by offset)");
  if (opts && opts->a) {
    for (int64_t i = 0; i < A.N; ++i)
      if (!std::isfinite(opts->a[i])) fail(HTLR_ERR_NUMERIC, "a(x) has NaN/Inf");
  }
}

}  // namespace htlr

using namespace htlr;

extern "C" {

const char* htlr_last_error(void) { return g_last_error.c_str(); }

htlr_status htlr_build(const double* points, htlr_kernel kernel, int d, int n, int p, int leaf,
                       const htlr_build_opts* opts, htlr_matrix* out) {
  if (!out) { g_last_error = "out is NULL"; return HTLR_ERR_INVALID; }
  *out = nullptr;
  htlr_matrix_s* A = nullptr;
  htlr_status st = guarded([&] {
    A = new htlr_matrix_s();
    init_handle(*A, points, kernel, d, n, p, leaf, opts);
    HTLR_HIP(hipGetDevice(&A->device));
    Builder bd{A, false};
    build_impl(*A, bd, opts ? opts->a : nullptr);
    A->device_bytes = bd.total;
  });
  if (st != HTLR_OK) {
    delete A;
    return st;
  }
  *out = A;
  return HTLR_OK;
}

htlr_status htlr_footprint(const double* points, htlr_kernel kernel, int d, int n, int p, int leaf,
                           const htlr_build_opts* opts, size_t* bytes) {
  if (!bytes) { g_last_error = "bytes is NULL"; return HTLR_ERR_INVALID; }
  return guarded([&] {
    htlr_matrix_s A;
    init_handle(A, points, kernel, d, n, p, leaf, opts);
    Builder bd{&A, true};
    build_impl(A, bd, nullptr);
    *bytes = bd.total;
  });
}

htlr_status htlr_info(htlr_matrix A, htlr_info_t* info) {
  if (!A || !info) { g_last_error = "null argument"; return HTLR_ERR_INVALID; }
  return guarded([&] {
    std::memset(info, 0, sizeof(*info));
    // quasi-uniform handles: the structure is that of the uniform-grid matrix
    const htlr_matrix_impl& S = A->quasi ? quasi_inner(*A) : *A;
    info->d = A->d;
    info->n = A->n;
    info->p = A->p;
    info->leaf_side = S.plan.m[S.L];
    info->levels = S.L;
    info->uniform = A->uniform ? 1 : 0;
    for (int l = 0; l <= S.L && l < 16; ++l) {
      info->adm_pairs[l] = S.plan.adm[l].nnz();
      info->unique_cores[l] = S.levels[l].ncore;
      info->level_rank[l] = S.levels[l].npairs > 0 ? S.levels[l].rank : 0;
    }
    info->near_pairs = S.plan.near.nnz();
    info->device_bytes = A->device_bytes;
    info->diag0 = S.D0;
    info->uniform_m = A->quasi ? S.n : 0;
    info->rank = S.rank;
  });
}

void htlr_free(htlr_matrix A) {
  if (!A) return;
  (void)hipDeviceSynchronize();
  delete A;
}

htlr_status htlr_plan_counts(const double* points, const double* edges, int d, int n, int leaf, double eta2,
                             int admissibility, int* levels, int64_t* adm_per_level, int64_t* near_pairs) {
  if (!levels || !adm_per_level || !near_pairs) { g_last_error = "null argument"; return HTLR_ERR_INVALID; }
  return guarded([&] {
    Grid g = make_grid(points, d, n, edges);
    Plan pl = make_plan(g, leaf, eta2, admissibility);
    *levels = pl.L;
    for (int l = 0; l < 16; ++l) adm_per_level[l] = l <= pl.L ? pl.adm[l].nnz() : 0;
    *near_pairs = pl.near.nnz();
  });
}

htlr_status htlr_plan_pairs(const double* points, const double* edges, int d, int n, int leaf, double eta2,
                            int admissibility, int level, int32_t* tau, int32_t* sigma, int64_t cap, int64_t* count) {
  if (!count) { g_last_error = "null argument"; return HTLR_ERR_INVALID; }
  return guarded([&] {
    Grid g = make_grid(points, d, n, edges);
    Plan pl = make_plan(g, leaf, eta2, admissibility);
    if (level > pl.L) fail(HTLR_ERR_INVALID, "level beyond the tree depth");
    const Csr& c = level >= 0 ? pl.adm[level] : pl.near;
    int64_t k = 0;
    for (int64_t t = 0; t + 1 < (int64_t)c.ptr.size(); ++t)
      for (int64_t q = c.ptr[t]; q < c.ptr[t + 1]; ++q, ++k)
        if (k < cap && tau && sigma) {
          tau[k] = (int32_t)t;
          sigma[k] = c.src[q];
        }
    *count = k;
  });
}

}  // extern "C"
