// Quasi-uniform grids through a uniform one (Sec. 3.3, eq. 3.9):
//
//     f = a o u + T Ahat S u,
//
// Ahat the HTLR matrix of the kernel on the uniform cell-centred grid of m^d
// cells (a = 0), S and T the cell-overlap transfers between the two grids
// (a vector read as piecewise constant on its cells):
//
//     S[t,i] = |Omega_t^uni cap Omega_i| / |Omega_t^uni|    (m^d x n^d),
//     T[i,t] = |Omega_i cap Omega_t^uni| / |Omega_i|        (n^d x m^d).
//
// Cells of a tensor grid are products of 1D intervals, so S and T are
// Kronecker products of 1D overlap matrices S_l (m x n) and T_l (n x m).  A
// row of a 1D overlap matrix covers a contiguous run of cells; it is stored
// as a band of fixed width w (the longest run, at most the number of input
// cells) starting at column lo[r], clamped so that the band stays inside the
// input, with zeros outside the run.
//
// k_transfer applies the Kronecker product directly: one thread per output
// point, w^d products per point from a w^d neighbourhood of the input, which
// neighbouring threads share in cache (first index fastest on both sides).
// It reads each input vector about once from HBM and writes each output
// once: HBM bound at (rows_in + rows_out) values per right-hand side.  The
// T transfer adds a_i u_i in the same pass.

#include <algorithm>
#include <cmath>
#include <cstring>

#include "htlr_device.h"
#include "htlr_handle.h"

namespace htlr {

extern thread_local std::string g_last_error;
htlr_status record(const Error& e);

struct QuasiData {
  int m = 0;                         // uniform cells per dimension
  int64_t M = 0;                     // m^d
  htlr_matrix inner = nullptr;       // Ahat (uniform grid, a = 0)
  // band of the 1D matrices, per direction (0: S, rows = m over n columns;
  // 1: T, rows = n over m columns): width, first column and values of row r
  // of dimension l at lo[l*rows + r] and val[(l*rows + r)*w + k]
  int w[2] = {0, 0};
  DevBuf lo[2], v64[2], v32[2];
  DevBuf a64, a32;                   // a(x_i) on the quasi-uniform grid (empty: a = 0)
  DevBuf uh, fh;                     // S u and Ahat S u, M x nrhs
  QuasiData() = default;
  QuasiData(const QuasiData&) = delete;
  QuasiData& operator=(const QuasiData&) = delete;
  ~QuasiData() {
    if (inner) htlr_free(inner);
  }
};

htlr_matrix_impl& quasi_inner(htlr_matrix_impl& A) { return *A.quasi->inner; }

// out[o] (+)= sum over the band of every dimension of
// val_1[o_1][k_1] ... val_D[o_D][k_D] in[lo_1[o_1] + k_1, ..., lo_D[o_D] + k_D],
// the last dimension outermost; plus a[o] u0[o] when a is given.  Grid:
// (ceil(nout^D / 256), nrhs).
template <typename T, int D>
__global__ void __launch_bounds__(256)
k_transfer(const T* __restrict__ in, T* __restrict__ out, const int* __restrict__ lo, const T* __restrict__ val,
           int w, int nin, int nout, int64_t Nin, int64_t Nout, const T* __restrict__ a, const T* __restrict__ u0) {
  const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (o >= Nout) return;
  const int r = blockIdx.y;
  const int o1 = (int)(o % nout);
  const int o2 = (int)((o / nout) % nout);
  const int l1 = lo[o1], l2 = lo[nout + o2];
  const T* v1 = val + (int64_t)o1 * w;
  const T* v2 = val + ((int64_t)nout + o2) * w;
  const T* x = in + (int64_t)r * Nin;
  T acc = 0;
  if (D == 3) {
    const int o3 = (int)(o / ((int64_t)nout * nout));
    const int l3 = lo[2 * nout + o3];
    const T* v3 = val + (2 * (int64_t)nout + o3) * w;
    for (int c = 0; c < w; ++c) {
      const T* xc = x + (int64_t)(l3 + c) * nin * nin;
      T acc2 = 0;
      for (int b = 0; b < w; ++b) {
        const T* xb = xc + (int64_t)(l2 + b) * nin + l1;
        T acc1 = 0;
        for (int k = 0; k < w; ++k) acc1 += v1[k] * xb[k];
        acc2 += v2[b] * acc1;
      }
      acc += v3[c] * acc2;
    }
  } else {
    for (int b = 0; b < w; ++b) {
      const T* xb = x + (int64_t)(l2 + b) * nin + l1;
      T acc1 = 0;
      for (int k = 0; k < w; ++k) acc1 += v1[k] * xb[k];
      acc += v2[b] * acc1;
    }
  }
  if (a) acc += a[o] * u0[(int64_t)r * Nout + o];
  out[(int64_t)r * Nout + o] = acc;
}

namespace {

// Length of [a0, a1] cap [b0, b1] (0 when they do not overlap).
double overlap(double a0, double a1, double b0, double b1) {
  return std::max(0.0, std::min(a1, b1) - std::max(a0, b0));
}

struct Band {
  int w = 0;
  std::vector<int> lo;               // d * rows
  std::vector<double> val;           // d * rows * w
};

// Row r of the 1D matrix with rows over the cells er (edges, rows + 1) and
// columns over the cells ec: overlap(cell r, cell c) / |cell r|.  The run of
// overlapping columns of every row is found by binary search on the edges.
Band make_band(const std::vector<std::vector<double>>& er, const std::vector<std::vector<double>>& ec) {
  const int d = (int)er.size();
  const int rows = (int)er[0].size() - 1, cols = (int)ec[0].size() - 1;
  std::vector<int> first((size_t)d * rows), last((size_t)d * rows);
  int w = 1;
  for (int l = 0; l < d; ++l)
    for (int r = 0; r < rows; ++r) {
      const double r0 = er[l][r], r1 = er[l][r + 1];
      // first column whose right edge lies beyond r0, last whose left edge lies before r1
      int c0 = (int)(std::upper_bound(ec[l].begin() + 1, ec[l].end(), r0) - ec[l].begin()) - 1;
      int c1 = (int)(std::lower_bound(ec[l].begin(), ec[l].end() - 1, r1) - ec[l].begin()) - 1;
      c0 = std::min(std::max(c0, 0), cols - 1);
      c1 = std::min(std::max(c1, c0), cols - 1);
      first[(size_t)l * rows + r] = c0;
      last[(size_t)l * rows + r] = c1;
      w = std::max(w, c1 - c0 + 1);
    }
  Band b;
  b.w = std::min(w, cols);
  b.lo.resize((size_t)d * rows);
  b.val.assign((size_t)d * rows * b.w, 0.0);
  for (int l = 0; l < d; ++l)
    for (int r = 0; r < rows; ++r) {
      const size_t i = (size_t)l * rows + r;
      const int lo = std::min(first[i], cols - b.w);
      b.lo[i] = lo;
      const double r0 = er[l][r], r1 = er[l][r + 1];
      for (int k = 0; k < b.w; ++k) {
        const int c = lo + k;
        b.val[i * b.w + k] = overlap(r0, r1, ec[l][c], ec[l][c + 1]) / (r1 - r0);
      }
    }
  return b;
}

template <typename T>
void upload(DevBuf& dst, const std::vector<T>& v) {
  dst.alloc(v.size() * sizeof(T));
  if (!v.empty()) HTLR_HIP(hipMemcpy(dst.ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
}

template <typename T>
void launch_transfer(int d, const T* in, T* out, const int* lo, const T* val, int w, int nin, int nout, int nrhs,
                     const T* a, const T* u0, hipStream_t st) {
  int64_t Nin = 1, Nout = 1;
  for (int l = 0; l < d; ++l) { Nin *= nin; Nout *= nout; }
  const int64_t blocks = (Nout + 255) / 256;
  if (blocks > 0x7fffffff) fail(HTLR_ERR_UNSUPPORTED, "grid too large for the transfer kernel");
  if (d == 3)
    hipLaunchKernelGGL((k_transfer<T, 3>), dim3((unsigned)blocks, nrhs), dim3(256), 0, st, in, out, lo, val, w, nin,
                       nout, Nin, Nout, a, u0);
  else
    hipLaunchKernelGGL((k_transfer<T, 2>), dim3((unsigned)blocks, nrhs), dim3(256), 0, st, in, out, lo, val, w, nin,
                       nout, Nin, Nout, a, u0);
  HTLR_HIP(hipGetLastError());
}

}  // namespace

size_t quasi_buffer_bytes(const htlr_matrix_impl& A, int nrhs, int prec) {
  return 2 * (size_t)A.quasi->M * nrhs * (prec == HTLR_FP64 ? 8 : 4);
}

void quasi_matvec(htlr_matrix_impl& A, const void* u, void* f, int nrhs, int prec, hipStream_t st) {
  QuasiData& Q = *A.quasi;
  htlr_matrix_impl& I = *Q.inner;
  const bool f64 = prec == HTLR_FP64;
  const size_t need = (size_t)Q.M * nrhs * (f64 ? 8 : 4);
  if (Q.uh.bytes < need) {
    Q.uh.alloc(need);
    Q.fh.alloc(need);
  }
  const int dir_s = 0, dir_t = 1;
  if (f64) {
    {
      ProfScope ps(A, "quasi_s", -1, st);
      launch_transfer<double>(A.d, (const double*)u, Q.uh.as<double>(), Q.lo[dir_s].as<int>(),
                              Q.v64[dir_s].as<double>(), Q.w[dir_s], A.n, Q.m, nrhs, nullptr, nullptr, st);
    }
    {
      std::lock_guard<std::mutex> li(I.ws_mu);
      product(I, Q.uh.ptr, Q.fh.ptr, nrhs, prec, st);
    }
    ProfScope ps(A, "quasi_t", -1, st);
    launch_transfer<double>(A.d, Q.fh.as<double>(), (double*)f, Q.lo[dir_t].as<int>(), Q.v64[dir_t].as<double>(),
                            Q.w[dir_t], Q.m, A.n, nrhs, Q.a64.as<double>(), (const double*)u, st);
  } else {
    {
      ProfScope ps(A, "quasi_s", -1, st);
      launch_transfer<float>(A.d, (const float*)u, Q.uh.as<float>(), Q.lo[dir_s].as<int>(), Q.v32[dir_s].as<float>(),
                             Q.w[dir_s], A.n, Q.m, nrhs, nullptr, nullptr, st);
    }
    {
      std::lock_guard<std::mutex> li(I.ws_mu);
      product(I, Q.uh.ptr, Q.fh.ptr, nrhs, prec, st);
    }
    ProfScope ps(A, "quasi_t", -1, st);
    launch_transfer<float>(A.d, Q.fh.as<float>(), (float*)f, Q.lo[dir_t].as<int>(), Q.v32[dir_t].as<float>(),
                           Q.w[dir_t], Q.m, A.n, nrhs, Q.a32.as<float>(), (const float*)u, st);
  }
}

}  // namespace htlr

using namespace htlr;

extern "C" {

htlr_status htlr_build_quasi(const double* points, htlr_kernel kernel, int d, int n, int m, int p, int leaf,
                             const htlr_build_opts* opts, htlr_matrix* out) {
  if (!out) { g_last_error = "out is NULL"; return HTLR_ERR_INVALID; }
  *out = nullptr;
  htlr_matrix_s* A = nullptr;
  try {
    g_last_error.clear();
    const Grid g = make_grid(points, d, n, opts ? opts->edges : nullptr);
    if (m < 1 || m > (1 << 15)) fail(HTLR_ERR_INVALID, "m out of range");
    auto Q = std::make_shared<QuasiData>();
    Q->m = m;
    Q->M = 1;
    int64_t N = 1;
    for (int l = 0; l < d; ++l) { Q->M *= m; N *= n; }
    htlr_build_opts io{};
    if (opts) io = *opts;
    io.a = nullptr;
    io.edges = nullptr;    // Ahat lives on the uniform grid of m cells
    const htlr_status bs = htlr_build(nullptr, kernel, d, m, p, leaf, &io, &Q->inner);
    if (bs != HTLR_OK) fail(bs, "uniform grid of the transfer: " + g_last_error);
    const htlr_matrix_impl& I = *Q->inner;
    A = new htlr_matrix_s();
    A->d = d;
    A->n = n;
    A->p = p;
    A->leaf = leaf;
    A->kid = kernel;
    A->N = N;
    A->P = I.P;
    A->rank = I.rank;
    A->L = I.L;
    A->uniform = g.uniform;
    A->eta2 = I.eta2;
    A->adm_kind = I.adm_kind;
    A->gl_order = I.gl_order;
    A->precisions = I.precisions;
    A->device = I.device;
    A->grid = g;
    // 1D cell edges: quasi-uniform (Voronoi, from the grid) and uniform k/m
    std::vector<std::vector<double>> eq(d), eu(d);
    for (int l = 0; l < d; ++l) {
      eq[l].assign(g.e.begin() + (size_t)l * (n + 1), g.e.begin() + (size_t)(l + 1) * (n + 1));
      eu[l].resize(m + 1);
      for (int k = 0; k <= m; ++k) eu[l][k] = (double)k / m;
    }
    const bool want32 = (I.precisions & ((1 << HTLR_FP32) | (1 << HTLR_BF16_CORE))) != 0;
    const bool want64 = (I.precisions & (1 << HTLR_FP64)) != 0;
    size_t bytes = I.device_bytes;
    for (int dir = 0; dir < 2; ++dir) {
      const Band b = dir == 0 ? make_band(eu, eq) : make_band(eq, eu);
      Q->w[dir] = b.w;
      upload(Q->lo[dir], b.lo);
      if (want64) upload(Q->v64[dir], b.val);
      if (want32) upload(Q->v32[dir], std::vector<float>(b.val.begin(), b.val.end()));
      bytes += Q->lo[dir].bytes + Q->v64[dir].bytes + Q->v32[dir].bytes;
    }
    if (opts && opts->a) {
      std::vector<double> a(opts->a, opts->a + N);
      for (double v : a)
        if (!std::isfinite(v)) fail(HTLR_ERR_NUMERIC, "a(x) has NaN/Inf");
      if (want64) upload(Q->a64, a);
      if (want32) upload(Q->a32, std::vector<float>(a.begin(), a.end()));
      bytes += Q->a64.bytes + Q->a32.bytes;
    }
    A->device_bytes = bytes;
    A->quasi = std::move(Q);
    *out = A;
    return HTLR_OK;
  } catch (const Error& e) {
    delete A;
    return record(e);
  } catch (const std::bad_alloc&) {
    delete A;
    g_last_error = "host allocation failed";
    return HTLR_ERR_OOM;
  } catch (const std::exception& e) {
    delete A;
    g_last_error = e.what();
    return HTLR_ERR_INVALID;
  }
}

}  // extern "C"
