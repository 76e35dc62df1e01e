// Rows of the uncompressed Nystrom product (eq. 1.3-1.4), for measuring the
// HTLR approximation error the way Sec. 5 does (e_apply;rand: relative
// 2-norm error against the exact A u on randomly chosen rows).
//
//   out_i = (a_i + D_i) u_i + sum_{j != i} k(x_i, x_j) |Omega_j| u_j
//
// One block per group of target rows; its threads stride over all N source
// points in natural order (first index fastest), so consecutive lanes read
// consecutive u values, and every source value a block loads serves all of
// its rows.  Per-thread partial sums are added in a fixed tree order, so the
// result is deterministic.  Everything in FP64.

#include <algorithm>

#include "htlr_device.h"
#include "htlr_handle.h"

namespace htlr {

extern thread_local std::string g_last_error;
htlr_status record(const Error& e);

namespace {

constexpr int kExactThreads = 256;
constexpr int kExactAcc = 8;       // rows x right-hand sides a block accumulates

// RC right-hand sides (columns r >= nrhs are skipped), kExactAcc / RC rows
// per block.  A row index outside [0, N) yields NaN in its output rows.
template <int KID, int RC>
__global__ __launch_bounds__(kExactThreads) void k_exact_rows(
    const double* __restrict__ u, double* __restrict__ out, const int64_t* __restrict__ rows, int nrows,
    const double* __restrict__ x, const double* __restrict__ w, const double* __restrict__ a,
    const double* __restrict__ D, double D0, int d, int n, int64_t N, int nrhs, int pm1) {
  constexpr int RPB = kExactAcc / RC;
  __shared__ double red[kExactThreads];
  const int tid = threadIdx.x;
  const int r0 = blockIdx.x * RPB;
  // target points of this block's rows (-1: no row, or an index out of range)
  int64_t ti[RPB];
  double tx[RPB], ty[RPB], tz[RPB];
#pragma unroll
  for (int q = 0; q < RPB; ++q) {
    ti[q] = -1;
    tx[q] = ty[q] = tz[q] = 0.0;
    const int64_t i = r0 + q < nrows ? rows[r0 + q] : -1;
    if (i >= 0 && i < N) {
      ti[q] = i;
      tx[q] = x[i % n];
      ty[q] = x[n + (i / n) % n];
      tz[q] = d == 3 ? x[2 * n + i / ((int64_t)n * n)] : 0.0;
    }
  }
  double acc[RPB][RC];
#pragma unroll
  for (int q = 0; q < RPB; ++q)
#pragma unroll
    for (int r = 0; r < RC; ++r) acc[q][r] = 0.0;
  // source index j = tid + k * kExactThreads, carried as (j0, j1, j2)
  int j0 = tid % n, j1 = (tid / n) % n, j2 = tid / (n * n);
  for (int64_t j = tid; j < N; j += kExactThreads) {
    const double y0 = x[j0], y1 = x[n + j1], y2 = d == 3 ? x[2 * n + j2] : 0.0;
    const double wj = w[j0] * w[n + j1] * (d == 3 ? w[2 * n + j2] : 1.0);
    double uj[RC];
#pragma unroll
    for (int r = 0; r < RC; ++r) uj[r] = r < nrhs ? u[j + (int64_t)r * N] : 0.0;
#pragma unroll
    for (int q = 0; q < RPB; ++q) {
      if (ti[q] < 0 || ti[q] == j) continue;
      const double kv = kvec<KID, double>(tx[q] - y0, ty[q] - y1, tz[q] - y2, d, pm1) * wj;
#pragma unroll
      for (int r = 0; r < RC; ++r) acc[q][r] += kv * uj[r];
    }
    j0 += kExactThreads;
    while (j0 >= n) {
      j0 -= n;
      if (++j1 == n) {
        j1 = 0;
        ++j2;
      }
    }
  }
  // fixed-order tree reduction of each (row, rhs) sum
#pragma unroll
  for (int q = 0; q < RPB; ++q)
#pragma unroll
    for (int r = 0; r < RC; ++r) {
      if (r0 + q >= nrows || r >= nrhs) continue;     // uniform across the block
      red[tid] = acc[q][r];
      __syncthreads();
      for (int s = kExactThreads / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
      }
      if (tid == 0) {
        const int64_t i = ti[q];
        double v = __builtin_nan("");
        if (i >= 0) v = (a[i] + (D ? D[i] : D0)) * u[i + (int64_t)r * N] + red[0];
        out[(r0 + q) + (int64_t)r * nrows] = v;
      }
      __syncthreads();
    }
}

template <int KID>
void launch_exact(const htlr_matrix_impl& A, const double* u, const int64_t* rows, int nrows, double* out, int nrhs,
                  hipStream_t st) {
  const double* D = A.uniform ? nullptr : A.D64.as<double>();
  const int rc = nrhs <= 1 ? 1 : nrhs <= 2 ? 2 : nrhs <= 4 ? 4 : 8;
  const unsigned blocks = (unsigned)((nrows + kExactAcc / rc - 1) / (kExactAcc / rc));
#define HTLR_EXACT_RC(RCV)                                                                                     \
  hipLaunchKernelGGL((k_exact_rows<KID, RCV>), dim3(blocks), dim3(kExactThreads), 0, st, u, out, rows, nrows, \
                     A.x64.as<double>(), A.w64.as<double>(), A.a64.as<double>(), D, A.D0, A.d, A.n, A.N, nrhs,  \
                     A.p - 1)
  switch (rc) {
    case 1: HTLR_EXACT_RC(1); break;
    case 2: HTLR_EXACT_RC(2); break;
    case 4: HTLR_EXACT_RC(4); break;
    default: HTLR_EXACT_RC(8); break;
  }
#undef HTLR_EXACT_RC
}

}  // namespace

}  // namespace htlr

using namespace htlr;

extern "C" {

htlr_status htlr_exact_rows(htlr_matrix A, const double* u, const int64_t* rows, int nrows, double* out, int nrhs,
                            void* stream) {
  try {
    g_last_error.clear();
    if (!A || !u || !rows || !out) fail(HTLR_ERR_INVALID, "null argument");
    if (A->quasi) fail(HTLR_ERR_UNSUPPORTED, "transfer-form handles: rows of the quasi-uniform operator are not built");
    if (nrows < 1) fail(HTLR_ERR_INVALID, "nrows must be positive");
    if (nrhs < 1 || nrhs > kExactAcc) fail(HTLR_ERR_INVALID, "nrhs out of range (1..8)");
    int dev = 0;
    HTLR_HIP(hipGetDevice(&dev));
    if (dev != A->device) fail(HTLR_ERR_INVALID, "current device differs from the build device");
    const hipStream_t st = (hipStream_t)stream;
    switch (A->kid) {
      case HTLR_K_INV_R: launch_exact<HTLR_K_INV_R>(*A, u, rows, nrows, out, nrhs, st); break;
      case HTLR_K_NEG_LOG: launch_exact<HTLR_K_NEG_LOG>(*A, u, rows, nrows, out, nrhs, st); break;
      case HTLR_K_EXP: launch_exact<HTLR_K_EXP>(*A, u, rows, nrows, out, nrhs, st); break;
      case HTLR_K_GAUSS: launch_exact<HTLR_K_GAUSS>(*A, u, rows, nrows, out, nrhs, st); break;
      case HTLR_K_POLY_TEST: launch_exact<HTLR_K_POLY_TEST>(*A, u, rows, nrows, out, nrhs, st); break;
      default: fail(HTLR_ERR_INVALID, "unknown kernel");
    }
    HTLR_HIP(hipGetLastError());
    return HTLR_OK;
  } catch (const Error& e) {
    return record(e);
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return HTLR_ERR_INVALID;
  }
}

}  // extern "C"
