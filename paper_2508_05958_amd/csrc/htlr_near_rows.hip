// Near field + diagonal on uniform grids with a radial kernel (the
// inadmissible leaves of eq. 4.1, evaluated on the fly): 2D leaves of M x M
// points (M = 8 or 16), and 3D leaves of 4 x 4 x 4 points.
//
// The kernel value between two points depends only on the squared index
// distance, read from the table h^2 k(h sqrt(s)) (entry 0 holds the diagonal
// integral D).  Between a target row i1 of leaf tau and a source row j1 of a
// near leaf sigma the M x M block depends only on i0 - j0, so its 2M - 1
// values, read once from LDS into registers, serve M * M * RC FMAs.
//
// One wave per (target leaf, chunk of RC right-hand sides); lane = (g, i1)
// with i1 = lane % M the target row and g = lane / M one of G = 64 / M groups
// that takes the source rows j1 = g, g + G, ...  Each near leaf is staged in
// the wave's own LDS slice.  At the end the G partial sums of a row are added
// across lanes in a fixed order (xor butterfly), so results are deterministic.

#include "htlr_device.h"
#include "htlr_handle.h"

namespace htlr {

namespace {

// LDS writes of this wave are visible to its later LDS reads.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kRowsWaves = 4;            // waves (work items) per workgroup
constexpr size_t kRowsLds = 64 * 1024;   // LDS per workgroup (table + staged leaves)

template <typename T, int M, int RC>
__global__ __launch_bounds__(64 * kRowsWaves) void k_near_rows2d(
    const T* __restrict__ u, T* __restrict__ f, const T* __restrict__ a, const int64_t* __restrict__ nptr,
    const int32_t* __restrict__ nsrc, const T* __restrict__ table, int tsize, int n, int B, int nrhs, int nitems) {
  constexpr int G = 64 / M;
  constexpr int LDU = M + 1;             // padded source row (odd stride in 8-byte words)
  constexpr int K = 2 * M - 1;
  extern __shared__ unsigned char smem_raw[];
  T* tab = reinterpret_cast<T*>(smem_raw);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  T* us = tab + ((tsize + 1) & ~1) + (size_t)wave * (M * LDU * RC);
  for (int s = threadIdx.x; s < tsize; s += 64 * kRowsWaves) tab[s] = table[s];
  __syncthreads();                       // the only workgroup barrier
  const int item = blockIdx.x * kRowsWaves + wave;
  if (item >= nitems) return;
  const int nchunk = (nrhs + RC - 1) / RC;
  const int tau = item / nchunk, r0 = (item % nchunk) * RC;
  const int tx = tau % B, ty = tau / B;
  const int i1 = lane % M, g = lane / M;
  const int64_t NN = (int64_t)n * n;
  T acc[RC][M];
#pragma unroll
  for (int r = 0; r < RC; ++r)
#pragma unroll
    for (int i0 = 0; i0 < M; ++i0) acc[r][i0] = T(0);

  for (int64_t e = nptr[tau]; e < nptr[tau + 1]; ++e) {
    const int sg = nsrc[e];
    const int sx = sg % B, sy = sg / B;
    const int ox = sx - tx, oy = sy - ty;
    wave_sync();                         // the previous leaf's reads are done
#pragma unroll
    for (int r = 0; r < RC; ++r) {
      const bool live = r0 + r < nrhs;
      const T* ur = u + (int64_t)(live ? r0 + r : 0) * NN;
#pragma unroll
      for (int k = lane; k < M * M; k += 64) {
        const int j0 = k % M, j1 = k / M;
        us[(r * M + j1) * LDU + j0] = live ? ur[(int64_t)(sx * M + j0) + (int64_t)n * (sy * M + j1)] : T(0);
      }
    }
    wave_sync();
    for (int j1 = g; j1 < M; j1 += G) {
      const int dy = (i1 - j1) - M * oy;
      const int dy2 = dy * dy;
      T kv[K];
#pragma unroll
      for (int t = 0; t < K; ++t) {
        const int dx = (t - (M - 1)) - M * ox;
        kv[t] = tab[dy2 + dx * dx];
      }
#pragma unroll
      for (int r = 0; r < RC; ++r) {
        T uv[M];
#pragma unroll
        for (int j0 = 0; j0 < M; ++j0) uv[j0] = us[(r * M + j1) * LDU + j0];
#pragma unroll
        for (int i0 = 0; i0 < M; ++i0)
#pragma unroll
          for (int j0 = 0; j0 < M; ++j0) acc[r][i0] += kv[i0 - j0 + M - 1] * uv[j0];
      }
    }
  }
  // add the G groups' partial sums of each row: butterfly over lane bits
#pragma unroll
  for (int off = 32; off >= M; off >>= 1)
#pragma unroll
    for (int r = 0; r < RC; ++r)
#pragma unroll
      for (int i0 = 0; i0 < M; ++i0) acc[r][i0] += __shfl_xor(acc[r][i0], off);
  if (g != 0) return;
  const int64_t row = (int64_t)(tx * M) + (int64_t)n * (ty * M + i1);
#pragma unroll
  for (int r = 0; r < RC; ++r) {
    if (r0 + r >= nrhs) break;
    const int64_t base = (int64_t)(r0 + r) * NN + row;
#pragma unroll
    for (int i0 = 0; i0 < M; ++i0) f[base + i0] = acc[r][i0] + a[row + i0] * u[base + i0];
  }
}

// 3D leaves of M x M x M points (M = 4): lane = (g, row) with row = (i1, i2)
// one of the M^2 target rows and g one of G = 64 / M^2 groups taking the
// source rows (j1, j2) = g, g + G, ... of each near leaf.  For a (target
// row, source row) pair the M x M block depends only on i0 - j0: 2M - 1 table
// values serve M * M * RC FMAs.  Groups are added by an xor butterfly in a
// fixed order.
template <typename T, int M, int RC>
__global__ __launch_bounds__(64 * kRowsWaves) void k_near_rows3d(
    const T* __restrict__ u, T* __restrict__ f, const T* __restrict__ a, const int64_t* __restrict__ nptr,
    const int32_t* __restrict__ nsrc, const T* __restrict__ table, int tsize, int n, int B, int nrhs, int nitems) {
  constexpr int M2 = M * M, M3 = M2 * M, G = 64 / M2;
  constexpr int K = 2 * M - 1;
  static_assert(G * M2 == 64, "rows per wave");
  extern __shared__ unsigned char smem_raw[];
  T* tab = reinterpret_cast<T*>(smem_raw);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  T* us = tab + ((tsize + 1) & ~1) + (size_t)wave * (M3 * RC);
  for (int s = threadIdx.x; s < tsize; s += 64 * kRowsWaves) tab[s] = table[s];
  __syncthreads();                       // the only workgroup barrier
  const int item = blockIdx.x * kRowsWaves + wave;
  if (item >= nitems) return;
  const int nchunk = (nrhs + RC - 1) / RC;
  const int tau = item / nchunk, r0 = (item % nchunk) * RC;
  const int tx = tau % B, ty = (tau / B) % B, tz = tau / (B * B);
  const int row = lane % M2, g = lane / M2;
  const int i1 = row % M, i2 = row / M;
  const int64_t N = (int64_t)n * n * n;
  T acc[RC][M];
#pragma unroll
  for (int r = 0; r < RC; ++r)
#pragma unroll
    for (int i0 = 0; i0 < M; ++i0) acc[r][i0] = T(0);

  for (int64_t e = nptr[tau]; e < nptr[tau + 1]; ++e) {
    const int sg = nsrc[e];
    const int sx = sg % B, sy = (sg / B) % B, sz = sg / (B * B);
    const int ox = sx - tx, oy = sy - ty, oz = sz - tz;
    wave_sync();                         // the previous leaf's reads are done
#pragma unroll
    for (int r = 0; r < RC; ++r) {
      const bool live = r0 + r < nrhs;
      const T* ur = u + (int64_t)(live ? r0 + r : 0) * N;
#pragma unroll
      for (int k = lane; k < M3; k += 64) {
        const int j0 = k % M, j1 = (k / M) % M, j2 = k / M2;
        us[r * M3 + k] = live ? ur[(int64_t)(sx * M + j0) + (int64_t)n * ((sy * M + j1) + (int64_t)n * (sz * M + j2))]
                              : T(0);
      }
    }
    wave_sync();
#pragma unroll
    for (int js = g; js < M2; js += G) {
      const int j1 = js % M, j2 = js / M;
      const int dy = (i1 - j1) - M * oy, dz = (i2 - j2) - M * oz;
      const int base = dy * dy + dz * dz;
      T kv[K];
#pragma unroll
      for (int t = 0; t < K; ++t) {
        const int dx = (t - (M - 1)) - M * ox;
        kv[t] = tab[base + dx * dx];
      }
#pragma unroll
      for (int r = 0; r < RC; ++r) {
        T uv[M];
#pragma unroll
        for (int j0 = 0; j0 < M; ++j0) uv[j0] = us[r * M3 + js * M + j0];
#pragma unroll
        for (int i0 = 0; i0 < M; ++i0)
#pragma unroll
          for (int j0 = 0; j0 < M; ++j0) acc[r][i0] += kv[i0 - j0 + M - 1] * uv[j0];
      }
    }
  }
#pragma unroll
  for (int off = 32; off >= M2; off >>= 1)
#pragma unroll
    for (int r = 0; r < RC; ++r)
#pragma unroll
      for (int i0 = 0; i0 < M; ++i0) acc[r][i0] += __shfl_xor(acc[r][i0], off);
  if (g != 0) return;
  const int64_t gr = (int64_t)(tx * M) + (int64_t)n * ((ty * M + i1) + (int64_t)n * (tz * M + i2));
#pragma unroll
  for (int r = 0; r < RC; ++r) {
    if (r0 + r >= nrhs) break;
    const int64_t base = (int64_t)(r0 + r) * N + gr;
#pragma unroll
    for (int i0 = 0; i0 < M; ++i0) f[base + i0] = acc[r][i0] + a[gr + i0] * u[base + i0];
  }
}

template <typename T>
int rows3d_rc(int nrhs) {
  const int cap = std::is_same<T, double>::value ? 4 : 8;
  int rc = 1;
  while (rc < cap && rc < nrhs) rc *= 2;
  return rc;
}

template <typename T>
size_t rows3d_lds(const htlr_matrix_impl& A, int rc) {
  return (((size_t)A.Tsize + 1) & ~size_t(1)) * sizeof(T) + (size_t)kRowsWaves * 64 * rc * sizeof(T);
}

template <typename T>
int rows2d_rc(int nrhs) {
  const int cap = std::is_same<T, double>::value ? 2 : 4;
  int rc = 1;
  while (rc < cap && rc < nrhs) rc *= 2;
  return rc;
}

template <typename T>
size_t rows2d_lds(const htlr_matrix_impl& A, int m, int rc) {
  return (((size_t)A.Tsize + 1) & ~size_t(1)) * sizeof(T) + (size_t)kRowsWaves * m * (m + 1) * rc * sizeof(T);
}

}  // namespace

bool near_rows2d_ok(const htlr_matrix_impl& A, int nrhs, int prec) {
  if (!A.uniform || A.d != 2 || A.kid == HTLR_K_POLY_TEST || A.Tsize <= 0) return false;
  const int m = A.plan.m[A.L];
  if (m != 8 && m != 16) return false;
  return prec == HTLR_FP64 ? rows2d_lds<double>(A, m, rows2d_rc<double>(nrhs)) <= kRowsLds
                           : rows2d_lds<float>(A, m, rows2d_rc<float>(nrhs)) <= kRowsLds;
}

template <typename T>
void launch_near_rows2d(htlr_matrix_impl& A, const T* u, T* f, int nrhs, hipStream_t st) {
  const bool f64 = std::is_same<T, double>::value;
  const int m = A.plan.m[A.L], B = A.plan.B[A.L];
  const int rc = rows2d_rc<T>(nrhs);
  const int nchunk = (nrhs + rc - 1) / rc;
  const int64_t nitems = A.levels[A.L].nbox * nchunk;
  if (nitems > 0x7fffffffLL) fail(HTLR_ERR_UNSUPPORTED, "too many near-field work items");
  const int blocks = (int)((nitems + kRowsWaves - 1) / kRowsWaves);
  const size_t sh = rows2d_lds<T>(A, m, rc);
  if (sh > kRowsLds) fail(HTLR_ERR_UNSUPPORTED, "near-field table exceeds LDS");
  const T* tab = f64 ? (const T*)A.T64.ptr : (const T*)A.T32.ptr;
  const T* a = f64 ? (const T*)A.a64.ptr : (const T*)A.a32.ptr;
  const int64_t* np = A.near_ptr.as<int64_t>();
  const int32_t* ns = A.near_src.as<int32_t>();
#define HTLR_ROWS2D(MV, RCV)                                                                                   \
  hipLaunchKernelGGL((k_near_rows2d<T, MV, RCV>), dim3(blocks), dim3(64 * kRowsWaves), sh, st, u, f, a, np, ns, \
                     tab, A.Tsize, A.n, B, nrhs, (int)nitems)
  if (m == 16) {
    if (rc == 1) HTLR_ROWS2D(16, 1);
    else if (rc == 2) HTLR_ROWS2D(16, 2);
    else if constexpr (!std::is_same<T, double>::value) HTLR_ROWS2D(16, 4);
  } else {
    if (rc == 1) HTLR_ROWS2D(8, 1);
    else if (rc == 2) HTLR_ROWS2D(8, 2);
    else if constexpr (!std::is_same<T, double>::value) HTLR_ROWS2D(8, 4);
  }
#undef HTLR_ROWS2D
  HTLR_HIP(hipGetLastError());
}

bool near_rows3d_ok(const htlr_matrix_impl& A, int nrhs, int prec) {
  if (!A.uniform || A.d != 3 || A.kid == HTLR_K_POLY_TEST || A.Tsize <= 0) return false;
  if (A.plan.m[A.L] != 4) return false;
  return prec == HTLR_FP64 ? rows3d_lds<double>(A, rows3d_rc<double>(nrhs)) <= kRowsLds
                           : rows3d_lds<float>(A, rows3d_rc<float>(nrhs)) <= kRowsLds;
}

template <typename T>
void launch_near_rows3d(htlr_matrix_impl& A, const T* u, T* f, int nrhs, hipStream_t st) {
  const bool f64 = std::is_same<T, double>::value;
  const int B = A.plan.B[A.L];
  const int rc = rows3d_rc<T>(nrhs);
  const int nchunk = (nrhs + rc - 1) / rc;
  const int64_t nitems = A.levels[A.L].nbox * nchunk;
  if (nitems > 0x7fffffffLL) fail(HTLR_ERR_UNSUPPORTED, "too many near-field work items");
  const int blocks = (int)((nitems + kRowsWaves - 1) / kRowsWaves);
  const size_t sh = rows3d_lds<T>(A, rc);
  if (sh > kRowsLds) fail(HTLR_ERR_UNSUPPORTED, "near-field table exceeds LDS");
  const T* tab = f64 ? (const T*)A.T64.ptr : (const T*)A.T32.ptr;
  const T* a = f64 ? (const T*)A.a64.ptr : (const T*)A.a32.ptr;
  const int64_t* np = A.near_ptr.as<int64_t>();
  const int32_t* ns = A.near_src.as<int32_t>();
#define HTLR_ROWS3D(RCV)                                                                                     \
  hipLaunchKernelGGL((k_near_rows3d<T, 4, RCV>), dim3(blocks), dim3(64 * kRowsWaves), sh, st, u, f, a, np, ns, \
                     tab, A.Tsize, A.n, B, nrhs, (int)nitems)
  if (rc == 1) HTLR_ROWS3D(1);
  else if (rc == 2) HTLR_ROWS3D(2);
  else if (rc == 4) HTLR_ROWS3D(4);
  else if constexpr (!std::is_same<T, double>::value) HTLR_ROWS3D(8);
#undef HTLR_ROWS3D
  HTLR_HIP(hipGetLastError());
}

template void launch_near_rows3d<double>(htlr_matrix_impl&, const double*, double*, int, hipStream_t);
template void launch_near_rows3d<float>(htlr_matrix_impl&, const float*, float*, int, hipStream_t);
template void launch_near_rows2d<double>(htlr_matrix_impl&, const double*, double*, int, hipStream_t);
template void launch_near_rows2d<float>(htlr_matrix_impl&, const float*, float*, int, hipStream_t);

}  // namespace htlr
