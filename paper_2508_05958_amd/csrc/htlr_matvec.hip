// HTLR matrix-vector product (Alg. 4.2, eq. 4.3) on the GPU.
//
// The recursion of Alg. 4.2 visits every leaf (tau, sigma) of the block
// cluster tree once.  Here the leaves are processed level by level, and
// each step is one launch over all boxes of a level:
//
//   near   f_tau  = a o u_tau + sum_{sigma in near(tau)} A_tau,sigma u_sigma
//          (inadmissible leaves, eq. 4.1, kernel values made on the fly),
//   up     W_sigma = (|Omega| o u_sigma) x_1 V_1^T ... x_d V_d^T,
//   core   H_tau  = sum_{sigma in adm(tau)} G_tau,sigma x_{[d+1..2d],[1..d]} W_sigma,
//   down   f_tau += H_tau x_1 U_1 ... x_d U_d,
//
// for every level that has admissible leaves.  W_sigma depends only on sigma,
// so it is computed once per box instead of once per leaf; the sum over the
// leaves of a row block is the same sum Alg. 4.2 forms, in a different order.
// Every output element is written by exactly one thread of one launch, and
// launches on a stream are ordered, so the product is deterministic.

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "htlr_device.h"
#include "htlr_handle.h"

namespace htlr {

htlr_status record(const Error& e);
extern thread_local std::string g_last_error;

constexpr int kThreads = 256;

template <typename TW, typename T> __device__ __forceinline__ TW store_cast(T v) { return (TW)v; }
template <> __device__ __forceinline__ uint16_t store_cast<uint16_t, float>(float v) { return f2bf(v); }

__device__ __forceinline__ int64_t lin3(int i0, int i1, int i2, int n) {
  return (int64_t)i0 + (int64_t)n * ((int64_t)i1 + (int64_t)n * i2);
}

// ---------------------------------------------------------------------------
// Near field + diagonal, uniform grid: the kernel value between two points
// depends on their integer index difference delta only.  Radial kernels read
// h^d k(h sqrt(|delta|^2)) from a table indexed by |delta|^2 (entry 0 is the
// diagonal integral D); the polynomial test kernel is evaluated directly.
template <int KID, typename T, int RC>
__global__ __launch_bounds__(kThreads) void k_near_uniform(
    const T* __restrict__ u, T* __restrict__ f, const T* __restrict__ a, const int64_t* __restrict__ nptr,
    const int32_t* __restrict__ nsrc, const T* __restrict__ table, int tsize, int d, int n, int m, int B,
    int nrhs, T h, T w0, T D0, int pm1) {
  extern __shared__ unsigned char smem_raw[];
  T* tab = reinterpret_cast<T*>(smem_raw);
  const bool radial = KID != HTLR_K_POLY_TEST;
  T* us = tab + (radial ? ((tsize + 1) & ~1) : 0);
  const int M = (d == 3) ? m * m * m : m * m;
  const int tid = threadIdx.x;
  const int tau = blockIdx.x;
  const int r0 = blockIdx.y * RC;
  int tb[3] = {tau % B, (tau / B) % B, d == 3 ? tau / (B * B) : 0};
  if (radial)
    for (int s = tid; s < tsize; s += kThreads) tab[s] = table[s];
  constexpr int IPT = 4;  // up to 4 * 256 target points per leaf
  T acc[IPT][RC];
  int Ii[IPT][3];
#pragma unroll
  for (int q = 0; q < IPT; ++q) {
    int i = tid + q * kThreads;
    int i0 = i % m, i1 = (i / m) % m, i2 = (d == 3) ? i / (m * m) : 0;
    Ii[q][0] = tb[0] * m + i0;
    Ii[q][1] = tb[1] * m + i1;
    Ii[q][2] = tb[2] * m + i2;
#pragma unroll
    for (int r = 0; r < RC; ++r) acc[q][r] = T(0);
  }
  for (int64_t e = nptr[tau]; e < nptr[tau + 1]; ++e) {
    const int sg = nsrc[e];
    const int sb[3] = {sg % B, (sg / B) % B, d == 3 ? sg / (B * B) : 0};
    __syncthreads();
    for (int idx = tid; idx < M * RC; idx += kThreads) {
      int j = idx % M, r = idx / M;
      int j0 = j % m, j1 = (j / m) % m, j2 = (d == 3) ? j / (m * m) : 0;
      int64_t g = lin3(sb[0] * m + j0, sb[1] * m + j1, d == 3 ? sb[2] * m + j2 : 0, n);
      if (d == 2) g = (int64_t)(sb[0] * m + j0) + (int64_t)n * (sb[1] * m + j1);
      us[r * M + j] = (r0 + r < nrhs) ? u[(int64_t)(r0 + r) * ((int64_t)n * n * (d == 3 ? n : 1)) + g] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
      if (tid + q * kThreads >= M) break;
      int jj = 0;
      const int nz = (d == 3) ? m : 1;
      for (int j2 = 0; j2 < nz; ++j2) {
        int d2 = (d == 3) ? Ii[q][2] - (sb[2] * m + j2) : 0;
        for (int j1 = 0; j1 < m; ++j1) {
          int d1 = Ii[q][1] - (sb[1] * m + j1);
          int base = d2 * d2 + d1 * d1;
          for (int j0 = 0; j0 < m; ++j0, ++jj) {
            int d0 = Ii[q][0] - (sb[0] * m + j0);
            T kv;
            if constexpr (radial) {
              kv = tab[base + d0 * d0];
            } else {
              if (d0 == 0 && d1 == 0 && d2 == 0) kv = D0;
              else kv = w0 * kvec<KID, T>(h * d0, h * d1, h * d2, d, pm1);
            }
#pragma unroll
            for (int r = 0; r < RC; ++r) acc[q][r] += kv * us[r * M + jj];
          }
        }
      }
    }
  }
  const int64_t N = (d == 3) ? (int64_t)n * n * n : (int64_t)n * n;
#pragma unroll
  for (int q = 0; q < IPT; ++q) {
    if (tid + q * kThreads >= M) break;
    int64_t g = (d == 3) ? lin3(Ii[q][0], Ii[q][1], Ii[q][2], n) : (int64_t)Ii[q][0] + (int64_t)n * Ii[q][1];
    T ai = a[g];
#pragma unroll
    for (int r = 0; r < RC; ++r)
      if (r0 + r < nrhs) f[(int64_t)(r0 + r) * N + g] = acc[q][r] + ai * u[(int64_t)(r0 + r) * N + g];
  }
}

// Near field + diagonal, uniform 3D grid with leaves of side m <= 8, one
// wave per (target leaf, rhs chunk).  Each lane owns one row of targets
// (i1, i2) and all m targets i0 along x.  For a source row (j1, j2) the
// m x m block between the target and source rows depends only on i0 - j0
// (the grid is uniform), so the 2m-1 kernel values are read once and reused
// for m*m*RC FMAs.
// With NW waves per leaf, wave w takes every NW-th source box and the
// partial sums are added in wave order through LDS.
template <int KID, typename T, int RC, int NW, bool FULL>
__global__ __launch_bounds__(64 * NW) void k_near_rows(
    const T* __restrict__ u, T* __restrict__ f, const T* __restrict__ a, const int64_t* __restrict__ nptr,
    const int32_t* __restrict__ nsrc, const T* __restrict__ table, int tsize, int n, int m, int B, int nrhs, T h,
    T w0, T D0, int pm1) {
  constexpr int MM = 8;
  extern __shared__ unsigned char smem_raw[];
  T* tab = reinterpret_cast<T*>(smem_raw);
  constexpr bool radial = KID != HTLR_K_POLY_TEST;
  const int M = m * m * m;
  const int wv = threadIdx.x >> 6;
  T* us_all = tab + (radial ? ((tsize + 1) & ~1) : 0);  // NW x [MM*64][RC], also the reduction buffer
  T* us = us_all + (size_t)wv * MM * 64 * RC;            // this wave's [M][RC]
  const int lane = threadIdx.x & 63;
  const int tau = blockIdx.x;
  const int r0 = blockIdx.y * RC;
  const int64_t N = (int64_t)n * n * n;
  const int tb0 = tau % B, tb1 = (tau / B) % B, tb2 = tau / (B * B);
  if (radial)
    for (int s = threadIdx.x; s < tsize; s += 64 * NW) tab[s] = table[s];
  const bool active = lane < m * m;
  const int i1 = lane % m, i2 = lane / m;
  const int I1 = tb1 * m + i1, I2 = tb2 * m + i2;
  T acc[MM][RC];
#pragma unroll
  for (int i = 0; i < MM; ++i)
#pragma unroll
    for (int r = 0; r < RC; ++r) acc[i][r] = T(0);
  const int64_t ebeg = nptr[tau], eend = nptr[tau + 1];
  for (int64_t e0 = ebeg; e0 < eend; e0 += NW) {
    const int64_t e = e0 + wv;
    const bool have = e < eend;
    const int sg = __builtin_amdgcn_readfirstlane(have ? nsrc[e] : 0);   // one source box per wave
    const int sb0 = sg % B, sb1 = (sg / B) % B, sb2 = sg / (B * B);
    __syncthreads();
    for (int idx = lane; have && idx < M * RC; idx += 64) {
      const int j = idx % M, r = idx / M;
      const int j0 = j % m, j1 = (j / m) % m, j2 = j / (m * m);
      us[j * RC + r] = (r0 + r < nrhs)
                           ? u[(int64_t)(r0 + r) * N + lin3(sb0 * m + j0, sb1 * m + j1, sb2 * m + j2, n)]
                           : T(0);
    }
    __syncthreads();
    if (!active || !have) continue;
    const int D = (tb0 - sb0) * m;   // I0 - J0 = D + (i0 - j0)
    int sq[2 * MM - 1];              // (D + dl)^2 for dl = -(MM-1)..MM-1, wave-uniform
#pragma unroll
    for (int k = 0; k < 2 * MM - 1; ++k) sq[k] = __builtin_amdgcn_readfirstlane((D + k - (MM - 1)) * (D + k - (MM - 1)));
    for (int j2 = 0; j2 < m; ++j2) {
      const int d2 = I2 - (sb2 * m + j2);
      for (int j1 = 0; j1 < m; ++j1) {
        const int d1 = I1 - (sb1 * m + j1);
        T tv[2 * MM - 1];
        if constexpr (radial) {
          const int base = d1 * d1 + d2 * d2;
#pragma unroll
          for (int k = 0; k < 2 * MM - 1; ++k) {
            const int dl = k - (MM - 1);
            const int dd = D + dl;
            if constexpr (FULL) tv[k] = tab[base + sq[k]];
            else tv[k] = (dl > -m && dl < m) ? tab[base + dd * dd] : T(0);
          }
        } else {
          const T f12 = w0 * ipow(T(1) + T(kPolyADev[1]) * (h * d1), pm1) * ipow(T(1) + T(kPolyADev[2]) * (h * d2), pm1);
#pragma unroll
          for (int k = 0; k < 2 * MM - 1; ++k) {
            const int dl = k - (MM - 1);
            const int dd = D + dl;
            const bool in = dl > -m && dl < m;
            const bool self = dd == 0 && d1 == 0 && d2 == 0;
            tv[k] = !in ? T(0) : (self ? D0 : f12 * ipow(T(1) + T(kPolyADev[0]) * (h * dd), pm1));
          }
        }
        const T* ur = us + (size_t)(m * j1 + m * m * j2) * RC;
#pragma unroll
        for (int j0 = 0; j0 < MM; ++j0) {
          if (!FULL && j0 >= m) break;
          T uv[RC];
#pragma unroll
          for (int r = 0; r < RC; ++r) uv[r] = ur[j0 * RC + r];
#pragma unroll
          for (int i0 = 0; i0 < MM; ++i0) {
            const T t = tv[i0 - j0 + MM - 1];
#pragma unroll
            for (int r = 0; r < RC; ++r) acc[i0][r] += t * uv[r];
          }
        }
      }
    }
  }
  if constexpr (NW > 1) {
    __syncthreads();
#pragma unroll
    for (int i0 = 0; i0 < MM; ++i0)
#pragma unroll
      for (int r = 0; r < RC; ++r) us[(i0 * RC + r) * 64 + lane] = acc[i0][r];
    __syncthreads();
    if (wv != 0) return;
#pragma unroll
    for (int i0 = 0; i0 < MM; ++i0)
#pragma unroll
      for (int r = 0; r < RC; ++r) {
        T v = T(0);
        for (int w = 0; w < NW; ++w) v += us_all[(size_t)w * MM * 64 * RC + (i0 * RC + r) * 64 + lane];
        acc[i0][r] = v;
      }
  }
  if (!active) return;
#pragma unroll
  for (int i0 = 0; i0 < MM; ++i0) {
    if (i0 >= m) break;
    const int64_t g = lin3(tb0 * m + i0, I1, I2, n);
    const T ai = a[g];
#pragma unroll
    for (int r = 0; r < RC; ++r)
      if (r0 + r < nrhs) f[(int64_t)(r0 + r) * N + g] = acc[i0][r] + ai * u[(int64_t)(r0 + r) * N + g];
  }
}

// Near field + diagonal on the matrix cores: uniform 3D grid, leaves of 8^3
// points, radial kernel, float.  For a target leaf and a chunk of 16
// right-hand sides, f_tau (512 x 16) += K_tau,sigma (512 x 512) u_sigma
// (512 x 16) for every near sigma, with 16x16x4 f32 MFMA: A = kernel values
// K(i, j) = T[|I - J|^2] read from the LDS table, B = u_sigma staged in LDS.
// Each of the 4 waves owns 128 target rows (8 MFMA tiles).
typedef float htlr_f32x4 __attribute__((ext_vector_type(4)));
typedef double htlr_f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
__device__ __forceinline__ void near_mfma_body(const T* __restrict__ u, T* __restrict__ f,
                                               const T* __restrict__ a, const int64_t* __restrict__ nptr,
                                               const int32_t* __restrict__ nsrc, const T* __restrict__ table,
                                               int tsize, int n, int B, int nrhs) {
  using V4 = typename std::conditional<std::is_same<T, double>::value, htlr_f64x4, htlr_f32x4>::type;
  constexpr int m = 8, M = 512;
  extern __shared__ unsigned char smem_raw[];
  T* tab = reinterpret_cast<T*>(smem_raw);
  const int tpad = (tsize + 3) & ~3;
  T* us = tab + tpad;                     // [M/2][16]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int tau = blockIdx.x;
  const int r0 = blockIdx.y * 16;
  const int64_t N = (int64_t)n * n * n;
  const int tb0 = tau % B, tb1 = (tau / B) % B, tb2 = tau / (B * B);
  for (int s = tid; s < tsize; s += 256) tab[s] = table[s];
  // A rows of this lane: i = wv*128 + t*16 + (lane & 15), t = 0..7
  //   ix = lane & 7, iy = (2 t + ((lane >> 3) & 1)) & 7, iz = 2 wv + t / 4
  const int l15 = lane & 15;
  const int Ix = tb0 * m + (l15 & 7);
  int Iy[4], Iz[2];
#pragma unroll
  for (int t = 0; t < 4; ++t) Iy[t] = tb1 * m + ((2 * t + (l15 >> 3)) & 7);
#pragma unroll
  for (int t = 0; t < 2; ++t) Iz[t] = tb2 * m + 2 * wv + t;
  V4 acc[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) acc[t] = V4{T(0), T(0), T(0), T(0)};
  const int jl = lane >> 4, rl = lane & 15;
  constexpr int JH = M / 2;               // source points staged at a time
  static_assert(JH == 256, "one staged source point per thread and half");
  // Staging is software pipelined: the 16 values (one source point, all
  // right-hand sides) this thread stages for the next half are loaded into
  // registers while the current half is computed.
  T pre[16];
  const int64_t e_beg = nptr[tau], e_end = nptr[tau + 1];
  auto load_half = [&](int64_t e, int half) {
    const int sg = nsrc[e];
    const int sb0 = sg % B, sb1 = (sg / B) % B, sb2 = sg / (B * B);
    const int j = half * JH + tid;
    const int64_t g = lin3(sb0 * m + (j & 7), sb1 * m + ((j >> 3) & 7), sb2 * m + (j >> 6), n);
#pragma unroll
    for (int r = 0; r < 16; ++r) pre[r] = (r0 + r < nrhs) ? u[(int64_t)(r0 + r) * N + g] : T(0);
  };
  if (e_beg < e_end) load_half(e_beg, 0);
  for (int64_t e = e_beg; e < e_end; ++e) {
    const int sg = nsrc[e];
    const int sb0 = sg % B, sb1 = (sg / B) % B, sb2 = sg / (B * B);
    for (int half = 0; half < 2; ++half) {
      const int jb = half * JH;
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 16; ++r) us[tid * 16 + r] = pre[r];
      __syncthreads();
      if (half == 0) load_half(e, 1);
      else if (e + 1 < e_end) load_half(e + 1, 0);
      for (int j0 = jb; j0 < jb + JH; j0 += 4) {
        const int j = j0 + jl;
        const int dx = Ix - (sb0 * m + (j & 7));
        const int jy = sb1 * m + ((j >> 3) & 7), jz = sb2 * m + (j >> 6);
        const T b = us[(j - jb) * 16 + rl];
        const int dx2 = dx * dx;
        int dy2[4], dz2[2];
#pragma unroll
        for (int t = 0; t < 4; ++t) { const int d = Iy[t] - jy; dy2[t] = d * d; }
#pragma unroll
        for (int t = 0; t < 2; ++t) { const int d = Iz[t] - jz; dz2[t] = d * d; }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const T av = tab[dx2 + dy2[t & 3] + dz2[t >> 2]];
          if constexpr (std::is_same<T, double>::value)
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b, acc[t], 0, 0, 0);
          else
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, b, acc[t], 0, 0, 0);
        }
      }
    }
  }
  const int r = lane & 15;
  if (r0 + r >= nrhs) return;
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      // accumulator layouts of 16x16x4: f32 register v holds row 4 (lane/16) + v,
      // f64 register v holds row lane/16 + 4 v; the column is lane % 16
      const int row = std::is_same<T, double>::value ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v;
      const int i = wv * 128 + t * 16 + row;
      const int64_t g = lin3(tb0 * m + (i & 7), tb1 * m + ((i >> 3) & 7), tb2 * m + (i >> 6), n);
      const int64_t o = (int64_t)(r0 + r) * N + g;
      f[o] = acc[t][v] + a[g] * u[o];
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_near_mfma(const T* __restrict__ u, T* __restrict__ f,
                                                    const T* __restrict__ a, const int64_t* __restrict__ nptr,
                                                    const int32_t* __restrict__ nsrc, const T* __restrict__ table,
                                                    int tsize, int n, int B, int nrhs) {
  near_mfma_body<T>(u, f, a, nptr, nsrc, table, tsize, n, B, nrhs);
}

// Single precision: at least 4 waves per SIMD (the compiler then fits the
// kernel in fewer registers; 3% faster at 128^3 x 16 than its own choice of 3).
template <>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_near_mfma<float>(
    const float* __restrict__ u, float* __restrict__ f, const float* __restrict__ a, const int64_t* __restrict__ nptr,
    const int32_t* __restrict__ nsrc, const float* __restrict__ table, int tsize, int n, int B, int nrhs) {
  near_mfma_body<float>(u, f, a, nptr, nsrc, table, tsize, n, B, nrhs);
}

// Near field + diagonal on a general tensor grid: kernel values evaluated from
// coordinates relative to the target box, weights |Omega_j| and per-point
// diagonal integrals D_i.
template <int KID, typename T, int RC>
__global__ __launch_bounds__(kThreads) void k_near_tensor(
    const T* __restrict__ u, T* __restrict__ f, const T* __restrict__ a, const T* __restrict__ D,
    const int64_t* __restrict__ nptr, const int32_t* __restrict__ nsrc, const double* __restrict__ x,
    const T* __restrict__ wdim, int d, int n, int m, int B, int nrhs, int pm1) {
  extern __shared__ unsigned char smem_raw[];
  constexpr bool kTab = uses_exp_table<KID, T>();
  double* etab = reinterpret_cast<double*>(smem_raw);                // [64] 2^(j/64), exponential kernels in FP64
  T* cs = reinterpret_cast<T*>(smem_raw + (kTab ? kExpTabBytes : 0));  // [3][m] source coordinates relative to the target box
  T* us = cs + 3 * m;                      // [RC][M] weighted source values
  const int M = (d == 3) ? m * m * m : m * m;
  const int tid = threadIdx.x;
  if constexpr (kTab)
    for (int i = tid; i < 64; i += kThreads) etab[i] = kExp2Frac64[i];
  const int tau = blockIdx.x;
  const int r0 = blockIdx.y * RC;
  const int64_t N = (d == 3) ? (int64_t)n * n * n : (int64_t)n * n;
  int tb[3] = {tau % B, (tau / B) % B, d == 3 ? tau / (B * B) : 0};
  double org[3];
  for (int l = 0; l < 3; ++l) org[l] = l < d ? x[l * n + tb[l] * m] : 0.0;
  constexpr int IPT = 4;
  T acc[IPT][RC];
  T xi[IPT][3];
  int li[IPT];
#pragma unroll
  for (int q = 0; q < IPT; ++q) {
    int i = tid + q * kThreads;
    li[q] = i;
    int ii[3] = {i % m, (i / m) % m, (d == 3) ? i / (m * m) : 0};
    for (int l = 0; l < 3; ++l) xi[q][l] = l < d ? (T)(x[l * n + tb[l] * m + ii[l]] - org[l]) : T(0);
#pragma unroll
    for (int r = 0; r < RC; ++r) acc[q][r] = T(0);
  }
  for (int64_t e = nptr[tau]; e < nptr[tau + 1]; ++e) {
    const int sg = nsrc[e];
    const int sb[3] = {sg % B, (sg / B) % B, d == 3 ? sg / (B * B) : 0};
    __syncthreads();
    for (int idx = tid; idx < 3 * m; idx += kThreads) {
      int l = idx / m, j = idx % m;
      cs[idx] = l < d ? (T)(x[l * n + sb[l] * m + j] - org[l]) : T(0);
    }
    for (int idx = tid; idx < M * RC; idx += kThreads) {
      int j = idx % M, r = idx / M;
      int jj[3] = {j % m, (j / m) % m, (d == 3) ? j / (m * m) : 0};
      int gi[3] = {sb[0] * m + jj[0], sb[1] * m + jj[1], d == 3 ? sb[2] * m + jj[2] : 0};
      int64_t g = (d == 3) ? lin3(gi[0], gi[1], gi[2], n) : (int64_t)gi[0] + (int64_t)n * gi[1];
      T wj = wdim[gi[0]] * wdim[n + gi[1]];
      if (d == 3) wj *= wdim[2 * n + gi[2]];
      us[r * M + j] = (r0 + r < nrhs) ? wj * u[(int64_t)(r0 + r) * N + g] : T(0);
    }
    __syncthreads();
    const bool self = (sg == tau);
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
      if (li[q] >= M) break;
      int jj = 0;
      const int nz = (d == 3) ? m : 1;
      for (int j2 = 0; j2 < nz; ++j2) {
        T dx2 = (d == 3) ? xi[q][2] - cs[2 * m + j2] : T(0);
        for (int j1 = 0; j1 < m; ++j1) {
          T dx1 = xi[q][1] - cs[m + j1];
          const T c12 = dx1 * dx1 + dx2 * dx2;
          for (int j0 = 0; j0 < m; ++j0, ++jj) {
            if (self && jj == li[q]) continue;
            T dx0 = xi[q][0] - cs[j0];
            T kv = kvec_c12_t<KID, T>(dx0, dx1, dx2, c12, d, pm1, etab);
#pragma unroll
            for (int r = 0; r < RC; ++r) acc[q][r] += kv * us[r * M + jj];
          }
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < IPT; ++q) {
    int i = li[q];
    if (i >= M) break;
    int ii[3] = {i % m, (i / m) % m, (d == 3) ? i / (m * m) : 0};
    int gi[3] = {tb[0] * m + ii[0], tb[1] * m + ii[1], d == 3 ? tb[2] * m + ii[2] : 0};
    int64_t g = (d == 3) ? lin3(gi[0], gi[1], gi[2], n) : (int64_t)gi[0] + (int64_t)n * gi[1];
    T diag = a[g] + D[g];
#pragma unroll
    for (int r = 0; r < RC; ++r)
      if (r0 + r < nrhs) f[(int64_t)(r0 + r) * N + g] = acc[q][r] + diag * u[(int64_t)(r0 + r) * N + g];
  }
}

// ---------------------------------------------------------------------------
// Up contraction: W_sigma = u~_sigma x_1 V_1^T ... x_d V_d^T, one block per
// (box, right-hand side, chunk), slice by slice along the last dimension.
// V is [m][p] (uniform: vstride = 0) or [d][B][m][p] (per box).  Large boxes
// of coarse levels are split over gridDim.z chunks of rpc slices; each chunk
// writes a partial W (part != nullptr), summed in chunk order by k_up_reduce.
template <typename T, typename TW>
__global__ __launch_bounds__(kThreads) void k_up(const T* __restrict__ u, TW* __restrict__ W,
                                                 const T* __restrict__ V, int uniform, int d, int n, int m,
                                                 int B, int p, int nrhs, int rpc, T* __restrict__ part, int rows) {
  extern __shared__ unsigned char smem_raw[];
  const int tid = threadIdx.x;
  const int box = blockIdx.x, r = blockIdx.y;
  const int lo = blockIdx.z * rpc, hi = min(m, lo + rpc);
  const int P = (d == 3) ? p * p * p : p * p;
  const int64_t N = (d == 3) ? (int64_t)n * n * n : (int64_t)n * n;
  int bb[3] = {box % B, (box / B) % B, d == 3 ? box / (B * B) : 0};
  auto Vk = [&](int k) -> const T* {
    return uniform ? V : V + ((size_t)k * B + bb[k]) * (size_t)m * p;
  };
  const T* V0 = Vk(0);
  const T* V1 = Vk(1);
  const T* V2 = d == 3 ? Vk(2) : nullptr;
  constexpr int WPT = 8;  // up to 8 * 256 core entries (p^d <= 2048)
  T acc[WPT];
#pragma unroll
  for (int q = 0; q < WPT; ++q) acc[q] = T(0);
  const T* ur = u + (int64_t)r * N;
  if (d == 3) {
    // a slice is staged in chunks of `rows` rows (all of it when it fits)
    T* sl = reinterpret_cast<T*>(smem_raw);   // rows*m
    T* t1 = sl + rows * m;                     // p*m
    T* t12 = t1 + p * m;                       // p*p
    for (int j2 = lo; j2 < hi; ++j2) {
      for (int ja = 0; ja < m; ja += rows) {
        const int nr = min(rows, m - ja);
        __syncthreads();
        for (int idx = tid; idx < m * nr; idx += kThreads) {
          int j0 = idx % m, jr = idx / m;
          sl[idx] = ur[lin3(bb[0] * m + j0, bb[1] * m + ja + jr, bb[2] * m + j2, n)];
        }
        __syncthreads();
        for (int idx = tid; idx < p * nr; idx += kThreads) {
          int s0 = idx % p, jr = idx / p;
          T v = T(0);
          for (int j0 = 0; j0 < m; ++j0) v += V0[j0 * p + s0] * sl[jr * m + j0];
          t1[(ja + jr) * p + s0] = v;  // [j1][s0]
        }
      }
      __syncthreads();
      for (int idx = tid; idx < p * p; idx += kThreads) {
        int s0 = idx % p, s1 = idx / p;
        T v = T(0);
        for (int j1 = 0; j1 < m; ++j1) v += V1[j1 * p + s1] * t1[j1 * p + s0];
        t12[idx] = v;  // [s1][s0]
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < WPT; ++q) {
        int t = tid + q * kThreads;
        if (t < P) acc[q] += V2[j2 * p + t / (p * p)] * t12[t % (p * p)];
      }
    }
  } else {
    // each row's p dot products of length m are split over kThreads / p
    // thread groups and combined through LDS in group order
    T* sl = reinterpret_cast<T*>(smem_raw);   // row, m
    T* red = sl + m;                           // kThreads partial sums
    T* t1 = red + kThreads;                    // p
    const int G = kThreads / p;
    const int s0g = tid % p, g = tid / p;
    for (int j1 = lo; j1 < hi; ++j1) {
      __syncthreads();
      for (int j0 = tid; j0 < m; j0 += kThreads) sl[j0] = ur[(int64_t)(bb[0] * m + j0) + (int64_t)n * (bb[1] * m + j1)];
      __syncthreads();
      if (g < G) {
        T v = T(0);
        for (int j0 = g; j0 < m; j0 += G) v += V0[j0 * p + s0g] * sl[j0];
        red[g * p + s0g] = v;
      }
      __syncthreads();
      if (tid < p) {
        T v = T(0);
        for (int k = 0; k < G; ++k) v += red[k * p + tid];
        t1[tid] = v;
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < WPT; ++q) {
        int t = tid + q * kThreads;
        if (t < P) acc[q] += V1[j1 * p + t / p] * t1[t % p];
      }
    }
  }
  if (part) {
    T* Po = part + (((int64_t)blockIdx.z * gridDim.x + box) * nrhs + r) * P;
#pragma unroll
    for (int q = 0; q < WPT; ++q) {
      int t = tid + q * kThreads;
      if (t < P) Po[t] = acc[q];
    }
    return;
  }
  TW* Wo = W + ((int64_t)box * nrhs + r) * P;
#pragma unroll
  for (int q = 0; q < WPT; ++q) {
    int t = tid + q * kThreads;
    if (t < P) Wo[t] = store_cast<TW>(acc[q]);
  }
}

// W = sum over the chunks of the partial up contractions, in chunk order.
template <typename T, typename TW>
__global__ void k_up_reduce(const T* __restrict__ part, TW* __restrict__ W, int64_t count, int chunks) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
    T v = part[i];
    for (int c = 1; c < chunks; ++c) v += part[c * count + i];
    W[i] = store_cast<TW>(v);
  }
}

// Down expansion: f_tau += H_tau x_1 U_1 ... x_d U_d, one block per (box,
// rhs, chunk of rpc slices along the last dimension; chunks write disjoint
// parts of f).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_down(const T* __restrict__ H, T* __restrict__ f,
                                                   const T* __restrict__ U, int uniform, int d, int n, int m,
                                                   int B, int p, int nrhs, int rpc) {
  extern __shared__ unsigned char smem_raw[];
  const int P = (d == 3) ? p * p * p : p * p;
  T* hs = reinterpret_cast<T*>(smem_raw);  // P
  T* z = hs + P;                           // p*p (3D: [t1][t0]) or p (2D)
  T* y = z + p * p;                        // m*p   [i1][t0] (3D)
  const int tid = threadIdx.x;
  const int box = blockIdx.x, r = blockIdx.y;
  const int lo = blockIdx.z * rpc, hi = min(m, lo + rpc);
  const int64_t N = (d == 3) ? (int64_t)n * n * n : (int64_t)n * n;
  int bb[3] = {box % B, (box / B) % B, d == 3 ? box / (B * B) : 0};
  auto Uk = [&](int k) -> const T* {
    return uniform ? U : U + ((size_t)k * B + bb[k]) * (size_t)m * p;
  };
  const T* U0 = Uk(0);
  const T* U1 = Uk(1);
  const T* U2 = d == 3 ? Uk(2) : nullptr;
  const T* Hb = H + ((int64_t)box * nrhs + r) * P;
  for (int t = tid; t < P; t += kThreads) hs[t] = Hb[t];
  T* fr = f + (int64_t)r * N;
  if (d == 3) {
    for (int i2 = lo; i2 < hi; ++i2) {
      __syncthreads();
      for (int idx = tid; idx < p * p; idx += kThreads) {
        T v = T(0);
        for (int t2 = 0; t2 < p; ++t2) v += U2[i2 * p + t2] * hs[t2 * p * p + idx];
        z[idx] = v;  // [t1][t0]
      }
      __syncthreads();
      for (int idx = tid; idx < m * p; idx += kThreads) {
        int t0 = idx % p, i1 = idx / p;
        T v = T(0);
        for (int t1 = 0; t1 < p; ++t1) v += U1[i1 * p + t1] * z[t1 * p + t0];
        y[idx] = v;  // [i1][t0]
      }
      __syncthreads();
      for (int idx = tid; idx < m * m; idx += kThreads) {
        int i0 = idx % m, i1 = idx / m;
        T v = T(0);
        for (int t0 = 0; t0 < p; ++t0) v += U0[i0 * p + t0] * y[i1 * p + t0];
        fr[lin3(bb[0] * m + i0, bb[1] * m + i1, bb[2] * m + i2, n)] += v;
      }
    }
  } else {
    for (int i1 = lo; i1 < hi; ++i1) {
      __syncthreads();
      for (int t0 = tid; t0 < p; t0 += kThreads) {
        T v = T(0);
        for (int t1 = 0; t1 < p; ++t1) v += U1[i1 * p + t1] * hs[t1 * p + t0];
        z[t0] = v;
      }
      __syncthreads();
      for (int i0 = tid; i0 < m; i0 += kThreads) {
        T v = T(0);
        for (int t0 = 0; t0 < p; ++t0) v += U0[i0 * p + t0] * z[t0];
        fr[(int64_t)(bb[0] * m + i0) + (int64_t)n * (bb[1] * m + i1)] += v;
      }
    }
  }
}

// Source or output tensor of (box, column r): the product's own buffer
// ([box][nrhs][P]), or with GRP the buffer of the matrix that owns column r
// in a grouped launch over several matrices that share their factors.
template <bool GRP, typename TW>
__device__ __forceinline__ TW* col_slot(TW* W, const ColTab* __restrict__ tab, int64_t box, int r, int nrhs, int P) {
  if constexpr (GRP) return (TW*)tab->base[r] + (box * tab->ld[r] + tab->rl[r]) * (int64_t)P;
  else return W + (box * nrhs + r) * (int64_t)P;
}

// Up contraction of a whole 2D box in one block (boxes of up to 64 x 64
// points): the box X is staged in LDS, then T1[j1][s0] = sum_j0 V0[j0][s0]
// X[j1][j0] and W[s1][s0] = sum_j1 V1[j1][s1] T1[j1][s0], two barriers per
// box instead of a few per row.
template <typename T, typename TW, bool GRP = false>
__global__ __launch_bounds__(kThreads) void k_up2d_box(const T* __restrict__ u, TW* __restrict__ W,
                                                       const T* __restrict__ V, int uniform, int n, int m, int B,
                                                       int p, int nrhs, const ColTab* __restrict__ tab) {
  extern __shared__ unsigned char smem_raw[];
  T* X = reinterpret_cast<T*>(smem_raw);   // m*m  [j1][j0]
  T* T1 = X + m * m;                       // m*p  [j1][s0]
  const int tid = threadIdx.x;
  const int box = blockIdx.x, r = blockIdx.y;
  const int b0 = box % B, b1 = box / B;
  const T* V0 = uniform ? V : V + (size_t)b0 * m * p;
  const T* V1 = uniform ? V : V + ((size_t)B + b1) * m * p;
  const T* ur = u + (int64_t)r * n * n;
  for (int idx = tid; idx < m * m; idx += kThreads) {
    const int j0 = idx % m, j1 = idx / m;
    X[idx] = ur[(int64_t)(b0 * m + j0) + (int64_t)n * (b1 * m + j1)];
  }
  __syncthreads();
  for (int idx = tid; idx < m * p; idx += kThreads) {
    const int s0 = idx % p, j1 = idx / p;
    T v = T(0);
    for (int j0 = 0; j0 < m; ++j0) v += V0[j0 * p + s0] * X[j1 * m + j0];
    T1[idx] = v;
  }
  __syncthreads();
  TW* Wo = col_slot<GRP>(W, tab, box, r, nrhs, p * p);
  for (int idx = tid; idx < p * p; idx += kThreads) {
    const int s0 = idx % p, s1 = idx / p;
    T v = T(0);
    for (int j1 = 0; j1 < m; ++j1) v += V1[j1 * p + s1] * T1[j1 * p + s0];
    Wo[idx] = store_cast<TW>(v);
  }
}

// Down expansion of a whole 2D box in one block (boxes of up to 64 x 64
// points): Z[i1][t0] = sum_t1 U1[i1][t1] H[t1][t0], then
// f[i1][i0] += sum_t0 U0[i0][t0] Z[i1][t0] (the sums of k_down, in its order).
template <typename T, bool GRP = false>
__global__ __launch_bounds__(kThreads) void k_down2d_box(const T* __restrict__ H, T* __restrict__ f,
                                                         const T* __restrict__ U, int uniform, int n, int m, int B,
                                                         int p, int nrhs, const ColTab* __restrict__ tab) {
  extern __shared__ unsigned char smem_raw[];
  T* hs = reinterpret_cast<T*>(smem_raw);  // p*p  [t1][t0]
  T* Z = hs + p * p;                       // m*p  [i1][t0]
  const int tid = threadIdx.x;
  const int box = blockIdx.x, r = blockIdx.y;
  const int b0 = box % B, b1 = box / B;
  const T* U0 = uniform ? U : U + (size_t)b0 * m * p;
  const T* U1 = uniform ? U : U + ((size_t)B + b1) * m * p;
  const T* Hb = col_slot<GRP>(H, tab, box, r, nrhs, p * p);
  for (int t = tid; t < p * p; t += kThreads) hs[t] = Hb[t];
  __syncthreads();
  for (int idx = tid; idx < m * p; idx += kThreads) {
    const int t0 = idx % p, i1 = idx / p;
    T v = T(0);
    for (int t1 = 0; t1 < p; ++t1) v += U1[i1 * p + t1] * hs[t1 * p + t0];
    Z[idx] = v;
  }
  __syncthreads();
  T* fr = f + (int64_t)r * n * n;
  for (int idx = tid; idx < m * m; idx += kThreads) {
    const int i0 = idx % m, i1 = idx / m;
    T v = T(0);
    for (int t0 = 0; t0 < p; ++t0) v += U0[i0 * p + t0] * Z[i1 * p + t0];
    fr[(int64_t)(b0 * m + i0) + (int64_t)n * (b1 * m + i1)] += v;
  }
}

// Up contraction of large 2D boxes (128 points per side and more): R rows
// staged at a time (R m <= 4096, R p <= kThreads), each of a stage's R p dots
// (length m) split over G = kThreads / (R p) threads and combined through LDS
// in group order; thread t < p^2 accumulates W[s1][s0] over the rows in order.
// Four barriers per stage of R rows.  Grid (boxes, rhs, row chunks); with
// several chunks the partial sums go to part (summed by k_up_reduce).
template <typename T, typename TW>
__global__ __launch_bounds__(kThreads) void k_up2d_rows(const T* __restrict__ u, TW* __restrict__ W,
                                                        const T* __restrict__ V, int uniform, int n, int m, int B,
                                                        int p, int nrhs, int rpc, int R, T* __restrict__ part) {
  extern __shared__ unsigned char smem_raw[];
  T* X = reinterpret_cast<T*>(smem_raw);   // R*m      [jr][j0]
  T* red = X + R * m;                      // kThreads partial dots
  T* T1 = red + kThreads;                  // R*p      [jr][s0]
  const int tid = threadIdx.x;
  const int box = blockIdx.x, r = blockIdx.y;
  const int lo = blockIdx.z * rpc, hi = min(m, lo + rpc);
  const int b0 = box % B, b1 = box / B;
  const T* V0 = uniform ? V : V + (size_t)b0 * m * p;
  const T* V1 = uniform ? V : V + ((size_t)B + b1) * m * p;
  const T* ur = u + (int64_t)r * n * n;
  const int P = p * p;
  const int s0 = tid % p, s1 = tid / p;
  T acc = T(0);
  for (int ja = lo; ja < hi; ja += R) {
    const int nr = min(R, hi - ja);
    const int nout = nr * p, G = kThreads / nout;
    __syncthreads();
    for (int idx = tid; idx < nr * m; idx += kThreads) {
      const int j0 = idx % m, jr = idx / m;
      X[idx] = ur[(int64_t)(b0 * m + j0) + (int64_t)n * (b1 * m + ja + jr)];
    }
    __syncthreads();
    {
      const int o = tid % nout, g = tid / nout;
      if (g < G) {
        const int c0 = o % p, jr = o / p;
        T v = T(0);
        for (int j0 = g; j0 < m; j0 += G) v += V0[j0 * p + c0] * X[jr * m + j0];
        red[g * nout + o] = v;
      }
    }
    __syncthreads();
    if (tid < nout) {
      T v = T(0);
      for (int k = 0; k < G; ++k) v += red[k * nout + tid];
      T1[tid] = v;
    }
    __syncthreads();
    if (tid < P)
      for (int jr = 0; jr < nr; ++jr) acc += V1[(ja + jr) * p + s1] * T1[jr * p + s0];
  }
  if (tid >= P) return;
  if (part) {
    part[(((int64_t)blockIdx.z * gridDim.x + box) * nrhs + r) * P + tid] = acc;
    return;
  }
  W[((int64_t)box * nrhs + r) * P + tid] = store_cast<TW>(acc);
}

// Down expansion of 2D boxes, R rows at a time (R m <= 4096 outputs):
// Z[ir][t0] = sum_t1 U1[i1][t1] H[t1][t0], then
// f[i1][i0] += sum_t0 U0[i0][t0] Z[ir][t0] (the sums of k_down, in its order).
// Grid (boxes, rhs, row chunks); chunks write disjoint rows of f.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_down2d(const T* __restrict__ H, T* __restrict__ f,
                                                     const T* __restrict__ U, int uniform, int n, int m, int B, int p,
                                                     int nrhs, int rpc, int R) {
  extern __shared__ unsigned char smem_raw[];
  T* hs = reinterpret_cast<T*>(smem_raw);  // p*p  [t1][t0]
  T* Z = hs + p * p;                       // R*p  [ir][t0]
  const int tid = threadIdx.x;
  const int box = blockIdx.x, r = blockIdx.y;
  const int lo = blockIdx.z * rpc, hi = min(m, lo + rpc);
  const int b0 = box % B, b1 = box / B;
  const T* U0 = uniform ? U : U + (size_t)b0 * m * p;
  const T* U1 = uniform ? U : U + ((size_t)B + b1) * m * p;
  const T* Hb = H + ((int64_t)box * nrhs + r) * p * p;
  for (int t = tid; t < p * p; t += kThreads) hs[t] = Hb[t];
  T* fr = f + (int64_t)r * n * n;
  for (int ia = lo; ia < hi; ia += R) {
    const int nr = min(R, hi - ia);
    __syncthreads();
    for (int idx = tid; idx < nr * p; idx += kThreads) {
      const int t0 = idx % p, ir = idx / p;
      T v = T(0);
      for (int t1 = 0; t1 < p; ++t1) v += U1[(ia + ir) * p + t1] * hs[t1 * p + t0];
      Z[idx] = v;
    }
    __syncthreads();
    for (int idx = tid; idx < nr * m; idx += kThreads) {
      const int i0 = idx % m, ir = idx / m;
      T v = T(0);
      for (int t0 = 0; t0 < p; ++t0) v += U0[i0 * p + t0] * Z[ir * p + t0];
      fr[(int64_t)(b0 * m + i0) + (int64_t)n * (b1 * m + ia + ir)] += v;
    }
  }
}

// Up contraction of small 3D boxes (up to 16 points per side) in one pass:
// nb boxes per block, each box staged in LDS, then
//   T1[j2][j1][s0] = sum_j0 V0[j0][s0] X[j2][j1][j0],
//   T2[j2][s1][s0] = sum_j1 V1[j1][s1] T1[j2][j1][s0],
//   W[s2][s1][s0]  = sum_j2 V2[j2][s2] T2[j2][s1][s0]
// (the sums of k_up, in its order), three barriers per block.
template <typename T, typename TW, bool GRP = false>
__global__ __launch_bounds__(kThreads) void k_up3d_small(const T* __restrict__ u, TW* __restrict__ W,
                                                         const T* __restrict__ V, int uniform, int n, int m, int B,
                                                         int p, int nrhs, int nb, int64_t nbox,
                                                         const ColTab* __restrict__ tab) {
  extern __shared__ unsigned char smem_raw[];
  const int m2 = m * m, m3 = m2 * m, pp = p * p, P = pp * p;
  const int per = m3 + m2 * p + m * pp;    // LDS values per box
  T* sh = reinterpret_cast<T*>(smem_raw);
  const int tid = threadIdx.x, r = blockIdx.y;
  const int64_t box0 = (int64_t)blockIdx.x * nb;
  const T* ur = u + (int64_t)r * n * n * n;
  auto Vk = [&](int k, int64_t box) -> const T* {
    if (uniform) return V;
    const int64_t bk = k == 0 ? box % B : (k == 1 ? (box / B) % B : box / ((int64_t)B * B));
    return V + ((size_t)k * B + bk) * (size_t)m * p;
  };
  for (int idx = tid; idx < nb * m3; idx += kThreads) {
    const int bl = idx / m3, q = idx % m3;
    const int64_t box = box0 + bl;
    if (box >= nbox) continue;
    const int j0 = q % m, j1 = (q / m) % m, j2 = q / m2;
    const int64_t b0 = box % B, b1 = (box / B) % B, b2 = box / ((int64_t)B * B);
    sh[bl * per + q] = ur[lin3((int)(b0 * m + j0), (int)(b1 * m + j1), (int)(b2 * m + j2), n)];
  }
  __syncthreads();
  for (int idx = tid; idx < nb * m2 * p; idx += kThreads) {
    const int bl = idx / (m2 * p), q = idx % (m2 * p);
    const int64_t box = box0 + bl;
    if (box >= nbox) continue;
    const int s0 = q % p, j12 = q / p;           // j12 = j1 + m j2
    const T* V0 = Vk(0, box);
    const T* X = sh + bl * per + j12 * m;
    T v = T(0);
    for (int j0 = 0; j0 < m; ++j0) v += V0[j0 * p + s0] * X[j0];
    sh[bl * per + m3 + q] = v;                   // T1[j2][j1][s0]
  }
  __syncthreads();
  for (int idx = tid; idx < nb * m * pp; idx += kThreads) {
    const int bl = idx / (m * pp), q = idx % (m * pp);
    const int64_t box = box0 + bl;
    if (box >= nbox) continue;
    const int s0 = q % p, s1 = (q / p) % p, j2 = q / pp;
    const T* V1 = Vk(1, box);
    const T* T1 = sh + bl * per + m3 + j2 * m * p;
    T v = T(0);
    for (int j1 = 0; j1 < m; ++j1) v += V1[j1 * p + s1] * T1[j1 * p + s0];
    sh[bl * per + m3 + m2 * p + q] = v;          // T2[j2][s1][s0]
  }
  __syncthreads();
  for (int idx = tid; idx < nb * P; idx += kThreads) {
    const int bl = idx / P, t = idx % P;
    const int64_t box = box0 + bl;
    if (box >= nbox) continue;
    const T* V2 = Vk(2, box);
    const T* T2 = sh + bl * per + m3 + m2 * p;
    T v = T(0);
    for (int j2 = 0; j2 < m; ++j2) v += V2[j2 * p + t / pp] * T2[j2 * pp + t % pp];
    col_slot<GRP>(W, tab, box, r, nrhs, P)[t] = store_cast<TW>(v);
  }
}

// Down expansion of small 3D boxes (up to 16 points per side) in one pass:
//   Z2[i2][t1][t0] = sum_t2 U2[i2][t2] H[t2][t1][t0],
//   Z1[i2][i1][t0] = sum_t1 U1[i1][t1] Z2[i2][t1][t0],
//   f[i2][i1][i0] += sum_t0 U0[i0][t0] Z1[i2][i1][t0]
// (the sums of k_down, in its order), nb boxes per block.
template <typename T, bool GRP = false>
__global__ __launch_bounds__(kThreads) void k_down3d_small(const T* __restrict__ H, T* __restrict__ f,
                                                           const T* __restrict__ U, int uniform, int n, int m, int B,
                                                           int p, int nrhs, int nb, int64_t nbox,
                                                           const ColTab* __restrict__ tab) {
  extern __shared__ unsigned char smem_raw[];
  const int m2 = m * m, m3 = m2 * m, pp = p * p, P = pp * p;
  const int per = P + m * pp + m2 * p;     // LDS values per box
  T* sh = reinterpret_cast<T*>(smem_raw);
  const int tid = threadIdx.x, r = blockIdx.y;
  const int64_t box0 = (int64_t)blockIdx.x * nb;
  auto Uk = [&](int k, int64_t box) -> const T* {
    if (uniform) return U;
    const int64_t bk = k == 0 ? box % B : (k == 1 ? (box / B) % B : box / ((int64_t)B * B));
    return U + ((size_t)k * B + bk) * (size_t)m * p;
  };
  for (int idx = tid; idx < nb * P; idx += kThreads) {
    const int bl = idx / P, t = idx % P;
    const int64_t box = box0 + bl;
    if (box >= nbox) continue;
    sh[bl * per + t] = col_slot<GRP>(H, tab, box, r, nrhs, P)[t];
  }
  __syncthreads();
  for (int idx = tid; idx < nb * m * pp; idx += kThreads) {
    const int bl = idx / (m * pp), q = idx % (m * pp);
    const int64_t box = box0 + bl;
    if (box >= nbox) continue;
    const int t01 = q % pp, i2 = q / pp;
    const T* U2 = Uk(2, box);
    const T* hs = sh + bl * per;
    T v = T(0);
    for (int t2 = 0; t2 < p; ++t2) v += U2[i2 * p + t2] * hs[t2 * pp + t01];
    sh[bl * per + P + q] = v;                    // Z2[i2][t1][t0]
  }
  __syncthreads();
  for (int idx = tid; idx < nb * m2 * p; idx += kThreads) {
    const int bl = idx / (m2 * p), q = idx % (m2 * p);
    const int64_t box = box0 + bl;
    if (box >= nbox) continue;
    const int t0 = q % p, i1 = (q / p) % m, i2 = q / (m * p);
    const T* U1 = Uk(1, box);
    const T* Z2 = sh + bl * per + P + i2 * pp;
    T v = T(0);
    for (int t1 = 0; t1 < p; ++t1) v += U1[i1 * p + t1] * Z2[t1 * p + t0];
    sh[bl * per + P + m * pp + q] = v;           // Z1[i2][i1][t0]
  }
  __syncthreads();
  T* fr = f + (int64_t)r * n * n * n;
  for (int idx = tid; idx < nb * m3; idx += kThreads) {
    const int bl = idx / m3, q = idx % m3;
    const int64_t box = box0 + bl;
    if (box >= nbox) continue;
    const int i0 = q % m, i12 = q / m;           // i12 = i1 + m i2
    const T* U0 = Uk(0, box);
    const T* Z1 = sh + bl * per + P + m * pp + i12 * p;
    T v = T(0);
    for (int t0 = 0; t0 < p; ++t0) v += U0[i0 * p + t0] * Z1[t0];
    const int64_t b0 = box % B, b1 = (box / B) % B, b2 = box / ((int64_t)B * B);
    fr[lin3((int)(b0 * m + i0), (int)(b1 * m + i12 % m), (int)(b2 * m + i12 / m), n)] += v;
  }
}

// Core apply with one stored core per offset (uniform grids), plain VALU
// version: one block per (target box, rhs chunk), one thread per core row t.
// G layout: GT = true -> [core][s][t], false -> [core][t][s].
template <typename TG, typename TW, typename TA, int RC, bool GT>
__global__ __launch_bounds__(kThreads) void k_core_simple(
    const TW* __restrict__ W, TA* __restrict__ H, const TG* __restrict__ G, const int64_t* __restrict__ ptr,
    const int32_t* __restrict__ src, const int32_t* __restrict__ cid, int P, int nrhs) {
  extern __shared__ unsigned char smem_raw[];
  TA* ws = reinterpret_cast<TA*>(smem_raw);  // [RC][P]
  const int tid = threadIdx.x;
  const int tau = blockIdx.x;
  const int r0 = blockIdx.y * RC;
  constexpr int TPT = 8;
  TA acc[TPT][RC];
#pragma unroll
  for (int q = 0; q < TPT; ++q)
#pragma unroll
    for (int r = 0; r < RC; ++r) acc[q][r] = TA(0);
  const int64_t PP = (int64_t)P * P;
  for (int64_t e = ptr[tau]; e < ptr[tau + 1]; ++e) {
    const int64_t sg = src[e];
    const TG* Gc = G + (int64_t)cid[e] * PP;
    __syncthreads();
    for (int idx = tid; idx < RC * P; idx += kThreads) {
      int r = idx / P, s = idx % P;
      ws[idx] = (r0 + r < nrhs) ? to_acc(W[(sg * nrhs + r0 + r) * P + s]) : TA(0);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < TPT; ++q) {
      int t = tid + q * kThreads;
      if (t >= P) break;
      for (int s = 0; s < P; ++s) {
        TA g = to_acc(GT ? Gc[(int64_t)s * P + t] : Gc[(int64_t)t * P + s]);
#pragma unroll
        for (int r = 0; r < RC; ++r) acc[q][r] += g * ws[r * P + s];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    int t = tid + q * kThreads;
    if (t >= P) break;
#pragma unroll
    for (int r = 0; r < RC; ++r)
      if (r0 + r < nrhs) H[((int64_t)tau * nrhs + r0 + r) * P + t] = acc[q][r];
  }
}

// Core apply on a general tensor grid: G(t, s) = k(xi_t - eta_s) generated on
// the fly from the Chebyshev points of both boxes (relative to the target
// box), one block per (target box, rhs chunk).
template <int KID, typename T, int RC>
__global__ __launch_bounds__(kThreads) void k_core_tensor(
    const T* __restrict__ W, T* __restrict__ H, const double* __restrict__ cheb, const int64_t* __restrict__ ptr,
    const int32_t* __restrict__ src, int d, int p, int B, int nrhs, int pm1) {
  extern __shared__ unsigned char smem_raw[];
  constexpr bool kTab = uses_exp_table<KID, T>();
  double* etab = reinterpret_cast<double*>(smem_raw);                // [64] 2^(j/64), exponential kernels in FP64
  T* ws = reinterpret_cast<T*>(smem_raw + (kTab ? kExpTabBytes : 0));  // [RC][P]
  const int P = (d == 3) ? p * p * p : p * p;
  T* ce = ws + RC * P;                      // [3][p] source points relative to the target origin
  const int tid = threadIdx.x;
  if constexpr (kTab)
    for (int i = tid; i < 64; i += kThreads) etab[i] = kExp2Frac64[i];
  const int tau = blockIdx.x;
  const int r0 = blockIdx.y * RC;
  int tb[3] = {tau % B, (tau / B) % B, d == 3 ? tau / (B * B) : 0};
  const double org[3] = {cheb[(0 * B + tb[0]) * p], cheb[(1 * B + tb[1]) * p],
                         d == 3 ? cheb[(2 * B + tb[2]) * p] : 0.0};
  constexpr int TPT = 8;
  T acc[TPT][RC];
  T xt[TPT][3];
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    int t = tid + q * kThreads;
    int tt[3] = {t % p, (t / p) % p, (d == 3) ? t / (p * p) : 0};
    for (int l = 0; l < 3; ++l) xt[q][l] = (l < d && t < P) ? (T)(cheb[(l * B + tb[l]) * p + tt[l]] - org[l]) : T(0);
#pragma unroll
    for (int r = 0; r < RC; ++r) acc[q][r] = T(0);
  }
  for (int64_t e = ptr[tau]; e < ptr[tau + 1]; ++e) {
    const int64_t sg = src[e];
    const int sb[3] = {(int)(sg % B), (int)((sg / B) % B), d == 3 ? (int)(sg / (B * B)) : 0};
    __syncthreads();
    for (int idx = tid; idx < RC * P; idx += kThreads) {
      int r = idx / P, s = idx % P;
      ws[idx] = (r0 + r < nrhs) ? W[(sg * nrhs + r0 + r) * P + s] : T(0);
    }
    for (int idx = tid; idx < 3 * p; idx += kThreads) {
      int l = idx / p, s = idx % p;
      ce[idx] = l < d ? (T)(cheb[(l * B + sb[l]) * p + s] - org[l]) : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < TPT; ++q) {
      int t = tid + q * kThreads;
      if (t >= P) break;
      int s = 0;
      const int nz = (d == 3) ? p : 1;
      for (int s2 = 0; s2 < nz; ++s2) {
        T dx2 = (d == 3) ? xt[q][2] - ce[2 * p + s2] : T(0);
        for (int s1 = 0; s1 < p; ++s1) {
          T dx1 = xt[q][1] - ce[p + s1];
          const T c12 = dx1 * dx1 + dx2 * dx2;
          for (int s0 = 0; s0 < p; ++s0, ++s) {
            T g = kvec_c12_t<KID, T>(xt[q][0] - ce[s0], dx1, dx2, c12, d, pm1, etab);
#pragma unroll
            for (int r = 0; r < RC; ++r) acc[q][r] += g * ws[r * P + s];
          }
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    int t = tid + q * kThreads;
    if (t >= P) break;
#pragma unroll
    for (int r = 0; r < RC; ++r)
      if (r0 + r < nrhs) H[((int64_t)tau * nrhs + r0 + r) * P + t] = acc[q][r];
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

#define HTLR_DISPATCH_RC(rc, ...)                                   \
  switch (rc) {                                                     \
    case 1: { constexpr int RC = 1; __VA_ARGS__; break; }           \
    case 4: { constexpr int RC = 4; __VA_ARGS__; break; }           \
    default: { constexpr int RC = 16; __VA_ARGS__; break; }         \
  }

constexpr size_t kLdsBudget = 64 * 1024;

// Right-hand sides per block (1, 4 or 16): enough for nrhs, within the LDS budget.
static int pick_rc(int nrhs, size_t fixed_bytes, size_t per_rc_bytes) {
  int rc = nrhs <= 1 ? 1 : (nrhs <= 4 ? 4 : 16);
  while (rc > 1 && fixed_bytes + rc * per_rc_bytes > kLdsBudget) rc = rc == 16 ? 4 : 1;
  if (fixed_bytes + rc * per_rc_bytes > kLdsBudget) fail(HTLR_ERR_UNSUPPORTED, "working set exceeds LDS");
  return rc;
}

// ---------------------------------------------------------------------------
// Work buffers


// Chunks of the up contraction and down expansion of a level: levels with
// few, large boxes spread each box over several blocks (at least 4 slices
// each), aiming at about 512 blocks.
static int chunk_target(const LevelData& lv, int d) {
  // 2D boxes of 128 points per side and more: about 2048 blocks (each block
  // stages row chunks, and a level of such boxes has few of them)
  return (d == 2 && lv.m >= 128) ? 2048 : 512;
}

static int level_chunks(const LevelData& lv, int nrhs, int d) {
  const int64_t base = lv.nbox * (int64_t)nrhs;
  const int target = chunk_target(lv, d);
  if (lv.m < 16 || base >= (target == 512 ? 256 : target)) return 1;
  return (int)std::max<int64_t>(1, std::min<int64_t>(lv.m / 4, (target + base - 1) / base));
}

// Elements of a level's partial up-contraction buffer, enough for every
// right-hand-side count up to nrhs (chunks x boxes x rhs <= target + boxes x rhs).
static size_t up_part_elems(const LevelData& lv, int nrhs, int P, int d) {
  if (level_chunks(lv, 1, d) <= 1) return 0;
  return (size_t)(chunk_target(lv, d) + lv.nbox * (int64_t)nrhs) * P;
}

size_t workspace_bytes(const htlr_matrix_impl& A, int nrhs, int prec) {
  (void)prec;
  size_t tot = 0;
  for (const LevelData& lv : A.levels) {
    if (lv.npairs == 0) continue;
    size_t cnt = (size_t)lv.nbox * nrhs * lv.P;
    tot += 2 * ((cnt * sizeof(double) + 255) & ~size_t(255));
    tot += up_part_elems(lv, nrhs, lv.P, A.d) * sizeof(double);
  }
  return tot;
}

// Work buffers are sized for 8-byte elements so that products of every
// precision share them; they are reallocated only when nrhs grows.
void ensure_workspace(htlr_matrix_impl& A, int nrhs, int prec) {
  (void)prec;
  Workspace& ws = A.ws;
  if (ws.nrhs >= nrhs) return;
  if (ws.frozen) fail(HTLR_ERR_INVALID, "nrhs exceeds the reserved work buffers");
  ws.W.clear();
  ws.H.clear();
  ws.UP.clear();
  ws.W.resize(A.L + 1);
  ws.H.resize(A.L + 1);
  ws.UP.resize(A.L + 1);
  ws.bytes = 0;
  for (const LevelData& lv : A.levels) {
    if (lv.npairs == 0) continue;
    size_t cnt = (size_t)lv.nbox * nrhs * lv.P;
    ws.W[lv.level].alloc(cnt * sizeof(double));
    ws.H[lv.level].alloc(cnt * sizeof(double));
    ws.UP[lv.level].alloc(up_part_elems(lv, nrhs, lv.P, A.d) * sizeof(double));
    ws.bytes += ws.W[lv.level].bytes + ws.H[lv.level].bytes + ws.UP[lv.level].bytes;
  }
  ws.zero.alloc((size_t)A.P * sizeof(double));
  HTLR_HIP(hipMemset(ws.zero.ptr, 0, ws.zero.bytes));
  ws.bytes += ws.zero.bytes;
  ws.nrhs = nrhs;
}

// ---------------------------------------------------------------------------
// Driver

const std::vector<hipStream_t>& side_streams(htlr_matrix_impl& A) {
  constexpr int kSideStreams = 4;
  if (A.side.empty()) {
    for (int i = 0; i < kSideStreams; ++i) {
      hipStream_t s = nullptr;
      HTLR_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      A.side.push_back(s);
    }
  }
  if (!A.ev_fork) {
    HTLR_HIP(hipEventCreateWithFlags(&A.ev_fork, hipEventDisableTiming));
    for (hipEvent_t& e : A.ev_level) HTLR_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  return A.side;
}

TuneParams find_tune(const htlr_matrix_impl& A, int nrhs, int prec) {
  auto it = A.tune.find({nrhs, prec});
  if (it != A.tune.end()) return it->second;
  TuneParams best;
  int bw = 0;
  for (auto& kv : A.tune)
    if (kv.first.second == prec && kv.first.first < nrhs && kv.first.first > bw) {
      bw = kv.first.first;
      best = kv.second;
    }
  return best;
}

// Kernel of a level's up contraction (and, with the same rule, of its down
// expansion) for a product with nrhs right-hand sides.
enum UpKind { kUpGeneric = 0, kUpSmall3d = 1, kUpBox2d = 2, kUpRows2d = 3 };

static int up_kind(const htlr_matrix_impl& A, const LevelData& lv, int nrhs, size_t tsize) {
  const int d = A.d, lm = lv.m, p = lv.rank;
  const int nch = level_chunks(lv, nrhs, d);
  if (d == 2 && nch == 1 && lm <= 64) return kUpBox2d;
  const size_t per3 = (size_t)lm * lm * lm + (size_t)lm * lm * p + (size_t)lm * p * p;
  if (d == 3 && nch == 1 && lm <= 16 && per3 * tsize <= kLdsBudget) return kUpSmall3d;
  if (d == 2 && lm >= 128) return kUpRows2d;
  return kUpGeneric;
}

static int down_kind(const htlr_matrix_impl& A, const LevelData& lv, int nrhs, size_t tsize) {
  const int d = A.d, lm = lv.m, p = lv.rank, P = lv.P;
  const int nch = level_chunks(lv, nrhs, d);
  const size_t per3d = (size_t)P + (size_t)lm * p * p + (size_t)lm * lm * p;
  if (d == 3 && nch == 1 && lm <= 16 && per3d * tsize <= kLdsBudget) return kUpSmall3d;
  if (d == 2 && nch == 1 && lm <= 64) return kUpBox2d;
  if (d == 2 && lm >= 128 && lm <= 256) return kUpRows2d;
  return kUpGeneric;
}

// Whether a level's up contraction and down expansion can run as one launch
// over several matrices with a column table (the one-pass box kernels).
static bool groupable_kind(int k) { return k == kUpSmall3d || k == kUpBox2d; }

// Up contraction of one level: W = (|Omega| o u) x_l V_l^T (Alg. 4.2).  With
// tab (device column table, nrhs = the launch's columns) each column's W goes
// to the buffer of the matrix that owns it.
template <typename T, typename TW>
static void launch_up(htlr_matrix_impl& A, LevelData& lv, const T* u, TW* W, T* upart, int nrhs, hipStream_t ls,
                      const ColTab* tab) {
  const int d = A.d, p = lv.rank, P = lv.P, n = A.n;
  const int lm = lv.m, lB = lv.B;
  const bool f64 = std::is_same<T, double>::value;
  const T* V = f64 ? (const T*)lv.V64.ptr : (const T*)lv.V32.ptr;
  const int uni = A.uniform ? 1 : 0;
  const int kind = up_kind(A, lv, nrhs, sizeof(T));
  if (tab && !groupable_kind(kind)) fail(HTLR_ERR_INVALID, "grouped up contraction of a level without box kernels");
  // 3D: rows of a slice staged at a time, as many as the LDS budget allows
  const int up_rows = d == 3 ? (int)std::max<int64_t>(1, std::min<int64_t>(lm, ((int64_t)(kLdsBudget / sizeof(T)) -
                                                       (int64_t)p * lm - (int64_t)p * p) / lm)) : 0;
  const size_t sh_up = (d == 3 ? (size_t)up_rows * lm + (size_t)p * lm + (size_t)p * p
                               : (size_t)lm + (size_t)kThreads + (size_t)p) * sizeof(T);
  if (sh_up > kLdsBudget) fail(HTLR_ERR_UNSUPPORTED, "box too large for the up contraction");
  const int nch = level_chunks(lv, nrhs, d), rpc = (lm + nch - 1) / nch;
  T* part = nch > 1 ? upart : nullptr;
  const int64_t wcount = lv.nbox * (int64_t)nrhs * P;
  if (kind == kUpSmall3d) {
    // 3D boxes up to 16 points per side whose stages fit in LDS: whole
    // boxes, several per block when small
    const size_t per3 = (size_t)lm * lm * lm + (size_t)lm * lm * p + (size_t)lm * p * p;
    const int S = std::max(std::max(lm * lm * lm, lm * lm * p), std::max(lm * p * p, p * p * p));
    int nb3 = std::max(1, kThreads / S);
    while (nb3 > 1 && nb3 * per3 * sizeof(T) > kLdsBudget) --nb3;
    const unsigned g3 = (unsigned)((lv.nbox + nb3 - 1) / nb3);
    if (tab)
      hipLaunchKernelGGL((k_up3d_small<T, TW, true>), dim3(g3, nrhs), dim3(kThreads), nb3 * per3 * sizeof(T), ls, u, W,
                         V, uni, n, lm, lB, p, nrhs, nb3, (int64_t)lv.nbox, tab);
    else
      hipLaunchKernelGGL((k_up3d_small<T, TW>), dim3(g3, nrhs), dim3(kThreads), nb3 * per3 * sizeof(T), ls, u, W, V,
                         uni, n, lm, lB, p, nrhs, nb3, (int64_t)lv.nbox, (const ColTab*)nullptr);
  } else if (kind == kUpBox2d) {
    // 2D boxes up to 64 points per side: one block contracts the whole box
    const size_t sh_box = ((size_t)lm * lm + (size_t)lm * p) * sizeof(T);
    if (tab)
      hipLaunchKernelGGL((k_up2d_box<T, TW, true>), dim3(lv.nbox, nrhs), dim3(kThreads), sh_box, ls, u, W, V, uni, n,
                         lm, lB, p, nrhs, tab);
    else
      hipLaunchKernelGGL((k_up2d_box<T, TW>), dim3(lv.nbox, nrhs), dim3(kThreads), sh_box, ls, u, W, V, uni, n, lm,
                         lB, p, nrhs, (const ColTab*)nullptr);
  } else if (kind == kUpRows2d) {
    // larger 2D boxes: staged rows with each dot split over the block
    const int Rr = std::max(1, std::min(std::min(rpc, 4096 / lm), kThreads / p));
    const size_t sh_rows = ((size_t)Rr * lm + (size_t)kThreads + (size_t)Rr * p) * sizeof(T);
    hipLaunchKernelGGL((k_up2d_rows<T, TW>), dim3(lv.nbox, nrhs, nch), dim3(kThreads), sh_rows, ls, u, W, V, uni, n,
                       lm, lB, p, nrhs, rpc, Rr, part);
  } else {
    hipLaunchKernelGGL((k_up<T, TW>), dim3(lv.nbox, nrhs, nch), dim3(kThreads), sh_up, ls, u, W, V, uni, d, n, lm, lB,
                       p, nrhs, rpc, part, up_rows);
  }
  if (nch > 1 && kind != kUpSmall3d && kind != kUpBox2d)
    hipLaunchKernelGGL((k_up_reduce<T, TW>), dim3((unsigned)std::min<int64_t>((wcount + 255) / 256, 4096)), dim3(256), 0,
                       ls, (const T*)part, W, wcount, nch);
  HTLR_HIP(hipGetLastError());
}

// Core apply of one level: H_tau = sum_sigma G_{tau sigma} W_sigma (Alg. 4.2).
template <typename T>
static void launch_core(htlr_matrix_impl& A, LevelData& lv, const void* W, T* H, const void* zero, int nrhs, int prec,
                        hipStream_t ls, bool noalloc) {
  const int d = A.d, p = lv.rank, P = lv.P, pm1 = A.p - 1;
  const int lB = lv.B;
  const bool f64 = std::is_same<T, double>::value;
  if (prec == HTLR_BF16_CORE) {
    if constexpr (!std::is_same<T, double>::value) {
      if (!A.uniform) fail(HTLR_ERR_UNSUPPORTED, "bfloat16 cores need a uniform grid");
      if (!lv.Gm16.ptr) fail(HTLR_ERR_UNSUPPORTED, "matrix built without bfloat16 cores");
      if (!noalloc && core_mfma_ok(A, lv, prec)) {
        launch_core_mfma(A, lv, prec, W, H, zero, nrhs, ls);
      } else {
        const int rc = pick_rc(nrhs, 0, (size_t)P * sizeof(float));
        const int nchunk = (nrhs + rc - 1) / rc;
        size_t sh = (size_t)rc * P * sizeof(float);
        HTLR_DISPATCH_RC(rc, hipLaunchKernelGGL((k_core_simple<uint16_t, uint16_t, float, RC, false>),
                                                dim3(lv.nbox, nchunk), dim3(kThreads), sh, ls, (const uint16_t*)W, H,
                                                lv.Gm16.as<uint16_t>(), lv.ptr.as<int64_t>(), lv.src.as<int32_t>(),
                                                lv.cid.as<int32_t>(), P, nrhs));
      }
    }
  } else if (A.uniform && !noalloc && core_mfma_ok(A, lv, prec)) {
    launch_core_mfma(A, lv, prec, W, H, zero, nrhs, ls);
  } else if (A.uniform) {
    const T* G = f64 ? (const T*)lv.Gm64.ptr : (const T*)lv.Gm32.ptr;
    if (!G) fail(HTLR_ERR_UNSUPPORTED, "matrix built without cores for this precision");
    const int rc = pick_rc(nrhs, 0, (size_t)P * sizeof(T));
    const int nchunk = (nrhs + rc - 1) / rc;
    size_t sh = (size_t)rc * P * sizeof(T);
    HTLR_DISPATCH_RC(rc, hipLaunchKernelGGL((k_core_simple<T, T, T, RC, false>), dim3(lv.nbox, nchunk), dim3(kThreads),
                                            sh, ls, (const T*)W, H, G, lv.ptr.as<int64_t>(), lv.src.as<int32_t>(),
                                            lv.cid.as<int32_t>(), P, nrhs));
  } else {
    const size_t tab = f64 ? kExpTabBytes : 0;   // reserved for the double-precision exponential kernels
    const int rc = pick_rc(nrhs, 3 * (size_t)p * sizeof(T) + tab, (size_t)P * sizeof(T));
    const int nchunk = (nrhs + rc - 1) / rc;
    size_t sh = ((size_t)rc * P + 3 * (size_t)p) * sizeof(T) + tab;
    HTLR_DISPATCH_KID(A.kid, HTLR_DISPATCH_RC(rc, hipLaunchKernelGGL((k_core_tensor<KID, T, RC>), dim3(lv.nbox, nchunk),
                                                                   dim3(kThreads), sh, ls, (const T*)W, H,
                                                                   lv.cheb64.as<double>(), lv.ptr.as<int64_t>(),
                                                                   lv.src.as<int32_t>(), d, p, lB, nrhs, pm1)));
  }
  HTLR_HIP(hipGetLastError());
}

// Near field and diagonal term (overwrites f): inadmissible leaves evaluated
// on the fly (eq. 4.1).
template <typename T>
static void launch_near(htlr_matrix_impl& A, const T* u, T* f, int nrhs, int prec, hipStream_t st, bool noalloc) {
  const int d = A.d, n = A.n, pm1 = A.p - 1;
  const bool f64 = std::is_same<T, double>::value;
  const Plan& pl = A.plan;
  const int m = pl.m[A.L], B = pl.B[A.L];
  const int M = d == 3 ? m * m * m : m * m;
  const T* a = f64 ? (const T*)A.a64.ptr : (const T*)A.a32.ptr;
  const int64_t nleaf = A.levels[A.L].nbox;
  const bool mfma_ok = A.uniform && d == 3 && m == 8 && A.kid != HTLR_K_POLY_TEST &&
                       (((size_t)A.Tsize + 3) & ~size_t(3)) * sizeof(T) + (size_t)256 * 16 * sizeof(T) <= kLdsBudget;
  // two or more right-hand sides: the near field as class tiles of the core
  // apply.  Measured at 128^3 (FP64): 16 RHS 59.4 -> 49.9 ms against the
  // table kernel; 12 RHS 59.9 -> 55.4; 8 RHS 32.5 -> 29.4, 4 RHS 16.7 ->
  // 15.9, 2 RHS 8.3 -> 7.9 against the automatic choice before it.  One
  // right-hand side keeps the leaf-column kernel (a tile would span 128 leaves).
  if (!noalloc && near_tiles_ok(A, nrhs) && (A.cur.near_kind == 4 || (A.cur.near_kind < 0 && nrhs >= 2))) {
    launch_near_tiles<T>(A, u, f, nrhs, st);
    return;
  }
  const bool near_leaves = !noalloc && use_near_leaves(A, nrhs, prec, A.ws.frozen);
  const bool near_mfma = !near_leaves && mfma_ok &&
                         (A.cur.near_kind == 1 || A.cur.near_kind == 2 || (A.cur.near_kind < 0 && nrhs >= 8));
  if (near_leaves) {
    launch_near_leaves<T>(A, u, f, nrhs, prec, st);
  } else if (near_mfma) {
    const size_t sh = (((size_t)A.Tsize + 3) & ~size_t(3)) * sizeof(T) + (size_t)256 * 16 * sizeof(T);
    const T* tab = f64 ? (const T*)A.T64.ptr : (const T*)A.T32.ptr;
    hipLaunchKernelGGL((k_near_mfma<T>), dim3(nleaf, (nrhs + 15) / 16), dim3(256), sh, st, u, f, a,
                       A.near_ptr.as<int64_t>(), A.near_src.as<int32_t>(), tab, A.Tsize, n, B, nrhs);
  } else if (A.uniform && d == 3 && A.cur.near_kind != 3 && near_rows3d_ok(A, nrhs, prec)) {
    launch_near_rows3d<T>(A, u, f, nrhs, st);
  } else if (A.uniform && d == 3 && m <= 8) {
    const bool radial = A.kid != HTLR_K_POLY_TEST;
    const T* tab = radial ? (f64 ? (const T*)A.T64.ptr : (const T*)A.T32.ptr) : nullptr;
    const size_t fixed = (radial ? ((A.Tsize + 1) & ~1) : 0) * sizeof(T);
    int rc = f64 ? (nrhs <= 1 ? 1 : (nrhs <= 2 ? 2 : 4)) : (nrhs <= 1 ? 1 : (nrhs <= 2 ? 2 : (nrhs <= 4 ? 4 : 8)));
    const size_t per_wave = (size_t)8 * 64 * sizeof(T);   // [MM*64] x rc
    while (rc > 1 && fixed + per_wave * rc > kLdsBudget) rc /= 2;
    const int nchunk = (nrhs + rc - 1) / rc;
    // waves per leaf: enough waves to fill the GPU, within the LDS budget
    // (8 waves per leaf cap registers at 128 per lane: only for the narrow chunks)
    const int nwmax = (f64 ? rc >= 2 : rc >= 4) ? 4 : 8;
    int nw = 1;
    if (A.cur.near_nw > 0) {
      while (nw < A.cur.near_nw && nw < nwmax && fixed + per_wave * rc * nw * 2 <= kLdsBudget) nw *= 2;
    } else {
      while (nw < nwmax && (int64_t)nleaf * nchunk * nw < 8192 && fixed + per_wave * rc * nw * 2 <= kLdsBudget) nw *= 2;
    }
    const bool full = m == 8;
    const size_t sh = fixed + per_wave * rc * nw;
    if (sh > kLdsBudget) fail(HTLR_ERR_UNSUPPORTED, "near-field working set exceeds LDS");
#define HTLR_NEAR_ROWS3(RCV, NWV, FV)                                                                              \
  HTLR_DISPATCH_KID(A.kid, hipLaunchKernelGGL((k_near_rows<KID, T, RCV, NWV, FV>), dim3(nleaf, nchunk), dim3(64 * NWV),  \
                                              sh, st, u, f, a, A.near_ptr.as<int64_t>(), A.near_src.as<int32_t>(), tab, \
                                              A.Tsize, n, m, B, nrhs, (T)A.h, (T)A.w0, (T)A.D0, pm1))
#define HTLR_NEAR_ROWS(RCV, NWV)                                   \
  if (full) { HTLR_NEAR_ROWS3(RCV, NWV, true); } else { HTLR_NEAR_ROWS3(RCV, NWV, false); }
#define HTLR_NEAR_NW(RCV)                                  \
  switch (nw) {                                            \
    case 1: HTLR_NEAR_ROWS(RCV, 1); break;                 \
    case 2: HTLR_NEAR_ROWS(RCV, 2); break;                 \
    case 4: HTLR_NEAR_ROWS(RCV, 4); break;                 \
    default: HTLR_NEAR_ROWS(RCV, 8); break;                \
  }
#define HTLR_NEAR_NW4(RCV)                                 \
  switch (nw) {                                            \
    case 1: HTLR_NEAR_ROWS(RCV, 1); break;                 \
    case 2: HTLR_NEAR_ROWS(RCV, 2); break;                 \
    default: HTLR_NEAR_ROWS(RCV, 4); break;                \
  }
    switch (rc) {
      case 1: HTLR_NEAR_NW(1); break;
      case 2:
        if constexpr (std::is_same<T, double>::value) { HTLR_NEAR_NW4(2); }
        else { HTLR_NEAR_NW(2); }
        break;
      case 4: HTLR_NEAR_NW4(4); break;
      default:
        if constexpr (!std::is_same<T, double>::value) { HTLR_NEAR_NW4(8); }
        else fail(HTLR_ERR_INVALID, "near-field chunk size");
        break;
    }
#undef HTLR_NEAR_NW4
#undef HTLR_NEAR_NW
#undef HTLR_NEAR_ROWS
#undef HTLR_NEAR_ROWS3
  } else if (A.uniform && d == 2 && A.cur.near_kind != 3 && near_rows2d_ok(A, nrhs, prec)) {
    launch_near_rows2d<T>(A, u, f, nrhs, st);
  } else if (A.uniform) {
    const bool radial = A.kid != HTLR_K_POLY_TEST;
    const T* tab = radial ? (f64 ? (const T*)A.T64.ptr : (const T*)A.T32.ptr) : nullptr;
    const size_t fixed = (radial ? ((A.Tsize + 1) & ~1) : 0) * sizeof(T);
    const int rc = pick_rc(nrhs, fixed, (size_t)M * sizeof(T));
    const int nchunk = (nrhs + rc - 1) / rc;
    size_t sh = fixed + (size_t)M * rc * sizeof(T);
    HTLR_DISPATCH_KID(A.kid, HTLR_DISPATCH_RC(rc, hipLaunchKernelGGL((k_near_uniform<KID, T, RC>), dim3(nleaf, nchunk),
                                                                   dim3(kThreads), sh, st, u, f, a,
                                                                   A.near_ptr.as<int64_t>(), A.near_src.as<int32_t>(),
                                                                   tab, A.Tsize, d, n, m, B, nrhs, (T)A.h, (T)A.w0,
                                                                   (T)A.D0, pm1)));
  } else {
    const T* D = f64 ? (const T*)A.D64.ptr : (const T*)A.D32.ptr;
    const T* wd = f64 ? (const T*)A.w64.ptr : (const T*)A.w32.ptr;
    const size_t tab = f64 ? kExpTabBytes : 0;   // reserved for the double-precision exponential kernels
    const int rc = pick_rc(nrhs, 3 * (size_t)m * sizeof(T) + tab, (size_t)M * sizeof(T));
    const int nchunk = (nrhs + rc - 1) / rc;
    size_t sh = (3 * (size_t)m + (size_t)M * rc) * sizeof(T) + tab;
    HTLR_DISPATCH_KID(A.kid, HTLR_DISPATCH_RC(rc, hipLaunchKernelGGL((k_near_tensor<KID, T, RC>), dim3(nleaf, nchunk),
                                                                   dim3(kThreads), sh, st, u, f, a, D,
                                                                   A.near_ptr.as<int64_t>(), A.near_src.as<int32_t>(),
                                                                   A.x64.as<double>(), wd, d, n, m, B, nrhs, pm1)));
  }
  HTLR_HIP(hipGetLastError());
}

// Down expansion of one level: f_tau += H_tau x_l U_l (Alg. 4.2).  With tab
// (device column table) each column's H comes from the buffer of the matrix
// that owns it.
template <typename T>
static void launch_down(htlr_matrix_impl& A, LevelData& lv, const T* H, T* f, int nrhs, hipStream_t st,
                        const ColTab* tab) {
  const int d = A.d, p = lv.rank, P = lv.P, n = A.n;
  const int lm = lv.m, lB = lv.B;
  const bool f64 = std::is_same<T, double>::value;
  const T* U = f64 ? (const T*)lv.U64.ptr : (const T*)lv.U32.ptr;
  const int uni = A.uniform ? 1 : 0;
  const size_t sh_dn = ((size_t)P + (d == 3 ? (size_t)p * p + (size_t)lm * p : (size_t)p)) * sizeof(T);
  if (sh_dn > kLdsBudget) fail(HTLR_ERR_UNSUPPORTED, "core too large for the down expansion");
  const int nch = level_chunks(lv, nrhs, d), rpc = (lm + nch - 1) / nch;
  const int kind = down_kind(A, lv, nrhs, sizeof(T));
  if (tab && !groupable_kind(kind)) fail(HTLR_ERR_INVALID, "grouped down expansion of a level without box kernels");
  // 2D: whole boxes up to 64 points per side, staged row chunks at 128 and
  // 256 points (measured faster than the row kernel there), the row kernel
  // for larger boxes
  if (kind == kUpSmall3d) {
    const size_t per3 = (size_t)P + (size_t)lm * p * p + (size_t)lm * lm * p;
    const int S = std::max(std::max(lm * lm * lm, lm * lm * p), std::max(lm * p * p, P));
    int nb3 = std::max(1, kThreads / S);
    while (nb3 > 1 && nb3 * per3 * sizeof(T) > kLdsBudget) --nb3;
    const dim3 grid((unsigned)((lv.nbox + nb3 - 1) / nb3), nrhs);
    if (tab)
      hipLaunchKernelGGL((k_down3d_small<T, true>), grid, dim3(kThreads), nb3 * per3 * sizeof(T), st, H, f, U, uni, n,
                         lm, lB, p, nrhs, nb3, (int64_t)lv.nbox, tab);
    else
      hipLaunchKernelGGL((k_down3d_small<T>), grid, dim3(kThreads), nb3 * per3 * sizeof(T), st, H, f, U, uni, n, lm,
                         lB, p, nrhs, nb3, (int64_t)lv.nbox, (const ColTab*)nullptr);
  } else if (kind == kUpBox2d) {
    const size_t sh = ((size_t)p * p + (size_t)lm * p) * sizeof(T);
    if (tab)
      hipLaunchKernelGGL((k_down2d_box<T, true>), dim3(lv.nbox, nrhs), dim3(kThreads), sh, st, H, f, U, uni, n, lm, lB,
                         p, nrhs, tab);
    else
      hipLaunchKernelGGL((k_down2d_box<T>), dim3(lv.nbox, nrhs), dim3(kThreads), sh, st, H, f, U, uni, n, lm, lB, p,
                         nrhs, (const ColTab*)nullptr);
  } else if (kind == kUpRows2d) {
    const int R2 = std::max(1, std::min(rpc, 4096 / lm));
    hipLaunchKernelGGL((k_down2d<T>), dim3(lv.nbox, nrhs, nch), dim3(kThreads),
                       ((size_t)p * p + (size_t)R2 * p) * sizeof(T), st, H, f, U, uni, n, lm, lB, p, nrhs, rpc, R2);
  } else {
    hipLaunchKernelGGL((k_down<T>), dim3(lv.nbox, nrhs, nch), dim3(kThreads), sh_dn, st, H, f, U, uni, d, n, lm, lB, p,
                       nrhs, rpc);
  }
  HTLR_HIP(hipGetLastError());
}

template <typename T>
static void check_shape(const htlr_matrix_impl& A) {
  const int d = A.d, m = A.plan.m[A.L];
  const int M = d == 3 ? m * m * m : m * m;
  if (M > 4 * kThreads) fail(HTLR_ERR_UNSUPPORTED, "leaf boxes larger than 1024 points");
  if (A.P > 8 * kThreads) fail(HTLR_ERR_UNSUPPORTED, "p^d larger than 2048");
}

// Whether the levels' launches are issued on the caller's stream one after
// another rather than concurrently on side streams.  Concurrency fills the
// chip when launches are small; when one level's core apply is many
// milliseconds of matrix-core work it fills the chip by itself, and running
// the other levels beside it only spoils its tail.  Measured at 128^3 x 16
// right-hand sides (level 4, 1.7e13 flop): serial is 3% faster in FP64 and
// 2% in FP32; in bfloat16, where the core apply is bound by memory traffic
// and the near field by the FP32 matrix rate, concurrency is 3% faster.
static bool levels_serial(const htlr_matrix_impl& A, int serial, int nrhs, int prec) {
  if (serial == 1) return true;
  if (serial == 2) return false;
  if (!A.uniform || prec == HTLR_BF16_CORE) return false;
  double fl = 0;
  for (const LevelData& lv : A.levels)
    if (lv.npairs > 0) fl = std::max(fl, 2.0 * (double)lv.npairs * lv.P * lv.P * nrhs);
  const double peak = prec == HTLR_FP64 ? 78.6e12 : 157.3e12;   // dense matrix-core flop/s
  return fl / peak > 20e-3;
}

template <typename T>
static void run_matvec(htlr_matrix_impl& A, const T* u, T* f, int nrhs, int prec, hipStream_t st,
                       const WorkView& wv) {
  A.cur = wv.noalloc ? TuneParams{} : find_tune(A, nrhs, prec);
  const bool prof = !wv.noalloc;
  check_shape<T>(A);
  // far field.  Each level's up and core launches run on a side stream,
  // concurrently with the near field and with the other levels; the down
  // expansions then add into f on the caller's stream in level order, so the
  // summation order is fixed.
  std::vector<LevelData*> act;
  for (LevelData& lv : A.levels)
    if (lv.npairs > 0) act.push_back(&lv);
  // (serial while profiling: each recorded duration is then one launch's alone)
  const bool fork = !wv.noalloc && !levels_serial(A, A.cur.serial, nrhs, prec) && !A.prof.on && !act.empty();
  const std::vector<hipStream_t>* side = fork ? &side_streams(A) : nullptr;
  if (fork) {
    HTLR_HIP(hipEventRecord(A.ev_fork, st));
    for (size_t i = 0; i < act.size() && i < side->size(); ++i)
      HTLR_HIP(hipStreamWaitEvent((*side)[i], A.ev_fork, 0));
  }
  for (size_t li = 0; li < act.size(); ++li) {
    LevelData& lv = *act[li];
    const hipStream_t ls = fork ? (*side)[li % side->size()] : st;
    const int l = lv.level;
    T* H = (T*)wv.H[l];
    {
      ProfScope ps(A, "up", l, ls, prof);
      if (prec == HTLR_BF16_CORE) {
        if constexpr (!std::is_same<T, double>::value)
          launch_up<float, uint16_t>(A, lv, u, (uint16_t*)wv.W[l], (float*)wv.UP[l], nrhs, ls, nullptr);
      } else {
        launch_up<T, T>(A, lv, u, (T*)wv.W[l], (T*)wv.UP[l], nrhs, ls, nullptr);
      }
    }
    {
      ProfScope ps(A, "core", l, ls, prof);
      launch_core<T>(A, lv, wv.W[l], H, wv.zero, nrhs, prec, ls, wv.noalloc);
    }
    if (fork) HTLR_HIP(hipEventRecord(A.ev_level[li], ls));
  }
  {
    ProfScope ps(A, "near", -1, st, prof);
    launch_near<T>(A, u, f, nrhs, prec, st, wv.noalloc);
  }
  for (size_t li = 0; li < act.size(); ++li) {
    LevelData& lv = *act[li];
    if (fork) HTLR_HIP(hipStreamWaitEvent(st, A.ev_level[li], 0));
    ProfScope ps(A, "down", lv.level, st, prof);
    launch_down<T>(A, lv, (const T*)wv.H[lv.level], f, nrhs, st, nullptr);
  }
}

void product_view(htlr_matrix_impl& A, const void* u, void* f, int nrhs, int prec, hipStream_t st,
                  const WorkView& wv) {
  if (prec == HTLR_FP64) run_matvec<double>(A, (const double*)u, (double*)f, nrhs, prec, st, wv);
  else run_matvec<float>(A, (const float*)u, (float*)f, nrhs, prec, st, wv);
}

void product(htlr_matrix_impl& A, const void* u, void* f, int nrhs, int prec, hipStream_t st) {
  ensure_workspace(A, nrhs, prec);
  WorkView wv;
  for (const LevelData& lv : A.levels) {
    if (lv.npairs == 0) continue;
    wv.W[lv.level] = A.ws.W[lv.level].ptr;
    wv.H[lv.level] = A.ws.H[lv.level].ptr;
    wv.UP[lv.level] = A.ws.UP[lv.level].ptr;
  }
  wv.zero = A.ws.zero.ptr;
  product_view(A, u, f, nrhs, prec, st, wv);
}

// Grouped product over matrices that share their factors (see
// product_group in htlr_handle.h).
template <typename T>
static int run_group(const std::vector<htlr_matrix_impl*>& As, const std::vector<int>& cols, const T* u, T* f,
                      int prec, hipStream_t st, ColTab* th, ColTab* td) {
  const size_t G = As.size();
  htlr_matrix_impl& A0 = *As[0];
  std::vector<int> c0(G);
  int C = 0;
  for (size_t g = 0; g < G; ++g) {
    c0[g] = C;
    C += cols[g];
  }
  if (C < 1 || C > kMaxGroupCols) fail(HTLR_ERR_INVALID, "grouped product: columns out of range");
  const int64_t N = A0.N;
  for (size_t g = 0; g < G; ++g) {
    const htlr_matrix_impl& A = *As[g];
    if (A.d != A0.d || A.n != A0.n || A.leaf != A0.leaf || A.orth != A0.orth || !A.uniform ||
        A.quasi || A.levels.size() != A0.levels.size())
      fail(HTLR_ERR_INVALID, "grouped product: matrices do not share their factors");
    for (size_t l = 0; l < A.levels.size(); ++l)
      if ((A.levels[l].npairs > 0) != (A0.levels[l].npairs > 0) || A.levels[l].rank != A0.levels[l].rank)
        fail(HTLR_ERR_INVALID, "grouped product: matrices differ in their levels");
    check_shape<T>(A);
    ensure_workspace(*As[g], cols[g], prec);
  }
  using TW = typename std::conditional<std::is_same<T, double>::value, double, float>::type;
  const bool bf = prec == HTLR_BF16_CORE;
  const size_t tsz = sizeof(T);
  std::vector<int> lev;
  for (const LevelData& lv : A0.levels)
    if (lv.npairs > 0) lev.push_back(lv.level);
  // a level runs as one launch when every matrix's own product, and the
  // grouped launch, take the same one-pass box kernel
  int nt = 0;
  std::vector<int> up_tab(A0.levels.size(), -1), dn_tab(A0.levels.size(), -1);
  for (int l : lev) {
    const int ku = up_kind(A0, A0.levels[l], C, tsz), kd = down_kind(A0, A0.levels[l], C, tsz);
    bool fu = groupable_kind(ku) && G > 1, fd = groupable_kind(kd) && G > 1;
    for (size_t g = 0; g < G; ++g) {
      fu = fu && up_kind(*As[g], As[g]->levels[l], cols[g], tsz) == ku;
      fd = fd && down_kind(*As[g], As[g]->levels[l], cols[g], tsz) == kd;
    }
    auto fill = [&](ColTab& t, bool out_w) {
      for (size_t g = 0; g < G; ++g)
        for (int r = 0; r < cols[g]; ++r) {
          t.base[c0[g] + r] = out_w ? As[g]->ws.W[l].ptr : As[g]->ws.H[l].ptr;
          t.ld[c0[g] + r] = cols[g];
          t.rl[c0[g] + r] = r;
        }
    };
    if (fu) { up_tab[l] = nt; fill(th[nt++], true); }
    if (fd) { dn_tab[l] = nt; fill(th[nt++], false); }
  }
  if (nt > 2 * kMaxLevels) fail(HTLR_ERR_INVALID, "grouped product: too many column tables");
  if (nt) HTLR_HIP(hipMemcpyAsync(td, th, nt * sizeof(ColTab), hipMemcpyHostToDevice, st));
  // up contractions
  for (int l : lev) {
    if (up_tab[l] >= 0) {
      if (bf) {
        if constexpr (!std::is_same<T, double>::value)
          launch_up<float, uint16_t>(A0, A0.levels[l], u, (uint16_t*)nullptr, nullptr, C, st, td + up_tab[l]);
      } else {
        launch_up<T, TW>(A0, A0.levels[l], u, (TW*)nullptr, nullptr, C, st, td + up_tab[l]);
      }
      continue;
    }
    for (size_t g = 0; g < G; ++g) {
      htlr_matrix_impl& A = *As[g];
      const T* ug = u + (int64_t)c0[g] * N;
      if (bf) {
        if constexpr (!std::is_same<T, double>::value)
          launch_up<float, uint16_t>(A, A.levels[l], ug, (uint16_t*)A.ws.W[l].ptr, (float*)A.ws.UP[l].ptr, cols[g],
                                     st, nullptr);
      } else {
        launch_up<T, TW>(A, A.levels[l], ug, (TW*)A.ws.W[l].ptr, (T*)A.ws.UP[l].ptr, cols[g], st, nullptr);
      }
    }
  }
  // core applies and near fields, per matrix
  for (size_t g = 0; g < G; ++g) {
    htlr_matrix_impl& A = *As[g];
    A.cur = find_tune(A, cols[g], prec);
    for (int l : lev) launch_core<T>(A, A.levels[l], A.ws.W[l].ptr, (T*)A.ws.H[l].ptr, A.ws.zero.ptr, cols[g], prec, st,
                                     false);
    launch_near<T>(A, u + (int64_t)c0[g] * N, f + (int64_t)c0[g] * N, cols[g], prec, st, false);
  }
  // down expansions in level order
  for (int l : lev) {
    if (dn_tab[l] >= 0) {
      launch_down<T>(A0, A0.levels[l], nullptr, f, C, st, td + dn_tab[l]);
      continue;
    }
    for (size_t g = 0; g < G; ++g) {
      htlr_matrix_impl& A = *As[g];
      launch_down<T>(A, A.levels[l], (const T*)A.ws.H[l].ptr, f + (int64_t)c0[g] * N, cols[g], st, nullptr);
    }
  }
  return nt;
}

int product_group(const std::vector<htlr_matrix_impl*>& As, const std::vector<int>& cols, const void* u, void* f,
                  int prec, hipStream_t st, ColTab* tab_host, ColTab* tab_dev) {
  if (As.empty() || As.size() != cols.size()) fail(HTLR_ERR_INVALID, "grouped product: bad member list");
  std::vector<htlr_matrix_impl*> order(As.begin(), As.end());
  std::sort(order.begin(), order.end());
  if (std::adjacent_find(order.begin(), order.end()) != order.end())
    fail(HTLR_ERR_INVALID, "grouped product: a matrix appears twice");
  std::vector<std::unique_lock<std::mutex>> locks;
  for (htlr_matrix_impl* A : order) locks.emplace_back(A->ws_mu);
  if (prec == HTLR_FP64) return run_group<double>(As, cols, (const double*)u, (double*)f, prec, st, tab_host, tab_dev);
  return run_group<float>(As, cols, (const float*)u, (float*)f, prec, st, tab_host, tab_dev);
}

// Carves the work buffers of a product with nrhs right-hand sides out of
// one region (each 256-byte aligned, in level order: W, H, UP, then the
// zero tensor); returns the bytes used.  With base NULL only the size is
// computed.
size_t carve_workview(const htlr_matrix_impl& A, int nrhs, char* base, WorkView* wv) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* q = base ? (void*)(base + off) : nullptr;
    off += (bytes + 255) & ~size_t(255);
    return q;
  };
  for (const LevelData& lv : A.levels) {
    if (lv.npairs == 0) continue;
    const size_t cnt = (size_t)lv.nbox * nrhs * lv.P;
    void* W = take(cnt * sizeof(double));
    void* H = take(cnt * sizeof(double));
    const size_t up = up_part_elems(lv, nrhs, lv.P, A.d) * sizeof(double);
    void* UP = up ? take(up) : nullptr;
    if (wv) {
      wv->W[lv.level] = W;
      wv->H[lv.level] = H;
      wv->UP[lv.level] = UP;
    }
  }
  const void* z = take((size_t)A.P * sizeof(double));
  if (wv) wv->zero = z;
  return off;
}


}  // namespace htlr

using namespace htlr;

extern "C" {

htlr_status htlr_workspace_bytes(htlr_matrix A, int nrhs, htlr_precision prec, size_t* bytes) {
  if (!A || !bytes || nrhs < 1) { g_last_error = "invalid argument"; return HTLR_ERR_INVALID; }
  try {
    *bytes = A->quasi ? workspace_bytes(quasi_inner(*A), nrhs, prec) + quasi_buffer_bytes(*A, nrhs, prec)
                      : workspace_bytes(*A, nrhs, prec);
  } catch (const Error& e) {
    return record(e);
  }
  return HTLR_OK;
}

htlr_status htlr_matvec(htlr_matrix A, const void* u, void* f, int nrhs, htlr_precision prec,
                        htlr_vec_dtype vec_dtype, void* stream) {
  try {
    g_last_error.clear();
    if (!A || !u || !f) fail(HTLR_ERR_INVALID, "null argument");
    if (nrhs < 1 || nrhs > 64) fail(HTLR_ERR_INVALID, "nrhs out of range (1..64)");
    if (prec != HTLR_FP64 && prec != HTLR_FP32 && prec != HTLR_BF16_CORE) fail(HTLR_ERR_INVALID, "unknown precision");
    if ((prec == HTLR_FP64) != (vec_dtype == HTLR_VEC_F64))
      fail(HTLR_ERR_UNSUPPORTED, "FP64 products take f64 vectors, FP32/BF16 products take f32 vectors");
    if (!(A->precisions & (1 << prec))) fail(HTLR_ERR_UNSUPPORTED, "matrix built without this precision");
    const size_t esz = vec_dtype == HTLR_VEC_F64 ? 8 : 4;
    const char* ub = (const char*)u;
    const char* fb = (const char*)f;
    const size_t span = (size_t)A->N * nrhs * esz;
    if (ub < fb + span && fb < ub + span) fail(HTLR_ERR_INVALID, "u and f overlap");
    int dev = 0;
    HTLR_HIP(hipGetDevice(&dev));
    if (dev != A->device) fail(HTLR_ERR_INVALID, "current device differs from the build device");
    std::lock_guard<std::mutex> lk(A->ws_mu);
    hipStream_t st = (hipStream_t)stream;
    if (A->quasi) quasi_matvec(*A, u, f, nrhs, prec, st);
    else product(*A, u, f, nrhs, prec, st);
    return HTLR_OK;
  } catch (const Error& e) {
    return record(e);
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return HTLR_ERR_INVALID;
  }
}

htlr_status htlr_autotune(htlr_matrix A, int nrhs, htlr_precision prec, htlr_tune_result* out) {
  try {
    g_last_error.clear();
    if (!A) fail(HTLR_ERR_INVALID, "null handle");
    // quasi-uniform handles: the transfers have no variants; tune Ahat
    if (A->quasi) return htlr_autotune(static_cast<htlr_matrix_s*>(&quasi_inner(*A)), nrhs, prec, out);
    if (nrhs < 1 || nrhs > 64) fail(HTLR_ERR_INVALID, "nrhs out of range (1..64)");
    if (prec != HTLR_FP64 && prec != HTLR_FP32 && prec != HTLR_BF16_CORE) fail(HTLR_ERR_INVALID, "unknown precision");
    if (!(A->precisions & (1 << prec))) fail(HTLR_ERR_UNSUPPORTED, "matrix built without this precision");
    if (A->ws.frozen) fail(HTLR_ERR_INVALID, "tune before reserving work buffers");
    htlr_tune_result res{};
    // cache lookup
    char key[256];
    std::string ranks;                  // level ranks, when the QR step truncated any
    bool truncated = false;
    for (const LevelData& lv : A->levels)
      if (lv.npairs > 0) {
        ranks += (ranks.empty() ? "_r" : ".") + std::to_string(lv.rank);
        truncated = truncated || lv.rank != A->p;
      }
    if (!truncated) ranks.clear();
    std::snprintf(key, sizeof(key), "d%d_n%d_p%d_leaf%d_k%d_%s_eta%.6g_adm%d_nrhs%d_prec%d%s", A->d, A->n, A->p, A->leaf,
                  A->kid, A->uniform ? "uniform" : "tensor", A->eta2, A->adm_kind, nrhs, (int)prec, ranks.c_str());
    const char* cache = std::getenv("HTLR_TUNE_CACHE");
    if (cache && *cache) {
      FILE* fp = std::fopen(cache, "r");
      if (fp) {
        char k2[256], line[512];
        TuneParams t;
        double md = 0, mb = 0;
        bool found = false;
        // key ks_target near_kind near_nw tile core_mode near_ks near_tpw near_ct serial ms_default ms_best
        // [order] (lines without the last field take order 0)
        while (std::fgets(line, sizeof(line), fp)) {
          t.order = 0;
          const int got = std::sscanf(line, "%255s %d %d %d %d %d %d %d %d %d %lf %lf %d", k2, &t.ks_target,
                                      &t.near_kind, &t.near_nw, &t.tile, &t.core_mode, &t.near_ks, &t.near_tpw,
                                      &t.near_ct, &t.serial, &md, &mb, &t.order);
          if ((got == 12 || got == 13) && std::strcmp(k2, key) == 0) {
            A->tune[{nrhs, (int)prec}] = t;
            res = htlr_tune_result{t.ks_target, t.near_kind, t.near_nw, 0, md, mb};
            found = true;
          }
        }
        std::fclose(fp);
        if (found) {
          if (out) *out = res;
          return HTLR_OK;
        }
      }
    }
    const size_t esz = prec == HTLR_FP64 ? 8 : 4;
    const size_t bytes = (size_t)A->N * nrhs * esz;
    DevBuf u, f;
    u.alloc(bytes);
    f.alloc(bytes);
    {
      // deterministic pseudo-random input (values do not affect timing)
      std::vector<unsigned char> host(bytes);
      uint64_t x = 88172645463325252ull;
      if (esz == 8) {
        double* hp = reinterpret_cast<double*>(host.data());
        for (size_t i = 0; i < bytes / 8; ++i) { x ^= x << 13; x ^= x >> 7; x ^= x << 17; hp[i] = (double)(x >> 11) * 0x1.0p-53 - 0.5; }
      } else {
        float* hp = reinterpret_cast<float*>(host.data());
        for (size_t i = 0; i < bytes / 4; ++i) { x ^= x << 13; x ^= x >> 7; x ^= x << 17; hp[i] = (float)((double)(x >> 11) * 0x1.0p-53 - 0.5); }
      }
      HTLR_HIP(hipMemcpy(u.ptr, host.data(), bytes, hipMemcpyHostToDevice));
    }
    hipStream_t st = nullptr;
    hipEvent_t e0, e1;
    HTLR_HIP(hipEventCreate(&e0));
    HTLR_HIP(hipEventCreate(&e1));
    auto time_with = [&](const TuneParams& t) -> double {
      A->tune[{nrhs, (int)prec}] = t;
      std::lock_guard<std::mutex> lk(A->ws_mu);
      ensure_workspace(*A, nrhs, prec);
      auto once = [&]() { product(*A, u.ptr, f.ptr, nrhs, prec, st); };
      once();   // warm-up (work lists, buffers)
      float best = 1e30f;
      for (int r = 0; r < 3; ++r) {
        HTLR_HIP(hipEventRecord(e0, st));
        once();
        HTLR_HIP(hipEventRecord(e1, st));
        HTLR_HIP(hipEventSynchronize(e1));
        float ms = 0;
        HTLR_HIP(hipEventElapsedTime(&ms, e0, e1));
        best = std::min(best, ms);
      }
      ++res.candidates;
      return best;
    };
    TuneParams best;                    // defaults
    res.ms_default = time_with(best);
    double best_ms = res.ms_default;
    if (core_mfma_any(*A, prec)) {
      for (int mode : {1, 2}) {
        TuneParams t = best;
        t.core_mode = mode;
        const double ms = time_with(t);
        if (ms < best_ms) { best_ms = ms; best = t; }
      }
      for (int tile : {1, 2, 3, 4, 5, 6, 7}) {
        TuneParams t = best;
        t.tile = tile;
        const double ms = time_with(t);
        if (ms < best_ms) { best_ms = ms; best = t; }
      }
      for (int target : {512, 1024, 2048, 4096, 8192}) {
        TuneParams t = best;
        t.ks_target = target;
        const double ms = time_with(t);
        if (ms < best_ms) { best_ms = ms; best = t; }
      }
      {
        const TuneParams base = best;
        const int ord = base.order >= 0 ? base.order : (prec == HTLR_BF16_CORE ? 0 : 2);
        for (int o = 0; o <= 2; ++o) {
          if (o == ord) continue;
          TuneParams t = base;
          t.order = o;
          const double ms = time_with(t);
          if (ms < best_ms) { best_ms = ms; best = t; }
        }
      }
    }
    const bool near_rows = A->uniform && A->d == 3 && A->plan.m[A->L] <= 8;
    const size_t tsz = (prec == HTLR_FP64 ? 8 : 4);
    const bool near_mfma = A->uniform && A->d == 3 && A->plan.m[A->L] == 8 && A->kid != HTLR_K_POLY_TEST &&
                           (((size_t)A->Tsize + 3) & ~size_t(3)) * tsz + (size_t)256 * 16 * tsz <= kLdsBudget;
    const bool near_lv = near_leaves_ok(*A, nrhs, prec);
    if (near_tiles_ok(*A, nrhs)) {
      TuneParams t = best;
      t.near_kind = 4;
      const double ms = time_with(t);
      if (ms < best_ms) { best_ms = ms; best = t; }
    }
    if (near_mfma) {
      TuneParams t = best;
      t.near_kind = 1;
      const double ms = time_with(t);
      if (ms < best_ms) { best_ms = ms; best = t; }
    }
    if (near_lv) {
      for (int ct : {1, 2})
      for (int tpw : {4, 8})
        for (int ks : {1, 2, 4, 8, 12, 16, 24, 32}) {
          TuneParams t = best;
          t.near_kind = 2;
          t.near_ct = ct;
          t.near_tpw = tpw;
          t.near_ks = ks;
          const double ms = time_with(t);
          if (ms < best_ms) { best_ms = ms; best = t; }
        }
    }
    if (near_mfma || near_lv) {
      TuneParams t = best;
      t.near_kind = 0;
      t.near_nw = 0;
      const double ms = time_with(t);
      if (ms < best_ms) { best_ms = ms; best = t; }
    }
    if (near_rows && best.near_kind == 0)
      for (int nw : {1, 2, 4, 8}) {
        TuneParams t = best;
        t.near_kind = 0;
        t.near_nw = nw;
        const double ms = time_with(t);
        if (ms < best_ms) { best_ms = ms; best = t; }
      }
    {
      // the other choice of level concurrency than the automatic one
      TuneParams t = best;
      t.serial = levels_serial(*A, best.serial, nrhs, (int)prec) ? 2 : 1;
      const double ms = time_with(t);
      if (ms < best_ms) { best_ms = ms; best = t; }
    }
    A->tune[{nrhs, (int)prec}] = best;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    res.ks_target = best.ks_target;
    res.near_kind = best.near_kind;
    res.near_waves = best.near_nw;
    res.ms_best = best_ms;
    if (cache && *cache) {
      FILE* fp = std::fopen(cache, "a");
      if (fp) {
        std::fprintf(fp, "%s %d %d %d %d %d %d %d %d %d %.6f %.6f %d\n", key, best.ks_target, best.near_kind,
                     best.near_nw, best.tile, best.core_mode, best.near_ks, best.near_tpw, best.near_ct, best.serial,
                     res.ms_default, best_ms, best.order);
        std::fclose(fp);
      }
    }
    if (out) *out = res;
    return HTLR_OK;
  } catch (const Error& e) {
    return record(e);
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return HTLR_ERR_INVALID;
  }
}

htlr_status htlr_profile_enable(htlr_matrix A, int enable) {
  if (!A) { g_last_error = "null handle"; return HTLR_ERR_INVALID; }
  std::lock_guard<std::mutex> lk(A->ws_mu);
  A->prof.clear();
  A->prof.on = enable != 0;
  if (A->quasi) {
    htlr_matrix_impl& I = quasi_inner(*A);
    std::lock_guard<std::mutex> li(I.ws_mu);
    I.prof.clear();
    I.prof.on = enable != 0;
  }
  return HTLR_OK;
}

htlr_status htlr_profile_read(htlr_matrix A, htlr_profile_entry* out, int cap, int* count) {
  if (!A || !count) { g_last_error = "null argument"; return HTLR_ERR_INVALID; }
  try {
    std::lock_guard<std::mutex> lk(A->ws_mu);
    std::vector<std::string> names;
    std::vector<double> tot;
    std::vector<int> cnt;
    std::vector<const Profiler::Rec*> recs;
    for (auto& r : A->prof.recs) recs.push_back(&r);
    if (A->quasi)
      for (auto& r : quasi_inner(*A).prof.recs) recs.push_back(&r);
    for (const Profiler::Rec* rp : recs) {
      const Profiler::Rec& r = *rp;
      HTLR_HIP(hipEventSynchronize(r.b));
      float ms = 0.f;
      HTLR_HIP(hipEventElapsedTime(&ms, r.a, r.b));
      size_t k = std::find(names.begin(), names.end(), r.name) - names.begin();
      if (k == names.size()) { names.push_back(r.name); tot.push_back(0.0); cnt.push_back(0); }
      tot[k] += ms;
      cnt[k] += 1;
    }
    *count = (int)names.size();
    for (int i = 0; i < (int)names.size() && i < cap && out; ++i) {
      std::memset(out[i].name, 0, sizeof(out[i].name));
      std::strncpy(out[i].name, names[i].c_str(), sizeof(out[i].name) - 1);
      out[i].launches = cnt[i];
      out[i].total_ms = tot[i];
    }
    return HTLR_OK;
  } catch (const Error& e) {
    return record(e);
  }
}

}  // extern "C"
