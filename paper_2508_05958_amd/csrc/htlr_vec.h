// Vector kernels shared by the solver and the request server: dot products
// with fixed-order block reductions, Gram-Schmidt updates, conversions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace htlr {
namespace {

constexpr int kRB = 256;       // threads per block of the vector kernels
constexpr int kRedBlocks = 512;

// partial[b][c] = sum over rows of block b of V[:, c] * w
__global__ __launch_bounds__(kRB) void k_dots_partial(const double* __restrict__ V, int64_t ldv, int ncols,
                                                       const double* __restrict__ w, int64_t N,
                                                       double* __restrict__ partial) {
  __shared__ double red[kRB];
  const int64_t chunk = (N + gridDim.x - 1) / gridDim.x;
  const int64_t lo = blockIdx.x * chunk, hi = lo + chunk < N ? lo + chunk : N;
  for (int c = 0; c < ncols; ++c) {
    double s = 0.0;
    const double* v = V + (int64_t)c * ldv;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kRB) s += v[i] * w[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = kRB / 2; st > 0; st >>= 1) {
      if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * ncols + c] = red[0];
    __syncthreads();
  }
}

// out[c] = sum over b of partial[b][c]: one block of kRB threads per column,
// each thread summing partials b = t, t + kRB, ..., then a fixed-order tree
// in LDS (a thread per column summing all nb partials in turn was a chain of
// nb dependent loads, tens of microseconds on every Gram-Schmidt step).
__global__ __launch_bounds__(kRB) void k_dots_final(const double* __restrict__ partial, int nb, int ncols,
                                                    double* __restrict__ out) {
  __shared__ double red[kRB];
  const int c = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += kRB) s += partial[(int64_t)b * ncols + c];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = kRB / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = red[0];
}

// w -= V[:, 0:ncols] h
__global__ void k_sub_vh(const double* __restrict__ V, int64_t ldv, int ncols, const double* __restrict__ h,
                         double* __restrict__ w, int64_t N) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < ncols; ++c) s += V[(int64_t)c * ldv + i] * h[c];
    w[i] -= s;
  }
}

// x += V[:, 0:ncols] y
__global__ void k_add_vy(const double* __restrict__ V, int64_t ldv, int ncols, const double* __restrict__ y,
                         double* __restrict__ x, int64_t N) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < ncols; ++c) s += V[(int64_t)c * ldv + i] * y[c];
    x[i] += s;
  }
}

__global__ void k_scale_to(const double* __restrict__ x, double a, double* __restrict__ y, int64_t N) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i];
}

__global__ void k_sub_to(const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ y,
                         int64_t N) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a[i] - b[i];
}

__global__ void k_add_to(double* __restrict__ x, const double* __restrict__ d, int64_t N) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
    x[i] += d[i];
}

__global__ void k_d2f(const double* __restrict__ x, float* __restrict__ y, int64_t N) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}

__global__ void k_f2d(const float* __restrict__ x, double* __restrict__ y, int64_t N) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (double)x[i];
}

__global__ void k_zero(double* __restrict__ x, int64_t N) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 0.0;
}

inline int vblocks(int64_t N) { return (int)std::min<int64_t>((N + 255) / 256, 8192); }

// Batched forms for the request server: one launch handles many vectors
// given by device pointer tables.

// y_j = (float) x_j for every column j of a batch (x_j of length N)
__global__ void k_gather_f32(const double* const* __restrict__ src, float* __restrict__ dst, int64_t N, int cols) {
  for (int j = 0; j < cols; ++j)
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
      dst[(int64_t)j * N + i] = (float)src[j][i];
}

__global__ void k_gather_f64(const double* const* __restrict__ src, double* __restrict__ dst, int64_t N, int cols) {
  for (int j = 0; j < cols; ++j)
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
      dst[(int64_t)j * N + i] = src[j][i];
}

}  // namespace
}  // namespace htlr
