// Device-side helpers: kernel functions k(x - y), bfloat16 conversion.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "htlr.h"

namespace htlr {

__device__ __constant__ static const double kPolyADev[3] = {0.50, 0.30, 0.20};

// Double-precision pieces of the kernels, written for their bounded
// arguments (finite s = r^2 > 0 of normal size; finite x <= 0 for e^x)
// without the special-case handling of the general library functions.
//
// Reciprocal square root: the hardware estimate y0 (about 23 correct bits)
// and two Newton steps y <- y (3/2 - (s/2) y^2), each doubling the correct
// bits.
__device__ __forceinline__ double rsqrt_f64(double s) {
  const double hs = 0.5 * s;
  double y = __builtin_amdgcn_rsq(s);
  y = y * fma(-hs * y, y, 1.5);
  return y * fma(-hs * y, y, 1.5);
}

// Square root: r0 = s y0 from the same estimate, then two Newton steps
// r <- r + (y0/2)(s - r^2) (the residual s - r^2 formed exactly by FMA).
__device__ __forceinline__ double sqrt_f64(double s) {
  const double y = __builtin_amdgcn_rsq(s), hy = 0.5 * y;
  double r = s * y;
  r = fma(fma(-r, r, s), hy, r);
  return fma(fma(-r, r, s), hy, r);
}

// e^x, x <= 0: Cody and Waite's reduction x = k ln 2 + f, k = rint(x / ln 2),
// with ln 2 split into the double nearest it and the remainder, so that
// |f| <= ln(2)/2; e^f by its Taylor polynomial of degree 13 (the truncation
// is below 4e-18 relative), coefficients 1/n!, by Horner's rule; 2^k by
// ldexp.  k is clamped at -1100, where the result is below 1e-300.
struct TaylorExpCoeffs {
  double c[14];
  constexpr TaylorExpCoeffs() : c{} {
    c[0] = 1.0;
    for (int n = 1; n < 14; ++n) c[n] = c[n - 1] / n;
  }
};

__device__ __forceinline__ double exp_neg_f64(double x) {
  constexpr TaylorExpCoeffs T;
  constexpr double kLog2e = 1.4426950408889634;      // 1 / ln 2
  constexpr double kLn2 = 0.6931471805599453;        // ln 2, nearest double
  constexpr double kLn2Lo = 2.3190468138462996e-17;  // ln 2 - kLn2
  const double k = fmax(__builtin_rint(x * kLog2e), -1100.0);
  const double f = fma(-k, kLn2Lo, fma(-k, kLn2, x));
  double p = T.c[13];
#pragma unroll
  for (int n = 12; n >= 0; --n) p = fma(p, f, T.c[n]);
  return __builtin_amdgcn_ldexp(p, (int)k);
}

// Radial kernels as functions of r^2 (r = |x - y|).
template <int KID>
__device__ __forceinline__ double kr2(double r2, int d) {
  if constexpr (KID == HTLR_K_INV_R) return rsqrt_f64(r2);
  else if constexpr (KID == HTLR_K_NEG_LOG) return -0.5 * log(r2);
  else if constexpr (KID == HTLR_K_EXP) return exp_neg_f64(-sqrt_f64(r2));
  else return exp_neg_f64(r2 * (-0.5 / d));
}

// Single precision: the hardware reciprocal square root, square root, 2^x
// and log2 instructions (about 1 ulp each), with exp(x) = 2^(x log2 e) and
// log(x) = ln 2 log2(x); far inside the accuracy of a single-precision
// product.  The arguments stay in the instructions' normal range: r^2 > 0,
// and the exponents are negative and of modest size on [0, 1]^d.
template <int KID>
__device__ __forceinline__ float kr2(float r2, int d) {
  constexpr float kLog2e = 1.44269504088896341f;      // log2(e)
  constexpr float kHalfLn2 = 0.346573590279972655f;   // ln(2) / 2
  if constexpr (KID == HTLR_K_INV_R) return __builtin_amdgcn_rsqf(r2);
  else if constexpr (KID == HTLR_K_NEG_LOG) return -kHalfLn2 * __builtin_amdgcn_logf(r2);
  else if constexpr (KID == HTLR_K_EXP) return __builtin_amdgcn_exp2f(-kLog2e * __builtin_amdgcn_sqrtf(r2));
  else return __builtin_amdgcn_exp2f(r2 * (-kLog2e / (2.0f * d)));
}

template <typename T>
__device__ __forceinline__ T ipow(T b, int e) {
  T r = T(1);
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

// k evaluated at the difference vector (dx0, dx1, dx2); pm1 = p - 1 (poly).
template <int KID, typename T>
__device__ __forceinline__ T kvec(T dx0, T dx1, T dx2, int d, int pm1) {
  if constexpr (KID == HTLR_K_POLY_TEST) {
    T v = ipow(T(1) + T(kPolyADev[0]) * dx0, pm1) * ipow(T(1) + T(kPolyADev[1]) * dx1, pm1);
    if (d == 3) v *= ipow(T(1) + T(kPolyADev[2]) * dx2, pm1);
    return v;
  } else {
    T r2 = dx0 * dx0 + dx1 * dx1 + dx2 * dx2;
    return kr2<KID>(r2, d);
  }
}

// k at (dx0, dx1, dx2) given c12 = dx1^2 + dx2^2 (formed once per source
// row by the caller): r^2 = dx0^2 + c12 for the radial kernels.
template <int KID, typename T>
__device__ __forceinline__ T kvec_c12(T dx0, T dx1, T dx2, T c12, int d, int pm1) {
  if constexpr (KID == HTLR_K_POLY_TEST) return kvec<KID, T>(dx0, dx1, dx2, d, pm1);
  else return kr2<KID>(fma(dx0, dx0, c12), d);
}

// bfloat16 stored as uint16_t; round to nearest even.
__device__ __host__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t x = __builtin_bit_cast(uint32_t, f);
  if ((x & 0x7f800000u) == 0x7f800000u) return (uint16_t)((x >> 16) | ((x & 0xffffu) ? 0x40u : 0u));
  x += 0x7fffu + ((x >> 16) & 1u);
  return (uint16_t)(x >> 16);
}

__device__ __host__ __forceinline__ float bf2f(uint16_t b) {
  return __builtin_bit_cast(float, (uint32_t)b << 16);
}

template <typename T> struct Acc { using type = T; };
template <> struct Acc<uint16_t> { using type = float; };

template <typename T> __device__ __forceinline__ T load_as(const T* p) { return *p; }
__device__ __forceinline__ float to_acc(float v) { return v; }
__device__ __forceinline__ double to_acc(double v) { return v; }
__device__ __forceinline__ float to_acc(uint16_t v) { return bf2f(v); }

template <typename T> __device__ __forceinline__ T from_acc(float v);
template <> __device__ __forceinline__ float from_acc<float>(float v) { return v; }
template <> __device__ __forceinline__ uint16_t from_acc<uint16_t>(float v) { return f2bf(v); }
template <typename T> __device__ __forceinline__ T from_acc_d(double v);
template <> __device__ __forceinline__ double from_acc_d<double>(double v) { return v; }

}  // namespace htlr
