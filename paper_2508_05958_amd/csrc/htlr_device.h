// Device-side helpers: kernel functions k(x - y), bfloat16 conversion.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

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

// e^x, x <= 0, by Tang's table-driven method: x = (64 m + j) ln(2)/64 + f
// with j = 0..63 and |f| <= ln(2)/128, so that e^x = 2^m 2^(j/64) e^f; e^f - 1
// by its Taylor polynomial of degree 5 (truncation below 4e-17).  tab holds
// 2^(j/64), j = 0..63 (kExp2Frac64, usually staged in LDS by the caller).
// The exponent is clamped as in exp_neg_f64.
__device__ __forceinline__ double exp_neg_f64_tab(double x, const double* tab) {
  constexpr double k64Log2e = 64.0 * 1.4426950408889634;      // 64 / ln 2
  constexpr double kLn2_64 = 0.6931471805599453 / 64.0;       // ln(2)/64, high part (exact scaling)
  constexpr double kLn2Lo_64 = 2.3190468138462996e-17 / 64.0;  // its remainder
  const double k = fmax(__builtin_rint(x * k64Log2e), -70400.0);
  const double f = fma(-k, kLn2Lo_64, fma(-k, kLn2_64, x));
  const int ki = (int)k;
  double q = fma(f, 1.0 / 120.0, 1.0 / 24.0);
  q = fma(q, f, 1.0 / 6.0);
  q = fma(q, f, 0.5);
  q = fma(q, f, 1.0);
  q = q * f;                                                  // e^f - 1
  const double t = tab[ki & 63];
  return __builtin_amdgcn_ldexp(fma(t, q, t), ki >> 6);
}

// 2^(j/64), j = 0..63, each the double nearest the exact value (computed to
// 50 significant digits), and the LDS bytes a kernel stages it in.
constexpr size_t kExpTabBytes = 64 * sizeof(double);
__device__ constexpr double kExp2Frac64[64] = {
    0x1.0000000000000p+0, 0x1.02c9a3e778061p+0, 0x1.059b0d3158574p+0, 0x1.0874518759bc8p+0,
    0x1.0b5586cf9890fp+0, 0x1.0e3ec32d3d1a2p+0, 0x1.11301d0125b51p+0, 0x1.1429aaea92de0p+0,
    0x1.172b83c7d517bp+0, 0x1.1a35beb6fcb75p+0, 0x1.1d4873168b9aap+0, 0x1.2063b88628cd6p+0,
    0x1.2387a6e756238p+0, 0x1.26b4565e27cddp+0, 0x1.29e9df51fdee1p+0, 0x1.2d285a6e4030bp+0,
    0x1.306fe0a31b715p+0, 0x1.33c08b26416ffp+0, 0x1.371a7373aa9cbp+0, 0x1.3a7db34e59ff7p+0,
    0x1.3dea64c123422p+0, 0x1.4160a21f72e2ap+0, 0x1.44e086061892dp+0, 0x1.486a2b5c13cd0p+0,
    0x1.4bfdad5362a27p+0, 0x1.4f9b2769d2ca7p+0, 0x1.5342b569d4f82p+0, 0x1.56f4736b527dap+0,
    0x1.5ab07dd485429p+0, 0x1.5e76f15ad2148p+0, 0x1.6247eb03a5585p+0, 0x1.6623882552225p+0,
    0x1.6a09e667f3bcdp+0, 0x1.6dfb23c651a2fp+0, 0x1.71f75e8ec5f74p+0, 0x1.75feb564267c9p+0,
    0x1.7a11473eb0187p+0, 0x1.7e2f336cf4e62p+0, 0x1.82589994cce13p+0, 0x1.868d99b4492edp+0,
    0x1.8ace5422aa0dbp+0, 0x1.8f1ae99157736p+0, 0x1.93737b0cdc5e5p+0, 0x1.97d829fde4e50p+0,
    0x1.9c49182a3f090p+0, 0x1.a0c667b5de565p+0, 0x1.a5503b23e255dp+0, 0x1.a9e6b5579fdbfp+0,
    0x1.ae89f995ad3adp+0, 0x1.b33a2b84f15fbp+0, 0x1.b7f76f2fb5e47p+0, 0x1.bcc1e904bc1d2p+0,
    0x1.c199bdd85529cp+0, 0x1.c67f12e57d14bp+0, 0x1.cb720dcef9069p+0, 0x1.d072d4a07897cp+0,
    0x1.d5818dcfba487p+0, 0x1.da9e603db3285p+0, 0x1.dfc97337b9b5fp+0, 0x1.e502ee78b3ff6p+0,
    0x1.ea4afa2a490dap+0, 0x1.efa1bee615a27p+0, 0x1.f50765b6e4540p+0, 0x1.fa7c1819e90d8p+0};

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

// Whether kvec_c12_t reads the table of 2^(j/64) for this kernel and type:
// the exponential kernels in double precision.
template <int KID, typename T>
constexpr bool uses_exp_table() {
  return std::is_same<T, double>::value && (KID == HTLR_K_EXP || KID == HTLR_K_GAUSS);
}

// kvec_c12, with e^x of the double-precision exponential kernels taken by
// exp_neg_f64_tab from etab (the staged kExp2Frac64; unused otherwise).
template <int KID, typename T>
__device__ __forceinline__ T kvec_c12_t(T dx0, T dx1, T dx2, T c12, int d, int pm1, const double* etab) {
  if constexpr (uses_exp_table<KID, T>()) {
    const double r2 = fma(dx0, dx0, c12);
    if constexpr (KID == HTLR_K_EXP) return exp_neg_f64_tab(-sqrt_f64(r2), etab);
    else return exp_neg_f64_tab(r2 * (-0.5 / d), etab);
  } else {
    return kvec_c12<KID, T>(dx0, dx1, dx2, c12, d, pm1);
  }
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
