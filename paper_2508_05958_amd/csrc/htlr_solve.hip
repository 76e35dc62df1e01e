// Solving A u = f (the "backward evaluation" of Sec. 1, eq. 1.2) with the
// HTLR product: restarted GMRES wrapped in iterative refinement.
//
// The paper stops at the product; the solver here is standard:
//   outer (FP64):  r = f - A x with the FP64 product; stop when
//                  ||r|| / ||f|| <= tol; otherwise solve A d = r
//                  approximately and set x += d;
//   inner:         GMRES(m), x0 = 0, Arnoldi with classical Gram-Schmidt
//                  applied twice, all Krylov vectors and projections in
//                  FP64; the products in the requested inner precision
//                  (vectors rounded to float around an FP32 or bfloat16-core
//                  product).  The small Hessenberg least-squares problem is
//                  solved on the host with Givens rotations.
// Reductions use fixed-order block partial sums, so a solve is
// deterministic.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "htlr_handle.h"
#include "htlr_vec.h"

namespace htlr {

extern thread_local std::string g_last_error;
htlr_status record(const Error& e);

#define HTLR_CHECK_MV(call)                                \
  do {                                                     \
    htlr_status s_ = (call);                               \
    if (s_ != HTLR_OK) ::htlr::fail(s_, g_last_error);     \
  } while (0)

namespace {


struct Solver {
  htlr_matrix_impl& A;
  hipStream_t st;
  int64_t N;
  int m;
  DevBuf V, w, r, d, partial, hdev, v32, w32;
  int fp64_mv = 0, inner_mv = 0;

  Solver(htlr_matrix_impl& a, hipStream_t s, int restart) : A(a), st(s), N(a.N), m(restart) {
    V.alloc((size_t)N * (m + 1) * sizeof(double));
    w.alloc(N * sizeof(double));
    r.alloc(N * sizeof(double));
    d.alloc(N * sizeof(double));
    partial.alloc((size_t)kRedBlocks * (m + 2) * sizeof(double));
    hdev.alloc((m + 2) * sizeof(double));
    v32.alloc(N * sizeof(float));
    w32.alloc(N * sizeof(float));
  }

  void matvec(int prec, const double* x, double* y) {
    if (prec == HTLR_FP64) {
      HTLR_CHECK_MV(htlr_matvec(&static_cast<htlr_matrix_s&>(A), x, y, 1, HTLR_FP64, HTLR_VEC_F64, st));
      ++fp64_mv;
    } else {
      hipLaunchKernelGGL(k_d2f, dim3(vblocks(N)), dim3(256), 0, st, x, v32.as<float>(), N);
      HTLR_CHECK_MV(htlr_matvec(&static_cast<htlr_matrix_s&>(A), v32.ptr, w32.ptr, 1, (htlr_precision)prec,
                                HTLR_VEC_F32, st));
      hipLaunchKernelGGL(k_f2d, dim3(vblocks(N)), dim3(256), 0, st, w32.as<float>(), y, N);
      ++inner_mv;
    }
  }

  // out[c] = <V[:, c], x> for c < ncols (device), copied to host
  void dots(const double* Vb, int ncols, const double* x, double* host) {
    hipLaunchKernelGGL(k_dots_partial, dim3(kRedBlocks), dim3(kRB), 0, st, Vb, N, ncols, x, N, partial.as<double>());
    hipLaunchKernelGGL(k_dots_final, dim3(ncols), dim3(kRB), 0, st, partial.as<double>(), kRedBlocks, ncols,
                       hdev.as<double>());
    HTLR_HIP(hipGetLastError());
    HTLR_HIP(hipMemcpyAsync(host, hdev.ptr, ncols * sizeof(double), hipMemcpyDeviceToHost, st));
    HTLR_HIP(hipStreamSynchronize(st));
  }

  double norm(const double* x) {
    double s = 0.0;
    dots(x, 1, x, &s);
    return std::sqrt(s);
  }

  // GMRES(m) on A d = b from d = 0; returns iterations used; *res = final
  // relative residual estimate (||b - A d|| / ||b|| from the recurrence).
  int gmres(int prec, const double* b, double* dout, double rtol, int maxit, double* res) {
    const double bn = norm(b);
    hipLaunchKernelGGL(k_zero, dim3(vblocks(N)), dim3(256), 0, st, dout, N);
    if (bn == 0.0) { *res = 0.0; return 0; }
    int it = 0;
    double rel = 1.0;
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), h(m + 2), h2(m + 2), y(m);
    double* Vp = V.as<double>();
    bool first = true;
    while (it < maxit) {
      // r = b - A d  (d = 0 on the first cycle)
      double beta;
      if (first) {
        HTLR_HIP(hipMemcpyAsync(r.ptr, b, N * sizeof(double), hipMemcpyDeviceToDevice, st));
        beta = bn;
      } else {
        matvec(prec, dout, w.as<double>());
        hipLaunchKernelGGL(k_sub_to, dim3(vblocks(N)), dim3(256), 0, st, b, w.as<double>(), r.as<double>(), N);
        beta = norm(r.as<double>());
      }
      first = false;
      rel = beta / bn;
      if (rel <= rtol) break;
      hipLaunchKernelGGL(k_scale_to, dim3(vblocks(N)), dim3(256), 0, st, r.as<double>(), 1.0 / beta, Vp, N);
      std::fill(g.begin(), g.end(), 0.0);
      g[0] = beta;
      int k = 0;
      for (; k < m && it < maxit; ++k) {
        double* vk = Vp + (int64_t)k * N;
        double* wk = Vp + (int64_t)(k + 1) * N;
        matvec(prec, vk, wk);
        // classical Gram-Schmidt, twice
        std::fill(h.begin(), h.end(), 0.0);
        for (int pass = 0; pass < 2; ++pass) {
          dots(Vp, k + 1, wk, h2.data());
          HTLR_HIP(hipMemcpyAsync(hdev.ptr, h2.data(), (k + 1) * sizeof(double), hipMemcpyHostToDevice, st));
          hipLaunchKernelGGL(k_sub_vh, dim3(vblocks(N)), dim3(256), 0, st, Vp, N, k + 1, hdev.as<double>(), wk, N);
          for (int j = 0; j <= k; ++j) h[j] += h2[j];
        }
        double hn = norm(wk);
        if (!std::isfinite(hn)) fail(HTLR_ERR_NUMERIC, "NaN/Inf in the Krylov basis");
        h[k + 1] = hn;
        if (hn > 0) hipLaunchKernelGGL(k_scale_to, dim3(vblocks(N)), dim3(256), 0, st, wk, 1.0 / hn, wk, N);
        // apply previous rotations, then a new one
        for (int j = 0; j < k; ++j) {
          double t = cs[j] * h[j] + sn[j] * h[j + 1];
          h[j + 1] = -sn[j] * h[j] + cs[j] * h[j + 1];
          h[j] = t;
        }
        double den = std::hypot(h[k], h[k + 1]);
        cs[k] = den > 0 ? h[k] / den : 1.0;
        sn[k] = den > 0 ? h[k + 1] / den : 0.0;
        h[k] = den;
        h[k + 1] = 0.0;
        g[k + 1] = -sn[k] * g[k];
        g[k] = cs[k] * g[k];
        for (int j = 0; j <= k; ++j) H[(size_t)j * m + k] = h[j];
        ++it;
        rel = std::fabs(g[k + 1]) / bn;
        if (rel <= rtol || hn == 0.0) { ++k; break; }
      }
      // y = R^{-1} g, d += V y
      for (int i = k - 1; i >= 0; --i) {
        double s = g[i];
        for (int j = i + 1; j < k; ++j) s -= H[(size_t)i * m + j] * y[j];
        y[i] = s / H[(size_t)i * m + i];
      }
      HTLR_HIP(hipMemcpyAsync(hdev.ptr, y.data(), k * sizeof(double), hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(k_add_vy, dim3(vblocks(N)), dim3(256), 0, st, Vp, N, k, hdev.as<double>(), dout, N);
      HTLR_HIP(hipGetLastError());
      if (rel <= rtol) break;
    }
    HTLR_HIP(hipStreamSynchronize(st));
    *res = rel;
    return it;
  }
};

}  // namespace
}  // namespace htlr

using namespace htlr;

extern "C" htlr_status htlr_solve(htlr_matrix A, const double* f, double* u, int nrhs, const htlr_solve_opts* opts,
                                  htlr_solve_info* info, void* stream) {
  try {
    g_last_error.clear();
    if (!A || !f || !u) fail(HTLR_ERR_INVALID, "null argument");
    if (nrhs != 1) fail(HTLR_ERR_UNSUPPORTED, "the solver takes one right-hand side");
    htlr_solve_opts o{};
    if (opts) o = *opts;
    const double tol = o.tol > 0 ? o.tol : 1e-10;
    const int restart = o.restart > 0 ? o.restart : 30;
    const int max_outer = o.max_outer > 0 ? o.max_outer : 20;
    const int max_inner = o.max_inner > 0 ? o.max_inner : 300;
    const int ip = o.inner_prec;
    if (ip != HTLR_FP64 && ip != HTLR_FP32 && ip != HTLR_BF16_CORE) fail(HTLR_ERR_INVALID, "unknown inner precision");
    if (restart > 1000) fail(HTLR_ERR_INVALID, "restart too large");
    const double inner_tol = o.inner_tol > 0 ? o.inner_tol : (ip == HTLR_FP32 ? 1e-6 : (ip == HTLR_BF16_CORE ? 1e-2 : tol));
    hipStream_t st = (hipStream_t)stream;
    Solver S(*A, st, restart);
    htlr_solve_info inf{};
    const int64_t N = A->N;
    const double fn = S.norm(f);
    if (!std::isfinite(fn)) fail(HTLR_ERR_NUMERIC, "f has NaN/Inf");
    hipLaunchKernelGGL(k_zero, dim3(vblocks(N)), dim3(256), 0, st, u, N);
    htlr_status status = HTLR_OK;
    if (fn == 0.0) {
      HTLR_HIP(hipStreamSynchronize(st));
      if (info) *info = inf;
      return HTLR_OK;
    }
    double rel = 1.0;
    for (int outer = 0;; ++outer) {
      // r = f - A u with the FP64 product; the first time u = 0, so r = f
      // exactly and the product is skipped
      if (outer == 0) {
        HTLR_HIP(hipMemcpyAsync(S.r.ptr, f, N * sizeof(double), hipMemcpyDeviceToDevice, st));
      } else {
        S.matvec(HTLR_FP64, u, S.w.as<double>());
        hipLaunchKernelGGL(k_sub_to, dim3(vblocks(N)), dim3(256), 0, st, f, S.w.as<double>(), S.r.as<double>(), N);
      }
      const double rn = outer == 0 ? fn : S.norm(S.r.as<double>());
      if (!std::isfinite(rn)) fail(HTLR_ERR_NUMERIC, "residual is NaN/Inf");
      rel = rn / fn;
      inf.outer_iters = outer;
      if (rel <= tol) break;
      if (outer >= max_outer) { status = HTLR_ERR_NOT_CONVERGED; break; }
      // inner solve of A d = r to max(inner_tol, tol ||f|| / ||r||)
      const double rtol = std::max(inner_tol, tol * fn / rn);
      DevBuf rb;
      rb.alloc(N * sizeof(double));
      HTLR_HIP(hipMemcpyAsync(rb.ptr, S.r.ptr, N * sizeof(double), hipMemcpyDeviceToDevice, st));
      double ires = 1.0;
      inf.inner_iters += S.gmres(ip, rb.as<double>(), S.d.as<double>(), rtol, max_inner, &ires);
      hipLaunchKernelGGL(k_add_to, dim3(vblocks(N)), dim3(256), 0, st, u, S.d.as<double>(), N);
      HTLR_HIP(hipGetLastError());
    }
    HTLR_HIP(hipStreamSynchronize(st));
    inf.rel_residual = rel;
    inf.matvecs_fp64 = S.fp64_mv;
    inf.matvecs_inner = S.inner_mv;
    if (info) *info = inf;
    if (status != HTLR_OK) g_last_error = "solver reached max_outer before tol";
    return status;
  } catch (const Error& e) {
    return record(e);
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return HTLR_ERR_INVALID;
  }
}
