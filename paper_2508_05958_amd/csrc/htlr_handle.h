// The HTLR matrix handle: everything htlr_build leaves resident in HBM, plus
// the work buffers of products.  Shared by construction, product and solver.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "htlr_internal.h"

namespace htlr {

#define HTLR_HIP(call)                                                                    \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      ::htlr::fail(e_ == hipErrorOutOfMemory ? HTLR_ERR_OOM : HTLR_ERR_HIP,               \
                   std::string(#call) + ": " + hipGetErrorString(e_));                   \
  } while (0)

// Device allocation owned by a handle.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : ptr(o.ptr), bytes(o.bytes) { o.ptr = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); ptr = o.ptr; bytes = o.bytes; o.ptr = nullptr; o.bytes = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t b) {
    release();
    if (b == 0) return;
    HTLR_HIP(hipMalloc(&ptr, b));
    bytes = b;
  }
  void release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
  }
  template <class T> T* as() const { return static_cast<T*>(ptr); }
};

// One level of the cluster tree that carries admissible leaves.
struct LevelData {
  int level = 0, B = 0, m = 0;
  int64_t nbox = 0, npairs = 0;
  DevBuf ptr, src, cid;              // CSR of admissible leaves; core id per entry (uniform)
  DevBuf U64, V64, U32, V32;         // factors: uniform [m][p]; tensor [d][B][m][p]
  DevBuf cheb64, cheb32;             // tensor grids: Chebyshev points [d][B][p]
  int ncore = 0;                     // uniform grids: one core per offset
  std::vector<int> offsets;          // 3 ints per core: sigma - tau in boxes
  DevBuf G64, G32, G16;              // cores, layout [core][s][t] (t fastest)
  DevBuf Gm16, Gm32, Gm64;           // cores for the matrix-core kernel, layout [core][t][s]
  DevBuf tile_ptr, tile_list;        // matrix-core kernel work lists (uniform)
  int ntile_cls = 0;                 // tiles per parity class
};

struct Workspace {
  int nrhs = 0;
  int prec = -1;
  std::vector<DevBuf> W, H, W16;     // per level
  DevBuf zero;                       // a zero source tensor (matrix-core kernel)
  size_t bytes = 0;
};

struct htlr_matrix_impl {
  int d = 0, n = 0, p = 0, leaf = 0, L = 0, P = 0, kid = 0;
  int64_t N = 0;
  bool uniform = false;
  double eta2 = 1.0;
  int adm_kind = 0, gl_order = 0, precisions = 7;
  double h = 0, w0 = 0, D0 = 0;
  int device = 0;
  Grid grid;
  Plan plan;
  DevBuf x64, x32, w64, w32;         // per-dimension nodes and cell lengths
  DevBuf a64, a32;                   // a(x_i), N values
  DevBuf D64, D32;                   // tensor grids: per-point diagonal integrals
  DevBuf near_ptr, near_src;         // inadmissible leaves (level L)
  DevBuf T64, T32;                   // uniform radial kernels: near-field table by squared distance
  int Tsize = 0;
  std::vector<LevelData> levels;     // index = level
  size_t device_bytes = 0;
  std::mutex ws_mu;
  Workspace ws;
};

}  // namespace htlr

struct htlr_matrix_s : htlr::htlr_matrix_impl {};
