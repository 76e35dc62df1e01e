// f = A u without device allocation: the product's work buffers (per level
// the source tensors W, the core apply's outputs H, the partial up
// contractions, and a zero tensor) live in one fixed-size array of this
// library's own device memory, `scratch`, instead of buffers the handle
// allocates on first use.  For callers that cannot call hipMalloc.
//
// Each device the library runs on holds its own copy of the array until the
// process ends.  Its device address is looked up once per device, with that
// device current, and kept; host code only ever passes that address to
// kernels (the array's name in host code is a host-side stand-in, not a
// device address).  Every call on a device shares the array, so calls that
// overlap on one device race; the buffers need no clearing, since every
// product writes each of them in full before reading it.

#include <mutex>

#include "htlr_handle.h"

namespace htlr {

extern thread_local std::string g_last_error;
htlr_status record(const Error& e);

namespace {

static __device__ __align__(256) unsigned char scratch[HTLR_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once).
char* scratch_on(int dev) {
  if (dev < 0 || dev >= kMaxDevices) fail(HTLR_ERR_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      fail(HTLR_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = (char*)ptr;
  }
  return g_scratch_ptr[dev];
}

}  // namespace
}  // namespace htlr

using namespace htlr;

extern "C" {

htlr_status htlr_matvec_noalloc(htlr_matrix A, const void* u, void* f, int nrhs, htlr_precision prec,
                                htlr_vec_dtype vec_dtype, void* stream) {
  try {
    g_last_error.clear();
    if (!A || !u || !f) fail(HTLR_ERR_INVALID, "null argument");
    if (nrhs < 1 || nrhs > 64) fail(HTLR_ERR_INVALID, "nrhs out of range (1..64)");
    if (prec != HTLR_FP64 && prec != HTLR_FP32 && prec != HTLR_BF16_CORE) fail(HTLR_ERR_INVALID, "unknown precision");
    if ((prec == HTLR_FP64) != (vec_dtype == HTLR_VEC_F64))
      fail(HTLR_ERR_UNSUPPORTED, "FP64 products take f64 vectors, FP32/BF16 products take f32 vectors");
    if (!(A->precisions & (1 << prec))) fail(HTLR_ERR_UNSUPPORTED, "matrix built without this precision");
    if (A->quasi) fail(HTLR_ERR_UNSUPPORTED, "transfer-form handles keep their own buffers: use htlr_matvec");
    const size_t esz = vec_dtype == HTLR_VEC_F64 ? 8 : 4;
    const char* ub = (const char*)u;
    const char* fb = (const char*)f;
    const size_t span = (size_t)A->N * nrhs * esz;
    if (ub < fb + span && fb < ub + span) fail(HTLR_ERR_INVALID, "u and f overlap");
    int dev = 0;
    HTLR_HIP(hipGetDevice(&dev));
    if (dev != A->device) fail(HTLR_ERR_INVALID, "current device differs from the build device");
    const size_t need = carve_workview(*A, nrhs, nullptr, nullptr);
    if (need > (size_t)HTLR_NOALLOC_SCRATCH_BYTES)
      fail(HTLR_ERR_INVALID, "work buffers of this product (" + std::to_string(need) +
                                 " bytes) exceed the fixed scratch of htlr_matvec_noalloc (" +
                                 std::to_string((size_t)HTLR_NOALLOC_SCRATCH_BYTES) + " bytes): use htlr_matvec");
    char* base = scratch_on(dev);
    WorkView wv;
    carve_workview(*A, nrhs, base, &wv);
    wv.noalloc = true;
    std::lock_guard<std::mutex> lk(A->ws_mu);
    product_view(*A, u, f, nrhs, prec, (hipStream_t)stream, wv);
    return HTLR_OK;
  } catch (const Error& e) {
    return record(e);
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return HTLR_ERR_INVALID;
  }
}

}  // extern "C"
