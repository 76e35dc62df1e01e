// GMRES with FP64 iterative refinement around the HTLR product.
#include "htlr_handle.h"

namespace htlr {
extern thread_local std::string g_last_error;
}

extern "C" htlr_status htlr_solve(htlr_matrix A, const double* f, double* u, int nrhs, const htlr_solve_opts* opts,
                                  htlr_solve_info* info, void* stream) {
  (void)A; (void)f; (void)u; (void)nrhs; (void)opts; (void)info; (void)stream;
  htlr::g_last_error = "solver not built yet";
  return HTLR_ERR_UNSUPPORTED;
}
