// placeholder, replaced by the GMRES driver
#include "ctx.h"
extern "C" {
hbf_status hbf_solve(hbf_ctx*, const void*, void*, int32_t, hbf_dtype, const hbf_solve_opts*, hbf_solve_info*, void*) {
  hbf::set_error("hbf_solve: not available");
  return HBF_ESTATE;
}
hbf_status hbf_solve_adjoint(hbf_ctx*, const void*, void*, int32_t, hbf_dtype, const hbf_solve_opts*, hbf_solve_info*, void*) {
  hbf::set_error("hbf_solve_adjoint: not available");
  return HBF_ESTATE;
}
}
