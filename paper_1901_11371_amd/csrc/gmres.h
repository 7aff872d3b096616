// GMRES building blocks (gmres.hip).
#pragma once

#include "kernels.h"

namespace hbf {

// out[i][r] = sum_n conj(V_i[n][r]) w[n][r] for i < nv (nv <= 64), FP64 accumulation.
hipError_t gm_dots(bool c128, const void* V, int64_t vstride, int nv, const void* w, int64_t n, int R, cd* partial,
                   size_t partial_len, cd* out, hipStream_t s);
// w -= sum_i V_i h_i ; u = sum_i V_i y_i
hipError_t gm_sub_combo(bool c128, const void* V, int64_t vstride, int nv, const cd* h, void* w, int64_t n, int R,
                        hipStream_t s);
hipError_t gm_combo(bool c128, const void* V, int64_t vstride, int nv, const cd* y, void* u, int64_t n, int R,
                    hipStream_t s);
// dst = src * f[r] (real factor per right-hand side)
hipError_t gm_scale(bool src128, const void* src, const double* f, bool dst128, void* dst, int64_t n, int R,
                    hipStream_t s);
hipError_t gm_sub64(const cd* a, const cd* b, cd* y, int64_t m, hipStream_t s);
hipError_t gm_add_to64(bool src128, const void* d, cd* x, int64_t m, hipStream_t s);
hipError_t gm_cast(bool src128, const void* a, bool dst128, void* b, int64_t m, hipStream_t s);
hipError_t gm_zero(void* p, int64_t ndoubles, hipStream_t s);
hipError_t gm_nonfinite(bool c128, const void* v, int64_t m, int* flag, hipStream_t s);

// per-RHS Hessenberg / Givens state
int64_t gm_small_per_rhs(int m);
hipError_t gm_cycle_start(double* small, int m, int R, const cd* nrm2, const double* target, double* inv,
                          double* resid, int* active, hipStream_t s);
hipError_t gm_h_accum(double* small, int m, int R, int j, const cd* h, hipStream_t s);
hipError_t gm_givens(double* small, int m, int R, int j, const cd* nrm2, double* inv, double* resid,
                     const double* target, int* active, hipStream_t s);
hipError_t gm_lsq(double* small, int m, int R, cd* y, hipStream_t s);

}  // namespace hbf
