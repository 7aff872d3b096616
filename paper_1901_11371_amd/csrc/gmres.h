// Krylov building blocks (gmres.hip).  A non-null `jdev` makes a kernel take
// the Arnoldi step index j from device memory (for captured step graphs).
#pragma once

#include "kernels.h"

namespace hbf {

// out[i][r] = sum_n conj(V_i[n][r]) w[n][r] for i < nv (nv <= 32), FP64 accumulation.
hipError_t gm_dots(bool c128, const void* V, int64_t vstride, int nv, const void* w, int64_t n, int R, cd* partial,
                   size_t partial_len, cd* out, hipStream_t s);
// the same for basis vectors 0..*jdev of a basis of at most m vectors
hipError_t gm_dots_dev(bool c128, const void* V, int64_t vstride, int m, const int* jdev, const void* w, int64_t n,
                       int R, cd* partial, size_t partial_len, cd* out, hipStream_t s);
// w -= sum_{i < nv} V_i h_i (nv = *jdev + 1 when jdev is given) ; u = sum_i V_i y_i
hipError_t gm_sub_combo(bool c128, const void* V, int64_t vstride, int nv, const int* jdev, const cd* h, void* w,
                        int64_t n, int R, hipStream_t s);
hipError_t gm_combo(bool c128, const void* V, int64_t vstride, int nv, const cd* y, void* u, int64_t n, int R,
                    hipStream_t s);
// dst = src * f[r] (real factor per right-hand side); with jdev, dst is basis
// vector *jdev + 1 of a basis of stride dstride
hipError_t gm_scale(bool src128, const void* src, const double* f, bool dst128, void* dst, int64_t dstride,
                    const int* jdev, int64_t n, int R, hipStream_t s);
hipError_t gm_copy_basis(bool c128, const void* V, int64_t vstride, const int* jdev, void* dst, int64_t m,
                         hipStream_t s);
hipError_t gm_copy(bool c128, const void* src, void* dst, int64_t m, hipStream_t s);
hipError_t gm_sub64(const cd* a, const cd* b, cd* y, int64_t m, hipStream_t s);
hipError_t gm_add_to64(bool src128, const void* d, cd* x, int64_t m, hipStream_t s);
hipError_t gm_cast(bool src128, const void* a, bool dst128, void* b, int64_t m, hipStream_t s);
hipError_t gm_zero(void* p, int64_t ndoubles, hipStream_t s);
hipError_t gm_set_int(int* p, int v, hipStream_t s);
hipError_t gm_nonfinite(bool c128, const void* v, int64_t m, int* flag, hipStream_t s);
// grad_z = -sum_r lam_r * conj(x_r), (nrhs, N) external layout, io dtype
hipError_t gm_impedance_grad(bool c128, const void* lam, const void* x, int64_t n, int R, void* out, hipStream_t s);

// per-RHS GMRES Hessenberg / Givens state
int64_t gm_small_per_rhs(int m);
hipError_t gm_cycle_start(double* small, int m, int R, const cd* nrm2, const double* target, double* inv,
                          double* resid, int* active, hipStream_t s);
hipError_t gm_h_accum(double* small, int m, int R, int j, const int* jdev, const cd* h, hipStream_t s);
hipError_t gm_givens(double* small, int m, int R, int j, const int* jdev, const cd* nrm2, double* inv, double* resid,
                     const double* target, int* active, hipStream_t s);
// step index += 1 (when jdev is given); *any_active = OR of the masks
hipError_t gm_step_end(int* jdev, const int* active, int R, int* any_active, hipStream_t s);
hipError_t gm_lsq(double* small, int m, int R, cd* y, hipStream_t s);
// Arnoldi steps each RHS took in the current cycle
hipError_t gm_read_iters(double* small, int m, int R, int* out, hipStream_t s);

// per-RHS TFQMR state (tq_state_bytes(R) bytes)
size_t tq_state_bytes(int R);
hipError_t tq_start(void* S, int R, const cd* nrm2, const double* target, double* inv, double* resid, int* active,
                    hipStream_t s);
hipError_t tq_rho0(void* S, int R, const cd* dot, hipStream_t s);
hipError_t tq_alpha(void* S, int R, const cd* sigma, int* active, hipStream_t s);
hipError_t tq_half(void* S, int R, const cd* wnrm2, double* resid, hipStream_t s);
hipError_t tq_commit(void* S, int R, int* active, hipStream_t s);
hipError_t tq_beta(void* S, int R, const cd* rhonew, int* active, hipStream_t s);
hipError_t tq_scales(const void* S, int R, double* f, hipStream_t s);
hipError_t tq_iters(const void* S, int R, int* out, hipStream_t s);
// y2 = y - alpha v; w -= alpha u; d = y + f d
hipError_t tq_e1(bool c128, const void* S, const int* active, void* y2, const void* y, const void* v, void* w,
                 const void* u, void* d, int64_t n, int R, hipStream_t s);
// xhat += eta d
hipError_t tq_e2(bool c128, const void* S, const int* active, void* xh, const void* d, int64_t n, int R,
                 hipStream_t s);
// w -= alpha u2; d = y2 + f d
hipError_t tq_e3(bool c128, const void* S, const int* active, void* w, const void* u2, const void* y2, void* d,
                 int64_t n, int R, hipStream_t s);
// y = w + beta y2
hipError_t tq_e4(bool c128, const void* S, const int* active, void* y, const void* w, const void* y2, int64_t n,
                 int R, hipStream_t s);
// v = u + beta (u2 + beta v)
hipError_t tq_e5(bool c128, const void* S, const int* active, void* v, const void* u, const void* u2, int64_t n,
                 int R, hipStream_t s);
// w = y = rt = r0 * inv[r]; d = xhat = 0
hipError_t tq_init(bool src128, const void* r0, const double* inv, bool c128, void* w, void* y, void* rt, void* d,
                   void* xh, int64_t n, int R, hipStream_t s);

}  // namespace hbf
