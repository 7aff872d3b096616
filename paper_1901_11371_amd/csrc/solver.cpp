// Solve driver: restarted, right-preconditioned GMRES (A M^{-1} u = r,
// d = M^{-1} u, M the approximate LU preconditioner built from the triangular
// parts of A, Sec. 3.1) inside an iterative-refinement loop.
//
// Each outer step computes the true residual r = b - A x in FP64 (complex128
// vectors; with complex64 factors the factors are widened and accumulated in
// FP64), then runs one GMRES(m) cycle on A d = r in the context precision
// (complex64 Krylov vectors with FP64 Gram-Schmidt dot products, FP64
// Hessenberg / Givens state) and updates x += d in FP64.  A cycle therefore
// restarts GMRES from the true residual, and the mixed-precision refinement
// recovers FP64 accuracy from complex64 inner solves.  All right-hand sides
// advance in lockstep; a right-hand side that has reached its target stops
// contributing (its Krylov column is zero).
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "ctx.h"
#include "gmres.h"

using namespace hbf;

namespace {

struct Err {
  hbf_status st;
  std::string msg;
};

void chk(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Err{HBF_EHIP, std::string(what) + ": " + hipGetErrorString(e)};
}
void chk(hbf_status s, const char* what) {
  if (s != HBF_OK) throw Err{s, std::string(what) + ": " + hbf::last_error()};
}

hbf_status solve_impl(hbf_ctx* c, const void* b, void* x, int32_t nrhs, hbf_dtype io, const hbf_solve_opts* opts,
                      hbf_solve_info* info, void* stream, bool adjoint) {
  const char* name = adjoint ? "hbf_solve_adjoint" : "hbf_solve";
  if (!c || !b || !x) { set_error(std::string(name) + ": NULL argument"); return HBF_EINVAL; }
  if (nrhs < 1 || nrhs > c->max_nrhs) { set_error(std::string(name) + ": nrhs out of range"); return HBF_EINVAL; }
  if (io != HBF_C64 && io != HBF_C128) { set_error(std::string(name) + ": bad io dtype"); return HBF_EINVAL; }
  hbf_solve_opts o{};
  if (opts) o = *opts;
  const double tol = o.tol > 0 ? o.tol : 1e-6;
  const int m = (o.restart > 0) ? std::min(o.restart, c->restart) : c->restart;
  if (m < 1 || m > 255) { set_error(std::string(name) + ": restart must be in [1, 255]"); return HBF_EINVAL; }
  const int max_iters = o.max_iters > 0 ? o.max_iters : 500;
  const int max_refine = o.max_refine > 0 ? o.max_refine : 10;
  const bool inner128 = c->dtype == HBF_C128;
  const bool mixed = !inner128 && o.mixed;
  const double inner_tol = o.inner_tol > 0 ? o.inner_tol : (mixed ? 1e-4 : 0.0);
  const int R = nrhs;
  const int64_t N = c->n;
  const int64_t NR = N * R;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (hipSetDevice(c->device) != hipSuccess) { set_error("hipSetDevice"); return HBF_EHIP; }

  try {
    cd* b64 = static_cast<cd*>(c->d_x64);
    cd* x64 = b64 + NR;
    cd* r64 = x64 + NR;
    cd* y64 = r64 + NR;
    const size_t ielt = c->elt;
    char* V = static_cast<char*>(c->d_krylov);
    const int64_t vstride = NR;  // elements between Krylov vectors
    auto Vj = [&](int j) { return static_cast<void*>(V + static_cast<size_t>(j) * NR * ielt); };
    void* w = c->d_w;
    void* z = c->d_vin;
    // small device state carved from d_small
    double* small = c->d_small;
    const int64_t per = gm_small_per_rhs(m);
    cd* h = reinterpret_cast<cd*>(small + per * R);
    cd* nrm2 = h + 256 * R;
    cd* ycoef = nrm2 + R;
    double* inv = reinterpret_cast<double*>(ycoef + 256 * R);
    double* resid = inv + R;
    double* target = resid + R;
    int* active = reinterpret_cast<int*>(target + R);
    cd* partial = reinterpret_cast<cd*>(c->d_red);
    const size_t plen = c->red_len / 2;

    chk(launch_to_internal(b, io == HBF_C128, b64, 1, N, R, s), "layout");
    chk(hipMemsetAsync(c->d_flag, 0, sizeof(int), s), "flag");
    chk(gm_nonfinite(true, b64, NR, c->d_flag, s), "check");
    int flag = 0;
    chk(hipMemcpyAsync(&flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, s), "flag");
    chk(hipStreamSynchronize(s), "sync");
    if (flag) throw Err{HBF_EINVAL, std::string(name) + ": non-finite value in the right-hand side"};
    bool x_zero = true;
    if (o.x0_given) {
      chk(launch_to_internal(x, io == HBF_C128, x64, 1, N, R, s), "layout");
      x_zero = false;
    } else {
      chk(gm_zero(x64, 2 * NR, s), "zero");
    }
    // ||b||
    chk(gm_dots(true, b64, vstride, 1, b64, N, R, partial, plen, nrm2, s), "norm");
    std::vector<cd> hn(R);
    chk(hipMemcpyAsync(hn.data(), nrm2, R * sizeof(cd), hipMemcpyDeviceToHost, s), "copy");
    chk(hipStreamSynchronize(s), "sync");
    std::vector<double> bnorm(R), relres(R, 1.0), tgt(R);
    for (int r = 0; r < R; ++r) bnorm[r] = std::sqrt(std::max(0.0, hn[r].x));
    std::vector<int> iters(R, 0), act(R);
    int total = 0, refine = 0;
    bool converged = false;
    for (;;) {
      // true residual r = b - A x in FP64
      if (x_zero) {
        chk(hipMemcpyAsync(r64, b64, NR * sizeof(cd), hipMemcpyDeviceToDevice, s), "copy");
      } else {
        chk(matvec_internal(c, x64, y64, R, true, adjoint, s), "residual matvec");
        chk(gm_sub64(b64, y64, r64, NR, s), "residual");
      }
      chk(gm_dots(true, r64, vstride, 1, r64, N, R, partial, plen, nrm2, s), "norm");
      chk(hipMemcpyAsync(hn.data(), nrm2, R * sizeof(cd), hipMemcpyDeviceToHost, s), "copy");
      chk(hipStreamSynchronize(s), "sync");
      bool all = true;
      for (int r = 0; r < R; ++r) {
        const double rn = std::sqrt(std::max(0.0, hn[r].x));
        relres[r] = bnorm[r] > 0 ? rn / bnorm[r] : 0.0;
        if (!(relres[r] <= tol)) all = false;
        // inner target: a fraction of the current residual, never below what the outer tolerance needs
        tgt[r] = (relres[r] <= tol) ? rn : std::max(inner_tol * rn, 0.5 * tol * bnorm[r]);
      }
      if (all) { converged = true; break; }
      if (total >= max_iters || refine >= max_refine + max_iters / m) break;
      // ---- one GMRES(m) cycle on A d = r ----
      chk(hipMemcpyAsync(target, tgt.data(), R * sizeof(double), hipMemcpyHostToDevice, s), "copy");
      chk(gm_cycle_start(small, m, R, nrm2, target, inv, resid, active, s), "cycle start");
      chk(gm_scale(true, r64, inv, inner128, Vj(0), N, R, s), "v0");
      chk(hipMemcpyAsync(act.data(), active, R * sizeof(int), hipMemcpyDeviceToHost, s), "copy");
      chk(hipStreamSynchronize(s), "sync");
      int used = 0;
      for (int j = 0; j < m; ++j) {
        std::vector<int> was = act;
        chk(precond_internal(c, Vj(j), z, R, adjoint, s), "preconditioner");
        chk(matvec_internal(c, z, w, R, inner128, adjoint, s), "matvec");
        for (int pass = 0; pass < 2; ++pass) {
          for (int i0 = 0; i0 <= j; i0 += 32)  // dot products in chunks of up to 32 basis vectors
            chk(gm_dots(inner128, Vj(i0), vstride, std::min(32, j + 1 - i0), w, N, R, partial, plen, h + i0 * R, s),
                "dots");
          chk(gm_sub_combo(inner128, V, vstride, j + 1, h, w, N, R, s), "orthogonalise");
          chk(gm_h_accum(small, m, R, j, h, s), "hessenberg");
        }
        chk(gm_dots(inner128, w, vstride, 1, w, N, R, partial, plen, nrm2, s), "norm");
        chk(gm_givens(small, m, R, j, nrm2, inv, resid, target, active, s), "givens");
        chk(gm_scale(inner128, w, inv, inner128, Vj(j + 1), N, R, s), "normalise");
        chk(hipMemcpyAsync(act.data(), active, R * sizeof(int), hipMemcpyDeviceToHost, s), "copy");
        chk(hipStreamSynchronize(s), "sync");
        ++total;
        used = j + 1;
        bool any = false;
        for (int r = 0; r < R; ++r) {
          if (was[r]) ++iters[r];
          any = any || act[r];
        }
        if (!any || total >= max_iters) break;
      }
      // d = M^{-1} (V y),  x += d
      chk(gm_lsq(small, m, R, ycoef, s), "least squares");
      chk(gm_combo(inner128, V, vstride, used, ycoef, w, N, R, s), "combine");
      chk(precond_internal(c, w, z, R, adjoint, s), "preconditioner");
      chk(gm_add_to64(inner128, z, x64, NR, s), "update");
      x_zero = false;
      ++refine;
    }
    chk(launch_to_external(x64, 1, x, io == HBF_C128, N, R, s), "layout");
    chk(hipStreamSynchronize(s), "sync");
    if (info) {
      for (int r = 0; r < R; ++r) {
        info[r].iters = iters[r];
        info[r].refinements = refine;
        info[r].converged = relres[r] <= tol ? 1 : 0;
        info[r].relres = relres[r];
      }
    }
    if (!converged) {
      set_error(std::string(name) + ": tolerance not reached within the iteration limit");
      return HBF_NOCONV;
    }
    return HBF_OK;
  } catch (const Err& e) {
    set_error(e.msg);
    (void)hipStreamSynchronize(s);
    return e.st;
  }
}

}  // namespace

extern "C" {

hbf_status hbf_solve(hbf_ctx* c, const void* b, void* x, int32_t nrhs, hbf_dtype io, const hbf_solve_opts* opts,
                     hbf_solve_info* info, void* stream) {
  return solve_impl(c, b, x, nrhs, io, opts, info, stream, false);
}

hbf_status hbf_solve_adjoint(hbf_ctx* c, const void* g, void* lam, int32_t nrhs, hbf_dtype io,
                             const hbf_solve_opts* opts, hbf_solve_info* info, void* stream) {
  return solve_impl(c, g, lam, nrhs, io, opts, info, stream, true);
}

}  // extern "C"
