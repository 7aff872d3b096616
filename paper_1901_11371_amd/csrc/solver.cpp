// Solve driver: a right-preconditioned Krylov method on A M^{-1} u = r
// (d = M^{-1} u, M the approximate LU preconditioner built from the
// triangular parts of A, Sec. 3.1) inside an iterative-refinement loop.
//
// Each outer step computes the true residual r = b - A x in FP64 (complex128
// vectors; with complex64 factors the factors are widened and accumulated in
// FP64), then runs one inner cycle on A d = r in the context precision and
// updates x += d in FP64:
//   * GMRES(m): restarted GMRES with classical Gram-Schmidt applied twice,
//     FP64 dot products and FP64 Hessenberg / Givens state;
//   * TFQMR: the transpose-free QMR method the paper solves with (Sec. 4),
//     which keeps no Krylov basis; a cycle runs until every right-hand side
//     meets its inner target (or the iteration budget ends).
// A cycle therefore restarts from the true residual, and the mixed-precision
// refinement recovers FP64 accuracy from complex64 inner solves.
//
// All right-hand sides advance in lockstep with per-RHS convergence masks on
// the device.  One Arnoldi step (preconditioner, matvec, two Gram-Schmidt
// passes, Givens update, normalisation) or one TFQMR iteration (two
// preconditioner applications and matvecs) is captured once as a HIP graph
// and replayed; the step index lives on the device.  The host reads the "any
// right-hand side still active" flag of step j only after step j + 1 is
// queued, so the device never waits for the host inside a cycle.
#include <algorithm>
#include <cmath>
#include <string>
#include <tuple>
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

// Carving of the context's small device state (d_small) for R right-hand
// sides and restart m.
struct SmallLayout {
  double* gm;       // GMRES per-RHS Hessenberg state
  cd* h;            // Gram-Schmidt coefficients [256][R]
  cd* nrm2;         // [R]
  cd* ycoef;        // [256][R]
  cd* dot;          // scratch dot products [R]
  double* inv;      // [R]
  double* resid;    // [R]
  double* target;   // [R]
  int* active;      // [R]
  int* iters;       // [R]
  void* tq;         // TFQMR state [R]
  int* jdev;        // step index
  int* any_active;  // OR of the masks after the last step
};

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

size_t carve(char* base, int m, int R, SmallLayout* L) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += align256(bytes);
    return p;
  };
  const size_t r = static_cast<size_t>(R);
  char* gm = take(static_cast<size_t>(gm_small_per_rhs(m)) * r * sizeof(double));
  char* h = take(256 * r * sizeof(cd));
  char* nrm2 = take(r * sizeof(cd));
  char* ycoef = take(256 * r * sizeof(cd));
  char* dot = take(r * sizeof(cd));
  char* inv = take(r * sizeof(double));
  char* resid = take(r * sizeof(double));
  char* target = take(r * sizeof(double));
  char* active = take(r * sizeof(int));
  char* iters = take(r * sizeof(int));
  char* tq = take(tq_state_bytes(R));
  char* ints = take(2 * sizeof(int));
  if (L) {
    L->gm = reinterpret_cast<double*>(gm);
    L->h = reinterpret_cast<cd*>(h);
    L->nrm2 = reinterpret_cast<cd*>(nrm2);
    L->ycoef = reinterpret_cast<cd*>(ycoef);
    L->dot = reinterpret_cast<cd*>(dot);
    L->inv = reinterpret_cast<double*>(inv);
    L->resid = reinterpret_cast<double*>(resid);
    L->target = reinterpret_cast<double*>(target);
    L->active = reinterpret_cast<int*>(active);
    L->iters = reinterpret_cast<int*>(iters);
    L->tq = tq;
    L->jdev = reinterpret_cast<int*>(ints);
    L->any_active = reinterpret_cast<int*>(ints) + 1;
  }
  return off;
}

// Everything one solve's kernels use.
struct Solve {
  hbf_ctx* c;
  int R, m;
  int64_t N, NR;
  bool adjoint, inner128;
  hipStream_t s;
  SmallLayout L;
  char* V;            // Krylov vectors (inner dtype)
  void* w;            // work vector
  void* z;            // preconditioned vector
  cd* partial;
  size_t plen;
  size_t ielt;
  void* Vj(int j) const { return V + static_cast<size_t>(j) * NR * ielt; }
};

// z = M^{-1} r for a vector in the context dtype: copy r to the sweeps' input
// and run them (no graph: the caller may be capturing).
void precond_into(const Solve& S, const void* r, void* z) {
  hbf_ctx* c = S.c;
  if (c->prec == HBF_PREC_NONE) {
    chk(gm_copy(S.inner128, r, z, S.NR, S.s), "copy");
    return;
  }
  chk(gm_copy(S.inner128, r, c->d_u, S.NR, S.s), "copy");
  chk(enqueue_sweeps(c, z, S.R, S.adjoint, S.s), "preconditioner");
}

// u = A M^{-1} y
void apply_am(const Solve& S, const void* y, void* u) {
  precond_into(S, y, S.z);
  chk(matvec_internal(S.c, S.z, u, S.R, S.inner128, S.adjoint, S.s), "matvec");
}

// One Arnoldi step j = *jdev: v = V_j; w = A M^{-1} v; two classical
// Gram-Schmidt passes against V_0..V_j (coefficients added into column j of
// H); H[j+1][j] = ||w||; Givens rotations; V_{j+1} = w / ||w||; j += 1.
void enqueue_arnoldi_step(const Solve& S) {
  hbf_ctx* c = S.c;
  const int* jd = S.L.jdev;
  if (c->prec == HBF_PREC_NONE) {
    chk(gm_copy_basis(S.inner128, S.V, S.NR, jd, S.z, S.NR, S.s), "basis");
  } else {
    chk(gm_copy_basis(S.inner128, S.V, S.NR, jd, c->d_u, S.NR, S.s), "basis");
    chk(enqueue_sweeps(c, S.z, S.R, S.adjoint, S.s), "preconditioner");
  }
  chk(matvec_internal(c, S.z, S.w, S.R, S.inner128, S.adjoint, S.s), "matvec");
  for (int pass = 0; pass < 2; ++pass) {
    chk(gm_dots_dev(S.inner128, S.V, S.NR, S.m, jd, S.w, S.N, S.R, S.partial, S.plen, S.L.h, S.s), "dots");
    chk(gm_sub_combo(S.inner128, S.V, S.NR, 0, jd, S.L.h, S.w, S.N, S.R, S.s), "orthogonalise");
    chk(gm_h_accum(S.L.gm, S.m, S.R, 0, jd, S.L.h, S.s), "hessenberg");
  }
  chk(gm_dots(S.inner128, S.w, S.NR, 1, S.w, S.N, S.R, S.partial, S.plen, S.L.nrm2, S.s), "norm");
  chk(gm_givens(S.L.gm, S.m, S.R, 0, jd, S.L.nrm2, S.L.inv, S.L.resid, S.L.target, S.L.active, S.s), "givens");
  chk(gm_scale(S.inner128, S.w, S.L.inv, S.inner128, S.V, S.NR, jd, S.N, S.R, S.s), "normalise");
  chk(gm_step_end(S.L.jdev, S.L.active, S.R, S.L.any_active, S.s), "step end");
}

// TFQMR vectors in the Krylov region
enum { TQ_W, TQ_Y, TQ_Y2, TQ_V, TQ_U, TQ_U2, TQ_D, TQ_X, TQ_RT, TQ_NVEC };

// One TFQMR iteration (two half steps) over all active right-hand sides.
void enqueue_tfqmr_iteration(const Solve& S) {
  void* W = S.Vj(TQ_W);
  void* Y = S.Vj(TQ_Y);
  void* Y2 = S.Vj(TQ_Y2);
  void* Vv = S.Vj(TQ_V);
  void* U = S.Vj(TQ_U);
  void* U2 = S.Vj(TQ_U2);
  void* D = S.Vj(TQ_D);
  void* X = S.Vj(TQ_X);
  void* RT = S.Vj(TQ_RT);
  const bool c128 = S.inner128;
  void* Q = S.L.tq;
  int* act = S.L.active;
  // alpha = rho / <rt, v>
  chk(gm_dots(c128, RT, S.NR, 1, Vv, S.N, S.R, S.partial, S.plen, S.L.dot, S.s), "dots");
  chk(tq_alpha(Q, S.R, S.L.dot, act, S.s), "alpha");
  // first half step
  chk(tq_e1(c128, Q, act, Y2, Y, Vv, W, U, D, S.N, S.R, S.s), "update");
  chk(gm_dots(c128, W, S.NR, 1, W, S.N, S.R, S.partial, S.plen, S.L.nrm2, S.s), "norm");
  chk(tq_half(Q, S.R, S.L.nrm2, S.L.resid, S.s), "half step");
  chk(tq_e2(c128, Q, act, X, D, S.N, S.R, S.s), "update");
  chk(tq_commit(Q, S.R, act, S.s), "masks");
  // second half step
  apply_am(S, Y2, U2);
  chk(tq_e3(c128, Q, act, W, U2, Y2, D, S.N, S.R, S.s), "update");
  chk(gm_dots(c128, W, S.NR, 1, W, S.N, S.R, S.partial, S.plen, S.L.nrm2, S.s), "norm");
  chk(tq_half(Q, S.R, S.L.nrm2, S.L.resid, S.s), "half step");
  chk(tq_e2(c128, Q, act, X, D, S.N, S.R, S.s), "update");
  chk(tq_commit(Q, S.R, act, S.s), "masks");
  // beta = <rt, w> / rho; y = w + beta y2; u = A M^{-1} y; v = u + beta (u2 + beta v)
  chk(gm_dots(c128, RT, S.NR, 1, W, S.N, S.R, S.partial, S.plen, S.L.dot, S.s), "dots");
  chk(tq_beta(Q, S.R, S.L.dot, act, S.s), "beta");
  chk(tq_e4(c128, Q, act, Y, W, Y2, S.N, S.R, S.s), "update");
  apply_am(S, Y, U);
  chk(tq_e5(c128, Q, act, Vv, U, U2, S.N, S.R, S.s), "update");
  chk(gm_step_end(nullptr, act, S.R, S.L.any_active, S.s), "step end");
}

// The captured graph of one step (kind 0: Arnoldi step, 1: TFQMR iteration),
// made on first use for this (kind, R, adjoint, m).
hipGraphExec_t step_graph(const Solve& S, int kind) {
  hbf_ctx* c = S.c;
  const auto key = std::make_tuple(kind, S.R, S.adjoint ? 1 : 0, kind == 0 ? S.m : 0);
  auto it = c->step_graphs.find(key);
  if (it != c->step_graphs.end()) return it->second;
  hipStream_t cs = nullptr;
  chk(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "graph stream");
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  std::string err;
  if (e == hipSuccess) {
    Solve S2 = S;
    S2.s = cs;
    try {
      if (kind == 0) enqueue_arnoldi_step(S2);
      else enqueue_tfqmr_iteration(S2);
    } catch (const Err& x) {
      err = x.msg;
    }
    e = hipStreamEndCapture(cs, &g);
  }
  if (e == hipSuccess && err.empty()) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  (void)hipStreamDestroy(cs);
  if (!err.empty()) throw Err{HBF_EHIP, "step capture: " + err};
  chk(e, "step graph");
  c->step_graphs.emplace(key, ge);
  return ge;
}

// Run up to `limit` steps; stop one step after the device reports that no
// right-hand side is active.  Returns the number of steps queued.
int run_steps(const Solve& S, int kind, int limit) {
  hbf_ctx* c = S.c;
  hipGraphExec_t ge = c->use_graphs ? step_graph(S, kind) : nullptr;
  int queued = 0;
  for (int j = 0; j < limit; ++j) {
    if (ge) chk(hipGraphLaunch(ge, S.s), "step launch");
    else if (kind == 0) enqueue_arnoldi_step(S);
    else enqueue_tfqmr_iteration(S);
    chk(hipMemcpyAsync(&c->h_flags[j & 1], S.L.any_active, sizeof(int), hipMemcpyDeviceToHost, S.s), "flag");
    chk(hipEventRecord(c->ev_step[j & 1], S.s), "event");
    ++queued;
    if (j >= 1) {
      chk(hipEventSynchronize(c->ev_step[(j - 1) & 1]), "event");
      if (c->h_flags[(j - 1) & 1] == 0) break;
    }
  }
  return queued;
}

hbf_status solve_impl(hbf_ctx* c, const void* b, void* x, int32_t nrhs, hbf_dtype io, const hbf_solve_opts* opts,
                      hbf_solve_info* info, void* stream, bool adjoint) {
  const char* name = adjoint ? "hbf_solve_adjoint" : "hbf_solve";
  if (!c || !b || !x) { set_error(std::string(name) + ": NULL argument"); return HBF_EINVAL; }
  if (nrhs < 1 || nrhs > c->max_nrhs) { set_error(std::string(name) + ": nrhs out of range"); return HBF_EINVAL; }
  if (io != HBF_C64 && io != HBF_C128) { set_error(std::string(name) + ": bad io dtype"); return HBF_EINVAL; }
  hbf_solve_opts o{};
  if (opts) o = *opts;
  if (o.method != HBF_GMRES && o.method != HBF_TFQMR) { set_error(std::string(name) + ": bad method"); return HBF_EINVAL; }
  const bool tfqmr = o.method == HBF_TFQMR;
  const double tol = o.tol > 0 ? o.tol : 1e-6;
  const int m = (o.restart > 0) ? std::min(o.restart, c->restart) : c->restart;
  if (m < 1 || m > 255) { set_error(std::string(name) + ": restart must be in [1, 255]"); return HBF_EINVAL; }
  const int max_iters = o.max_iters > 0 ? o.max_iters : 500;
  const int tq_cycle = o.restart > 0 ? o.restart : 250;
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
    Solve S;
    S.c = c;
    S.R = R;
    S.m = m;
    S.N = N;
    S.NR = NR;
    S.adjoint = adjoint;
    S.inner128 = inner128;
    S.s = s;
    carve(reinterpret_cast<char*>(c->d_small), m, R, &S.L);
    S.V = static_cast<char*>(c->d_krylov);
    S.w = c->d_w;
    S.z = c->d_vin;
    S.partial = reinterpret_cast<cd*>(c->d_red);
    S.plen = c->red_len / 2;
    S.ielt = c->elt;

    chk(launch_to_internal(b, io == HBF_C128, b64, 1, c->vmap, R, s), "layout");
    chk(gm_set_int(c->d_flag, 0, s), "flag");
    chk(gm_nonfinite(true, b64, NR, c->d_flag, s), "check");
    int flag = 0;
    chk(hipMemcpyAsync(&flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, s), "flag");
    chk(hipStreamSynchronize(s), "sync");
    if (flag) throw Err{HBF_EINVAL, std::string(name) + ": non-finite value in the right-hand side"};
    bool x_zero = true;
    if (o.x0_given) {
      chk(launch_to_internal(x, io == HBF_C128, x64, 1, c->vmap, R, s), "layout");
      x_zero = false;
    } else {
      chk(gm_zero(x64, 2 * NR, s), "zero");
    }
    // ||b||
    chk(gm_dots(true, b64, NR, 1, b64, N, R, S.partial, S.plen, S.L.nrm2, s), "norm");
    std::vector<cd> hn(R);
    chk(hipMemcpyAsync(hn.data(), S.L.nrm2, R * sizeof(cd), hipMemcpyDeviceToHost, s), "copy");
    chk(hipStreamSynchronize(s), "sync");
    std::vector<double> bnorm(R), relres(R, 1.0), tgt(R);
    for (int r = 0; r < R; ++r) bnorm[r] = std::sqrt(std::max(0.0, hn[r].x));
    std::vector<int> iters(R, 0), it_cycle(R);
    int total = 0, refine = 0;
    bool converged = false;
    for (;;) {
      // true residual r = b - A x in FP64
      if (x_zero) {
        chk(gm_copy(true, b64, r64, NR, s), "copy");
      } else {
        chk(matvec_internal(c, x64, y64, R, true, adjoint, s), "residual matvec");
        chk(gm_sub64(b64, y64, r64, NR, s), "residual");
      }
      chk(gm_dots(true, r64, NR, 1, r64, N, R, S.partial, S.plen, S.L.nrm2, s), "norm");
      chk(hipMemcpyAsync(hn.data(), S.L.nrm2, R * sizeof(cd), hipMemcpyDeviceToHost, s), "copy");
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
      chk(hipMemcpyAsync(S.L.target, tgt.data(), R * sizeof(double), hipMemcpyHostToDevice, s), "copy");
      int limit = max_iters - total;
      // complex64 TFQMR: its recurrence residual drifts from the true one
      // over long cycles (FP32 vectors), so a cycle ends after tq_cycle
      // iterations and the FP64 residual restarts it
      if (tfqmr && !inner128) limit = std::min(limit, tq_cycle);
      int steps = 0;
      if (!tfqmr) {
        // ---- one GMRES(m) cycle on A d = r ----
        chk(gm_cycle_start(S.L.gm, m, R, S.L.nrm2, S.L.target, S.L.inv, S.L.resid, S.L.active, s), "cycle start");
        chk(gm_scale(true, r64, S.L.inv, inner128, S.Vj(0), 0, nullptr, N, R, s), "v0");
        chk(gm_set_int(S.L.jdev, 0, s), "step index");
        steps = run_steps(S, 0, std::min(m, limit));
        // d = M^{-1} (V y),  x += d
        chk(gm_lsq(S.L.gm, m, R, S.L.ycoef, s), "least squares");
        chk(gm_combo(inner128, S.V, NR, steps, S.L.ycoef, S.w, N, R, s), "combine");
        chk(gm_read_iters(S.L.gm, m, R, S.L.iters, s), "iterations");
      } else {
        // ---- one TFQMR cycle on A d = r ----
        chk(tq_start(S.L.tq, R, S.L.nrm2, S.L.target, S.L.inv, S.L.resid, S.L.active, s), "cycle start");
        chk(tq_init(true, r64, S.L.inv, inner128, S.Vj(TQ_W), S.Vj(TQ_Y), S.Vj(TQ_RT), S.Vj(TQ_D), S.Vj(TQ_X), N, R,
                    s),
            "cycle start");
        apply_am(S, S.Vj(TQ_Y), S.Vj(TQ_U));
        chk(gm_copy(inner128, S.Vj(TQ_U), S.Vj(TQ_V), NR, s), "copy");
        chk(gm_dots(inner128, S.Vj(TQ_RT), NR, 1, S.Vj(TQ_W), N, R, S.partial, S.plen, S.L.dot, s), "dots");
        chk(tq_rho0(S.L.tq, R, S.L.dot, s), "cycle start");
        steps = run_steps(S, 1, limit);
        // d = M^{-1} (||r|| xhat)
        chk(tq_scales(S.L.tq, R, S.L.inv, s), "scale");
        chk(gm_scale(inner128, S.Vj(TQ_X), S.L.inv, inner128, S.w, 0, nullptr, N, R, s), "scale");
        chk(tq_iters(S.L.tq, R, S.L.iters, s), "iterations");
      }
      chk(precond_internal(c, S.w, S.z, R, adjoint, s), "preconditioner");
      chk(gm_add_to64(inner128, S.z, x64, NR, s), "update");
      chk(hipMemcpyAsync(it_cycle.data(), S.L.iters, R * sizeof(int), hipMemcpyDeviceToHost, s), "copy");
      chk(hipStreamSynchronize(s), "sync");
      for (int r = 0; r < R; ++r) iters[r] += it_cycle[r];
      total += steps;
      x_zero = false;
      ++refine;
    }
    chk(launch_to_external(x64, 1, x, io == HBF_C128, c->vmap, R, s), "layout");
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

namespace hbf {

size_t solver_small_bytes(int m, int R) { return carve(nullptr, m, R, nullptr); }

int solver_krylov_vectors(int m) { return std::max(m + 1, static_cast<int>(TQ_NVEC)); }

}  // namespace hbf

extern "C" {

hbf_status hbf_solve(hbf_ctx* c, const void* b, void* x, int32_t nrhs, hbf_dtype io, const hbf_solve_opts* opts,
                     hbf_solve_info* info, void* stream) {
  return solve_impl(c, b, x, nrhs, io, opts, info, stream, false);
}

hbf_status hbf_solve_adjoint(hbf_ctx* c, const void* g, void* lam, int32_t nrhs, hbf_dtype io,
                             const hbf_solve_opts* opts, hbf_solve_info* info, void* stream) {
  return solve_impl(c, g, lam, nrhs, io, opts, info, stream, true);
}

hbf_status hbf_impedance_grad(hbf_ctx* c, const void* lam, const void* x, int32_t nrhs, hbf_dtype io, void* grad_z,
                              void* stream) {
  if (!c || !lam || !x || !grad_z) { set_error("hbf_impedance_grad: NULL argument"); return HBF_EINVAL; }
  if (nrhs < 1) { set_error("hbf_impedance_grad: nrhs must be >= 1"); return HBF_EINVAL; }
  if (io != HBF_C64 && io != HBF_C128) { set_error("hbf_impedance_grad: bad io dtype"); return HBF_EINVAL; }
  if (hipSetDevice(c->device) != hipSuccess) { set_error("hipSetDevice"); return HBF_EHIP; }
  const hipError_t e = gm_impedance_grad(io == HBF_C128, lam, x, c->n_ext, nrhs, grad_z, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) { set_error(std::string("hbf_impedance_grad: ") + hipGetErrorString(e)); return HBF_EHIP; }
  return HBF_OK;
}

}  // extern "C"
