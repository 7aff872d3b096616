/*
 * hbf.h -- C ABI of the H-IDBF-LU library for MI355X (gfx950).
 *
 * The library builds the hierarchical interpolative-decomposition butterfly
 * factorisation (H-IDBF) of the 2D TM_z EFIE impedance matrix of an open PEC
 * curve (paper Sec. 3.1 entry formula; Algorithm 1 for the hierarchy; the
 * appendix's linear-scaling ID, LRCS, MSCS and recursive MSCS for each
 * off-diagonal block), and runs its per-iteration hot path on the GPU:
 *   - y = A x with the compressed operator (Algorithm 2),
 *   - z = P^{-1} r with the approximate LU preconditioner built from the
 *     triangular parts of A (Sec. 3.1, definitions of L~ and U~; block
 *     forward/back substitution, Algorithms 3 and 4),
 *   - restarted right-preconditioned GMRES with mixed-precision iterative
 *     refinement, for many right-hand sides at once, and its adjoint.
 *
 * Conventions (all entry points):
 *   - Unknowns: one pulse basis function per segment; segment i is the chord
 *     between nodes i and i+1 of the curve (curves concatenated in order).
 *     Any N > n0 (leaf size n0 = `leaf`): the leaves are the pieces of the
 *     bisection of [0, N) with first halves ceil(m/2) down to at most n0
 *     unknowns (the leaf partition of Algorithms 3 and 4).  Internally N is
 *     padded to n0 2^V with unknowns that are decoupled from the others
 *     (identity rows and columns); no padding is visible at the interface.
 *   - Vectors passed to matvec/precond/solve are DEVICE pointers owned by the
 *     caller, shape (nrhs, N), C-contiguous, interleaved re/im
 *     (complex64: 2 x float, complex128: 2 x double), i.e. torch's layout.
 *   - The operator is the unscaled physical A = Z + diag(z) (z = 0 unless an
 *     impedance is given).  The rescaling of Sec. 3.1 is internal.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).
 *     matvec and precond_apply are stream-ordered and asynchronous;
 *     solve / solve_adjoint return when the result is complete.
 *   - No exception crosses the ABI.  Every call returns an hbf_status; the
 *     text of the last error of the calling thread is hbf_last_error().
 *   - One context may be used by one stream at a time; calls that overlap on
 *     one context race on its workspace.
 *   - All workspace is allocated at build time, sized by max_nrhs; the hot
 *     calls (matvec, precond_apply, solve) allocate nothing on the device.
 */
#ifndef HBF_H
#define HBF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hbf_ctx hbf_ctx; /* opaque; owns every device buffer it uses */

typedef enum {
  HBF_OK = 0,
  HBF_NOCONV = 1,       /* warning: solve stopped at max_iters; outputs hold the best iterate */
  HBF_EINVAL = -1,      /* invalid argument (sizes, NaN input, nrhs > max_nrhs, ...) */
  HBF_ENOMEM = -2,      /* host or device allocation failed */
  HBF_EHIP = -3,        /* a HIP runtime call failed */
  HBF_ESINGULAR = -4,   /* a leaf block is singular to working precision */
  HBF_ESTATE = -5       /* call not valid in the context's state */
} hbf_status;

typedef enum { HBF_C64 = 0, HBF_C128 = 1 } hbf_dtype;

/* Preconditioner reading.
 * HBF_PREC_BLOCK_LU (default): P = (D + A_low) D^{-1} (D + A_up), D the exact
 *   n0 x n0 diagonal leaf blocks (leaf solves via FP64 partially pivoted LU).
 * HBF_PREC_PAPER_TRI: the paper's point-wise factors for the rescaled matrix,
 *   P = (I + a A_sl)(diag A + A_su), a = 1 / A[i*,i*], i* = argmax |A_ii|.
 * HBF_PREC_NONE: identity. */
typedef enum { HBF_PREC_BLOCK_LU = 0, HBF_PREC_PAPER_TRI = 1, HBF_PREC_NONE = 2 } hbf_prec;

/* Curves: host arrays.  Curve c owns nodes [node_off[c], node_off[c+1]),
 * node k at (xy[2k], xy[2k+1]).  Total segments = node_off[ncurves] - ncurves. */
typedef struct {
  int32_t ncurves;
  const int64_t* node_off; /* ncurves + 1 entries */
  const double* xy;        /* 2 * node_off[ncurves] doubles */
} hbf_curve;

typedef struct {
  hbf_dtype dtype;   /* factor storage: complex64 (FP32 accumulation) or complex128 */
  hbf_prec prec;     /* preconditioner reading (see above) */
  double eta0;       /* free-space impedance; <= 0 selects 376.730313668 */
  const double* z;   /* host, 2N doubles (interleaved), per-unknown impedance; NULL = 0 */
  int32_t max_nrhs;  /* largest nrhs of any later call; <= 0 selects 1 */
  int32_t restart;   /* GMRES restart length used to size the Krylov workspace; <= 0 selects 30 */
  int32_t device;    /* HIP device ordinal */
  int32_t nthreads;  /* host threads for the construction; <= 0 = all hardware threads */
  int32_t cache_plan; /* 1: keep this host factorisation in a one-entry process cache, so a later
                         build of the same curve/kappa/leaf/tol/preconditioner (any dtype) skips
                         the host construction; 0: no caching (a cache hit is still used) */
  int32_t superleaf;  /* leaf solves of the sweeps invert diagonal blocks of 2^superleaf leaves
                         exactly (2 or 3; <= 0 selects 2) */
  int32_t verbose;    /* 1: one progress line per construction phase and H-level on stderr */
  int32_t host_entries; /* hbf_build: 1 = evaluate the construction's kernel entries and IDs on the
                           host; 0 (default) = on the device, in batches: the entries of every ID's
                           first sample and probe, the dense and super-leaf blocks and the middle
                           couplings, and the column ID of every first sample (the probe checks and
                           any larger samples stay on the host).  hbf_plan_build: 2 = take the same
                           batched path, served on the host */
} hbf_build_opts;

/* Krylov method of the inner solves. */
typedef enum { HBF_GMRES = 0, HBF_TFQMR = 1 } hbf_method;

typedef struct {
  double tol;          /* relative residual target ||b - A x|| / ||b|| (<= 0: 1e-6) */
  int32_t restart;     /* GMRES restart length m (<= 0: build-time value; capped by it).  TFQMR
                          with complex64 inner vectors: the longest inner cycle (<= 0: 250), after
                          which the FP64 residual restarts it (the FP32 recurrence residual drifts
                          from the true residual over long cycles) */
  int32_t max_iters;   /* total inner GMRES iterations per solve (<= 0: 500) */
  int32_t max_refine;  /* outer refinement steps (<= 0: 10) */
  int32_t mixed;       /* 1: inner GMRES in complex64 with FP32 factors and FP64 Arnoldi,
                          outer FP64 residual + refinement; 0: everything in the ctx dtype */
  int32_t x0_given;    /* 1: x holds the initial guess on entry; 0: start from x = 0 */
  double inner_tol;    /* relative tolerance of each inner cycle (<= 0: 1e-4 when mixed) */
  int32_t method;      /* hbf_method: restarted GMRES(m) (default) or TFQMR (the paper's solver,
                          Sec. 4; no Krylov basis, two matvecs and preconditioner applications per
                          iteration) */
} hbf_solve_opts;

typedef struct {
  int32_t iters;        /* inner iterations, all cycles (GMRES: Arnoldi steps; TFQMR: iterations of
                           two operator applications each) */
  int32_t refinements;  /* outer refinement steps */
  int32_t converged;    /* 1 if relres <= tol */
  double relres;        /* final ||b - A x|| / ||b||, FP64 with the stored operator */
} hbf_solve_info;

typedef struct {
  int64_t n, leaf, levels;       /* N, n0, V (the leaf partition's depth) */
  int64_t n_blocks;              /* butterfly-compressed off-diagonal blocks */
  int64_t n_units;               /* small dense operations of one matvec */
  int32_t max_rank;              /* largest skeleton size of any ID */
  double mean_rank;              /* mean skeleton size over all IDs */
  int64_t bytes_butterfly;       /* bytes of the butterfly factors (T and S matrices) */
  int64_t bytes_dense;           /* bytes of dense diagonal + neighbour leaf blocks */
  int64_t bytes_index;           /* bytes of permutation / descriptor data read by a matvec */
  int64_t bytes_precond;         /* bytes of the leaf inverses */
  int64_t bytes_workspace;       /* device workspace (skeleton arena, Krylov basis, ...) */
  double build_seconds;          /* host construction + upload time */
  double scale_re, scale_im;     /* a = 1 / A[i*, i*] */
  /* Algorithmic bytes of one single-RHS application: every unit's matrices,
   * permutations and 64-byte descriptor once, plus the input and output
   * N-vectors in the context dtype.  Each further RHS adds 2 N-vectors. */
  int64_t apply_bytes_matvec;    /* y = A x (Algorithm 2) */
  int64_t apply_bytes_precond;   /* z = P^{-1} r (both sweeps, and s = D t in the block reading) */
  int64_t launches_matvec;       /* kernel launches of one matvec */
  int64_t arena_rows;            /* rows of skeleton vectors (sum of all ID ranks) per RHS */
  /* One preconditioner application is a chain of dependent steps (Algorithms
   * 3 and 4 are sequential over the diagonal tree): kernel launches, and the
   * steps inside them (a subtree program's steps are separated by workgroup
   * barriers; a stage launch is one step). */
  int64_t launches_precond;
  int64_t steps_precond;
  int64_t n_internal;            /* n0 2^V: N padded with decoupled unknowns (= N when N = n0 2^V) */
} hbf_stats_t;

/* Build the H-IDBF of A = Z + diag(z) for the curve at wavenumber `kappa`
 * (Sec. 3.1 entry formula; Algorithm 1; each off-diagonal block of size
 * N/2^v compressed by an IDBF with log2(N/n0) - v levels, appendix) with leaf
 * size `leaf` and relative ID tolerance `tol`, upload it, factor the leaf
 * blocks in FP64 on the GPU, and allocate all workspace.
 * On failure *out is NULL and nothing is leaked. */
hbf_status hbf_build(const hbf_curve* curve, double kappa, int32_t leaf, double tol,
                     const hbf_build_opts* opts, hbf_ctx** out);

/* Replace the per-unknown impedance z (host, 2N doubles) and refactor the
 * leaf blocks (the off-diagonal factors do not depend on z). */
hbf_status hbf_set_impedance(hbf_ctx* ctx, const double* z_host);

/* y = A x (adjoint = 0) or y = A^H x (adjoint = 1) with the compressed
 * operator (Algorithm 2; the adjoint traverses the factors in reverse order
 * with conjugate-transposed blocks).  `io` is the dtype of x and y; a
 * complex128 io on a complex64 context reads the complex64 factors and
 * accumulates in FP64.  x and y must not overlap. */
hbf_status hbf_matvec(hbf_ctx* ctx, const void* x, void* y, int32_t nrhs, hbf_dtype io,
                      int32_t adjoint, void* stream);

/* hbf_matvec without any device allocation or use of the context's
 * workspace, for callers that cannot allocate (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * kernels and results as hbf_matvec.  Its scratch (the skeleton vectors,
 * arena_rows x nrhs x 16 bytes, plus two (N, nrhs) layout buffers when
 * nrhs > 1) is one fixed 64 MiB array per device, held until the process
 * ends; a call that needs more returns HBF_EINVAL.  Every call on a device
 * shares that array, so calls that overlap on one device race. */
hbf_status hbf_matvec_noalloc(hbf_ctx* ctx, const void* x, void* y, int32_t nrhs, hbf_dtype io,
                              int32_t adjoint, void* stream);

/* z = P^{-1} r (adjoint = 0) or z = P^{-H} r (adjoint = 1): block forward
 * substitution over the lower part followed by block back substitution over
 * the upper part (Algorithms 3 and 4), with the leaf solves of the chosen
 * preconditioner reading.  io must equal the context dtype. */
hbf_status hbf_precond_apply(hbf_ctx* ctx, const void* r, void* z, int32_t nrhs, hbf_dtype io,
                             int32_t adjoint, void* stream);

/* Solve A x = b for nrhs right-hand sides (columns of the problem statement
 * A x = b of Sec. 3.1) by right-preconditioned restarted GMRES, with
 * mixed-precision iterative refinement when opts->mixed.  b and x are
 * device (nrhs, N) arrays of dtype io (complex128 recommended for mixed).
 * info (host, nrhs entries) may be NULL.  Returns HBF_NOCONV if any RHS
 * missed the tolerance (x then holds the best iterate). */
hbf_status hbf_solve(hbf_ctx* ctx, const void* b, void* x, int32_t nrhs, hbf_dtype io,
                     const hbf_solve_opts* opts, hbf_solve_info* info, void* stream);

/* Solve A^H lam = g (the adjoint system used for gradients), using the
 * adjoint operator and P^{-H} as right preconditioner. */
hbf_status hbf_solve_adjoint(hbf_ctx* ctx, const void* g, void* lam, int32_t nrhs, hbf_dtype io,
                             const hbf_solve_opts* opts, hbf_solve_info* info, void* stream);

/* grad_z = -sum_r lam_r (.) conj(x_r): the gradient of a real objective with
 * respect to the per-unknown impedance z of A = Z + diag(z), given the forward
 * solutions x = A^{-1} b and the adjoint solutions lam = A^{-H} g (A depends
 * on z only through its diagonal; Sec. 3.1 defines the system).  lam and x are
 * device (nrhs, N) arrays of dtype io; grad_z is a device array of N entries
 * of dtype io, overwritten.  Stream-ordered and asynchronous. */
hbf_status hbf_impedance_grad(hbf_ctx* ctx, const void* lam, const void* x, int32_t nrhs, hbf_dtype io,
                              void* grad_z, void* stream);

/* Set an execution parameter of the context (used by the autotuner; results
 * do not depend on them beyond rounding):
 *   "prog_levels"   subtrees of <= 2^value leaves are swept by one workgroup
 *                   program (0..12; default 5),
 *   "pipe_max_r"    stage launches with nrhs <= value use pipelined wave teams
 *                   (default 4),
 *   "prog_pipe"     1 = pipelined wave teams inside the sweep programs,
 *   "r1_max_blocks" persistent grid size (workgroups) of the pipelined and
 *                   one-RHS stage kernels; 0 = as many as the device holds at
 *                   once,
 *   "wave_units"    1 = one wave per unit for two-RHS stages,
 *   "lane_split"    1 = in the pipelined kernels, up to 32 lanes share the
 *                   dot product of one output of a unit with few outputs,
 *   "sweep_pipe_max_r"  as pipe_max_r, for the sweeps' stage launches
 *                   (default 4),
 *   "sweep_rc1"     1 = the sweeps' stage launches with nrhs > sweep_pipe_max_r
 *                   use the pipelined kernel with one RHS per workgroup chunk,
 *   "prog_lds"      1 = sweep programs whose vectors fit keep them in LDS
 *                   (default 1),
 *   "mv_direct"     1 = matvec stages of single-unit groups run over copies of
 *                   their unit descriptors in launch order (default 1),
 *   "lane_units"    1 = with one RHS, those forward stages give each lane one
 *                   output row of a run of units (default 1; needs mv_direct),
 *   "lane_max_entries"  ... for stages whose units average at most this many
 *                   matrix entries (default 640),
 *   "lane_scatter_split"  1 = in those stages, a row-ID transfer row that is
 *                   redundant in both IDs takes two lanes, one per ID's dot
 *                   product (default 1),
 *   "use_graphs"    1 = replay the preconditioner sweeps and the solvers' steps
 *                   from HIP graphs,
 *   "mfma"          1 = complex64 stage launches with nrhs >= mfma_min_r run
 *                   as complex GEMMs on the FP32 matrix cores (default 1),
 *   "mfma_min_r"    smallest nrhs for the matrix-core stage launches (default 8),
 *   "mfma_tiles"    right-hand sides per wave of the matvec's matrix-core
 *                   launches, in 16-column tiles: 1, 2 or 4 (default 4),
 *   "sweep_mfma_tiles"  the same for the sweeps' stage launches (default 1),
 *   "mfma_split_rows"  matrix-core launches of fewer than this many waves
 *                   (unit groups x RHS chunks) run the 16-row output tiles of
 *                   a group on parallel waves; bigger ones, or all with 0,
 *                   take a group's tiles in turn on one wave (default 2048).
 * Unknown keys or out-of-range values return HBF_EINVAL. */
hbf_status hbf_tune(hbf_ctx* ctx, const char* key, int64_t value);

/* Sizes and ranks of the built factorisation. */
hbf_status hbf_stats(const hbf_ctx* ctx, hbf_stats_t* out);

/* N of the context (-1 for NULL). */
int64_t hbf_size(const hbf_ctx* ctx);

/* Release every resource of the context (NULL is a no-op). */
void hbf_free(hbf_ctx* ctx);

/* Message of the last failed call on this thread ("" if none). */
const char* hbf_last_error(void);

/* ---- construction checks (host only, no GPU) --------------------------------
 * hbf_plan_* build the same host-side factorisation as hbf_build without
 * touching a GPU and evaluate it in FP64 on the host.  They exist so the
 * construction can be checked on machines without a GPU; no hot-path entry
 * point uses them. */
typedef struct hbf_plan hbf_plan;
hbf_status hbf_plan_build(const hbf_curve* curve, double kappa, int32_t leaf, double tol,
                          const hbf_build_opts* opts, hbf_plan** out);
/* y = A x (or A^H x) with the plan's factors in FP64; x, y host complex128 (nrhs, N). */
hbf_status hbf_plan_apply(const hbf_plan* plan, const double* x, double* y, int32_t nrhs,
                          int32_t adjoint);
/* z = P^{-1} r (or P^{-H} r) by the plan's sweep schedules in FP64 with host
 * leaf inverses; r, z host complex128 (nrhs, N). */
hbf_status hbf_plan_precond(const hbf_plan* plan, const double* r, double* z, int32_t nrhs,
                            int32_t adjoint);
/* Entries A[rows[a], cols[b]] from the library's own kernel evaluation
 * (host complex128, row-major nr x nc). */
hbf_status hbf_plan_entries(const hbf_plan* plan, const int64_t* rows, int64_t nr,
                            const int64_t* cols, int64_t nc, double* out);
hbf_status hbf_plan_stats(const hbf_plan* plan, hbf_stats_t* out);
void hbf_plan_free(hbf_plan* plan);
/* H0^(2)(x) = J0(x) - i Y0(x) by the library's own FP64 evaluation. */
void hbf_hankel2_0(const double* x, int64_t n, double* out /* 2n */);

#ifdef __cplusplus
}
#endif
#endif /* HBF_H */
