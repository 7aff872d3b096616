// Internal data structures of the H-IDBF-LU library (host side and the layout
// shared with the device kernels).
#pragma once

#include <complex>
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "../../include/hbf.h"

namespace hbf {

using cplx = std::complex<double>;

cplx hankel2_0(double x);

void set_error(const std::string& msg);

// ---------------------------------------------------------------------------
// One "unit": a small dense operation of the factor chain of one butterfly
// block (or a dense leaf block).  All units are stored in one table that the
// device kernels read directly, so the layout is fixed (64 bytes).
//
// Forward semantics, with src = concatenation of the input segments and
// dst = concatenation of the output segments:
//   GATHER  (column-ID transfer, the V factors):   two IDs a, b with ranks
//           k[0], k[1] = out_len[0], out_len[1]:
//             out_o[i] = src[perm_o[i]] + sum_t T_o(i, t) src[perm_o[k_o + t]]
//           T_o is k_o x (n_src - k_o), stored column-major; perm_o has n_src
//           bytes (skeleton positions first).
//   SCATTER (row-ID transfer, the U factors):       two IDs with ranks
//           k[0], k[1] = in_len[0], in_len[1]:
//             dst += Lambda_o [I; T_o^T] in_o, i.e. for q = invperm_o[p]:
//             dst[p] += (q < k_o) ? in_o[q] : sum_j T_o(j, q - k_o) in_o[j]
//           T_o is k_o x (n_dst - k_o), stored row-major; invperm_o has n_dst
//           bytes.
//   DENSE   dst = M src, M n_dst x n_src stored column-major.
// Adjoint semantics swap the roles of the input and output segments and use
// conjugate-transposed matrices.
// ---------------------------------------------------------------------------
enum UnitType : uint8_t { UNIT_GATHER = 0, UNIT_SCATTER = 1, UNIT_DENSE = 2 };
enum BufId : uint8_t { BUF_X = 0, BUF_Y = 1, BUF_ARENA = 2 };

struct alignas(16) Unit {
  int64_t mat;         // offset (complex entries) of the unit's matrices in the factor array
  int64_t perm;        // byte offset of the unit's permutations
  int32_t in_off[2];   // row offsets of the input segments
  int32_t out_off[2];  // row offsets of the output segments
  int16_t in_len[2];   // lengths (0 = absent)
  int16_t out_len[2];
  int16_t k[2];        // ranks of the two IDs (GATHER/SCATTER)
  uint8_t type;
  uint8_t in_buf;      // BufId of the input segments
  uint8_t out_buf;     // BufId of the output segments
  uint8_t pad0;
  int32_t mat_len;     // complex entries of the unit's matrices (padded to even)
  int32_t pad1[3];
};
static_assert(sizeof(Unit) == 64, "Unit must be 64 bytes");

// Program step table entries: first unit, end unit, flags (1 accumulate,
// 2 forward mode, 4 all units are dense 8-row slabs with one input and one
// output segment, 8 those slabs widen with the unit index), first 16-entry
// granule of the step's matrices and the number of granules they span.
constexpr int kStepInts = 5;

// A launch of the stage kernel: a range of groups; a group is a list of units
// whose outputs cover the same rows and are summed (direct=1: each group is
// the single unit unit_begin + g).
struct Launch {
  int32_t direct;
  int32_t first;       // first group (or first unit when direct; first step of a program)
  int32_t count;       // number of groups (number of steps of a program)
  int32_t max_src;     // largest source length of any unit in the launch
  int32_t max_dst;
  int32_t max_mat;     // largest matrix (complex entries) of any unit
  int32_t max_in = 0;  // largest input length (forward orientation) of any unit
  int32_t max_out = 0; // largest output length (forward orientation) of any unit
  int32_t out_leaf;    // 1 if the launch writes rows of the external vector (uses alpha/beta)
  int32_t kind;        // 0 butterfly/dense, 1 leaf solve
  int32_t prog = 0;    // 1: a sequential program over steps [first, first+count) of the step table
  int32_t force_fwd = 0;  // 1: apply the units in forward mode even in an adjoint schedule
  int32_t single = 1;     // 1: every group is one unit (no accumulation across units)
  int32_t ucopy = 0;      // 1: direct over the device's launch-order unit copies
  // one-RHS forward launches of single units: the launch's waves of the
  // lane-per-output kernel (entries [lw_first, lw_first + lw_count) of the
  // context's wave tables; lw_count = 0: none)
  int32_t lw_first = 0, lw_count = 0;
  int32_t lw_mean = 0;    // mean matrix entries per unit of the launch
  int32_t lw_split = 0;   // 1: some lane of those waves has a split role
  // program kept in LDS (lv_rows > 0): its steps index the rewritten unit
  // copies of Sweeps::punits, whose vector segments are LDS rows: the
  // program's rows [prow0, prow0 + prows) of X at [0, prows), of Y at
  // [prows, 2 prows), and every skeleton segment it touches after them
  int32_t lv_rows = 0;
  int32_t prow0 = 0, prows = 0;
};
enum : uint8_t { BUF_LDS = 3 };  // a segment of a program's LDS-resident vectors



// Per-butterfly-block bookkeeping.
struct BlockInfo {
  int64_t row0, col0, n;
  int L, D;
  int hlevel;          // v (1-based); the pair is the diagonal node (v-1, pair)
  int64_t pair;
  int lower;           // 1: F21 (rows = second child), 0: F12
  // unit ranges of the 2D+1 block levels, in forward order
  std::vector<int32_t> lvl_begin, lvl_end;
};

// The whole host-side factorisation.
struct Plan {
  // problem.  Unknowns are stored in the library's order: N real unknowns
  // (the caller's) padded to n = n0 2^V.  The bisection of [0, N) into leaves
  // of at most n0 (first half ceil(m/2), the leaf partition of Algorithms 3
  // and 4) places real leaf b at the start of library leaf lib_leaf(b); the
  // other library rows are ghost unknowns with A = identity on them and no
  // coupling, so the library operator is A (+) I and its block
  // preconditioner P (+) I.  For N = n0 2^V the map is the identity.
  int64_t n = 0;                  // library size n0 2^V
  int64_t n_real = 0;             // the caller's N
  std::vector<int32_t> lib_of;    // real index -> library index (empty: identity)
  std::vector<uint8_t> ghost;     // per library index: 1 for a ghost unknown (empty: none)
  int n0 = 0;
  int V = 0;                 // log2(N / n0)
  double kappa = 0, eta0 = 0, tol = 0;
  std::vector<double> cx, cy, w;  // segment centres and lengths
  std::vector<cplx> z;            // per-unknown impedance (may be empty)
  cplx scale = 1.0;               // a = 1/A[i*,i*]

  // factors
  std::vector<Unit> units;
  std::vector<cplx> fac;          // all unit matrices, FP64
  std::vector<uint8_t> perm;      // all permutations
  int64_t arena_rows = 0;
  std::vector<BlockInfo> blocks;
  // dense units: diag_unit[b] (A_bb), l0_unit[pair at level V] (lower and upper)
  std::vector<int32_t> diag_unit;
  std::vector<int32_t> l0_lower_unit, l0_upper_unit;  // per pair of the last level
  // super-leaf solve units: super-leaf S of 2^sl leaves owns units
  // [sl_*[S], sl_*[S] + sl_units), one per slab of sl_slab rows of each leaf
  // row block; matrices are filled by the leaf factorisation (on the device,
  // or on the host for the checks)
  int sl = 2;
  int sl_slab = 8;                // rows of a super-leaf unit (a slab of a leaf row block)
  int sl_units = 0;               // units per super-leaf and set
  std::vector<int32_t> sl_fwd, sl_bwd, sl_adj_fwd, sl_adj_bwd;
  int64_t leaf_fac_begin = 0;     // first complex entry of the super-leaf region
  int64_t leaf_fac_len = 0;

  // matvec schedules (forward and adjoint): launches over group tables
  std::vector<int32_t> group_off, group_units;
  std::vector<Launch> mv_fwd, mv_adj;

  // stats
  int max_rank = 0;
  double sum_rank = 0;
  int64_t n_ids = 0;
  int64_t bytes_butterfly_c128 = 0, bytes_dense_c128 = 0;
  double build_seconds = 0;

  cplx entry(int64_t i, int64_t j) const;
  cplx self_entry(int64_t i) const;
  bool is_ghost(int64_t i) const { return !ghost.empty() && ghost[i]; }
  int64_t lib(int64_t i) const { return lib_of.empty() ? i : lib_of[i]; }
};

// A product of index sets whose kernel entries the construction needs:
// out[c * nrows + a] = swap ? entry(cols[c], rows[a]) : entry(rows[a], cols[c]).
// out == nullptr: the matrix is only needed by an IdJob and stays with the evaluator.
struct EntryJob {
  const int32_t* rows;
  int32_t nrows;
  const int32_t* cols;
  int32_t ncols;
  int32_t swap;
  cplx* out;
};

// The column ID of the matrix of entry job `job` (rows = samples, columns =
// candidates), computed like column_id: rank *k, pivot order perm (ncols
// bytes), interpolation matrix T (k x (ncols - k), row-major, at most
// ncols^2 / 4 entries).
struct IdJob {
  int32_t job;
  int32_t kmax;
  double eps;
  int32_t* k;
  uint8_t* perm;
  cplx* T;
};

// Batched evaluation of kernel entries (and optionally of the column IDs of
// some of the evaluated matrices) for the construction: prepare() once the
// plan's geometry, impedance and padding are final, then any number of eval()
// calls (each blocking until its outputs are written).
class EntryEval {
 public:
  virtual ~EntryEval() = default;
  virtual void prepare(const Plan& P) = 0;
  virtual void eval(const std::vector<EntryJob>& jobs, const std::vector<IdJob>& ids) = 0;
  void eval(const std::vector<EntryJob>& jobs) { eval(jobs, {}); }
};

// Column ID of the s x n matrix M (column-major, overwritten): k, perm, T as
// described for IdJob (plan.cpp).
void column_id_into(std::vector<cplx>& M, int s, int n, double eps, int kmax, int32_t* k, uint8_t* perm, cplx* T);

// The device evaluator (entries.hip): FP64 entries on the given HIP device.
std::unique_ptr<EntryEval> make_device_entry_eval(int device);

// Build the plan.  Throws std::runtime_error on invalid input.  With `eval`,
// the kernel entries of the ID samples and probes and of the dense blocks are
// evaluated through it in batches; the IDs themselves run on the host.
void build_plan(Plan& p, const hbf_curve* curve, double kappa, int leaf, double tol,
                const hbf_build_opts* opts, EntryEval* eval = nullptr);

// Host FP64 evaluation of the plan: y = A x or A^H x for nrhs vectors
// (x, y are (nrhs, N) complex128).
void plan_apply(const Plan& p, const cplx* x, cplx* y, int nrhs, bool adjoint);

// Add a group of units to a group table; returns the group index.
int32_t add_group(Plan& p, const std::vector<int32_t>& unit_ids);

// Number of worker threads for the construction.
int build_threads(const hbf_build_opts* opts);

}  // namespace hbf
