// Device context of the H-IDBF-LU library.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <tuple>
#include <utility>
#include <vector>

#include "hbf_internal.h"
#include "kernels.h"
#include "schedule.h"

struct hbf_ctx {
  hbf::Plan P;       // host plan (factor entries released after upload)
  hbf::Sweeps S;
  hbf_dtype dtype = HBF_C64;
  hbf_prec prec = HBF_PREC_BLOCK_LU;
  int device = 0;
  int max_nrhs = 1;
  int restart = 30;
  int64_t n = 0;                // library rows (padded size)
  int64_t n_ext = 0;            // the caller's N
  int32_t* d_real_of = nullptr; // padding map on the device (null when n == N)
  int32_t* d_lib_of = nullptr;
  hbf::VecMap vmap;             // conversions between the caller's and the library layout
  bool padded() const { return n != n_ext; }
  int elt = 8;                 // bytes per factor entry
  bool wave_units = true;      // one wave per group for one- or two-RHS launches
  bool prog_pipe = true;       // pipelined wave teams in the sweep programs
  bool lane_split = true;      // pipelined kernels: several lanes share one output of a small unit
  bool sweep_rc1 = false;      // sweep stage launches above pipe_max_r: pipelined kernel, one RHS per chunk
  int sweep_pipe_max_r = 4;    // pipe_max_r for the sweeps' stage launches
  bool prog_lds = true;        // sweep programs keep their vectors in LDS where they fit
  bool mv_direct = true;       // matvec launches of single-unit groups run direct over unit copies
  int pipe_max_r = 4;          // stage launches with nrhs <= this use the pipelined wave teams
  bool mfma = true;            // complex64 stage launches with nrhs >= mfma_min_r run on the matrix cores
  int mfma_min_r = 8;
  int mfma_tiles = 4;          // 16-RHS tiles per wave of the matrix-core matvec launches (1, 2, 4)
  int sweep_mfma_tiles = 1;    // ... of the sweeps' matrix-core stage launches
  int mfma_split_rows = 2048;  // matrix-core launches of fewer waves: one wave per 16-row output tile
  int r1_max_blocks = 0;       // persistent grid size of the stage kernels (0: resident capacity)

  // device memory
  void* d_fac = nullptr;       // factors + leaf inverses (storage dtype)
  uint8_t* d_perm = nullptr;
  hbf::Unit* d_units = nullptr;
  int32_t* d_gofs = nullptr;
  int32_t* d_gunits = nullptr;
  int32_t* d_steps = nullptr;  // program steps of the sweeps
  hbf::Unit* d_punits = nullptr;  // unit copies of the programs with LDS-resident vectors
  hbf::Unit* d_lunits = nullptr;  // launch-order unit copies of the direct matvec launches
  int32_t* d_lwaves = nullptr;    // lane-per-output matvec launches: first unit of each wave
  uint16_t* d_lmap = nullptr;     // ... and each lane's unit offset and output row
  uint16_t* d_lrole = nullptr;    // ... and its role (kLane* bits)
  bool lane_units = true;      // one-RHS forward matvec launches of single units: one lane per output
  int lane_max_entries = 640;  // ... for launches whose units average at most this many matrix entries
  bool lane_scatter_split = true;  // SCATTER rows redundant in both IDs on two lanes
  std::vector<hbf::Launch> mv_fwd, mv_adj;  // matvec schedules as launched (mv_direct)
  void* d_arena = nullptr;     // skeleton vectors, arena_rows x max_nrhs x 16 bytes
  void* d_vin = nullptr;       // internal-layout vectors, n x max_nrhs x 16 bytes each
  void* d_vout = nullptr;
  void* d_u = nullptr;         // preconditioner work
  void* d_t = nullptr;
  void* d_pz = nullptr;        // preconditioner output of the captured graphs
  bool use_graphs = true;      // replay the preconditioner sweeps from captured HIP graphs
  std::map<std::pair<int, int>, hipGraphExec_t> pc_graphs;  // (nrhs, adjoint) -> graph
  // solver step graphs: (kind 0 Arnoldi step / 1 TFQMR iteration, nrhs, adjoint, restart) -> graph
  std::map<std::tuple<int, int, int, int>, hipGraphExec_t> step_graphs;
  int* h_flags = nullptr;      // pinned host copies of the "any RHS active" flag of the last two steps
  hipEvent_t ev_step[2] = {nullptr, nullptr};
  hbf::cd* d_diag64 = nullptr; // FP64 diagonal leaf blocks (with z), column-major
  int* d_flag = nullptr;
  // solver workspace
  void* d_krylov = nullptr;    // (restart+1) Krylov vectors, N x max_nrhs, inner dtype
  void* d_w = nullptr;         // one work vector (inner dtype)
  void* d_x64 = nullptr;       // FP64 outer vectors: x, r, b, d (N x max_nrhs each)
  double* d_red = nullptr;     // reduction scratch
  double* d_small = nullptr;   // per-RHS Krylov state (solver_small_bytes)
  size_t red_len = 0;

  std::vector<hbf::cd> diag_noz;  // host FP64 leaf blocks without z (for set_impedance)
  std::vector<hbf::cd> sl_noz;    // host FP64 super-leaf blocks without z (row-major)
  hbf_stats_t stats{};
  double build_seconds = 0;
  size_t workspace_bytes = 0;
};

namespace hbf {

// Run a schedule on the device.  vec_c128: vectors are complex128 (with
// complex64 factors this selects FP64 accumulation).  sweep: the launches
// belong to the preconditioner sweeps (their stage launches may run one RHS
// per chunk in the pipelined kernel whatever the RHS count).
// arena: skeleton-vector buffer of at least arena_rows x R x 16 bytes (NULL:
// the context's own).
hipError_t run_launches(hbf_ctx* c, const std::vector<Launch>& L, bool adjoint, void* X, void* Y, int R,
                        bool vec_c128, double alpha_re, double alpha_im, hipStream_t s, bool sweep = false,
                        void* arena = nullptr);

hbf_status matvec_internal(hbf_ctx* c, void* xin, void* yout, int R, bool vec_c128, bool adjoint, hipStream_t s,
                           void* arena = nullptr);
// The preconditioner sweeps on the context's work vectors: input in d_u
// (overwritten), output z (context dtype, internal layout).  Launches only,
// so the caller may capture them.
hipError_t enqueue_sweeps(hbf_ctx* c, void* zout, int R, bool adjoint, hipStream_t s);
// Device bytes of the solver's per-RHS state for restart m and R right-hand
// sides, and the number of Krylov-region vectors a solve needs.
size_t solver_small_bytes(int m, int R);
int solver_krylov_vectors(int m);
hbf_status precond_internal(hbf_ctx* c, const void* rin, void* zout, int R, bool adjoint, hipStream_t s);

}  // namespace hbf
