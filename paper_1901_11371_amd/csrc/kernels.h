// Device kernels of the H-IDBF-LU hot path (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "hbf_internal.h"

namespace hbf {

template <class T>
struct cx {
  T x, y;
};
using cf = cx<float>;
using cd = cx<double>;

// Arguments of one launch of the stage kernel.
struct StageArgs {
  const Unit* units;
  const int32_t* gofs;    // group offsets (group-list launches)
  const int32_t* gunits;  // unit ids of the groups
  const void* fac;        // factor entries (storage dtype)
  const uint8_t* perm;    // permutations
  void* buf[3];           // BUF_X, BUF_Y, BUF_ARENA (vector dtype), rows x R
  int32_t first, direct;  // first group / unit, 1 = one unit per group
  int32_t R, rc, nchunks; // RHS count, RHS per workgroup, RHS chunks
  int32_t acc;            // 1: dst += alpha * result; 0: dst = result
  double alpha_re, alpha_im;
  int32_t ch;             // matrix chunk capacity (entries) in LDS
  int32_t src_cap;        // LDS source capacity (rows x rc entries)
  int32_t split = 1;      // 1: up to 32 lanes may share one output of a small unit (pipelined kernels)
  int32_t single = 0;     // 1: every group is one unit (lanes may then share an output)
  int32_t lv_rows = 0;    // program with LDS-resident vectors: LDS rows (0: vectors in memory)
  int32_t prow0 = 0, prows = 0;  // ... and its rows of the X and Y vectors
};

constexpr int kStageThreads = 256;
constexpr int kOutPerThread = 4;
constexpr int kProgWaves = 16;
constexpr int kProgThreads = 64 * kProgWaves;
constexpr int kProgOutPerThread = 4;
constexpr int kWaveOutPerThread = 4;

// Launch helpers (defined in stage.hip).  F: factor storage, V: vectors, A: accumulation.
hipError_t launch_stage_c64(const StageArgs& a, int ngroups, bool adjoint, size_t lds, hipStream_t s);
hipError_t launch_stage_c128(const StageArgs& a, int ngroups, bool adjoint, size_t lds, hipStream_t s);
hipError_t launch_stage_c64_hi(const StageArgs& a, int ngroups, bool adjoint, size_t lds, hipStream_t s);
// Software-pipelined wave teams (stage_pipe.hip): stage launches over
// ngroups groups x nchunks RHS chunks, and sweep programs.
int pipe_team_lds(int elt_acc, int elt_fac);
int prog_team_lds_lv(int elt_fac);
// Largest vector footprint (rows of elt_vec bytes) a sweep program can keep in
// LDS next to its staging areas.
int prog_lds_rows_budget(int elt_fac, int elt_vec);
// Resident-capacity queries of the stage kernels (call outside stream capture).
void prepare_launch_shapes();
hipError_t launch_pipe_c64(const StageArgs& a, int ngroups, int nchunks, bool adjoint, int max_blocks, hipStream_t s);
hipError_t launch_pipe_c128(const StageArgs& a, int ngroups, int nchunks, bool adjoint, int max_blocks, hipStream_t s);
hipError_t launch_pipe_c64_hi(const StageArgs& a, int ngroups, int nchunks, bool adjoint, int max_blocks,
                              hipStream_t s);
hipError_t launch_prog_pipe_c64(const StageArgs& a, const int32_t* steps, int s0, int s1, bool adjoint,
                                hipStream_t s);
hipError_t launch_prog_pipe_c128(const StageArgs& a, const int32_t* steps, int s0, int s1, bool adjoint,
                                 hipStream_t s);
// Many right-hand sides with complex64 factors and vectors: one wave per group,
// complex GEMMs on FP32 matrix cores (stage_mfma.hip).
// tiles: 16-RHS column tiles per wave (1, 2 or 4); mtiles: waves per group
// and RHS chunk, each taking every mtiles-th 16-row output tile (1: one wave
// takes them all)
hipError_t launch_stage_mfma_c64(const StageArgs& a, int ngroups, int tiles, int mtiles, bool adjoint,
                                 hipStream_t s);
// One right-hand side, forward, launches of single units: one lane per output;
// wave w covers units from wfirst[w] on, lane l of it the output named by
// lmap[64 w + l] ((unit offset) << 8 | row; 0xffff idle) in the role
// lrole[64 w + l] (kLane* bits below; nullptr: every lane kLaneWhole)
// (stage_lanes.hip).
hipError_t launch_lanes_c64(const StageArgs& a, const int32_t* wfirst, const uint16_t* lmap, const uint16_t* lrole,
                            int nwaves, hipStream_t s);
hipError_t launch_lanes_c64_hi(const StageArgs& a, const int32_t* wfirst, const uint16_t* lmap,
                               const uint16_t* lrole, int nwaves, hipStream_t s);
hipError_t launch_lanes_c128(const StageArgs& a, const int32_t* wfirst, const uint16_t* lmap, const uint16_t* lrole,
                             int nwaves, hipStream_t s);
// Lane roles.  Without kLaneSplit the lane computes its output row whole
// (role kLaneWhole).  A SCATTER row that is redundant in both IDs can be split
// over two lanes of one wave, each running the dot product of one ID: the
// owner (kLaneOwner) adds the skeleton entries and the partner's part (lane
// given in bits 8-13 when kLanePartner is set) and writes the row.
enum : uint16_t {
  kLaneDot0 = 1,
  kLaneDot1 = 2,
  kLaneOwner = 4,
  kLaneSplit = 8,
  kLanePartner = 0x4000,
  kLaneWhole = kLaneDot0 | kLaneDot1 | kLaneOwner,
};
// Wave-per-group variant (4 groups per workgroup, wave_lds bytes of LDS each).
hipError_t launch_stage_wave_c64(const StageArgs& a, int ngroups, int wave_lds, bool adjoint, hipStream_t s);
hipError_t launch_stage_wave_c128(const StageArgs& a, int ngroups, int wave_lds, bool adjoint, hipStream_t s);
hipError_t launch_stage_wave_c64_hi(const StageArgs& a, int ngroups, int wave_lds, bool adjoint, hipStream_t s);
// Sequential programs (sweeps over small subtrees): steps [s0, s1) of the
// step table (3 ints per step: first unit, end unit, accumulate flag), one
// workgroup per RHS chunk, wave_lds bytes of LDS per wave.
hipError_t launch_program_c64(const StageArgs& a, const int32_t* steps, int s0, int s1, int wave_lds, bool adjoint,
                              hipStream_t s);
hipError_t launch_program_c128(const StageArgs& a, const int32_t* steps, int s0, int s1, int wave_lds, bool adjoint,
                               hipStream_t s);

// (nrhs, N) external layout <-> (N, R) internal layout, with dtype conversion.
// The caller's N unknowns and the library's n >= N rows (device arrays; both
// null when n == N and the order is the identity): real_of[i] is the caller's
// index of library row i, or -1 for a padding row; lib_of[j] the library row
// of the caller's unknown j.
struct VecMap {
  int64_t n_int = 0, n_ext = 0;
  const int32_t* real_of = nullptr;
  const int32_t* lib_of = nullptr;
};
// (R, N) caller layout <-> (n, R) library layout with a dtype cast; padding
// rows of the library layout are written as zero.
hipError_t launch_to_internal(const void* ext, int ext_c128, void* in, int in_c128, const VecMap& m, int R,
                              hipStream_t s);
hipError_t launch_to_external(const void* in, int in_c128, void* ext, int ext_c128, const VecMap& m, int R,
                              hipStream_t s);

// Super-leaf factorisation in FP64 of super-leaves [S0, S0+nb): A holds their
// exact diagonal blocks (row-major ns x ns each, batch-local); the inverses of
// the lower and upper blocks of L~ / U~ are written as four unit sets at
// base[set] + S * per_superleaf (complex entries): per leaf row block, slabs
// of `slab` rows, each column-major slab x width.  work holds nb * 3 ns^2
// complex doubles.
struct SuperleafOut {
  int64_t base[4];
  int64_t per_superleaf;
  int32_t slab;
};
hipError_t launch_superleaf_factor(const cd* A, int64_t S0, int64_t nb, int ns, int n0, int mode, double sre,
                                  double sim, void* fac, int fac_c128, SuperleafOut so, int* flag, cd* work,
                                  hipStream_t s);

}  // namespace hbf
