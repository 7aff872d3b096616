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
};

constexpr int kStageThreads = 256;
constexpr int kOutPerThread = 4;
constexpr int kProgWaves = 8;
constexpr int kProgThreads = 64 * kProgWaves;
constexpr int kProgOutPerThread = 4;
constexpr int kWaveOutPerThread = 4;

// Launch helpers (defined in stage.hip).  F: factor storage, V: vectors, A: accumulation.
hipError_t launch_stage_c64(const StageArgs& a, int ngroups, bool adjoint, size_t lds, hipStream_t s);
hipError_t launch_stage_c128(const StageArgs& a, int ngroups, bool adjoint, size_t lds, hipStream_t s);
hipError_t launch_stage_c64_hi(const StageArgs& a, int ngroups, bool adjoint, size_t lds, hipStream_t s);
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
hipError_t launch_to_internal(const void* ext, int ext_c128, void* in, int in_c128, int64_t n, int R, hipStream_t s);
hipError_t launch_to_external(const void* in, int in_c128, void* ext, int ext_c128, int64_t n, int R, hipStream_t s);

// Leaf factorisation in FP64 of leaves [b0, b0+nb): D (n0 x n0 blocks,
// column-major, complex double) -> inverses written to out (storage dtype) at
// out_fwd_off + b*stride (and out_bwd_off + b*stride for the second matrix of
// the point-wise reading).  work holds nb * 2 n0^2 complex doubles.
hipError_t launch_leaf_factor(const cd* D, int64_t b0, int64_t nb, int n0, int mode, double sre, double sim,
                              void* out, int out_c128, int64_t out_fwd_off, int64_t out_bwd_off,
                              int64_t stride, int* flag, cd* work, hipStream_t s);

}  // namespace hbf
