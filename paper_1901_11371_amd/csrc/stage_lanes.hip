// Stage launches of one right-hand side over small units, one lane per output.
//
// The factor chain's middle levels consist of hundreds of thousands of units
// of a few hundred matrix entries each (ranks around 9).  A kernel that gives
// a unit to a whole wave spends most of its instructions on the unit's
// bookkeeping (staging, guards, reductions), not on its data.  Here a wave
// takes a run of consecutive units whose outputs together fill its 64 lanes,
// and each lane computes one output row of one unit on its own (lane_unit.h).
// The permutation bytes and source entries a lane reads are shared by the
// lanes of its ID (one address per wave group), the matrices are read once.
// The host packs each launch into waves (a run of units with at most 64
// outputs in total, or a 64-row slice of a larger unit) and gives every lane
// its unit and row in a table, so a lane starts with two loads (its table
// entry, its unit's descriptor) and no scan.  A SCATTER row sums the dot
// products of both IDs where it is redundant in both; the host may give such a
// row two lanes, one per ID, so that no lane of the wave runs both loops
// while its neighbours wait (the owner lane adds its partner's part by a
// shuffle and writes the row).
#include "lane_unit.h"

namespace hbf {

namespace {

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <class V>
__device__ __forceinline__ V* buffer(const StageArgs& a, int i) {
  return reinterpret_cast<V*>(i == BUF_X ? a.buf[BUF_X] : (i == BUF_Y ? a.buf[BUF_Y] : a.buf[BUF_ARENA]));
}

// Output o of unit U (forward), one right-hand side, vectors in memory: the
// lane's part of it in its role (kLane* bits).
template <class F, class V, class A>
__device__ __forceinline__ cx<A> lane_value(const StageArgs& a, const Unit& U, int o, int role) {
  const lanes::Src<V> src{buffer<V>(a, U.in_buf), U.in_off[0], U.in_off[1], U.in_len[0]};
  const cx<F>* fac = reinterpret_cast<const cx<F>*>(a.fac);
  if (role & kLaneSplit) return lanes::scatter_part<F, A>(U, o, role, fac, a.perm, src);
  return lanes::unit_output<F, A>(U, o, fac, a.perm, src);
}

constexpr int kLaneWaves = 4;  // waves per workgroup

// Wave w takes the units from wfirst[w] on; lmap[64 w + lane] names the
// lane's output: (unit offset in the run) << 8 | output row, 0xffff = idle.
// SPLIT (launches with split SCATTER rows): lrole[64 w + lane] is the lane's
// role, and every lane of the wave takes part in the exchange of the split
// rows' partial sums; otherwise every lane computes its row whole.
template <class F, class V, class A, bool SPLIT>
__global__ void __launch_bounds__(64 * kLaneWaves) k_stage_lanes(StageArgs a, const int32_t* wfirst,
                                                                const uint16_t* lmap, const uint16_t* lrole,
                                                                int nwaves) {
  const int w = uni(static_cast<int>(blockIdx.x) * kLaneWaves + static_cast<int>(threadIdx.x >> 6));
  if (w >= nwaves) return;
  const int lane = threadIdx.x & 63;
  const int64_t e = static_cast<int64_t>(w) * 64 + lane;
  const int m = lmap[e];
  const int role = SPLIT ? lrole[e] : kLaneWhole;
  if (!SPLIT && m == 0xffff) return;
  cx<A> val{0, 0};
  Unit U{};
  if (m != 0xffff) {
    U = a.units[uni(wfirst[w]) + (m >> 8)];
    val = lane_value<F, V, A>(a, U, m & 0xff, role);
  }
  if constexpr (SPLIT) {
    const int from = (role & kLanePartner) ? (role >> 8) & 63 : lane;
    const A px = __shfl(val.x, from), py = __shfl(val.y, from);
    if (m == 0xffff || !(role & kLaneOwner)) return;
    if (role & kLanePartner) {
      val.x += px;
      val.y += py;
    }
  }
  const int o = m & 0xff;
  V* db = buffer<V>(a, U.out_buf);
  const int len_o = U.out_len[0];
  lanes::store<V, A>(db + (o < len_o ? U.out_off[0] + o : U.out_off[1] + (o - len_o)), val, a.acc, a.alpha_re,
                     a.alpha_im);
}

// lrole == nullptr: a launch without split rows
template <class F, class V, class A>
hipError_t launch_lanes(const StageArgs& a, const int32_t* wfirst, const uint16_t* lmap, const uint16_t* lrole,
                        int nwaves, hipStream_t s) {
  if (nwaves <= 0) return hipSuccess;
  const unsigned blocks = static_cast<unsigned>((nwaves + kLaneWaves - 1) / kLaneWaves);
  if (lrole)
    hipLaunchKernelGGL((k_stage_lanes<F, V, A, true>), dim3(blocks), dim3(64 * kLaneWaves), 0, s, a, wfirst, lmap,
                       lrole, nwaves);
  else
    hipLaunchKernelGGL((k_stage_lanes<F, V, A, false>), dim3(blocks), dim3(64 * kLaneWaves), 0, s, a, wfirst, lmap,
                       lrole, nwaves);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_lanes_c64(const StageArgs& a, const int32_t* wfirst, const uint16_t* lmap, const uint16_t* lrole,
                            int nwaves, hipStream_t s) {
  return launch_lanes<float, cf, float>(a, wfirst, lmap, lrole, nwaves, s);
}
hipError_t launch_lanes_c64_hi(const StageArgs& a, const int32_t* wfirst, const uint16_t* lmap,
                               const uint16_t* lrole, int nwaves, hipStream_t s) {
  return launch_lanes<float, cd, double>(a, wfirst, lmap, lrole, nwaves, s);
}
hipError_t launch_lanes_c128(const StageArgs& a, const int32_t* wfirst, const uint16_t* lmap, const uint16_t* lrole,
                             int nwaves, hipStream_t s) {
  return launch_lanes<double, cd, double>(a, wfirst, lmap, lrole, nwaves, s);
}

}  // namespace hbf
