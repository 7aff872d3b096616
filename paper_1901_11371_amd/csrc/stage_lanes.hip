// Stage launches of one right-hand side over small units, one lane per output.
//
// The factor chain's middle levels consist of hundreds of thousands of units
// of a few hundred matrix entries each (ranks around 9).  A kernel that gives
// a unit to a whole wave spends most of its instructions on the unit's
// bookkeeping (staging, guards, reductions), not on its data.  Here a wave
// takes a run of consecutive units whose outputs together fill its 64 lanes,
// and each lane computes one output row of one unit on its own:
//   GATHER  (column-ID transfer, forward):  out_o[i] = src[perm_o[i]]
//           + sum_t T_o(i, t) src[perm_o[k_o + t]]; T_o column-major, so at
//           each t the lanes of one ID read consecutive entries;
//   SCATTER (row-ID transfer, forward):     out[p] = sum over the two IDs of
//           in_o[q] if q = invperm_o[p] < k_o, else sum_j T_o(j, q - k_o) in_o[j];
//   DENSE:  out[o] = sum_t M(o, t) src[t], column-major, lanes read rows of a column.
// The permutation bytes and source entries a lane reads are shared by the
// lanes of its ID (one address per wave group), the matrices are read once.
// The host packs each launch into waves (a run of units with at most 64
// outputs in total, or one larger unit whose outputs the lanes take in turn).
#include "kernels.h"

namespace hbf {

namespace {

template <class T>
__device__ __forceinline__ void mac(cx<T>& acc, cx<T> a, cx<T> b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
template <class A, class S>
__device__ __forceinline__ cx<A> widen(cx<S> v) {
  return cx<A>{static_cast<A>(v.x), static_cast<A>(v.y)};
}
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <class V>
__device__ __forceinline__ V* buffer(const StageArgs& a, int i) {
  return reinterpret_cast<V*>(i == BUF_X ? a.buf[BUF_X] : (i == BUF_Y ? a.buf[BUF_Y] : a.buf[BUF_ARENA]));
}

// Output o of unit U (forward), one right-hand side.
template <class F, class V, class A>
__device__ __forceinline__ void lane_output(const StageArgs& a, const Unit& U, int o) {
  const int type = U.type;
  const int k0 = U.k[0], k1 = U.k[1];
  const int len0 = U.in_len[0];
  const int f_in = len0 + U.in_len[1];
  const int f_out = U.out_len[0] + U.out_len[1];
  const int off0 = U.in_off[0], off1 = U.in_off[1];
  const V* sb = buffer<V>(a, U.in_buf);
  const cx<F>* fac = reinterpret_cast<const cx<F>*>(a.fac) + U.mat;
  const uint8_t* pp = a.perm + U.perm;
  auto src = [&](int s) -> cx<A> { return widen<A>(sb[s < len0 ? off0 + s : off1 + (s - len0)]); };
  cx<A> val{0, 0};
  if (type == UNIT_GATHER) {
    const int id = o < k0 ? 0 : 1;
    const int i = id ? o - k0 : o;
    const int k = id ? k1 : k0;
    const int r = f_in - k;
    const cx<F>* T = fac + (id ? k0 * (f_in - k0) : 0) + i;
    const uint8_t* pm = pp + id * f_in;
    val = src(pm[i]);
#pragma unroll 4
    for (int t = 0; t < r; ++t) mac(val, widen<A>(T[t * k]), src(pm[k + t]));
  } else if (type == UNIT_SCATTER) {
#pragma unroll
    for (int id = 0; id < 2; ++id) {
      const int k = id ? k1 : k0;
      const int r = f_out - k;
      const int q = pp[id * f_out + o];
      const int sbase = id ? k0 : 0;
      if (q < k) {
        const cx<A> v = src(sbase + q);
        val.x += v.x;
        val.y += v.y;
      } else {
        const cx<F>* T = fac + (id ? k0 * (f_out - k0) : 0) + (q - k);
#pragma unroll 4
        for (int j = 0; j < k; ++j) mac(val, widen<A>(T[j * r]), src(sbase + j));
      }
    }
  } else {
#pragma unroll 4
    for (int t = 0; t < f_in; ++t) mac(val, widen<A>(fac[t * f_out + o]), src(t));
  }
  V* db = buffer<V>(a, U.out_buf);
  const int len_o = U.out_len[0];
  V* dp = db + (o < len_o ? U.out_off[0] + o : U.out_off[1] + (o - len_o));
  if (a.acc) {
    const A are = static_cast<A>(a.alpha_re), aim = static_cast<A>(a.alpha_im);
    const cx<A> cu = widen<A>(*dp);
    val = cx<A>{cu.x + are * val.x - aim * val.y, cu.y + are * val.y + aim * val.x};
  }
  using VT = decltype(dp->x);
  *dp = V{static_cast<VT>(val.x), static_cast<VT>(val.y)};
}

constexpr int kLaneWaves = 4;  // waves per workgroup

// wfirst[w] .. wfirst[w + 1]: the units of wave w (indices into a.units).
template <class F, class V, class A>
__global__ void __launch_bounds__(64 * kLaneWaves) k_stage_lanes(StageArgs a, const int32_t* wfirst, int nwaves) {
  const int w = uni(static_cast<int>(blockIdx.x) * kLaneWaves + static_cast<int>(threadIdx.x >> 6));
  if (w >= nwaves) return;
  const int lane = threadIdx.x & 63;
  const int u0 = uni(wfirst[w]), u1 = uni(wfirst[w + 1]);
  // the lane's unit and output for outputs pbase + lane of the run
  int total = 0;
  for (int u = u0; u < u1; ++u) total += uni(a.units[u].out_len[0] + a.units[u].out_len[1]);
  for (int pbase = 0; pbase < total; pbase += 64) {
    const int p = pbase + lane;
    int mu = -1, mo = 0, off = 0;
    for (int u = u0; u < u1; ++u) {
      const int n = uni(a.units[u].out_len[0] + a.units[u].out_len[1]);
      if (p >= off && p < off + n) {
        mu = u;
        mo = p - off;
      }
      off += n;
    }
    if (mu >= 0) {
      const Unit U = a.units[mu];
      lane_output<F, V, A>(a, U, mo);
    }
  }
}

template <class F, class V, class A>
hipError_t launch_lanes(const StageArgs& a, const int32_t* wfirst, int nwaves, hipStream_t s) {
  if (nwaves <= 0) return hipSuccess;
  const unsigned blocks = static_cast<unsigned>((nwaves + kLaneWaves - 1) / kLaneWaves);
  hipLaunchKernelGGL((k_stage_lanes<F, V, A>), dim3(blocks), dim3(64 * kLaneWaves), 0, s, a, wfirst, nwaves);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_lanes_c64(const StageArgs& a, const int32_t* wfirst, int nwaves, hipStream_t s) {
  return launch_lanes<float, cf, float>(a, wfirst, nwaves, s);
}
hipError_t launch_lanes_c64_hi(const StageArgs& a, const int32_t* wfirst, int nwaves, hipStream_t s) {
  return launch_lanes<float, cd, double>(a, wfirst, nwaves, s);
}
hipError_t launch_lanes_c128(const StageArgs& a, const int32_t* wfirst, int nwaves, hipStream_t s) {
  return launch_lanes<double, cd, double>(a, wfirst, nwaves, s);
}

}  // namespace hbf
