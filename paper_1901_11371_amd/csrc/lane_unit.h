// One output row of one unit of the factor chain, applied forward to one
// right-hand side by a single lane (the lane-per-output kernel of the matvec
// stages).  src[s] is source entry s of the unit (0 <= s < n_src, Src below).
//   GATHER  (column-ID transfer):  out_o[i] = src[perm_o[i]]
//           + sum_t T_o(i, t) src[perm_o[k_o + t]]; T_o is column-major, so at
//           each t the lanes of one ID read consecutive entries;
//   SCATTER (row-ID transfer):     out[p] = sum over the two IDs of in_o[q] if
//           q = invperm_o[p] < k_o, else sum_j T_o(j, q - k_o) in_o[j];
//   DENSE:  out[o] = sum_t M(o, t) src[t], column-major.
// scatter_part computes one lane's part of a SCATTER row split over two lanes.
#pragma once

#include "kernels.h"

namespace hbf {
namespace lanes {

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

// The source entries of a unit in memory: entry s < len0 is sb[off0 + s],
// entry s >= len0 is sb[off1 + s - len0].
template <class V>
struct Src {
  const V* sb;
  int off0, off1, len0;
  __device__ __forceinline__ V at(int s) const { return sb[s < len0 ? off0 + s : off1 + (s - len0)]; }
  // first entry of segment `id` (entries 0 .. len0-1 or len0 .. end)
  __device__ __forceinline__ const V* seg(int id) const { return sb + (id ? off1 : off0); }
};

// Dot product of k consecutive source entries [sbase, sbase + k) with the
// matrix entries T[0], T[stride], ...: when the range is one segment (a
// SCATTER ID's inputs are the skeleton of that ID, one segment each) the
// lane walks one pointer, otherwise it maps every index.
template <class F, class A, class V>
__device__ __forceinline__ void dot_range(cx<A>& val, const cx<F>* T, int stride, const Src<V>& src, int sbase,
                                          int k) {
  const bool one = sbase + k <= src.len0 || sbase >= src.len0;
  if (one) {
    const V* sp = sbase < src.len0 ? src.seg(0) + sbase : src.seg(1) + (sbase - src.len0);
#pragma unroll 4
    for (int j = 0; j < k; ++j) {
      mac(val, widen<A>(*T), widen<A>(sp[j]));
      T += stride;
    }
  } else {
#pragma unroll 4
    for (int j = 0; j < k; ++j) {
      mac(val, widen<A>(*T), widen<A>(src.at(sbase + j)));
      T += stride;
    }
  }
}

template <class F, class A, class V>
__device__ __forceinline__ cx<A> unit_output(const Unit& U, int o, const cx<F>* fac_all, const uint8_t* perm_all,
                                             const Src<V>& src) {
  const int type = U.type;
  const int k0 = U.k[0], k1 = U.k[1];
  const int f_in = U.in_len[0] + U.in_len[1];
  const int f_out = U.out_len[0] + U.out_len[1];
  const cx<F>* fac = fac_all + U.mat;
  const uint8_t* pp = perm_all + U.perm;
  cx<A> val{0, 0};
  if (type == UNIT_GATHER) {
    const int id = o < k0 ? 0 : 1;
    const int i = id ? o - k0 : o;
    const int k = id ? k1 : k0;
    const int r = f_in - k;
    const cx<F>* T = fac + (id ? k0 * (f_in - k0) : 0) + i;
    const uint8_t* pm = pp + id * f_in;
    const uint8_t* pr = pm + k;
    val = widen<A>(src.at(pm[i]));
#pragma unroll 4
    for (int t = 0; t < r; ++t) {
      mac(val, widen<A>(*T), widen<A>(src.at(pr[t])));
      T += k;
    }
  } else if (type == UNIT_SCATTER) {
#pragma unroll
    for (int id = 0; id < 2; ++id) {
      const int k = id ? k1 : k0;
      const int r = f_out - k;
      const int q = pp[id * f_out + o];
      const int sbase = id ? k0 : 0;
      if (q < k) {
        const cx<A> v = widen<A>(src.at(sbase + q));
        val.x += v.x;
        val.y += v.y;
      } else {
        dot_range<F, A>(val, fac + (id ? k0 * (f_out - k0) : 0) + (q - k), r, src, sbase, k);
      }
    }
  } else {
    dot_range<F, A>(val, fac + o, f_out, src, 0, f_in);
  }
  return val;
}

// The part of SCATTER output row o that a lane of role `role` (kLane* bits)
// computes when the row's two ID dot products may run on two lanes: the owner
// adds the row's skeleton entries (q < k) of both IDs, and a lane runs the dot
// product of at most one ID, so the lanes of a wave share one loop.
template <class F, class A, class V>
__device__ __forceinline__ cx<A> scatter_part(const Unit& U, int o, int role, const cx<F>* fac_all,
                                              const uint8_t* perm_all, const Src<V>& src) {
  const int k0 = U.k[0], k1 = U.k[1];
  const int f_out = U.out_len[0] + U.out_len[1];
  const uint8_t* pp = perm_all + U.perm;
  cx<A> val{0, 0};
  if (role & kLaneOwner) {
    const int q0 = pp[o], q1 = pp[f_out + o];
    if (q0 < k0) {
      const cx<A> v = widen<A>(src.at(q0));
      val.x += v.x;
      val.y += v.y;
    }
    if (q1 < k1) {
      const cx<A> v = widen<A>(src.at(k0 + q1));
      val.x += v.x;
      val.y += v.y;
    }
  }
  if (role & (kLaneDot0 | kLaneDot1)) {
    const int id = (role & kLaneDot0) ? 0 : 1;
    const int k = id ? k1 : k0;
    const int r = f_out - k;
    const int q = pp[id * f_out + o];
    dot_range<F, A>(val, fac_all + U.mat + (id ? k0 * (f_out - k0) : 0) + (q - k), r, src, id ? k0 : 0, k);
  }
  return val;
}

// dst = val (acc == 0) or dst + alpha val
template <class V, class A>
__device__ __forceinline__ void store(V* dp, cx<A> val, int acc, double alpha_re, double alpha_im) {
  if (acc) {
    const A are = static_cast<A>(alpha_re), aim = static_cast<A>(alpha_im);
    const cx<A> cu = widen<A>(*dp);
    val = cx<A>{cu.x + are * val.x - aim * val.y, cu.y + are * val.y + aim * val.x};
  }
  using VT = decltype(dp->x);
  *dp = V{static_cast<VT>(val.x), static_cast<VT>(val.y)};
}

}  // namespace lanes
}  // namespace hbf
