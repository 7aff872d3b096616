// Software-pipelined wave teams.  Most units of the H-IDBF factor chain are
// tiny (a few hundred matrix entries), so a kernel that loads a unit, waits,
// computes and only then loads the next one is bound by memory latency.  Here
// every wave is a team that walks over a list of work items (unit, matrix
// chunk); while it computes item i from LDS, the loads of item i+1 (sources,
// permutations and a 4 KB matrix chunk, into registers) are already in
// flight, and the descriptor of the unit after that is fetched one step
// earlier still.  Used for the matvec and sweep stages with few right-hand
// sides per team and for the sweep programs.
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "kernels.h"

namespace hbf {

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kPW = 4;                  // 16-byte words per lane per matrix chunk
constexpr int kChunkW = 64 * kPW;       // words per chunk (4 KB)
constexpr int kSrcPL = 4;               // source entries per lane (256 max)
constexpr int kPermPL = 8;              // permutation bytes per lane (512 max)
constexpr int kOpt = 4;                 // outputs per lane (256 max)
constexpr int kStepWin = 128;           // program steps staged in LDS at a time
constexpr int kDescMax = 64;            // unit descriptors per program step staged in LDS
constexpr int kPrefDist = 3;            // program steps the prefetch wave may run ahead
constexpr int kPrefSlots = 32;          // 128-byte lines per prefetch-wave lane and step
constexpr int kLook = kPrefDist > 2 ? kPrefDist : 2;  // steps read ahead of the current one
// Waves of a program workgroup: 16 with complex64 factors; 12 with complex128,
// whose wider registers would otherwise spill at 4 waves per SIMD.
template <class F>
constexpr int prog_waves() {
  return sizeof(F) == 4 ? 16 : 12;
}

template <class T>
__device__ __forceinline__ void cmac(cx<T>& acc, cx<T> a, cx<T> b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
template <class T>
__device__ __forceinline__ void cmac_conj(cx<T>& acc, cx<T> a, cx<T> b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
}
template <class A, class F>
__device__ __forceinline__ cx<A> up(cx<F> v) {
  return cx<A>{static_cast<A>(v.x), static_cast<A>(v.y)};
}
__device__ __forceinline__ int cdiv_pos(int a, int b) { return a <= 0 ? 0 : (a + b - 1) / b; }
__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Buffer i of the launch, selected by uniform branches (no runtime index into
// the argument array).
__device__ __forceinline__ void* bufp(const StageArgs& a, int i) {
  return i == BUF_X ? a.buf[BUF_X] : (i == BUF_Y ? a.buf[BUF_Y] : a.buf[BUF_ARENA]);
}

// Unit fields a team needs, in the team's own orientation (source/destination).
struct UDesc {
  int64_t mat, perm;
  int s_buf, s_off0, s_off1, s_len0, n_src;
  int d_buf, d_off0, d_off1, d_len0, n_dst;
  int type, k0, k1, f_in, f_out, mat_len, plen, nwords;
};

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni64(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane(static_cast<int>(v & 0xffffffff));
  const int hi = __builtin_amdgcn_readfirstlane(static_cast<int>(v >> 32));
  return (static_cast<int64_t>(hi) << 32) | static_cast<uint32_t>(lo);
}

template <bool ADJ, class F>
__device__ __forceinline__ UDesc read_desc(const Unit* U) {
  UDesc d;
  d.mat = U->mat;
  d.perm = U->perm;
  d.type = U->type;
  d.k0 = U->k[0];
  d.k1 = U->k[1];
  d.f_in = U->in_len[0] + U->in_len[1];
  d.f_out = U->out_len[0] + U->out_len[1];
  d.mat_len = U->mat_len;
  d.plen = (d.type == UNIT_GATHER) ? d.f_in : (d.type == UNIT_SCATTER) ? d.f_out : 0;
  d.nwords = (d.mat_len * static_cast<int>(sizeof(cx<F>)) + 15) / 16;
  if (!ADJ) {
    d.s_buf = U->in_buf; d.s_off0 = U->in_off[0]; d.s_off1 = U->in_off[1]; d.s_len0 = U->in_len[0];
    d.n_src = d.f_in;
    d.d_buf = U->out_buf; d.d_off0 = U->out_off[0]; d.d_off1 = U->out_off[1]; d.d_len0 = U->out_len[0];
    d.n_dst = d.f_out;
  } else {
    d.s_buf = U->out_buf; d.s_off0 = U->out_off[0]; d.s_off1 = U->out_off[1]; d.s_len0 = U->out_len[0];
    d.n_src = d.f_out;
    d.d_buf = U->in_buf; d.d_off0 = U->in_off[0]; d.d_off1 = U->in_off[1]; d.d_len0 = U->in_len[0];
    d.n_dst = d.f_in;
  }
  return d;
}

// A unit descriptor staged in LDS, moved to scalar registers.
__device__ __forceinline__ Unit unit_from_lds(const Unit* p) {
  const int* w = reinterpret_cast<const int*>(p);
  int v[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = uni(w[i]);
  Unit u;
  __builtin_memcpy(&u, v, sizeof(Unit));
  return u;
}

// The register slot of one prefetched work item.
template <class V>
struct Slot {
  u32x4 mw[kPW];
  V sv[kSrcPL];
  uint8_t pv[kPermPL];
};

// Team work list: groups g = first_group + team, + nteams, ...; a group is
// units [q0, q1) (direct or through the group table); an item is a
// (unit, matrix chunk) pair.  Units without matrix entries still form one item.
struct Cursor {
  int g, q, q1, c;  // group, unit position, end of the group's units, chunk
};

template <class F, class V, class A, bool ADJ>
__device__ __forceinline__ void issue_static(const StageArgs& a, const UDesc& d, int c, int lane, Slot<V>& s) {
  const u32x4* gm = reinterpret_cast<const u32x4*>(reinterpret_cast<const cx<F>*>(a.fac) + d.mat);
#pragma unroll
  for (int j = 0; j < kPW; ++j) {
    const int w = c * kChunkW + lane + 64 * j;
    if (w < d.nwords) s.mw[j] = __builtin_nontemporal_load(&gm[w]);
  }
  if (c == 0 && d.plen > 0) {
    const uint8_t* pp = a.perm + d.perm;
#pragma unroll
    for (int j = 0; j < kPermPL; ++j) {
      const int e = lane + 64 * j;
      if (e < 2 * d.plen) s.pv[j] = pp[e];
    }
  }
}

template <class F, class V, class A, bool ADJ>
__device__ __forceinline__ void issue_src(const StageArgs& a, const UDesc& d, int lane, int R, int r0, int nr,
                                          Slot<V>& s) {
  const V* sb = reinterpret_cast<const V*>(bufp(a, d.s_buf));
#pragma unroll
  for (int j = 0; j < kSrcPL; ++j) {
    const int e = lane + 64 * j;
    if (e < d.n_src * nr) {
      const int t = e / nr, rr = e - t * nr;
      const int row = (t < d.s_len0) ? d.s_off0 + t : d.s_off1 + (t - d.s_len0);
      s.sv[j] = sb[static_cast<int64_t>(row) * R + r0 + rr];
    }
  }
}

template <class F, class V, class A, bool ADJ>
__device__ __forceinline__ void issue(const StageArgs& a, const UDesc& d, int c, int lane, int R, int r0, int nr,
                                      Slot<V>& s) {
  issue_static<F, V, A, ADJ>(a, d, c, lane, s);
  if (c == 0) issue_src<F, V, A, ADJ>(a, d, lane, R, r0, nr, s);
}

// Stage the slot's item in LDS (sources and permutations for a unit's first
// chunk; SRC = false: the sources are read in place from LDS-resident vectors).
template <class F, class V, class A, bool SRC = true>
__device__ __forceinline__ void commit(const UDesc& d, int c, int lane, int nr, const Slot<V>& slot, cx<A>* s_src,
                                       uint8_t* s_p, uint8_t* s_q, u32x4* s_m4) {
  // The source and matrix staging areas have fixed sizes (64 kSrcPL entries,
  // kChunkW words), so every lane writes all of its slots: entries past the
  // item's data hold stale values that nothing reads, and no exec-masked
  // block per element is needed.
  if (c == 0) {
    if constexpr (SRC) {
#pragma unroll
      for (int j = 0; j < kSrcPL; ++j) s_src[lane + 64 * j] = up<A>(slot.sv[j]);
    }
#pragma unroll
    for (int j = 0; j < kPermPL; ++j) {
      const int e = lane + 64 * j;
      if (e < 2 * d.plen) {
        const int o = e >= d.plen ? 1 : 0, p = e - o * d.plen;
        s_p[o * 256 + p] = slot.pv[j];
        s_q[o * 256 + slot.pv[j]] = static_cast<uint8_t>(p);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < kPW; ++j) s_m4[lane + 64 * j] = slot.mw[j];
}

// Accumulate one item (a matrix chunk of one unit) into the lane's outputs.
// Lanes per output: with fewer than 64 outputs, P = 2^i lanes share one
// output's dot product (each takes every P-th term); write_dst reduces them.
// Only for items that are written on their own (`split`): the units of a
// group accumulate into the same registers and must agree on the mapping.
__device__ __forceinline__ int lanes_per_output_log2(int nout, bool split) {
  int lp = 0;
  if (split)
    while (lp < 5 && (nout << (lp + 1)) <= 64) ++lp;
  return lp;
}

// srcf(t, rr): source entry t of RHS rr of the unit (staged in LDS, or read
// in place from a program's LDS-resident vectors).
template <class F, class A, bool ADJ, class SrcF>
__device__ __forceinline__ void compute_item(const UDesc& d, int c, int lane, int nr, const SrcF& srcf,
                                             const uint8_t* s_p, const uint8_t* s_q, const cx<F>* s_mat,
                                             cx<A>* acc, bool split) {
  constexpr int kChunkE = kChunkW * 16 / static_cast<int>(sizeof(cx<F>));
  const int e0 = c * kChunkE;
  const int e1 = min(d.mat_len, e0 + kChunkE);
  const int type = d.type;
  const int k0 = d.k0, k1 = d.k1, f_in = d.f_in, f_out = d.f_out;
  const int lp = lanes_per_output_log2(d.n_dst * nr, split);
  const int P = 1 << lp;
  const int part = lane & (P - 1);
  const bool first_chunk = (c == 0) && part == 0;
  const bool whole = (c == 0) && d.mat_len <= kChunkE;  // the item holds all of the unit's matrices
#pragma unroll
  for (int j = 0; j < kOpt; ++j) {
    const int p = (P > 1) ? (lane >> lp) : lane + 64 * j;
    if (P > 1 && j > 0) break;
    if (p >= d.n_dst * nr) break;
    const int o = p / nr;
    const int rr = p - o * nr;
    cx<A> s = acc[j];
    auto S = [&](int t) -> cx<A> { return srcf(t, rr); };
    auto MAC = [&](int e, int t) {
      const cx<A> m = up<A>(s_mat[e - e0]);
      if (ADJ) cmac_conj(s, m, S(t));
      else cmac(s, m, S(t));
    };
    if (type == UNIT_DENSE) {
      if (!ADJ) {
        int tlo = 0, thi = f_in;
        if (!whole) {
          tlo = cdiv_pos(e0 - o, f_out);
          thi = min(f_in, cdiv_pos(e1 - o, f_out));
        }
        for (int t = tlo + part; t < thi; t += P) MAC(t * f_out + o, t);
      } else {
        const int base = o * f_out;
        const int ilo = max(0, e0 - base), ihi = min(f_out, e1 - base);
        for (int i = ilo + part; i < ihi; i += P) MAC(base + i, i);
      }
    } else if (type == UNIT_GATHER) {
      if (!ADJ) {
        const int id = (o < k0) ? 0 : 1;
        const int i = id ? o - k0 : o;
        const int k = id ? k1 : k0;
        const int r = f_in - k;
        const int base = id ? k0 * (f_in - k0) : 0;
        const uint8_t* pm = s_p + id * 256;
        if (first_chunk) {
          const cx<A> v = S(pm[i]);
          s.x += v.x;
          s.y += v.y;
        }
        int tlo = 0, thi = r;
        if (!whole) {
          tlo = cdiv_pos(e0 - base - i, k);
          thi = min(r, cdiv_pos(e1 - base - i, k));
        }
        for (int t = tlo + part; t < thi; t += P) MAC(base + t * k + i, pm[k + t]);
      } else {
#pragma unroll
        for (int id = 0; id < 2; ++id) {
          const int k = id ? k1 : k0;
          const int base = id ? k0 * (f_in - k0) : 0;
          const int sbase = id ? k0 : 0;
          const int qq = s_q[id * 256 + o];
          if (qq < k) {
            if (first_chunk) {
              const cx<A> v = S(sbase + qq);
              s.x += v.x;
              s.y += v.y;
            }
          } else {
            const int cb = base + (qq - k) * k;
            const int ilo = max(0, e0 - cb), ihi = min(k, e1 - cb);
            for (int i = ilo + part; i < ihi; i += P) MAC(cb + i, sbase + i);
          }
        }
      }
    } else {  // UNIT_SCATTER
      if (!ADJ) {
#pragma unroll
        for (int id = 0; id < 2; ++id) {
          const int k = id ? k1 : k0;
          const int r = f_out - k;
          const int base = id ? k0 * (f_out - k0) : 0;
          const int sbase = id ? k0 : 0;
          const int qq = s_p[id * 256 + o];
          if (qq < k) {
            if (first_chunk) {
              const cx<A> v = S(sbase + qq);
              s.x += v.x;
              s.y += v.y;
            }
          } else {
            const int t = qq - k;
            int jlo = 0, jhi = k;
            if (!whole) {
              jlo = cdiv_pos(e0 - base - t, r);
              jhi = min(k, cdiv_pos(e1 - base - t, r));
            }
            for (int jj = jlo + part; jj < jhi; jj += P) MAC(base + jj * r + t, sbase + jj);
          }
        }
      } else {
        const int id = (o < k0) ? 0 : 1;
        const int jj = id ? o - k0 : o;
        const int k = id ? k1 : k0;
        const int r = f_out - k;
        const int base = id ? k0 * (f_out - k0) : 0;
        const uint8_t* pm = s_q + id * 256;
        if (first_chunk) {
          const cx<A> v = S(pm[jj]);
          s.x += v.x;
          s.y += v.y;
        }
        const int rb = base + jj * r;
        const int tlo = max(0, e0 - rb), thi = min(r, e1 - rb);
        for (int t = tlo + part; t < thi; t += P) MAC(rb + t, pm[k + t]);
      }
    }
    acc[j] = s;
  }
}

// Write a finished unit's (or group's) destination and clear the accumulators
// (LVD: the destination rows are rows of a program's LDS-resident vectors lvv).
template <class V, class A, bool LVD = false>
__device__ __forceinline__ void write_dst(const StageArgs& a, const UDesc& d, int acc_mode, double alpha_re,
                                          double alpha_im, int lane, int R, int r0, int nr, cx<A>* acc,
                                          bool split, V* lvv = nullptr) {
  V* db = LVD ? lvv : reinterpret_cast<V*>(bufp(a, d.d_buf));
  const A are = static_cast<A>(alpha_re), aim = static_cast<A>(alpha_im);
  const int lp = lanes_per_output_log2(d.n_dst * nr, split);
  const int P = 1 << lp;
  if (P > 1) {
    for (int off = P / 2; off >= 1; off /= 2) {
      acc[0].x += __shfl_xor(acc[0].x, off);
      acc[0].y += __shfl_xor(acc[0].y, off);
    }
  }
#pragma unroll
  for (int j = 0; j < kOpt; ++j) {
    const int p = (P > 1) ? (lane >> lp) : lane + 64 * j;
    if (P > 1 && (j > 0 || (lane & (P - 1)) != 0)) {
      acc[j] = cx<A>{0, 0};
      continue;
    }
    if (p >= d.n_dst * nr) break;
    const int o = p / nr;
    const int rr = p - o * nr;
    const int row = (o < d.d_len0) ? d.d_off0 + o : d.d_off1 + (o - d.d_len0);
    V* dp = LVD ? &db[row] : &db[static_cast<int64_t>(row) * R + r0 + rr];
    cx<A> v = acc[j];
    if (acc_mode) {
      const cx<A> cu = up<A>(*dp);
      v = cx<A>{cu.x + are * v.x - aim * v.y, cu.y + are * v.y + aim * v.x};
    }
    using VT = decltype(dp->x);
    *dp = V{static_cast<VT>(v.x), static_cast<VT>(v.y)};
    acc[j] = cx<A>{0, 0};
  }
}

template <class F, class V, class A, bool ADJ>
__device__ void team_run(const StageArgs& a, int first_group, int ngroups, int team, int nteams, int lane,
                         unsigned char* lds, int R, int r0, int nr) {
  // LDS: src (256 complex A), perm 2x256, iperm 2x256, matrix chunk (kChunkW words)
  cx<A>* s_src = reinterpret_cast<cx<A>*>(lds);
  uint8_t* s_p = reinterpret_cast<uint8_t*>(s_src + 256);
  uint8_t* s_q = s_p + 512;
  u32x4* s_m4 = reinterpret_cast<u32x4*>(s_q + 512);
  const cx<F>* s_mat = reinterpret_cast<const cx<F>*>(s_m4);
  constexpr int kChunkE = kChunkW * 16 / static_cast<int>(sizeof(cx<F>));

  auto unit_of = [&](int q) -> const Unit* { return &a.units[uni(a.direct ? q : a.gunits[q])]; };
  auto group_range = [&](int gi, int& q0, int& q1) {
    const int g = first_group + gi;
    if (a.direct) {
      q0 = g;
      q1 = g + 1;
    } else {
      q0 = uni(a.gofs[g]);
      q1 = uni(a.gofs[g + 1]);
    }
  };

  int gi = team;
  if (gi >= ngroups) return;
  Cursor cur;
  cur.g = gi;
  group_range(gi, cur.q, cur.q1);
  cur.c = 0;
  UDesc d = read_desc<ADJ, F>(unit_of(cur.q));
  Slot<V> slot;
  issue<F, V, A, ADJ>(a, d, 0, lane, R, r0, nr, slot);
  // Direct launches: the descriptor of the team's next unit is fetched one
  // unit ahead by a vector load (lane l < 16 holds its dword l), so moving to
  // a unit waits on no scalar load; vector loads complete in order, so the
  // wait for an item's data never waits on this one.
  int vdesc = 0;
  auto load_vdesc = [&](int g) {
    if (g < ngroups && lane < 16) vdesc = reinterpret_cast<const int*>(a.units + first_group + g)[lane];
  };
  if (a.direct) load_vdesc(gi + nteams);

  cx<A> acc[kOpt];
#pragma unroll
  for (int j = 0; j < kOpt; ++j) acc[j] = cx<A>{0, 0};

  for (;;) {
    const int nch = d.nwords > 0 ? (d.nwords + kChunkW - 1) / kChunkW : 1;
    commit<F, V, A>(d, cur.c, lane, nr, slot, s_src, s_p, s_q, s_m4);
    wsync();
    // ---- advance the cursor and prefetch the next item ----
    Cursor nxt = cur;
    bool group_end = false;
    if (cur.c + 1 < nch) {
      nxt.c = cur.c + 1;
    } else if (cur.q + 1 < cur.q1) {
      nxt.q = cur.q + 1;
      nxt.c = 0;
    } else {
      group_end = true;
      nxt.g = cur.g + nteams;
      if (nxt.g < ngroups) {
        group_range(nxt.g, nxt.q, nxt.q1);
        nxt.c = 0;
      } else {
        nxt.q = -1;
      }
    }
    UDesc dn = d;
    if (nxt.q >= 0) {
      if (nxt.c == 0) {
        if (a.direct) {
          int w[16];
#pragma unroll
          for (int i = 0; i < 16; ++i) w[i] = __builtin_amdgcn_readlane(vdesc, i);
          Unit u;
          __builtin_memcpy(&u, w, sizeof(Unit));
          dn = read_desc<ADJ, F>(&u);
        } else {
          dn = read_desc<ADJ, F>(unit_of(nxt.q));
        }
      }
      issue<F, V, A, ADJ>(a, dn, nxt.c, lane, R, r0, nr, slot);
      if (a.direct && nxt.c == 0) load_vdesc(nxt.g + nteams);
    }
    const auto srcf = [&](int t, int rr) -> cx<A> { return s_src[t * nr + rr]; };
    compute_item<F, A, ADJ>(d, cur.c, lane, nr, srcf, s_p, s_q, s_mat, acc, (a.direct || a.single) && a.split);
    if (group_end)
      write_dst<V, A>(a, d, a.acc, a.alpha_re, a.alpha_im, lane, R, r0, nr, acc, (a.direct || a.single) && a.split);
    wsync();
    if (nxt.q < 0) break;
    cur = nxt;
    d = dn;
  }
}

// A dense 8-row slab unit (column-major 8 x w matrix, one input and one
// output segment, one RHS), forward: the wave streams the matrix straight into
// registers with coalesced 16-byte loads (lane l, load k: word l + 64 k, so a
// wave instruction reads one contiguous kilobyte), together with the matching
// input entries; lanes holding the same rows reduce by shuffles.
template <class F, class V, class A, bool LV>
__device__ __forceinline__ void slab_unit(const StageArgs& a, const UDesc& d, int lane, int R, int r0, V* lvv) {
  constexpr int EP = 16 / static_cast<int>(sizeof(cx<F>));  // complex entries per 16-byte word
  constexpr int G = 8 / EP;                                  // words per column
  constexpr int B = 4;                                       // words in flight per lane
  const u32x4* gm = reinterpret_cast<const u32x4*>(reinterpret_cast<const cx<F>*>(a.fac) + d.mat);
  const V* xb = LV ? lvv : reinterpret_cast<const V*>(bufp(a, d.s_buf));
  const int nw = d.n_src * G;
  cx<A> acc[EP];
#pragma unroll
  for (int q = 0; q < EP; ++q) acc[q] = cx<A>{0, 0};
  for (int k0 = 0; k0 < nw; k0 += 64 * B) {
    u32x4 m[B];
    V xv[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int wi = k0 + 64 * b + lane;
      if (wi < nw) {
        m[b] = __builtin_nontemporal_load(&gm[wi]);
        xv[b] = LV ? xb[d.s_off0 + wi / G] : xb[static_cast<int64_t>(d.s_off0 + wi / G) * R + r0];
      }
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int wi = k0 + 64 * b + lane;
      if (wi < nw) {
        const cx<A> x = up<A>(xv[b]);
        if constexpr (EP == 2) {
          cmac(acc[0], cx<A>{__uint_as_float(m[b][0]), __uint_as_float(m[b][1])}, x);
          cmac(acc[1], cx<A>{__uint_as_float(m[b][2]), __uint_as_float(m[b][3])}, x);
        } else {
          const double re = __hiloint2double(static_cast<int>(m[b][1]), static_cast<int>(m[b][0]));
          const double im = __hiloint2double(static_cast<int>(m[b][3]), static_cast<int>(m[b][2]));
          cmac(acc[0], cx<A>{static_cast<A>(re), static_cast<A>(im)}, x);
        }
      }
    }
  }
#pragma unroll
  for (int off = G; off < 64; off <<= 1) {
#pragma unroll
    for (int q = 0; q < EP; ++q) {
      acc[q].x += __shfl_xor(acc[q].x, off);
      acc[q].y += __shfl_xor(acc[q].y, off);
    }
  }
  if (lane < G) {
    V* db = LV ? lvv : reinterpret_cast<V*>(bufp(a, d.d_buf));
    using VT = decltype(db->x);
#pragma unroll
    for (int q = 0; q < EP; ++q) {
      const int row = d.d_off0 + EP * lane + q;
      db[LV ? static_cast<int64_t>(row) : static_cast<int64_t>(row) * R + r0] =
          V{static_cast<VT>(acc[q].x), static_cast<VT>(acc[q].y)};
    }
  }
}

// A sweep program run by one workgroup per RHS chunk: steps in order, each a
// range of independent units shared by the compute waves (unit
// u0 + wave + kCompute i, kCompute = prog_waves - 1).  The step table is staged in LDS in windows of
// kStepWin steps.  The last wave of the workgroup takes no units: it loads the
// descriptors of the first kDescMax units of step st + 2 into a ring of three
// LDS step buffers, and touches one dword of every 128-byte line of the
// matrices of the next kPrefDist steps so that they are in L2 when the compute
// waves ask for them (a wave's wait for its own operands would otherwise also
// wait for these loads).  A compute wave prefetches one item ahead: the next
// chunk, its next unit of the same step, or its first unit of the next step
// (also when it has nothing to do in the current one); the permutations and
// matrix chunk of that item are requested before the step barrier (they do
// not depend on the sweep), its sources only after.
template <class F, class V, class A, bool ADJ, bool NR1, bool LV>
__device__ void prog_run(const StageArgs& a, const int32_t* steps, int s0, int s1, int wave, int lane,
                         unsigned char* lds, int32_t* s_steps, Unit* ring, int* s_ctr, V* lvv, int R, int r0,
                         int nr) {
  constexpr int kCompute = prog_waves<F>() - 1;  // waves that take units; the last one prefetches
  const int tid = threadIdx.x;
  int w0 = s0;  // first step of the staged window
  auto load_window = [&](int from) {
    const int cnt = kStepInts * min(kStepWin, s1 - from);
    for (int e = tid; e < cnt; e += blockDim.x) s_steps[e] = steps[kStepInts * from + e];
  };
  auto st_u0 = [&](int st) { return uni(s_steps[kStepInts * (st - w0)]); };
  auto st_u1 = [&](int st) { return uni(s_steps[kStepInts * (st - w0) + 1]); };
  auto st_fl = [&](int st) { return uni(s_steps[kStepInts * (st - w0) + 2]); };
  auto st_g0 = [&](int st) { return uni(s_steps[kStepInts * (st - w0) + 3]); };
  auto st_ng = [&](int st) { return uni(s_steps[kStepInts * (st - w0) + 4]); };
  // window reload before step st: every wave has passed the previous step's
  // barrier, so no reads of the old window remain (uniform over the workgroup)
  auto maybe_reload = [&](int st) {
    if (st + kLook >= w0 + kStepWin && st + kLook < s1) {
      w0 = st;
      load_window(st);
      __syncthreads();
    }
  };
  // slab steps (one RHS) run through slab_unit: the compute waves claim their
  // units, widest first, from a counter in LDS that is cleared (behind one
  // extra barrier) at the start of the step; they take no lookahead item
  auto is_slab = [&](int st) { return NR1 && ((st_fl(st) >> 2) & 1); };
  load_window(s0);
  if constexpr (LV) {  // the program's rows of X and Y into LDS
    const V* X = reinterpret_cast<const V*>(a.buf[BUF_X]);
    const V* Y = reinterpret_cast<const V*>(a.buf[BUF_Y]);
    for (int e = tid; e < a.prows; e += blockDim.x) {
      lvv[e] = X[static_cast<int64_t>(a.prow0 + e) * R + r0];
      lvv[a.prows + e] = Y[static_cast<int64_t>(a.prow0 + e) * R + r0];
    }
  }
  __syncthreads();
  {  // ring slots of the first two steps
    for (int st = s0; st < min(s1, s0 + 2); ++st) {
      const int b0 = st_u0(st), nu = min(kDescMax, st_u1(st) - b0);
      if (tid < 4 * nu)
        reinterpret_cast<u32x4*>(ring + (st % 3) * kDescMax + (tid >> 2))[tid & 3] =
            reinterpret_cast<const u32x4*>(a.units + b0 + (tid >> 2))[tid & 3];
    }
  }
  __syncthreads();

  if (wave == kCompute) {
    // ---------------- prefetch wave ----------------
    constexpr int kLine = 128;
    const int64_t gbytes = 16 * static_cast<int64_t>(sizeof(cx<F>));
    const char* fac = reinterpret_cast<const char*>(a.fac);
    unsigned sink = 0;
    int pst = s0 + 1, pdone = 0;  // cursor: step and lines of it already touched
    for (int st = s0; st < s1; ++st) {
      maybe_reload(st);
      if (is_slab(st)) __syncthreads();
      u32x4 rv[4];
      int rcount = 0;
      if (st + 2 < s1) {
        const int b0 = st_u0(st + 2), nu = min(kDescMax, st_u1(st + 2) - b0);
        rcount = nu;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int e = lane + 64 * j;
          if (e < 4 * nu) rv[j] = reinterpret_cast<const u32x4*>(a.units + b0 + (e >> 2))[e & 3];
        }
      }
      if (pst <= st) {
        pst = st + 1;
        pdone = 0;
      }
      const int lim = min(s1 - 1, st + kPrefDist);
      int nl = pst <= lim ? static_cast<int>(st_ng(pst) * gbytes / kLine) : 0;
      int pv[kPrefSlots];
#pragma unroll
      for (int j = 0; j < kPrefSlots; ++j) {
        while (pst <= lim && pdone >= nl) {
          ++pst;
          pdone = 0;
          nl = pst <= lim ? static_cast<int>(st_ng(pst) * gbytes / kLine) : 0;
        }
        pv[j] = 0;
        if (pst <= lim) {
          const int line = pdone + lane;
          if (line < nl)
            pv[j] = *reinterpret_cast<const int*>(fac + st_g0(pst) * gbytes + static_cast<int64_t>(line) * kLine);
          pdone += 64;
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int e = lane + 64 * j;
        if (e < 4 * rcount)
          reinterpret_cast<u32x4*>(ring + ((st + 2) % 3) * kDescMax + (e >> 2))[e & 3] = rv[j];
      }
#pragma unroll
      for (int j = 0; j < kPrefSlots; ++j) sink ^= static_cast<unsigned>(pv[j]);
      __syncthreads();
    }
    if (a.R < 0) reinterpret_cast<unsigned*>(a.buf[BUF_X])[tid] = sink;  // never taken (R >= 1): keeps the loads
    return;
  }

  // ---------------- compute waves ----------------
  // (LV: no source staging; the wave's LDS starts with the permutations)
  cx<A>* s_src = reinterpret_cast<cx<A>*>(lds);
  uint8_t* s_p = LV ? reinterpret_cast<uint8_t*>(lds) : reinterpret_cast<uint8_t*>(s_src + 256);
  uint8_t* s_q = s_p + 512;
  u32x4* s_m4 = reinterpret_cast<u32x4*>(s_q + 512);
  const cx<F>* s_mat = reinterpret_cast<const cx<F>*>(s_m4);
  // descriptor of unit q of step st, in the orientation the step applies it in
  auto desc_at = [&](int q, int st) -> UDesc {
    const int i = q - st_u0(st);
    const int fl = st_fl(st);
    Unit u;
    if (i < kDescMax) u = unit_from_lds(&ring[(st % 3) * kDescMax + i]);
    else u = a.units[q];
    if (ADJ && ((fl >> 1) & 1)) return read_desc<false, F>(&u);
    return read_desc<ADJ, F>(&u);
  };
  bool have = false;       // the item (cq, cc) of step cst has been requested
  bool src_ready = false;  // ... including its sources
  int cq = 0, cc = 0, cst = s0;
  UDesc d{};
  Slot<V> slot;
  cx<A> acc[kOpt];
#pragma unroll
  for (int j = 0; j < kOpt; ++j) acc[j] = cx<A>{0, 0};
  for (int st = s0; st < s1; ++st) {
    maybe_reload(st);
    const int u0 = st_u0(st), u1 = st_u1(st), flags = st_fl(st);
    if (is_slab(st)) {
      if (tid == 0) *s_ctr = 0;
      __syncthreads();
      const bool rev = (flags >> 3) & 1;
      for (;;) {
        int idx = 0;
        if (lane == 0) idx = atomicAdd(s_ctr, 1);
        idx = uni(idx);
        if (idx >= u1 - u0) break;
        slab_unit<F, V, A, LV>(a, desc_at(rev ? u1 - 1 - idx : u0 + idx, st), lane, R, r0, lvv);
      }
    } else if (!have && u0 + wave < u1) {
      cq = u0 + wave;
      cc = 0;
      cst = st;
      d = desc_at(cq, st);
      issue_static<F, V, A, ADJ>(a, d, 0, lane, slot);
      have = true;
      src_ready = false;
    }
    while (have && cst == st) {
      if (!LV && cc == 0 && !src_ready) issue_src<F, V, A, ADJ>(a, d, lane, R, r0, nr, slot);
      const int nch = d.nwords > 0 ? (d.nwords + kChunkW - 1) / kChunkW : 1;
      commit<F, V, A, !LV>(d, cc, lane, nr, slot, s_src, s_p, s_q, s_m4);
      wsync();
      // next item
      int nq = cq, nc = cc + 1, nst = st;
      bool nhave = true;
      bool unit_end = false;
      if (nc >= nch) {
        unit_end = true;
        nc = 0;
        if (cq + kCompute < u1) {
          nq = cq + kCompute;
        } else if (st + 1 < s1 && !is_slab(st + 1) && st_u0(st + 1) + wave < st_u1(st + 1)) {
          nq = st_u0(st + 1) + wave;
          nst = st + 1;
        } else {
          nhave = false;
        }
      }
      UDesc dn = d;
      src_ready = false;
      if (nhave) {
        if (nc == 0) dn = desc_at(nq, nst);
        issue_static<F, V, A, ADJ>(a, dn, nc, lane, slot);
        if (!LV && nc == 0 && nst == st) {  // same step: its sources are final already
          issue_src<F, V, A, ADJ>(a, dn, lane, R, r0, nr, slot);
          src_ready = true;
        }
      }
      const bool fwd = ADJ && ((flags >> 1) & 1);
      if constexpr (LV) {
        const auto srcf = [&](int t, int) -> cx<A> {
          return up<A>(lvv[t < d.s_len0 ? d.s_off0 + t : d.s_off1 + (t - d.s_len0)]);
        };
        if (fwd) compute_item<F, A, false>(d, cc, lane, nr, srcf, s_p, s_q, s_mat, acc, a.split);
        else compute_item<F, A, ADJ>(d, cc, lane, nr, srcf, s_p, s_q, s_mat, acc, a.split);
      } else {
        const auto srcf = [&](int t, int rr) -> cx<A> { return s_src[t * nr + rr]; };
        if (fwd) compute_item<F, A, false>(d, cc, lane, nr, srcf, s_p, s_q, s_mat, acc, a.split);
        else compute_item<F, A, ADJ>(d, cc, lane, nr, srcf, s_p, s_q, s_mat, acc, a.split);
      }
      if (unit_end) {
        const double are = (flags & 1) ? a.alpha_re : 0.0, aim = (flags & 1) ? a.alpha_im : 0.0;
        write_dst<V, A, LV>(a, d, flags & 1, are, aim, lane, R, r0, nr, acc, a.split, lvv);
      }
      wsync();
      have = nhave;
      cq = nq;
      cc = nc;
      cst = nst;
      d = dn;
    }
    // a wave without work in this step requests its first item of the next one
    if (!have && st + 1 < s1 && !is_slab(st + 1) && st_u0(st + 1) + wave < st_u1(st + 1)) {
      cq = st_u0(st + 1) + wave;
      cc = 0;
      cst = st + 1;
      d = desc_at(cq, st + 1);
      issue_static<F, V, A, ADJ>(a, d, 0, lane, slot);
      have = true;
      src_ready = false;
    }
    __syncthreads();
  }
  if constexpr (LV) {  // the program's rows of X and Y back to memory (every step has passed its barrier)
    V* X = reinterpret_cast<V*>(a.buf[BUF_X]);
    V* Y = reinterpret_cast<V*>(a.buf[BUF_Y]);
    for (int e = tid; e < a.prows; e += kCompute * 64) {
      X[static_cast<int64_t>(a.prow0 + e) * R + r0] = lvv[e];
      Y[static_cast<int64_t>(a.prow0 + e) * R + r0] = lvv[a.prows + e];
    }
  }
}

// Stage launch: teams = waves; team t handles groups t, t + nteams, ... for RHS chunk `chunk`.
// NR1: every RHS chunk holds one right-hand side (nr == 1 at compile time).
template <class F, class V, class A, bool ADJ, bool NR1>
__global__ void __launch_bounds__(256) k_stage_pipe(StageArgs a, int ngroups, int team_lds) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int chunk = blockIdx.y;
  const int r0 = chunk * a.rc;
  const int nr = NR1 ? 1 : min(a.rc, a.R - r0);
  const int team = blockIdx.x * 4 + wave;
  const int nteams = gridDim.x * 4;
  team_run<F, V, A, ADJ>(a, a.first, ngroups, team, nteams, lane, smem + static_cast<size_t>(wave) * team_lds, a.R,
                         r0, nr);
}

// Sweep program kernel: one workgroup per RHS chunk.
template <class F, class V, class A, bool ADJ, bool NR1, bool LV>
__global__ void __launch_bounds__(64 * prog_waves<F>()) k_program_pipe(StageArgs a, const int32_t* steps, int s0, int s1,
                                                                  int team_lds) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int chunk = blockIdx.x;
  const int r0 = chunk * a.rc;
  const int nr = NR1 ? 1 : min(a.rc, a.R - r0);
  Unit* ring = reinterpret_cast<Unit*>(smem + static_cast<size_t>(prog_waves<F>()) * team_lds);
  int32_t* s_steps = reinterpret_cast<int32_t*>(ring + 3 * kDescMax);
  int* s_ctr = reinterpret_cast<int*>(s_steps + kStepInts * kStepWin);
  V* lvv = reinterpret_cast<V*>(s_ctr + 4);
  prog_run<F, V, A, ADJ, NR1, LV>(a, steps, s0, s1, wave, lane, smem + static_cast<size_t>(wave) * team_lds, s_steps,
                                  ring, s_ctr, lvv, a.R, r0, nr);
}

}  // namespace

int pipe_team_lds(int elt_acc, int elt_fac) {
  (void)elt_fac;
  return 256 * elt_acc + 1024 + kChunkW * 16;
}

// Per-wave LDS of a program with LDS-resident vectors (no source staging).
int prog_team_lds_lv(int elt_fac) {
  (void)elt_fac;
  return 1024 + kChunkW * 16;
}

int prog_lds_rows_budget(int elt_fac, int elt_vec) {
  const int waves = elt_fac == 8 ? prog_waves<float>() : prog_waves<double>();
  const int base = prog_team_lds_lv(elt_fac) * waves + 3 * kDescMax * static_cast<int>(sizeof(Unit)) +
                   kStepInts * static_cast<int>(sizeof(int32_t)) * kStepWin + 16;
  return (160 * 1024 - base) / elt_vec;
}

// Workgroups of `kernel` the device holds at once (every CU filled to the
// occupancy its registers and `lds` bytes of LDS allow).
static int resident_blocks(const void* kernel, int block, size_t lds) {
  static std::mutex mu;
  static std::map<std::tuple<const void*, size_t, int, int>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  const auto key = std::make_tuple(kernel, lds, block, dev);
  std::lock_guard<std::mutex> lk(mu);
  const auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, lds) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  const int n = per_cu * cus;
  cache[key] = n;
  return n;
}

// max_blocks > 0 caps the grid's x size; 0 sizes it to the resident capacity
// (the teams are persistent: a second partial round of workgroups would only
// start once the first round has finished its share).
template <class F, class V, class A>
static void (*pipe_kernel(bool adjoint, bool nr1))(StageArgs, int, int) {
  return adjoint ? (nr1 ? k_stage_pipe<F, V, A, true, true> : k_stage_pipe<F, V, A, true, false>)
                 : (nr1 ? k_stage_pipe<F, V, A, false, true> : k_stage_pipe<F, V, A, false, false>);
}

template <class F, class V, class A>
static int pipe_lds1() {
  return pipe_team_lds(static_cast<int>(sizeof(cx<A>)), static_cast<int>(sizeof(cx<F>)));
}

// Occupancy queries of every stage-kernel variant, made outside any stream
// capture (a query is not a stream operation, but it need not run while a
// graph is being recorded).
template <class F, class V, class A>
static void prepare_pipe() {
  for (int v = 0; v < 4; ++v)
    resident_blocks(reinterpret_cast<const void*>(pipe_kernel<F, V, A>(v & 1, v >> 1)), 256,
                    static_cast<size_t>(pipe_lds1<F, V, A>()) * 4);
}

template <class F, class V, class A>
static hipError_t launch_pipe(const StageArgs& a, int ngroups, int nchunks, bool adjoint, int max_blocks,
                              hipStream_t s) {
  const int lds1 = pipe_lds1<F, V, A>();
  const bool nr1 = a.rc == 1;
  void (*kern)(StageArgs, int, int) = pipe_kernel<F, V, A>(adjoint, nr1);
  int cap = max_blocks;
  if (cap <= 0) {
    const int res = resident_blocks(reinterpret_cast<const void*>(kern), 256, static_cast<size_t>(lds1) * 4);
    cap = res > 0 ? std::max(1, res / std::max(1, nchunks)) : 2048;
  }
  int bx = (ngroups + 3) / 4;
  if (bx > cap) bx = cap;
  if (bx < 1) bx = 1;
  const dim3 grid(static_cast<unsigned>(bx), static_cast<unsigned>(nchunks));
  hipLaunchKernelGGL(kern, grid, dim3(256), lds1 * 4, s, a, ngroups, lds1);
  return hipGetLastError();
}

template <class F, class V, class A>
static hipError_t launch_prog_pipe(const StageArgs& a, const int32_t* steps, int s0, int s1, bool adjoint,
                                   hipStream_t s) {
  const bool lv = a.lv_rows > 0;
  const int lds1 = lv ? prog_team_lds_lv(static_cast<int>(sizeof(cx<F>)))
                      : pipe_team_lds(static_cast<int>(sizeof(cx<A>)), static_cast<int>(sizeof(cx<F>)));
  const dim3 grid(static_cast<unsigned>(a.nchunks));
  const size_t lds = static_cast<size_t>(lds1) * prog_waves<F>() + 3 * kDescMax * sizeof(Unit) +
                     kStepInts * sizeof(int32_t) * kStepWin + 16 + (lv ? sizeof(V) * a.lv_rows : 0);
  const dim3 block(64 * prog_waves<F>());
  const bool nr1 = a.rc == 1;
  if (lv && !nr1) return hipErrorInvalidValue;
  if (lv && adjoint)
    hipLaunchKernelGGL((k_program_pipe<F, V, A, true, true, true>), grid, block, lds, s, a, steps, s0, s1, lds1);
  else if (lv)
    hipLaunchKernelGGL((k_program_pipe<F, V, A, false, true, true>), grid, block, lds, s, a, steps, s0, s1, lds1);
  else if (adjoint && nr1)
    hipLaunchKernelGGL((k_program_pipe<F, V, A, true, true, false>), grid, block, lds, s, a, steps, s0, s1, lds1);
  else if (adjoint)
    hipLaunchKernelGGL((k_program_pipe<F, V, A, true, false, false>), grid, block, lds, s, a, steps, s0, s1, lds1);
  else if (nr1)
    hipLaunchKernelGGL((k_program_pipe<F, V, A, false, true, false>), grid, block, lds, s, a, steps, s0, s1, lds1);
  else
    hipLaunchKernelGGL((k_program_pipe<F, V, A, false, false, false>), grid, block, lds, s, a, steps, s0, s1, lds1);
  return hipGetLastError();
}

void prepare_launch_shapes() {
  prepare_pipe<float, cf, float>();
  prepare_pipe<double, cd, double>();
  prepare_pipe<float, cd, double>();
}

hipError_t launch_pipe_c64(const StageArgs& a, int ngroups, int nchunks, bool adjoint, int max_blocks, hipStream_t s) {
  return launch_pipe<float, cf, float>(a, ngroups, nchunks, adjoint, max_blocks, s);
}
hipError_t launch_pipe_c128(const StageArgs& a, int ngroups, int nchunks, bool adjoint, int max_blocks,
                            hipStream_t s) {
  return launch_pipe<double, cd, double>(a, ngroups, nchunks, adjoint, max_blocks, s);
}
hipError_t launch_pipe_c64_hi(const StageArgs& a, int ngroups, int nchunks, bool adjoint, int max_blocks,
                              hipStream_t s) {
  return launch_pipe<float, cd, double>(a, ngroups, nchunks, adjoint, max_blocks, s);
}
hipError_t launch_prog_pipe_c64(const StageArgs& a, const int32_t* steps, int s0, int s1, bool adjoint,
                                hipStream_t s) {
  return launch_prog_pipe<float, cf, float>(a, steps, s0, s1, adjoint, s);
}
hipError_t launch_prog_pipe_c128(const StageArgs& a, const int32_t* steps, int s0, int s1, bool adjoint,
                                 hipStream_t s) {
  return launch_prog_pipe<double, cd, double>(a, steps, s0, s1, adjoint, s);
}

}  // namespace hbf
