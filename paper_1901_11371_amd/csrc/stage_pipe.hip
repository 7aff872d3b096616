// Software-pipelined wave teams.  Most units of the H-IDBF factor chain are
// tiny (a few hundred matrix entries), so a kernel that loads a unit, waits,
// computes and only then loads the next one is bound by memory latency.  Here
// every wave is a team that walks over a list of work items (unit, matrix
// chunk); while it computes item i from LDS, the loads of item i+1 (sources,
// permutations and a 4 KB matrix chunk, into registers) are already in
// flight, and the descriptor of the unit after that is fetched one step
// earlier still.  Used for the matvec and sweep stages with few right-hand
// sides per team and for the sweep programs.
#include "kernels.h"

namespace hbf {

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kPW = 4;                  // 16-byte words per lane per matrix chunk
constexpr int kChunkW = 64 * kPW;       // words per chunk (4 KB)
constexpr int kSrcPL = 4;               // source entries per lane (256 max)
constexpr int kPermPL = 8;              // permutation bytes per lane (512 max)
constexpr int kOpt = 4;                 // outputs per lane (256 max)

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
__device__ __forceinline__ void issue(const StageArgs& a, const UDesc& d, int c, int lane, int R, int r0, int nr,
                                      Slot<V>& s) {
  const u32x4* gm = reinterpret_cast<const u32x4*>(reinterpret_cast<const cx<F>*>(a.fac) + d.mat);
#pragma unroll
  for (int j = 0; j < kPW; ++j) {
    const int w = c * kChunkW + lane + 64 * j;
    if (w < d.nwords) s.mw[j] = __builtin_nontemporal_load(&gm[w]);
  }
  if (c == 0) {
    const V* sb = reinterpret_cast<const V*>(a.buf[d.s_buf]);
#pragma unroll
    for (int j = 0; j < kSrcPL; ++j) {
      const int e = lane + 64 * j;
      if (e < d.n_src * nr) {
        const int t = e / nr, rr = e - t * nr;
        const int row = (t < d.s_len0) ? d.s_off0 + t : d.s_off1 + (t - d.s_len0);
        s.sv[j] = sb[static_cast<int64_t>(row) * R + r0 + rr];
      }
    }
#pragma unroll
    for (int j = 0; j < kPermPL; ++j) {
      const int e = lane + 64 * j;
      if (e < 2 * d.plen) s.pv[j] = a.perm[d.perm + e];
    }
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

  cx<A> acc[kOpt];
#pragma unroll
  for (int j = 0; j < kOpt; ++j) acc[j] = cx<A>{0, 0};

  for (;;) {
    // ---- commit the current item to LDS ----
    const int nch = d.nwords > 0 ? (d.nwords + kChunkW - 1) / kChunkW : 1;
    if (cur.c == 0) {
#pragma unroll
      for (int j = 0; j < kSrcPL; ++j) {
        const int e = lane + 64 * j;
        if (e < d.n_src * nr) s_src[e] = up<A>(slot.sv[j]);
      }
#pragma unroll
      for (int j = 0; j < kPermPL; ++j) {
        const int e = lane + 64 * j;
        if (e < 2 * d.plen) {
          const int o = e / d.plen, p = e - o * d.plen;
          s_p[o * 256 + p] = slot.pv[j];
          s_q[o * 256 + slot.pv[j]] = static_cast<uint8_t>(p);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < kPW; ++j) {
      const int w = cur.c * kChunkW + lane + 64 * j;
      if (w < d.nwords) s_m4[lane + 64 * j] = slot.mw[j];
    }
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
      if (nxt.c == 0) dn = read_desc<ADJ, F>(unit_of(nxt.q));
      issue<F, V, A, ADJ>(a, dn, nxt.c, lane, R, r0, nr, slot);
    }
    // ---- compute the current item ----
    {
      const int e0 = cur.c * kChunkE;
      const int e1 = min(d.mat_len, e0 + kChunkE);
      const bool first_chunk = cur.c == 0;
      const int type = d.type;
      const int k0 = d.k0, k1 = d.k1, f_in = d.f_in, f_out = d.f_out;
#pragma unroll
      for (int j = 0; j < kOpt; ++j) {
        const int p = lane + 64 * j;
        if (p >= d.n_dst * nr) break;
        const int o = p / nr;
        const int rr = p - o * nr;
        cx<A> s = acc[j];
        auto S = [&](int t) { return s_src[t * nr + rr]; };
        auto MAC = [&](int e, int t) {
          const cx<A> m = up<A>(s_mat[e - e0]);
          if (ADJ) cmac_conj(s, m, S(t));
          else cmac(s, m, S(t));
        };
        if (type == UNIT_DENSE) {
          if (!ADJ) {
            const int tlo = cdiv_pos(e0 - o, f_out), thi = min(f_in, cdiv_pos(e1 - o, f_out));
            for (int t = tlo; t < thi; ++t) MAC(t * f_out + o, t);
          } else {
            const int base = o * f_out;
            const int ilo = max(0, e0 - base), ihi = min(f_out, e1 - base);
            for (int i = ilo; i < ihi; ++i) MAC(base + i, i);
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
            const int tlo = cdiv_pos(e0 - base - i, k), thi = min(r, cdiv_pos(e1 - base - i, k));
            for (int t = tlo; t < thi; ++t) MAC(base + t * k + i, pm[k + t]);
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
                for (int i = ilo; i < ihi; ++i) MAC(cb + i, sbase + i);
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
                const int jlo = cdiv_pos(e0 - base - t, r), jhi = min(k, cdiv_pos(e1 - base - t, r));
                for (int jj = jlo; jj < jhi; ++jj) MAC(base + jj * r + t, sbase + jj);
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
            for (int t = tlo; t < thi; ++t) MAC(rb + t, pm[k + t]);
          }
        }
        acc[j] = s;
      }
    }
    // ---- end of a group: write its destination ----
    if (group_end) {
      V* db = reinterpret_cast<V*>(a.buf[d.d_buf]);
      const A are = static_cast<A>(a.alpha_re), aim = static_cast<A>(a.alpha_im);
#pragma unroll
      for (int j = 0; j < kOpt; ++j) {
        const int p = lane + 64 * j;
        if (p >= d.n_dst * nr) break;
        const int o = p / nr;
        const int rr = p - o * nr;
        const int row = (o < d.d_len0) ? d.d_off0 + o : d.d_off1 + (o - d.d_len0);
        V* dp = &db[static_cast<int64_t>(row) * R + r0 + rr];
        cx<A> v = acc[j];
        if (a.acc) {
          const cx<A> cu = up<A>(*dp);
          v = cx<A>{cu.x + are * v.x - aim * v.y, cu.y + are * v.y + aim * v.x};
        }
        using VT = decltype(dp->x);
        *dp = V{static_cast<VT>(v.x), static_cast<VT>(v.y)};
        acc[j] = cx<A>{0, 0};
      }
    }
    wsync();
    if (nxt.q < 0) break;
    cur = nxt;
    d = dn;
  }
}

// Stage launch: teams = waves; team t handles groups t, t + nteams, ... for RHS chunk `chunk`.
template <class F, class V, class A, bool ADJ>
__global__ void __launch_bounds__(256) k_stage_pipe(StageArgs a, int ngroups, int team_lds) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int chunk = blockIdx.y;
  const int r0 = chunk * a.rc;
  const int nr = min(a.rc, a.R - r0);
  const int team = blockIdx.x * 4 + wave;
  const int nteams = gridDim.x * 4;
  team_run<F, V, A, ADJ>(a, a.first, ngroups, team, nteams, lane, smem + static_cast<size_t>(wave) * team_lds, a.R,
                         r0, nr);
}

// Sweep program: one workgroup per RHS chunk runs the steps in order; the
// waves share each step's units (one unit per team).
template <class F, class V, class A, bool ADJ>
__global__ void __launch_bounds__(64 * kProgWaves) k_program_pipe(StageArgs a, const int32_t* steps, int s0, int s1,
                                                                  int team_lds) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int chunk = blockIdx.x;
  const int r0 = chunk * a.rc;
  const int nr = min(a.rc, a.R - r0);
  unsigned char* my = smem + static_cast<size_t>(wave) * team_lds;
  const double are = a.alpha_re, aim = a.alpha_im;
  for (int st = s0; st < s1; ++st) {
    const int u0 = uni(steps[3 * st]), u1 = uni(steps[3 * st + 1]), flags = uni(steps[3 * st + 2]);
    StageArgs b = a;
    b.acc = flags & 1;
    b.alpha_re = (flags & 1) ? are : 0.0;
    b.alpha_im = (flags & 1) ? aim : 0.0;
    b.direct = 1;
    if (ADJ && ((flags >> 1) & 1))
      team_run<F, V, A, false>(b, u0, u1 - u0, wave, kProgWaves, lane, my, a.R, r0, nr);
    else
      team_run<F, V, A, ADJ>(b, u0, u1 - u0, wave, kProgWaves, lane, my, a.R, r0, nr);
    __syncthreads();
  }
}

}  // namespace

int pipe_team_lds(int elt_acc, int elt_fac) {
  (void)elt_fac;
  return 256 * elt_acc + 1024 + kChunkW * 16;
}

template <class F, class V, class A>
static hipError_t launch_pipe(const StageArgs& a, int ngroups, int nchunks, bool adjoint, int max_blocks,
                              hipStream_t s) {
  const int lds1 = pipe_team_lds(static_cast<int>(sizeof(cx<A>)), static_cast<int>(sizeof(cx<F>)));
  int bx = (ngroups + 3) / 4;
  if (bx > max_blocks) bx = max_blocks;
  if (bx < 1) bx = 1;
  const dim3 grid(static_cast<unsigned>(bx), static_cast<unsigned>(nchunks));
  if (adjoint) hipLaunchKernelGGL((k_stage_pipe<F, V, A, true>), grid, dim3(256), lds1 * 4, s, a, ngroups, lds1);
  else hipLaunchKernelGGL((k_stage_pipe<F, V, A, false>), grid, dim3(256), lds1 * 4, s, a, ngroups, lds1);
  return hipGetLastError();
}

template <class F, class V, class A>
static hipError_t launch_prog_pipe(const StageArgs& a, const int32_t* steps, int s0, int s1, bool adjoint,
                                   hipStream_t s) {
  const int lds1 = pipe_team_lds(static_cast<int>(sizeof(cx<A>)), static_cast<int>(sizeof(cx<F>)));
  const dim3 grid(static_cast<unsigned>(a.nchunks));
  if (adjoint)
    hipLaunchKernelGGL((k_program_pipe<F, V, A, true>), grid, dim3(64 * kProgWaves), lds1 * kProgWaves, s, a, steps,
                       s0, s1, lds1);
  else
    hipLaunchKernelGGL((k_program_pipe<F, V, A, false>), grid, dim3(64 * kProgWaves), lds1 * kProgWaves, s, a, steps,
                       s0, s1, lds1);
  return hipGetLastError();
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
