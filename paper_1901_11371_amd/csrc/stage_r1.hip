// Single-right-hand-side stage kernel.  With one RHS the H-IDBF apply is a
// pure stream of the factor bytes; this kernel keeps as many of them in flight
// as possible:
//  * each wave is an independent team that walks over groups of units
//    (persistent loop), so a workgroup never waits on a barrier;
//  * a unit's sources, permutations and first matrix chunk are requested
//    together; matrix chunks go straight from HBM to registers (the next
//    chunk is requested before the current one is consumed) and are never
//    staged in LDS;
//  * every lane multiplies the matrix entries it holds with the gathered
//    sources and adds the products into the wave's LDS accumulator for the
//    destination segment with LDS atomics.  Only the owning wave touches its
//    accumulator, and a wave's LDS operations execute in order, so the result
//    is the same from run to run.
#include "kernels.h"

namespace hbf {

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;               // waves per workgroup
constexpr int kWordsPerLane = 4;        // 16-byte words per lane per matrix chunk
constexpr int kChunkWords = 64 * kWordsPerLane;

struct R1Lds {
  // per-wave LDS layout (bytes): acc (2 * 256 A), src (256 A-complex), perm 2x256, iperm 2x256
  static constexpr int kMax = 256;
};

template <class A>
__device__ __forceinline__ void lds_add(A* p, A v) {
  atomicAdd(p, v);
}

template <class F, class V, class A, bool ADJ>
__global__ void __launch_bounds__(64 * kWaves) k_stage_r1(StageArgs a, int ngroups) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  constexpr int M = R1Lds::kMax;
  const size_t per_wave = 2 * M * sizeof(A) + 2 * M * sizeof(A) + 4 * M;
  unsigned char* base = smem + per_wave * wave;
  A* acc = reinterpret_cast<A*>(base);                      // 2*M (re, im interleaved)
  A* src = acc + 2 * M;                                     // 2*M
  uint8_t* perm = reinterpret_cast<uint8_t*>(src + 2 * M);  // 2 x M: forward permutations
  uint8_t* iperm = perm + 2 * M;                            // 2 x M: their inverses

  const int total_waves = gridDim.x * kWaves;
  for (int gw = blockIdx.x * kWaves + wave; gw < ngroups; gw += total_waves) {
    const int g = a.first + gw;
    int q0, q1;
    if (a.direct) {
      q0 = g;
      q1 = g + 1;
    } else {
      q0 = a.gofs[g];
      q1 = a.gofs[g + 1];
    }
    const Unit* U0 = &a.units[a.direct ? q0 : a.gunits[q0]];
    const int d_buf = ADJ ? U0->in_buf : U0->out_buf;
    const int d_off0 = ADJ ? U0->in_off[0] : U0->out_off[0];
    const int d_off1 = ADJ ? U0->in_off[1] : U0->out_off[1];
    const int d_len0 = ADJ ? U0->in_len[0] : U0->out_len[0];
    const int n_dst = d_len0 + (ADJ ? U0->in_len[1] : U0->out_len[1]);
    for (int e = lane; e < 2 * n_dst; e += 64) acc[e] = A(0);

    for (int q = q0; q < q1; ++q) {
      const Unit* U = &a.units[a.direct ? q : a.gunits[q]];
      const int type = U->type;
      const int s_buf = ADJ ? U->out_buf : U->in_buf;
      const int s_off0 = ADJ ? U->out_off[0] : U->in_off[0];
      const int s_off1 = ADJ ? U->out_off[1] : U->in_off[1];
      const int s_len0 = ADJ ? U->out_len[0] : U->in_len[0];
      const int n_src = s_len0 + (ADJ ? U->out_len[1] : U->in_len[1]);
      const int k0 = U->k[0], k1 = U->k[1];
      const int f_in = U->in_len[0] + U->in_len[1];
      const int f_out = U->out_len[0] + U->out_len[1];
      const int mat_len = U->mat_len;
      const int plen = (type == UNIT_GATHER) ? f_in : (type == UNIT_SCATTER) ? f_out : 0;
      const u32x4* gm = reinterpret_cast<const u32x4*>(reinterpret_cast<const cx<F>*>(a.fac) + U->mat);
      const int nwords = (mat_len * static_cast<int>(sizeof(cx<F>)) + 15) / 16;

      // ---- issue every load of the unit ----
      const V* sb = reinterpret_cast<const V*>(a.buf[s_buf]);
      V sv[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int t = lane + 64 * j;
        if (t < n_src) sv[j] = sb[(t < s_len0) ? s_off0 + t : s_off1 + (t - s_len0)];
      }
      uint8_t pv[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int e = lane + 64 * j;
        if (e < 2 * plen) pv[j] = a.perm[U->perm + e];
      }
      u32x4 mw[kWordsPerLane];
#pragma unroll
      for (int j = 0; j < kWordsPerLane; ++j) {
        const int w = lane + 64 * j;
        if (w < nwords) mw[j] = __builtin_nontemporal_load(&gm[w]);
      }
      // ---- sources and permutations to LDS ----
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int t = lane + 64 * j;
        if (t < n_src) {
          src[2 * t] = static_cast<A>(sv[j].x);
          src[2 * t + 1] = static_cast<A>(sv[j].y);
        }
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int e = lane + 64 * j;
        if (e < 2 * plen) {
          const int o = e / plen, p = e - o * plen;
          // GATHER stores forward permutations, SCATTER their inverses
          if (type == UNIT_GATHER) {
            perm[o * M + p] = pv[j];
            iperm[o * M + pv[j]] = static_cast<uint8_t>(p);
          } else {
            iperm[o * M + p] = pv[j];
            perm[o * M + pv[j]] = static_cast<uint8_t>(p);
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

      // ---- identity parts of the interpolative decompositions ----
      if (type == UNIT_GATHER || type == UNIT_SCATTER) {
        const int ktot = k0 + k1;
        for (int x = lane; x < ktot; x += 64) {
          const int o = (x < k0) ? 0 : 1;
          const int j = o ? x - k0 : x;
          const int sbase = o ? k0 : 0;
          int di, si;
          if (type == UNIT_GATHER) {
            if (!ADJ) { di = sbase + j; si = perm[o * M + j]; }
            else { di = perm[o * M + j]; si = sbase + j; }
          } else {
            if (!ADJ) { di = perm[o * M + j]; si = sbase + j; }
            else { di = sbase + j; si = perm[o * M + j]; }
          }
          lds_add(&acc[2 * di], src[2 * si]);
          lds_add(&acc[2 * di + 1], src[2 * si + 1]);
        }
      }

      // ---- matrix entries, chunk by chunk straight from registers ----
      constexpr int epw = 16 / static_cast<int>(sizeof(cx<F>));  // entries per 16-byte word
      const int r0 = (type == UNIT_GATHER) ? f_in - k0 : f_out - k0;
      const int r1 = (type == UNIT_GATHER) ? f_in - k1 : f_out - k1;
      const int split = k0 * r0;  // first entry of the second ID's matrix
      for (int c0 = 0; c0 < nwords; c0 += kChunkWords) {
        u32x4 nx[kWordsPerLane];
        const bool more = c0 + kChunkWords < nwords;
        if (more) {
#pragma unroll
          for (int j = 0; j < kWordsPerLane; ++j) {
            const int w = c0 + kChunkWords + lane + 64 * j;
            if (w < nwords) nx[j] = __builtin_nontemporal_load(&gm[w]);
          }
        }
#pragma unroll
        for (int j = 0; j < kWordsPerLane; ++j) {
          const int w = c0 + lane + 64 * j;
          if (w >= nwords) continue;
          const cx<F>* ent = reinterpret_cast<const cx<F>*>(&mw[j]);
#pragma unroll
          for (int h = 0; h < epw; ++h) {
            const int e = w * epw + h;
            if (e >= mat_len) continue;
            const cx<F> m = ent[h];
            if (m.x == F(0) && m.y == F(0)) continue;  // padding
            int di, si;
            if (type == UNIT_DENSE) {
              const int i = e % f_out, t = e / f_out;
              if (!ADJ) { di = i; si = t; } else { di = t; si = i; }
            } else {
              const int o = (e < split) ? 0 : 1;
              const int ee = o ? e - split : e;
              const int k = o ? k1 : k0;
              const int r = o ? r1 : r0;
              const int sbase = o ? k0 : 0;
              if (type == UNIT_GATHER) {
                const int i = ee % k, t = ee / k;  // column-major k x r
                const int red = perm[o * M + k + t];
                if (!ADJ) { di = sbase + i; si = red; } else { di = red; si = sbase + i; }
              } else {
                const int jj = ee / r, t = ee - (ee / r) * r;  // row-major k x r
                const int red = perm[o * M + k + t];
                if (!ADJ) { di = red; si = sbase + jj; } else { di = sbase + jj; si = red; }
              }
            }
            const A sx = src[2 * si], sy = src[2 * si + 1];
            const A mx = static_cast<A>(m.x), my = ADJ ? -static_cast<A>(m.y) : static_cast<A>(m.y);
            lds_add(&acc[2 * di], mx * sx - my * sy);
            lds_add(&acc[2 * di + 1], mx * sy + my * sx);
          }
        }
        if (more) {
#pragma unroll
          for (int j = 0; j < kWordsPerLane; ++j) mw[j] = nx[j];
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // ---- write the destination ----
    V* db = reinterpret_cast<V*>(a.buf[d_buf]);
    const A are = static_cast<A>(a.alpha_re), aim = static_cast<A>(a.alpha_im);
    for (int o = lane; o < n_dst; o += 64) {
      const int row = (o < d_len0) ? d_off0 + o : d_off1 + (o - d_len0);
      A vx = acc[2 * o], vy = acc[2 * o + 1];
      if (a.acc) {
        const V cur = db[row];
        const A cx_ = static_cast<A>(cur.x), cy_ = static_cast<A>(cur.y);
        const A nx_ = cx_ + are * vx - aim * vy;
        const A ny_ = cy_ + are * vy + aim * vx;
        vx = nx_;
        vy = ny_;
      }
      using VT = decltype(db->x);
      db[row] = V{static_cast<VT>(vx), static_cast<VT>(vy)};
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

template <class F, class V, class A>
hipError_t launch_r1(const StageArgs& a, int ngroups, bool adjoint, int max_blocks, hipStream_t s) {
  constexpr int M = R1Lds::kMax;
  const size_t per_wave = 2 * M * sizeof(A) + 2 * M * sizeof(A) + 4 * M;
  const size_t lds = per_wave * kWaves;
  int blocks = (ngroups + kWaves - 1) / kWaves;
  if (blocks > (max_blocks > 0 ? max_blocks : 2048)) blocks = max_blocks > 0 ? max_blocks : 2048;
  if (blocks < 1) blocks = 1;
  if (adjoint) hipLaunchKernelGGL((k_stage_r1<F, V, A, true>), dim3(blocks), dim3(64 * kWaves), lds, s, a, ngroups);
  else hipLaunchKernelGGL((k_stage_r1<F, V, A, false>), dim3(blocks), dim3(64 * kWaves), lds, s, a, ngroups);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_stage_r1_c64(const StageArgs& a, int ngroups, bool adjoint, int max_blocks, hipStream_t s) {
  return launch_r1<float, cf, float>(a, ngroups, adjoint, max_blocks, s);
}
hipError_t launch_stage_r1_c128(const StageArgs& a, int ngroups, bool adjoint, int max_blocks, hipStream_t s) {
  return launch_r1<double, cd, double>(a, ngroups, adjoint, max_blocks, s);
}
hipError_t launch_stage_r1_c64_hi(const StageArgs& a, int ngroups, bool adjoint, int max_blocks, hipStream_t s) {
  return launch_r1<float, cd, double>(a, ngroups, adjoint, max_blocks, s);
}

}  // namespace hbf
