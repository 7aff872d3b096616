// The stage kernel: executes a batch of small dense operations ("units") of
// the H-IDBF factor chain -- the column-ID transfers of the V factors, the
// dense coupling blocks of the middle factor, the row-ID transfers of the U
// factors and the dense leaf blocks -- for R right-hand sides at once.
//
// One workgroup handles one group of units (units whose outputs cover the same
// rows; their results are summed in registers) for a chunk of `rc` RHS.  For
// each unit it stages the source vectors and the permutations in LDS, streams
// the unit's matrices from HBM into LDS in contiguous, 16-byte-vectorised
// chunks, and accumulates its outputs.  The factor bytes are read once per
// RHS chunk and never reshaped; with one RHS the kernel is a pure stream of
// the factors (memory bound), with many RHS each staged matrix entry is
// reused rc times from LDS.
#include "kernels.h"

namespace hbf {

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <class T>
__device__ __forceinline__ void cmac(cx<T>& acc, cx<T> a, cx<T> b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
// acc += conj(a) * b
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

template <class F, class A, bool ADJ>
__device__ __forceinline__ void mac(cx<A>& acc, cx<F> m, cx<A> s) {
  if constexpr (ADJ) cmac_conj(acc, up<A>(m), s);
  else cmac(acc, up<A>(m), s);
}

__device__ __forceinline__ int ceil_div_pos(int a, int b) {  // ceil(a/b) for b > 0, clamped at >= 0
  return a <= 0 ? 0 : (a + b - 1) / b;
}

// Synchronisation of a team: the whole workgroup, or one wavefront.
struct BlockSync {
  __device__ __forceinline__ void operator()() const { __syncthreads(); }
};
struct WaveSync {
  __device__ __forceinline__ void operator()() const {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
};

// One team (TEAM threads) evaluates the group of units [q0, q1) (unit ids
// q directly, or through the group table) for RHS chunk `chunk` and writes
// its destination.  smem is the team's LDS region.
template <class F, class V, class A, bool ADJ, int TEAM, int OPT, class Sync>
__device__ __forceinline__ void process_group(const StageArgs& a, int q0, int q1, bool direct, int chunk, int tid,
                                              unsigned char* smem, Sync sync) {
  const int r0 = chunk * a.rc;
  const int nr = min(a.rc, a.R - r0);
  const int R = a.R;

  cx<A>* s_src = reinterpret_cast<cx<A>*>(smem);
  cx<F>* s_mat = reinterpret_cast<cx<F>*>(smem + static_cast<size_t>(a.src_cap) * sizeof(cx<A>));
  uint8_t* s_p = reinterpret_cast<uint8_t*>(s_mat + a.ch);  // stored permutations, 2 x 256
  uint8_t* s_q = s_p + 512;                                  // their inverses, 2 x 256

  // destination segments (shared by all units of the group)
  const Unit* U0 = &a.units[direct ? q0 : a.gunits[q0]];
  const int d_buf = ADJ ? U0->in_buf : U0->out_buf;
  const int d_off0 = ADJ ? U0->in_off[0] : U0->out_off[0];
  const int d_off1 = ADJ ? U0->in_off[1] : U0->out_off[1];
  const int d_len0 = ADJ ? U0->in_len[0] : U0->out_len[0];
  const int d_len1 = ADJ ? U0->in_len[1] : U0->out_len[1];
  const int n_dst = d_len0 + d_len1;
  const int n_out = n_dst * nr;

  cx<A> acc[OPT];
#pragma unroll
  for (int j = 0; j < OPT; ++j) acc[j] = cx<A>{0, 0};

  for (int q = q0; q < q1; ++q) {
    const Unit* U = &a.units[direct ? q : a.gunits[q]];
    const int type = U->type;
    const int s_buf = ADJ ? U->out_buf : U->in_buf;
    const int s_off0 = ADJ ? U->out_off[0] : U->in_off[0];
    const int s_off1 = ADJ ? U->out_off[1] : U->in_off[1];
    const int s_len0 = ADJ ? U->out_len[0] : U->in_len[0];
    const int s_len1 = ADJ ? U->out_len[1] : U->in_len[1];
    const int n_src = s_len0 + s_len1;
    const int k0 = U->k[0], k1 = U->k[1];
    const int f_in = U->in_len[0] + U->in_len[1];    // forward source length
    const int f_out = U->out_len[0] + U->out_len[1]; // forward destination length
    const int64_t mat = U->mat;
    const int mat_len = U->mat_len;

    sync();  // LDS of the previous unit is free
    // stage the sources
    {
      const V* sb = reinterpret_cast<const V*>(a.buf[s_buf]);
      for (int e = tid; e < n_src * nr; e += TEAM) {
        const int t = e / nr;
        const int rr = e - t * nr;
        const int row = (t < s_len0) ? s_off0 + t : s_off1 + (t - s_len0);
        s_src[e] = up<A>(sb[static_cast<int64_t>(row) * R + r0 + rr]);
      }
    }
    // stage permutations (GATHER: 2 x f_in bytes; SCATTER: 2 x f_out bytes)
    int plen = 0;
    if (type == UNIT_GATHER) plen = f_in;
    else if (type == UNIT_SCATTER) plen = f_out;
    if (plen) {
      const uint8_t* pp = a.perm + U->perm;
      for (int e = tid; e < 2 * plen; e += TEAM) {
        const int o = e / plen, j = e - o * plen;
        const uint8_t v = pp[e];
        s_p[o * 256 + j] = v;
        s_q[o * 256 + v] = static_cast<uint8_t>(j);
      }
    }
    // matrices, chunk by chunk
    const cx<F>* gm = reinterpret_cast<const cx<F>*>(a.fac) + mat;
    for (int e0 = 0; e0 < mat_len; e0 += a.ch) {
      const int e1 = min(mat_len, e0 + a.ch);
      sync();
      {
        const u32x4* g4 = reinterpret_cast<const u32x4*>(gm + e0);
        u32x4* l4 = reinterpret_cast<u32x4*>(s_mat);
        const int nw = ((e1 - e0) * static_cast<int>(sizeof(cx<F>)) + 15) / 16;
        for (int w = tid; w < nw; w += TEAM) l4[w] = __builtin_nontemporal_load(&g4[w]);
      }
      sync();
      const bool first_chunk = (e0 == 0);
#pragma unroll
      for (int j = 0; j < OPT; ++j) {
        const int p = tid + j * TEAM;
        if (p >= n_out) break;
        const int o = p / nr;
        const int rr = p - o * nr;
        cx<A> s = acc[j];
        auto S = [&](int t) { return s_src[t * nr + rr]; };
        if (type == UNIT_DENSE) {
          if (!ADJ) {
            // out[o] = sum_t M(o, t) src[t], M column-major f_out x f_in
            const int tlo = ceil_div_pos(e0 - o, f_out), thi = min(f_in, ceil_div_pos(e1 - o, f_out));
            for (int t = tlo; t < thi; ++t) mac<F, A, false>(s, s_mat[t * f_out + o - e0], S(t));
          } else {
            // out[t=o] = sum_i conj(M(i, o)) src[i]
            const int base = o * f_out;
            const int ilo = max(0, e0 - base), ihi = min(f_out, e1 - base);
            for (int i = ilo; i < ihi; ++i) mac<F, A, true>(s, s_mat[base + i - e0], S(i));
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
            const int tlo = ceil_div_pos(e0 - base - i, k), thi = min(r, ceil_div_pos(e1 - base - i, k));
            for (int t = tlo; t < thi; ++t) mac<F, A, false>(s, s_mat[base + t * k + i - e0], S(pm[k + t]));
          } else {
            // o indexes the forward source; sum over both IDs
#pragma unroll
            for (int id = 0; id < 2; ++id) {
              const int k = id ? k1 : k0;
              const int r = f_in - k;
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
                const int t = qq - k;
                const int cb = base + t * k;
                const int ilo = max(0, e0 - cb), ihi = min(k, e1 - cb);
                for (int i = ilo; i < ihi; ++i) mac<F, A, true>(s, s_mat[cb + i - e0], S(sbase + i));
              }
              (void)r;
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
              const int qq = s_p[id * 256 + o];  // stored inverse permutation
              if (qq < k) {
                if (first_chunk) {
                  const cx<A> v = S(sbase + qq);
                  s.x += v.x;
                  s.y += v.y;
                }
              } else {
                const int t = qq - k;
                const int jlo = ceil_div_pos(e0 - base - t, r), jhi = min(k, ceil_div_pos(e1 - base - t, r));
                for (int jj = jlo; jj < jhi; ++jj) mac<F, A, false>(s, s_mat[base + jj * r + t - e0], S(sbase + jj));
              }
            }
          } else {
            // o indexes [in_a; in_b]: in_id[j] = src[perm[j]] + sum_t conj(T(j,t)) src[perm[k+t]]
            const int id = (o < k0) ? 0 : 1;
            const int jj = id ? o - k0 : o;
            const int k = id ? k1 : k0;
            const int r = f_out - k;
            const int base = id ? k0 * (f_out - k0) : 0;
            const uint8_t* pm = s_q + id * 256;  // forward permutation = inverse of the stored one
            if (first_chunk) {
              const cx<A> v = S(pm[jj]);
              s.x += v.x;
              s.y += v.y;
            }
            const int rb = base + jj * r;
            const int tlo = max(0, e0 - rb), thi = min(r, e1 - rb);
            for (int t = tlo; t < thi; ++t) mac<F, A, true>(s, s_mat[rb + t - e0], S(pm[k + t]));
          }
        }
        acc[j] = s;
      }
    }
    if (mat_len == 0) {
      // units without matrices (not produced by the builder) contribute nothing
    }
  }
  // write the destination
  V* db = reinterpret_cast<V*>(a.buf[d_buf]);
  const A are = static_cast<A>(a.alpha_re), aim = static_cast<A>(a.alpha_im);
#pragma unroll
  for (int j = 0; j < OPT; ++j) {
    const int p = tid + j * TEAM;
    if (p >= n_out) break;
    const int o = p / nr;
    const int rr = p - o * nr;
    const int row = (o < d_len0) ? d_off0 + o : d_off1 + (o - d_len0);
    V* dp = &db[static_cast<int64_t>(row) * R + r0 + rr];
    cx<A> v = acc[j];
    if (a.acc) {
      const cx<A> cur = up<A>(*dp);
      v = cx<A>{cur.x + are * v.x - aim * v.y, cur.y + are * v.y + aim * v.x};
    }
    using VT = decltype(dp->x);
    *dp = V{static_cast<VT>(v.x), static_cast<VT>(v.y)};
  }
}

template <class F, class V, class A, bool ADJ>
__global__ void __launch_bounds__(kStageThreads) k_stage(StageArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int gi = blockIdx.x / a.nchunks;
  const int chunk = blockIdx.x - gi * a.nchunks;
  const int g = a.first + gi;
  int q0, q1;
  if (a.direct) {
    q0 = g;
    q1 = g + 1;
  } else {
    q0 = a.gofs[g];
    q1 = a.gofs[g + 1];
  }
  process_group<F, V, A, ADJ, kStageThreads, kOutPerThread>(a, q0, q1, a.direct != 0, chunk, threadIdx.x, smem,
                                                            BlockSync{});
}

// Wave-per-group variant: each of the 4 waves of a workgroup evaluates its own
// group with its own LDS slice (more independent factor streams in flight
// when one group's matrices are small, e.g. one right-hand side).
template <class F, class V, class A, bool ADJ>
__global__ void __launch_bounds__(kStageThreads) k_stage_wave(StageArgs a, int ngroups, int wave_lds) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int wave = threadIdx.x / 64;
  const int lane = threadIdx.x - wave * 64;
  const int gt = blockIdx.x * (kStageThreads / 64) + wave;
  if (gt >= ngroups * a.nchunks) return;
  const int gi = gt / a.nchunks;
  const int chunk = gt - gi * a.nchunks;
  const int g = a.first + gi;
  int q0, q1;
  if (a.direct) {
    q0 = g;
    q1 = g + 1;
  } else {
    q0 = a.gofs[g];
    q1 = a.gofs[g + 1];
  }
  process_group<F, V, A, ADJ, 64, kWaveOutPerThread>(a, q0, q1, a.direct != 0, chunk, lane,
                                                     smem + static_cast<size_t>(wave) * wave_lds, WaveSync{});
}

// A sequential program of steps run by one workgroup per RHS chunk: each step
// is a range of independent units (one block level, a dense neighbour block or
// a leaf solve); the waves take the units of a step round-robin, and the
// workgroup synchronises between steps.  Used for the sweeps over subtrees
// whose blocks are too small to fill the GPU.
template <class F, class V, class A, bool ADJ>
__global__ void __launch_bounds__(kProgThreads) k_program(StageArgs a, const int32_t* steps, int s0, int s1,
                                                          int wave_lds) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int wave = threadIdx.x / 64;
  const int lane = threadIdx.x - wave * 64;
  unsigned char* my = smem + static_cast<size_t>(wave) * wave_lds;
  const int chunk = blockIdx.x;
  const double are = a.alpha_re, aim = a.alpha_im;
  for (int st = s0; st < s1; ++st) {
    const int u0 = steps[kStepInts * st], u1 = steps[kStepInts * st + 1], flags = steps[kStepInts * st + 2];
    const int acc = flags & 1;
    const bool fwd_mode = (flags >> 1) & 1;
    StageArgs b = a;
    b.acc = acc;
    b.alpha_re = acc ? are : 0.0;
    b.alpha_im = acc ? aim : 0.0;
    for (int u = u0 + wave; u < u1; u += kProgWaves) {
      if (ADJ && fwd_mode)
        process_group<F, V, A, false, 64, kProgOutPerThread>(b, u, u + 1, true, chunk, lane, my, WaveSync{});
      else
        process_group<F, V, A, ADJ, 64, kProgOutPerThread>(b, u, u + 1, true, chunk, lane, my, WaveSync{});
    }
    __threadfence_block();
    __syncthreads();
  }
}

template <class F, class V, class A>
hipError_t launch_program(const StageArgs& a, const int32_t* steps, int s0, int s1, int wave_lds, bool adjoint,
                          hipStream_t s) {
  const dim3 grid(static_cast<unsigned>(a.nchunks));
  const size_t lds = static_cast<size_t>(wave_lds) * kProgWaves;
  if (adjoint)
    hipLaunchKernelGGL((k_program<F, V, A, true>), grid, dim3(kProgThreads), lds, s, a, steps, s0, s1, wave_lds);
  else
    hipLaunchKernelGGL((k_program<F, V, A, false>), grid, dim3(kProgThreads), lds, s, a, steps, s0, s1, wave_lds);
  return hipGetLastError();
}

template <class F, class V, class A>
hipError_t launch_stage_wave(const StageArgs& a, int ngroups, int wave_lds, bool adjoint, hipStream_t s) {
  const int per = kStageThreads / 64;
  const int64_t teams = static_cast<int64_t>(ngroups) * a.nchunks;
  const dim3 grid(static_cast<unsigned>((teams + per - 1) / per));
  const size_t lds = static_cast<size_t>(wave_lds) * per;
  if (adjoint)
    hipLaunchKernelGGL((k_stage_wave<F, V, A, true>), grid, dim3(kStageThreads), lds, s, a, ngroups, wave_lds);
  else
    hipLaunchKernelGGL((k_stage_wave<F, V, A, false>), grid, dim3(kStageThreads), lds, s, a, ngroups, wave_lds);
  return hipGetLastError();
}

template <class F, class V, class A>
hipError_t launch_stage(const StageArgs& a, int ngroups, bool adjoint, size_t lds, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>(ngroups) * static_cast<unsigned>(a.nchunks));
  if (adjoint) hipLaunchKernelGGL((k_stage<F, V, A, true>), grid, dim3(kStageThreads), lds, s, a);
  else hipLaunchKernelGGL((k_stage<F, V, A, false>), grid, dim3(kStageThreads), lds, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// layout conversion (nrhs, N) <-> (n, R) with dtype cast and the padding map
// ---------------------------------------------------------------------------
template <class S, class D>
__global__ void k_to_internal(const cx<S>* ext, cx<D>* in, int64_t n, int64_t n_ext, int R, const int32_t* real_of) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n * R) return;
  const int64_t i = e / R;
  const int r = static_cast<int>(e - i * R);
  const int64_t j = real_of ? real_of[i] : i;
  cx<S> v{0, 0};
  if (j >= 0) v = ext[static_cast<int64_t>(r) * n_ext + j];
  in[e] = cx<D>{static_cast<D>(v.x), static_cast<D>(v.y)};
}
template <class S, class D>
__global__ void k_to_external(const cx<S>* in, cx<D>* ext, int64_t n_ext, int R, const int32_t* lib_of) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n_ext * R) return;
  const int r = static_cast<int>(e / n_ext);
  const int64_t j = e - static_cast<int64_t>(r) * n_ext;
  const int64_t i = lib_of ? lib_of[j] : j;
  const cx<S> v = in[i * R + r];
  ext[e] = cx<D>{static_cast<D>(v.x), static_cast<D>(v.y)};
}

// ---------------------------------------------------------------------------
// Leaf factorisation in FP64 (one workgroup per leaf).  mode 0: block
// reading, inverse of the leaf block by Gauss-Jordan elimination with partial
// pivoting; mode 1: the paper's point-wise reading, inverses of
// I + a*strict_lower(D) and of upper(D).
// ---------------------------------------------------------------------------
__device__ __forceinline__ cd cdiv(cd a, cd b) {
  const double den = b.x * b.x + b.y * b.y;
  return cd{(a.x * b.x + a.y * b.y) / den, (a.y * b.x - a.x * b.y) / den};
}
__device__ __forceinline__ cd cmul(cd a, cd b) { return cd{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }

// Gauss-Jordan elimination on W = [M | I] (n x 2n, row-major, global
// scratch), in place: on return W[:, n:2n] = M^{-1}.  Partial pivoting on
// request; a zero pivot sets *flag.
__device__ void gauss_jordan_inplace(cd* W, int n, bool pivot, int* flag) {
  const int tid = threadIdx.x;
  const int w = 2 * n;
  __shared__ int s_piv;
  __shared__ double s_best[256];
  __shared__ int s_arg[256];
  __shared__ int s_bad;
  if (tid == 0) s_bad = 0;
  __syncthreads();
  for (int c = 0; c < n; ++c) {
    if (pivot) {
      double best = -1.0;
      int arg = c;
      for (int r = c + tid; r < n; r += blockDim.x) {
        const cd v = W[static_cast<int64_t>(r) * w + c];
        const double m = v.x * v.x + v.y * v.y;
        if (m > best) { best = m; arg = r; }
      }
      s_best[tid] = best;
      s_arg[tid] = arg;
      __syncthreads();
      if (tid == 0) {
        double b = -1.0;
        int ar = c;
        for (int t = 0; t < static_cast<int>(blockDim.x); ++t)
          if (s_best[t] > b || (s_best[t] == b && s_arg[t] < ar)) { b = s_best[t]; ar = s_arg[t]; }
        s_piv = ar;
      }
      __syncthreads();
      const int p = s_piv;
      if (p != c) {
        for (int j = tid; j < w; j += blockDim.x) {
          const cd t = W[static_cast<int64_t>(p) * w + j];
          W[static_cast<int64_t>(p) * w + j] = W[static_cast<int64_t>(c) * w + j];
          W[static_cast<int64_t>(c) * w + j] = t;
        }
      }
      __syncthreads();
    }
    const cd piv = W[static_cast<int64_t>(c) * w + c];
    if (!(piv.x * piv.x + piv.y * piv.y > 0.0)) {
      if (tid == 0) {
        atomicExch(flag, 1);
        s_bad = 1;
      }
    }
    __syncthreads();
    if (s_bad) return;
    for (int j = tid; j < w; j += blockDim.x) W[static_cast<int64_t>(c) * w + j] = cdiv(W[static_cast<int64_t>(c) * w + j], piv);
    __syncthreads();
    for (int e = tid; e < n * w; e += blockDim.x) {
      const int r = e / w, j = e - r * w;
      if (r == c || j == c) continue;
      const cd f = W[static_cast<int64_t>(r) * w + c];
      if (f.x == 0.0 && f.y == 0.0) continue;
      const cd v = W[static_cast<int64_t>(c) * w + j];
      const cd m = cmul(f, v);
      W[static_cast<int64_t>(r) * w + j] = cd{W[static_cast<int64_t>(r) * w + j].x - m.x, W[static_cast<int64_t>(r) * w + j].y - m.y};
    }
    __syncthreads();
    for (int r = tid; r < n; r += blockDim.x)
      if (r != c) W[static_cast<int64_t>(r) * w + c] = cd{0.0, 0.0};
    __syncthreads();
  }
}

// Super-leaf factorisation in FP64: one workgroup per super-leaf.  A holds
// the exact entries of the super-leaf's diagonal block (row-major ns x ns).
// The lower and upper blocks of L~ / U~ are inverted by Gauss-Jordan (with
// partial pivoting in the block reading, where they have full n0 x n0
// diagonal blocks) and written as the four unit sets (row slabs).
template <class F>
__global__ void __launch_bounds__(256) k_superleaf_factor(const cd* A, int64_t S0, int ns, int n0, int mode,
                                                          double sre, double sim, cx<F>* fac, SuperleafOut so,
                                                          int* flag, cd* work) {
  const int64_t S = S0 + blockIdx.x;
  const cd* As = A + static_cast<int64_t>(blockIdx.x) * ns * ns;
  cd* W = work + static_cast<int64_t>(blockIdx.x) * ns * 2 * ns;
  cd* Linv = work + static_cast<int64_t>(gridDim.x) * ns * 2 * ns + static_cast<int64_t>(blockIdx.x) * ns * ns;
  const int w = 2 * ns;
  const int tid = threadIdx.x;
  for (int pass = 0; pass < 2; ++pass) {
    const bool lower = pass == 0;
    for (int e = tid; e < ns * w; e += blockDim.x) {
      const int r = e / w, j = e - r * w;
      cd v{0.0, 0.0};
      if (j < ns) {
        const cd a = As[static_cast<int64_t>(r) * ns + j];
        if (mode == 0) {
          const int br = r / n0, bj = j / n0;
          if (lower ? (br >= bj) : (br <= bj)) v = a;
        } else if (lower) {
          if (r > j) v = cmul(cd{sre, sim}, a);
          else if (r == j) v = cd{1.0, 0.0};
        } else if (r <= j) {
          v = a;
        }
      } else {
        v = cd{(j - ns == r) ? 1.0 : 0.0, 0.0};
      }
      W[e] = v;
    }
    __syncthreads();
    gauss_jordan_inplace(W, ns, mode == 0, flag);
    __syncthreads();
    if (lower) {
      for (int e = tid; e < ns * ns; e += blockDim.x) {
        const int r = e / ns, c = e - r * ns;
        Linv[e] = W[static_cast<int64_t>(r) * w + ns + c];
      }
      __syncthreads();
    }
  }
  // W[:, ns:] holds Uinv, Linv the lower inverse; write the four sets
  const int sl = ns / n0;
  for (int set = 0; set < 4; ++set) {
    const bool lower_shape = (set == 0 || set == 2);
    int64_t off = so.base[set] + S * so.per_superleaf;
    for (int i = 0; i < sl; ++i) {
      const int c0 = lower_shape ? 0 : i * n0;
      const int wid = lower_shape ? (i + 1) * n0 : (sl - i) * n0;
      const int sw = so.slab * wid;  // entries of one slab (column-major slab x wid)
      for (int e = tid; e < n0 * wid; e += blockDim.x) {
        const int j = e / sw, rem = e - j * sw;
        const int c = rem / so.slab, r = rem - c * so.slab;
        const int gr = i * n0 + j * so.slab + r, gc = c0 + c;
        cd v;
        if (set == 0) v = Linv[static_cast<int64_t>(gr) * ns + gc];
        else if (set == 1) v = W[static_cast<int64_t>(gr) * w + ns + gc];
        else if (set == 2) { v = W[static_cast<int64_t>(gc) * w + ns + gr]; v.y = -v.y; }
        else { v = Linv[static_cast<int64_t>(gc) * ns + gr]; v.y = -v.y; }
        fac[off + e] = cx<F>{static_cast<F>(v.x), static_cast<F>(v.y)};
      }
      off += static_cast<int64_t>(n0) * wid;
    }
  }
}

unsigned blocks_for(int64_t n, int t) { return static_cast<unsigned>((n + t - 1) / t); }

}  // namespace

hipError_t launch_stage_c64(const StageArgs& a, int ngroups, bool adjoint, size_t lds, hipStream_t s) {
  return launch_stage<float, cf, float>(a, ngroups, adjoint, lds, s);
}
hipError_t launch_stage_c128(const StageArgs& a, int ngroups, bool adjoint, size_t lds, hipStream_t s) {
  return launch_stage<double, cd, double>(a, ngroups, adjoint, lds, s);
}
hipError_t launch_stage_c64_hi(const StageArgs& a, int ngroups, bool adjoint, size_t lds, hipStream_t s) {
  return launch_stage<float, cd, double>(a, ngroups, adjoint, lds, s);
}
hipError_t launch_stage_wave_c64(const StageArgs& a, int ngroups, int wave_lds, bool adjoint, hipStream_t s) {
  return launch_stage_wave<float, cf, float>(a, ngroups, wave_lds, adjoint, s);
}
hipError_t launch_stage_wave_c128(const StageArgs& a, int ngroups, int wave_lds, bool adjoint, hipStream_t s) {
  return launch_stage_wave<double, cd, double>(a, ngroups, wave_lds, adjoint, s);
}
hipError_t launch_stage_wave_c64_hi(const StageArgs& a, int ngroups, int wave_lds, bool adjoint, hipStream_t s) {
  return launch_stage_wave<float, cd, double>(a, ngroups, wave_lds, adjoint, s);
}
hipError_t launch_program_c64(const StageArgs& a, const int32_t* steps, int s0, int s1, int wave_lds, bool adjoint,
                              hipStream_t s) {
  return launch_program<float, cf, float>(a, steps, s0, s1, wave_lds, adjoint, s);
}
hipError_t launch_program_c128(const StageArgs& a, const int32_t* steps, int s0, int s1, int wave_lds, bool adjoint,
                               hipStream_t s) {
  return launch_program<double, cd, double>(a, steps, s0, s1, wave_lds, adjoint, s);
}

hipError_t launch_to_internal(const void* ext, int ext_c128, void* in, int in_c128, const VecMap& m, int R,
                              hipStream_t s) {
  const int64_t n = m.n_int, ne = m.n_ext;
  const int32_t* map = m.real_of;
  const unsigned nb = blocks_for(n * R, 256);
  if (ext_c128 && in_c128)
    hipLaunchKernelGGL((k_to_internal<double, double>), nb, 256, 0, s, (const cd*)ext, (cd*)in, n, ne, R, map);
  else if (ext_c128)
    hipLaunchKernelGGL((k_to_internal<double, float>), nb, 256, 0, s, (const cd*)ext, (cf*)in, n, ne, R, map);
  else if (in_c128)
    hipLaunchKernelGGL((k_to_internal<float, double>), nb, 256, 0, s, (const cf*)ext, (cd*)in, n, ne, R, map);
  else
    hipLaunchKernelGGL((k_to_internal<float, float>), nb, 256, 0, s, (const cf*)ext, (cf*)in, n, ne, R, map);
  return hipGetLastError();
}

hipError_t launch_to_external(const void* in, int in_c128, void* ext, int ext_c128, const VecMap& m, int R,
                              hipStream_t s) {
  const int64_t ne = m.n_ext;
  const int32_t* map = m.lib_of;
  const unsigned nb = blocks_for(ne * R, 256);
  if (ext_c128 && in_c128)
    hipLaunchKernelGGL((k_to_external<double, double>), nb, 256, 0, s, (const cd*)in, (cd*)ext, ne, R, map);
  else if (ext_c128)
    hipLaunchKernelGGL((k_to_external<float, double>), nb, 256, 0, s, (const cf*)in, (cd*)ext, ne, R, map);
  else if (in_c128)
    hipLaunchKernelGGL((k_to_external<double, float>), nb, 256, 0, s, (const cd*)in, (cf*)ext, ne, R, map);
  else
    hipLaunchKernelGGL((k_to_external<float, float>), nb, 256, 0, s, (const cf*)in, (cf*)ext, ne, R, map);
  return hipGetLastError();
}


hipError_t launch_superleaf_factor(const cd* A, int64_t S0, int64_t nb, int ns, int n0, int mode, double sre,
                                  double sim, void* fac, int fac_c128, SuperleafOut so, int* flag, cd* work,
                                  hipStream_t s) {
  if (fac_c128)
    hipLaunchKernelGGL((k_superleaf_factor<double>), dim3(static_cast<unsigned>(nb)), dim3(256), 0, s, A, S0, ns, n0,
                       mode, sre, sim, (cd*)fac, so, flag, work);
  else
    hipLaunchKernelGGL((k_superleaf_factor<float>), dim3(static_cast<unsigned>(nb)), dim3(256), 0, s, A, S0, ns, n0,
                       mode, sre, sim, (cf*)fac, so, flag, work);
  return hipGetLastError();
}

}  // namespace hbf
