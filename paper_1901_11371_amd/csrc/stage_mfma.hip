// Stage launches for many right-hand sides on the matrix cores.
//
// With R right-hand sides every unit of the factor chain is a small complex
// GEMM: out (n_dst x R) = M (n_dst x n_src) * in (n_src x R), where M is the
// unit's operator in natural row / column order.  For the butterfly transfer
// units M is not stored densely: an ID's skeleton columns are unit columns and
// its redundant columns are the interpolation matrix T, so each element of M
// is formed on the fly from T and the permutation bytes
//   GATHER  (column ID, V factors):  M[o][s] = q < k ? [q == i] : T(i, q - k),
//           o = (ID, i), q = position of source s in the ID's pivot order;
//   SCATTER (row ID, U factors):     M[p][j] = q < k ? [q == jj] : T(jj, q - k),
//           j = (ID, jj), q = position of output p in the ID's pivot order;
//   DENSE:  the stored column-major block.
// The adjoint uses M^H.  The complex product is four real products on
// v_mfma_f32_16x16x4_f32 (re*re - im*im, re*im + im*re) with FP32
// accumulation: one wave takes one group of units (units writing the same
// rows, summed in the accumulators) for NT 16-column tiles of right-hand
// sides (NT = 1, 2 or 4: 16, 32 or 64 RHS per wave, an execution parameter),
// one 16-row output tile at a time, 4 source rows per step.
#include <algorithm>
#include <cstdint>

#include "kernels.h"

namespace hbf {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMfmaWaves = 4;  // waves (groups) per workgroup

struct UnitView {
  int64_t mat, perm;
  int type, k0, k1, f_in, f_out;
  int s_off0, s_off1, s_len0;  // source segments in the launch's orientation
  int s_buf;
};

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <bool ADJ>
__device__ __forceinline__ UnitView view(const Unit* U) {
  UnitView v;
  v.mat = U->mat;
  v.perm = U->perm;
  v.type = uni(U->type);
  v.k0 = uni(U->k[0]);
  v.k1 = uni(U->k[1]);
  v.f_in = uni(U->in_len[0] + U->in_len[1]);
  v.f_out = uni(U->out_len[0] + U->out_len[1]);
  if (!ADJ) {
    v.s_buf = uni(U->in_buf);
    v.s_off0 = uni(U->in_off[0]);
    v.s_off1 = uni(U->in_off[1]);
    v.s_len0 = uni(U->in_len[0]);
  } else {
    v.s_buf = uni(U->out_buf);
    v.s_off0 = uni(U->out_off[0]);
    v.s_off1 = uni(U->out_off[1]);
    v.s_len0 = uni(U->out_len[0]);
  }
  return v;
}

// Element (o, s) of the unit's forward operator (o < f_out, s < f_in).
// inv: for GATHER, the positions of the sources in the two IDs' pivot orders
// (LDS, 2 x 256 bytes).
__device__ __forceinline__ cf fwd_elem(const UnitView& u, const cf* fac, const uint8_t* perm, const uint8_t* inv,
                                       int o, int s) {
  if (u.type == UNIT_DENSE) return fac[u.mat + static_cast<int64_t>(s) * u.f_out + o];
  if (u.type == UNIT_GATHER) {
    const int id = o < u.k0 ? 0 : 1;
    const int i = id ? o - u.k0 : o;
    const int k = id ? u.k1 : u.k0;
    const int q = inv[id * 256 + s];
    if (q < k) return cf{q == i ? 1.0f : 0.0f, 0.0f};
    const int64_t base = id ? static_cast<int64_t>(u.k0) * (u.f_in - u.k0) : 0;
    return fac[u.mat + base + static_cast<int64_t>(q - k) * k + i];
  }
  // SCATTER: the stored bytes are the inverse pivot order of each ID over the outputs
  const int id = s < u.k0 ? 0 : 1;
  const int jj = id ? s - u.k0 : s;
  const int k = id ? u.k1 : u.k0;
  const int q = perm[u.perm + id * u.f_out + o];
  if (q < k) return cf{q == jj ? 1.0f : 0.0f, 0.0f};
  const int r = u.f_out - k;
  const int64_t base = id ? static_cast<int64_t>(u.k0) * (u.f_out - u.k0) : 0;
  return fac[u.mat + base + static_cast<int64_t>(jj) * r + (q - k)];
}

__device__ __forceinline__ f32x4 mfma(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Wave gt takes group gt / (nrchunks * mtiles), RHS chunk and the output
// tiles mt0, mt0 + mtiles, ... of that group (mtiles = 1: all of them, one
// after another; more: the group's 16-row output tiles run on parallel waves,
// which shortens the dependent chain of a launch of few groups with many rows).
template <bool ADJ, int kNT>
__global__ void __launch_bounds__(64 * kMfmaWaves) k_stage_mfma(StageArgs a, int ngroups, int nrchunks, int mtiles) {
  __shared__ uint8_t s_inv[kMfmaWaves][512];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int gt = blockIdx.x * kMfmaWaves + wave;
  if (gt >= ngroups * nrchunks * mtiles) return;
  const int gi = gt / (nrchunks * mtiles);
  const int rem = gt - gi * nrchunks * mtiles;
  const int chunk = rem / mtiles;
  const int mt0 = rem - chunk * mtiles;
  const int g = a.first + gi;
  int q0, q1;
  if (a.direct) {
    q0 = g;
    q1 = g + 1;
  } else {
    q0 = a.gofs[g];
    q1 = a.gofs[g + 1];
  }
  const int R = a.R;
  const int r0 = chunk * 16 * kNT;
  const int nr = min(16 * kNT, R - r0);
  const cf* fac = static_cast<const cf*>(a.fac);
  uint8_t* inv = s_inv[wave];

  // destination segments (shared by the group's units)
  const Unit* U0 = &a.units[a.direct ? q0 : a.gunits[q0]];
  const int d_buf = uni(ADJ ? U0->in_buf : U0->out_buf);
  const int d_off0 = uni(ADJ ? U0->in_off[0] : U0->out_off[0]);
  const int d_off1 = uni(ADJ ? U0->in_off[1] : U0->out_off[1]);
  const int d_len0 = uni(ADJ ? U0->in_len[0] : U0->out_len[0]);
  const int n_dst = uni(d_len0 + (ADJ ? U0->in_len[1] : U0->out_len[1]));
  cf* db = static_cast<cf*>(d_buf == BUF_X ? a.buf[BUF_X] : (d_buf == BUF_Y ? a.buf[BUF_Y] : a.buf[BUF_ARENA]));

  const int li = lane & 15;  // A row / B column / C column within the tile
  const int lk = lane >> 4;  // A and B: k index within the step; C: row group
  const int ntiles = (nr + 15) >> 4;

  for (int mt = mt0; mt * 16 < n_dst; mt += mtiles) {
    f32x4 acc_re[kNT], acc_im[kNT];
#pragma unroll
    for (int t = 0; t < kNT; ++t) {
      acc_re[t] = f32x4{0, 0, 0, 0};
      acc_im[t] = f32x4{0, 0, 0, 0};
    }
    const int m = mt * 16 + li;  // output row of this lane's A element
    for (int q = q0; q < q1; ++q) {
      const Unit* U = &a.units[a.direct ? q : a.gunits[q]];
      const UnitView u = view<ADJ>(U);
      if (u.type == UNIT_GATHER) {
        // positions of the sources in the two pivot orders
        __builtin_amdgcn_wave_barrier();
        const uint8_t* pp = a.perm + u.perm;
        for (int e = lane; e < 2 * u.f_in; e += 64) {
          const int id = e >= u.f_in ? 1 : 0;
          const int j = e - id * u.f_in;
          inv[id * 256 + pp[e]] = static_cast<uint8_t>(j);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
      const int n_src = ADJ ? u.f_out : u.f_in;
      const cf* sb = static_cast<const cf*>(u.s_buf == BUF_X ? a.buf[BUF_X]
                                                             : (u.s_buf == BUF_Y ? a.buf[BUF_Y] : a.buf[BUF_ARENA]));
      for (int k0 = 0; k0 < n_src; k0 += 4) {
        const int kk = k0 + lk;
        // A element (m, kk) of the operator in the launch's orientation
        cf av{0.0f, 0.0f};
        if (m < n_dst && kk < n_src) {
          if (!ADJ) {
            av = fwd_elem(u, fac, a.perm, inv, m, kk);
          } else {
            av = fwd_elem(u, fac, a.perm, inv, kk, m);
            av.y = -av.y;
          }
        }
        // B elements: source row kk, RHS columns of each tile
        const int row = kk < u.s_len0 ? u.s_off0 + kk : u.s_off1 + (kk - u.s_len0);
        const cf* srow = sb + static_cast<int64_t>(row) * R + r0 + li;
        const float nim = -av.y;
#pragma unroll
        for (int t = 0; t < kNT; ++t) {
          if (t < ntiles) {
            cf bv{0.0f, 0.0f};
            if (kk < n_src && t * 16 + li < nr) bv = srow[t * 16];
            acc_re[t] = mfma(av.x, bv.x, acc_re[t]);
            acc_re[t] = mfma(nim, bv.y, acc_re[t]);
            acc_im[t] = mfma(av.x, bv.y, acc_im[t]);
            acc_im[t] = mfma(av.y, bv.x, acc_im[t]);
          }
        }
      }
      if (u.type == UNIT_GATHER) __builtin_amdgcn_wave_barrier();
    }
    // write the tile: lane holds rows 4 lk + v, column li of each RHS tile
    const float are = static_cast<float>(a.alpha_re), aim = static_cast<float>(a.alpha_im);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int o = mt * 16 + 4 * lk + v;
      if (o >= n_dst) continue;
      const int row = o < d_len0 ? d_off0 + o : d_off1 + (o - d_len0);
      cf* drow = db + static_cast<int64_t>(row) * R + r0 + li;
#pragma unroll
      for (int t = 0; t < kNT; ++t) {
        if (t < ntiles && t * 16 + li < nr) {
          cf val{acc_re[t][v], acc_im[t][v]};
          if (a.acc) {
            const cf cur = drow[t * 16];
            val = cf{cur.x + are * val.x - aim * val.y, cur.y + are * val.y + aim * val.x};
          }
          drow[t * 16] = val;
        }
      }
    }
  }
}

template <int NT>
hipError_t launch_nt(const StageArgs& a, int ngroups, int mtiles, bool adjoint, hipStream_t s) {
  const int nrchunks = (a.R + 16 * NT - 1) / (16 * NT);
  mtiles = std::max(1, mtiles);
  const int64_t waves = static_cast<int64_t>(ngroups) * nrchunks * mtiles;
  if (waves > INT32_MAX) return hipErrorInvalidValue;
  const unsigned blocks = static_cast<unsigned>((waves + kMfmaWaves - 1) / kMfmaWaves);
  if (blocks == 0) return hipSuccess;
  if (adjoint)
    hipLaunchKernelGGL((k_stage_mfma<true, NT>), dim3(blocks), dim3(64 * kMfmaWaves), 0, s, a, ngroups, nrchunks,
                       mtiles);
  else
    hipLaunchKernelGGL((k_stage_mfma<false, NT>), dim3(blocks), dim3(64 * kMfmaWaves), 0, s, a, ngroups, nrchunks,
                       mtiles);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_stage_mfma_c64(const StageArgs& a, int ngroups, int tiles, int mtiles, bool adjoint,
                                 hipStream_t s) {
  if (tiles >= 4) return launch_nt<4>(a, ngroups, mtiles, adjoint, s);
  if (tiles == 2) return launch_nt<2>(a, ngroups, mtiles, adjoint, s);
  return launch_nt<1>(a, ngroups, mtiles, adjoint, s);
}

}  // namespace hbf
