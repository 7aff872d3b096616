// GMRES building blocks for R right-hand sides in lockstep, vectors in the
// internal (N, R) layout.  Reductions (dot products and norms) accumulate in
// FP64 with a fixed two-pass order (per-block partial sums, then a sum over
// blocks), so results are deterministic.  The small Hessenberg / Givens
// bookkeeping runs on the device, one thread per right-hand side, in FP64.
#include "gmres.h"

namespace hbf {

namespace {

template <class T>
__device__ __forceinline__ cd ld(const cx<T>* p, int64_t i) {
  const cx<T> v = p[i];
  return cd{static_cast<double>(v.x), static_cast<double>(v.y)};
}
template <class T>
__device__ __forceinline__ void st(cx<T>* p, int64_t i, cd v) {
  p[i] = cx<T>{static_cast<T>(v.x), static_cast<T>(v.y)};
}

// Block layout: threadIdx.x -> rhs within a tile of RT, threadIdx.y -> rows.
constexpr int kRows = 256;

// partial[b][i][r] = sum over the block's rows of conj(V_i[n][r]) * w[n][r], i < nv
template <class T, int MAXV>
__global__ void k_dots(const cx<T>* V, int64_t vstride, int nv, const cx<T>* w, int64_t n, int R, cd* partial,
                       int rows_per_block) {
  const int r = blockIdx.y * blockDim.x + threadIdx.x;
  const int64_t row0 = static_cast<int64_t>(blockIdx.x) * rows_per_block;
  const int64_t row1 = min<int64_t>(n, row0 + rows_per_block);
  cd acc[MAXV];
#pragma unroll
  for (int i = 0; i < MAXV; ++i) acc[i] = cd{0, 0};
  if (r < R) {
    for (int64_t row = row0 + threadIdx.y; row < row1; row += blockDim.y) {
      const cd b = ld(w, row * R + r);
#pragma unroll
      for (int i = 0; i < MAXV; ++i) {
        if (i < nv) {
          const cd a = ld(V + i * vstride, row * R + r);
          acc[i].x += a.x * b.x + a.y * b.y;
          acc[i].y += a.x * b.y - a.y * b.x;
        }
      }
    }
  }
  __shared__ cd red[kRows];
  for (int i = 0; i < nv && i < MAXV; ++i) {
    red[threadIdx.y * blockDim.x + threadIdx.x] = acc[i];
    __syncthreads();
    for (int s = blockDim.y / 2; s > 0; s >>= 1) {
      if (threadIdx.y < s) {
        cd& d = red[threadIdx.y * blockDim.x + threadIdx.x];
        const cd o = red[(threadIdx.y + s) * blockDim.x + threadIdx.x];
        d.x += o.x;
        d.y += o.y;
      }
      __syncthreads();
    }
    if (threadIdx.y == 0 && r < R) partial[(static_cast<int64_t>(blockIdx.x) * nv + i) * R + r] = red[threadIdx.x];
    __syncthreads();
  }
}

// out[i][r] = sum_b partial[b][i][r]
__global__ void k_sum_partials(const cd* partial, int nb, int nv, int R, cd* out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nv * R) return;
  cd s{0, 0};
  for (int b = 0; b < nb; ++b) {
    const cd v = partial[static_cast<int64_t>(b) * nv * R + e];
    s.x += v.x;
    s.y += v.y;
  }
  out[e] = s;
}

// w[n][r] -= sum_i V_i[n][r] h[i][r]
template <class T>
__global__ void k_sub_combo(const cx<T>* V, int64_t vstride, int nv, const cd* h, cx<T>* w, int64_t n, int R) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n * R) return;
  const int r = static_cast<int>(e % R);
  cd acc = ld(w, e);
  for (int i = 0; i < nv; ++i) {
    const cd a = ld(V + i * vstride, e);
    const cd c = h[i * R + r];
    acc.x -= a.x * c.x - a.y * c.y;
    acc.y -= a.x * c.y + a.y * c.x;
  }
  st(w, e, acc);
}

// u[n][r] = sum_i V_i[n][r] y[i][r]
template <class T>
__global__ void k_combo(const cx<T>* V, int64_t vstride, int nv, const cd* y, cx<T>* u, int64_t n, int R) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n * R) return;
  const int r = static_cast<int>(e % R);
  cd acc{0, 0};
  for (int i = 0; i < nv; ++i) {
    const cd a = ld(V + i * vstride, e);
    const cd c = y[i * R + r];
    acc.x += a.x * c.x - a.y * c.y;
    acc.y += a.x * c.y + a.y * c.x;
  }
  st(u, e, acc);
}

// dst[n][r] = src[n][r] * s[r] (s real; s = 0 yields 0)
template <class S, class D>
__global__ void k_scale(const cx<S>* src, const double* s, cx<D>* dst, int64_t n, int R) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n * R) return;
  const double f = s[e % R];
  const cd v = ld(src, e);
  st(dst, e, cd{v.x * f, v.y * f});
}

// FP64 vectors: y = a - b (r = b - A x), x += cast(d)
__global__ void k_sub64(const cd* a, const cd* b, cd* y, int64_t m) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= m) return;
  y[e] = cd{a[e].x - b[e].x, a[e].y - b[e].y};
}
template <class T>
__global__ void k_add_to64(const cx<T>* d, cd* x, int64_t m) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const cd v = ld(d, e);
  x[e] = cd{x[e].x + v.x, x[e].y + v.y};
}
template <class S, class D>
__global__ void k_cast(const cx<S>* a, cx<D>* b, int64_t m) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= m) return;
  st(b, e, ld(a, e));
}
__global__ void k_fill_zero(double* p, int64_t m) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < m) p[e] = 0.0;
}

// ---- small per-RHS state ----------------------------------------------------
// Layout per rhs (doubles): H (m+1) x m complex (column j at j*(m+1)), cs[m],
// sn[m] complex, g[m+1] complex, then scalars.
struct Small {
  int m;
  __device__ __host__ int64_t per() const { return 2 * ((m + 1) * m + 2 * m + (m + 1)) + 8; }
  __device__ cd* H(double* base, int r) const { return reinterpret_cast<cd*>(base + r * per()); }
  __device__ cd* cs(double* base, int r) const { return H(base, r) + (m + 1) * m; }
  __device__ cd* sn(double* base, int r) const { return cs(base, r) + m; }
  __device__ cd* g(double* base, int r) const { return sn(base, r) + m; }
  __device__ double* scal(double* base, int r) const { return reinterpret_cast<double*>(g(base, r) + (m + 1)); }
};

// start of a cycle: beta[r] = sqrt(nrm2[r]); inv[r] = active ? 1/beta : 0;
// g = (beta, 0, ...); H = 0.  active[r] = beta > target[r].
__global__ void k_cycle_start(double* small, int m, int R, const cd* nrm2, const double* target, double* inv,
                              double* resid, int* active) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  Small S{m};
  const double beta = sqrt(max(0.0, nrm2[r].x));
  cd* H = S.H(small, r);
  for (int e = 0; e < (m + 1) * m; ++e) H[e] = cd{0, 0};
  cd* g = S.g(small, r);
  for (int e = 0; e <= m; ++e) g[e] = cd{0, 0};
  g[0] = cd{beta, 0};
  const int act = (beta > target[r]) && isfinite(beta) ? 1 : 0;
  active[r] = act;
  inv[r] = act ? 1.0 / beta : 0.0;
  resid[r] = beta;
  double* sc = S.scal(small, r);
  sc[0] = beta;
  sc[1] = 0;  // number of columns used
}

// add h (the CGS pass) into column j of H
__global__ void k_h_accum(double* small, int m, int R, int j, const cd* h) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  Small S{m};
  cd* H = S.H(small, r) + j * (m + 1);
  for (int i = 0; i <= j; ++i) {
    H[i].x += h[i * R + r].x;
    H[i].y += h[i * R + r].y;
  }
}

// column j complete: H[j+1][j] = sqrt(nrm2); inv = 1/H[j+1][j] (0 on breakdown);
// apply previous rotations, make a new one, update g; resid = |g[j+1]|.
// Inactive right-hand sides keep their state.
__global__ void k_givens(double* small, int m, int R, int j, const cd* nrm2, double* inv, double* resid,
                         const double* target, int* active) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  Small S{m};
  double* sc = S.scal(small, r);
  if (!active[r]) {
    inv[r] = 0.0;
    return;
  }
  cd* H = S.H(small, r) + j * (m + 1);
  cd* cs = S.cs(small, r);
  cd* sn = S.sn(small, r);
  cd* g = S.g(small, r);
  const double hn = sqrt(max(0.0, nrm2[r].x));
  H[j + 1] = cd{hn, 0};
  const double beta = sc[0];
  inv[r] = (hn > 1e-300 && hn > 1e-14 * beta) ? 1.0 / hn : 0.0;
  for (int i = 0; i < j; ++i) {
    const cd a = H[i], b = H[i + 1];
    const cd c = cs[i], s = sn[i];
    // [conj(c) conj(s); -s c] [a; b]
    H[i] = cd{c.x * a.x + c.y * a.y + s.x * b.x + s.y * b.y, c.x * a.y - c.y * a.x + s.x * b.y - s.y * b.x};
    H[i + 1] = cd{-(s.x * a.x - s.y * a.y) + (c.x * b.x - c.y * b.y), -(s.x * a.y + s.y * a.x) + (c.x * b.y + c.y * b.x)};
  }
  const cd a = H[j], b = H[j + 1];
  const double den = hypot(hypot(a.x, a.y), hypot(b.x, b.y));
  cd c{1, 0}, s{0, 0};
  if (den > 0) {
    c = cd{a.x / den, a.y / den};
    s = cd{b.x / den, b.y / den};
  }
  cs[j] = c;
  sn[j] = s;
  H[j] = cd{den, 0};
  H[j + 1] = cd{0, 0};
  const cd gj = g[j];
  g[j + 1] = cd{-(s.x * gj.x - s.y * gj.y), -(s.x * gj.y + s.y * gj.x)};
  g[j] = cd{c.x * gj.x + c.y * gj.y, c.x * gj.y - c.y * gj.x};
  sc[1] = j + 1;
  const double res = hypot(g[j + 1].x, g[j + 1].y);
  resid[r] = res;
  if (res <= target[r] || inv[r] == 0.0) active[r] = 0;
}

// y = H(0:k, 0:k)^{-1} g(0:k), k = columns used by the rhs; y[i][r] layout
__global__ void k_lsq(double* small, int m, int R, cd* y) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  Small S{m};
  const int k = static_cast<int>(S.scal(small, r)[1]);
  const cd* H = S.H(small, r);
  const cd* g = S.g(small, r);
  for (int i = m - 1; i >= k; --i) y[i * R + r] = cd{0, 0};
  for (int i = k - 1; i >= 0; --i) {
    cd acc = g[i];
    for (int t = i + 1; t < k; ++t) {
      const cd h = H[t * (m + 1) + i];
      const cd v = y[t * R + r];
      acc.x -= h.x * v.x - h.y * v.y;
      acc.y -= h.x * v.y + h.y * v.x;
    }
    const cd d = H[i * (m + 1) + i];
    const double den = d.x * d.x + d.y * d.y;
    y[i * R + r] = den > 0 ? cd{(acc.x * d.x + acc.y * d.y) / den, (acc.y * d.x - acc.x * d.y) / den} : cd{0, 0};
  }
}

// any non-finite value in an (N, R) vector -> flag
template <class T>
__global__ void k_nonfinite(const cx<T>* v, int64_t m, int* flag) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const cx<T> a = v[e];
  if (!isfinite(static_cast<double>(a.x)) || !isfinite(static_cast<double>(a.y))) atomicExch(flag, 1);
}

inline unsigned nblk(int64_t m, int t = 256) { return static_cast<unsigned>((m + t - 1) / t); }

template <class T>
hipError_t dots_impl(const void* V, int64_t vstride, int nv, const void* w, int64_t n, int R, cd* partial,
                     size_t partial_len, cd* out, hipStream_t s) {
  const int RT = R >= 64 ? 64 : (R >= 16 ? 16 : (R >= 4 ? 4 : 1));
  const dim3 blk(RT, kRows / RT);
  int64_t nb = std::min<int64_t>(1024, (n + 255) / 256);
  while (nb > 1 && static_cast<size_t>(nb) * nv * R > partial_len) nb /= 2;
  const int rpb = static_cast<int>((n + nb - 1) / nb);
  const dim3 grid(static_cast<unsigned>(nb), static_cast<unsigned>((R + RT - 1) / RT));
  const cx<T>* Vp = static_cast<const cx<T>*>(V);
  const cx<T>* wp = static_cast<const cx<T>*>(w);
  if (nv <= 1)
    hipLaunchKernelGGL((k_dots<T, 1>), grid, blk, 0, s, Vp, vstride, nv, wp, n, R, partial, rpb);
  else if (nv <= 8)
    hipLaunchKernelGGL((k_dots<T, 8>), grid, blk, 0, s, Vp, vstride, nv, wp, n, R, partial, rpb);
  else if (nv <= 16)
    hipLaunchKernelGGL((k_dots<T, 16>), grid, blk, 0, s, Vp, vstride, nv, wp, n, R, partial, rpb);
  else if (nv <= 32)
    hipLaunchKernelGGL((k_dots<T, 32>), grid, blk, 0, s, Vp, vstride, nv, wp, n, R, partial, rpb);
  else
    hipLaunchKernelGGL((k_dots<T, 64>), grid, blk, 0, s, Vp, vstride, nv, wp, n, R, partial, rpb);
  hipLaunchKernelGGL(k_sum_partials, nblk(static_cast<int64_t>(nv) * R), 256, 0, s, partial, static_cast<int>(nb), nv,
                     R, out);
  return hipGetLastError();
}

}  // namespace

hipError_t gm_dots(bool c128, const void* V, int64_t vstride, int nv, const void* w, int64_t n, int R, cd* partial,
                   size_t partial_len, cd* out, hipStream_t s) {
  if (nv > 64) return hipErrorInvalidValue;
  return c128 ? dots_impl<double>(V, vstride, nv, w, n, R, partial, partial_len, out, s)
              : dots_impl<float>(V, vstride, nv, w, n, R, partial, partial_len, out, s);
}

hipError_t gm_sub_combo(bool c128, const void* V, int64_t vstride, int nv, const cd* h, void* w, int64_t n, int R,
                        hipStream_t s) {
  if (c128)
    hipLaunchKernelGGL((k_sub_combo<double>), nblk(n * R), 256, 0, s, (const cd*)V, vstride, nv, h, (cd*)w, n, R);
  else
    hipLaunchKernelGGL((k_sub_combo<float>), nblk(n * R), 256, 0, s, (const cf*)V, vstride, nv, h, (cf*)w, n, R);
  return hipGetLastError();
}

hipError_t gm_combo(bool c128, const void* V, int64_t vstride, int nv, const cd* y, void* u, int64_t n, int R,
                    hipStream_t s) {
  if (c128)
    hipLaunchKernelGGL((k_combo<double>), nblk(n * R), 256, 0, s, (const cd*)V, vstride, nv, y, (cd*)u, n, R);
  else
    hipLaunchKernelGGL((k_combo<float>), nblk(n * R), 256, 0, s, (const cf*)V, vstride, nv, y, (cf*)u, n, R);
  return hipGetLastError();
}

hipError_t gm_scale(bool src128, const void* src, const double* f, bool dst128, void* dst, int64_t n, int R,
                    hipStream_t s) {
  const unsigned nb = nblk(n * R);
  if (src128 && dst128) hipLaunchKernelGGL((k_scale<double, double>), nb, 256, 0, s, (const cd*)src, f, (cd*)dst, n, R);
  else if (src128) hipLaunchKernelGGL((k_scale<double, float>), nb, 256, 0, s, (const cd*)src, f, (cf*)dst, n, R);
  else if (dst128) hipLaunchKernelGGL((k_scale<float, double>), nb, 256, 0, s, (const cf*)src, f, (cd*)dst, n, R);
  else hipLaunchKernelGGL((k_scale<float, float>), nb, 256, 0, s, (const cf*)src, f, (cf*)dst, n, R);
  return hipGetLastError();
}

hipError_t gm_sub64(const cd* a, const cd* b, cd* y, int64_t m, hipStream_t s) {
  hipLaunchKernelGGL(k_sub64, nblk(m), 256, 0, s, a, b, y, m);
  return hipGetLastError();
}

hipError_t gm_add_to64(bool src128, const void* d, cd* x, int64_t m, hipStream_t s) {
  if (src128) hipLaunchKernelGGL((k_add_to64<double>), nblk(m), 256, 0, s, (const cd*)d, x, m);
  else hipLaunchKernelGGL((k_add_to64<float>), nblk(m), 256, 0, s, (const cf*)d, x, m);
  return hipGetLastError();
}

hipError_t gm_cast(bool src128, const void* a, bool dst128, void* b, int64_t m, hipStream_t s) {
  if (src128 && dst128) hipLaunchKernelGGL((k_cast<double, double>), nblk(m), 256, 0, s, (const cd*)a, (cd*)b, m);
  else if (src128) hipLaunchKernelGGL((k_cast<double, float>), nblk(m), 256, 0, s, (const cd*)a, (cf*)b, m);
  else if (dst128) hipLaunchKernelGGL((k_cast<float, double>), nblk(m), 256, 0, s, (const cf*)a, (cd*)b, m);
  else hipLaunchKernelGGL((k_cast<float, float>), nblk(m), 256, 0, s, (const cf*)a, (cf*)b, m);
  return hipGetLastError();
}

hipError_t gm_zero(void* p, int64_t ndoubles, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_zero, nblk(ndoubles), 256, 0, s, static_cast<double*>(p), ndoubles);
  return hipGetLastError();
}

hipError_t gm_nonfinite(bool c128, const void* v, int64_t m, int* flag, hipStream_t s) {
  if (c128) hipLaunchKernelGGL((k_nonfinite<double>), nblk(m), 256, 0, s, (const cd*)v, m, flag);
  else hipLaunchKernelGGL((k_nonfinite<float>), nblk(m), 256, 0, s, (const cf*)v, m, flag);
  return hipGetLastError();
}

int64_t gm_small_per_rhs(int m) { return Small{m}.per(); }

hipError_t gm_cycle_start(double* small, int m, int R, const cd* nrm2, const double* target, double* inv,
                          double* resid, int* active, hipStream_t s) {
  hipLaunchKernelGGL(k_cycle_start, nblk(R, 64), 64, 0, s, small, m, R, nrm2, target, inv, resid, active);
  return hipGetLastError();
}

hipError_t gm_h_accum(double* small, int m, int R, int j, const cd* h, hipStream_t s) {
  hipLaunchKernelGGL(k_h_accum, nblk(R, 64), 64, 0, s, small, m, R, j, h);
  return hipGetLastError();
}

hipError_t gm_givens(double* small, int m, int R, int j, const cd* nrm2, double* inv, double* resid,
                     const double* target, int* active, hipStream_t s) {
  hipLaunchKernelGGL(k_givens, nblk(R, 64), 64, 0, s, small, m, R, j, nrm2, inv, resid, target, active);
  return hipGetLastError();
}

hipError_t gm_lsq(double* small, int m, int R, cd* y, hipStream_t s) {
  hipLaunchKernelGGL(k_lsq, nblk(R, 64), 64, 0, s, small, m, R, y);
  return hipGetLastError();
}

}  // namespace hbf
