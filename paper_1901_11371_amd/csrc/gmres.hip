// Krylov building blocks for R right-hand sides in lockstep, vectors in the
// internal (N, R) layout (RHS fastest).
//
// Reductions (dot products and norms) accumulate in FP64 in a fixed order:
// inside a wavefront by xor-shuffles over the lanes that hold the same
// right-hand side, across the waves of a block through LDS, then per-block
// partial sums are added in block order; results are deterministic.
//
// The per-RHS scalar state (GMRES Hessenberg / Givens, TFQMR coefficients)
// lives on the device and is advanced by one-thread-per-RHS kernels in FP64.
// Kernels of one Arnoldi step or one TFQMR iteration take the step index and
// the convergence masks from device memory, so one captured HIP graph serves
// every step and the host never reads state in the middle of an iteration.
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
__device__ __forceinline__ cd cmul(cd a, cd b) { return cd{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ cd cdiv(cd a, cd b) {
  const double den = b.x * b.x + b.y * b.y;
  return cd{(a.x * b.x + a.y * b.y) / den, (a.y * b.x - a.x * b.y) / den};
}

// Block layout of the reductions: threadIdx.x -> rhs within a tile of RT,
// threadIdx.y -> rows; 256 threads = 4 waves.
constexpr int kRows = 256;
constexpr int kWaves = kRows / 64;

// Sum of v over the lanes of the wave that share lane % RT (xor strides
// RT..32); every lane ends with the sum of its class.
template <int RT>
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int s = 32; s >= RT; s >>= 1) v += __shfl_xor(v, s);
  return v;
}

// Number of vectors of a chunked dot product: the static count, or, with a
// device step index j, the basis vectors [c0, j] clamped to the chunk.
__device__ __forceinline__ int chunk_count(int nv_static, const int* jdev, int c0) {
  if (!jdev) return nv_static;
  return min(nv_static, *jdev + 1 - c0);
}

// partial[b][i][r] = sum over the block's rows of conj(V_i[n][r]) * w[n][r], i < nv
template <class T, int MAXV, int RT>
__global__ void k_dots(const cx<T>* V, int64_t vstride, int nv_static, const int* jdev, int c0, const cx<T>* w,
                       int64_t n, int R, cd* partial, int rows_per_block) {
  const int nv = chunk_count(nv_static, jdev, c0);
  if (nv <= 0) return;
  V += static_cast<int64_t>(c0) * vstride;
  const int r = blockIdx.y * RT + threadIdx.x;
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
  __shared__ cd red[kWaves][64];
  const int lin = threadIdx.y * RT + threadIdx.x;
  const int wave = lin >> 6, lane = lin & 63;
  for (int i = 0; i < nv && i < MAXV; ++i) {
    const double sx = wave_sum<RT>(acc[i].x);
    const double sy = wave_sum<RT>(acc[i].y);
    if (lane < RT) red[wave][lane] = cd{sx, sy};
    __syncthreads();
    if (threadIdx.y == 0 && r < R) {
      // lane tx of every wave holds that wave's sum for rhs tile entry tx
      cd s = red[0][threadIdx.x];
#pragma unroll
      for (int q = 1; q < kWaves; ++q) {
        const cd o = red[q][threadIdx.x];
        s.x += o.x;
        s.y += o.y;
      }
      partial[(static_cast<int64_t>(blockIdx.x) * nv + i) * R + r] = s;
    }
    __syncthreads();
  }
}

// out[i][r] = sum_b partial[b][i][r]
__global__ void k_sum_partials(const cd* partial, int nb, int nv_static, const int* jdev, int c0, int R, cd* out) {
  const int nv = chunk_count(nv_static, jdev, c0);
  if (nv <= 0) return;
  out += static_cast<int64_t>(c0) * R;
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

// w[n][r] -= sum_i V_i[n][r] h[i][r], i < nv (nv = j + 1 with a device index)
template <class T>
__global__ void k_sub_combo(const cx<T>* V, int64_t vstride, int nv_static, const int* jdev, const cd* h, cx<T>* w,
                            int64_t n, int R) {
  const int nv = jdev ? *jdev + 1 : nv_static;
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

// dst[n][r] = src[n][r] * s[r] (s real; s = 0 yields 0); with a device index j
// the destination is basis vector j + 1 of dst (stride dstride)
template <class S, class D>
__global__ void k_scale(const cx<S>* src, const double* s, cx<D>* dst, int64_t dstride, const int* jdev, int64_t n,
                        int R) {
  if (jdev) dst += static_cast<int64_t>(*jdev + 1) * dstride;
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n * R) return;
  const double f = s[e % R];
  const cd v = ld(src, e);
  st(dst, e, cd{v.x * f, v.y * f});
}

// dst = basis vector *jdev of V
template <class T>
__global__ void k_copy_basis(const cx<T>* V, int64_t vstride, const int* jdev, cx<T>* dst, int64_t m) {
  const cx<T>* src = V + static_cast<int64_t>(*jdev) * vstride;
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < m) dst[e] = src[e];
}
template <class T>
__global__ void k_copy(const cx<T>* src, cx<T>* dst, int64_t m) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < m) dst[e] = src[e];
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
__global__ void k_set_int(int* p, int v) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *p = v;
}

// ---- GMRES per-RHS state ----------------------------------------------------
// Layout per rhs (doubles): H (m+1) x m complex (column j at j*(m+1)), cs[m],
// sn[m] complex, g[m+1] complex, then scalars: [0] beta, [1] columns used,
// [2] Arnoldi steps of the current cycle.
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
  sc[2] = 0;  // Arnoldi steps of this cycle
}

// add h (the CGS pass) into column j of H
__global__ void k_h_accum(double* small, int m, int R, int j_static, const int* jdev, const cd* h) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const int j = jdev ? *jdev : j_static;
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
__global__ void k_givens(double* small, int m, int R, int j_static, const int* jdev, const cd* nrm2, double* inv,
                         double* resid, const double* target, int* active) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const int j = jdev ? *jdev : j_static;
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
  sc[2] += 1;
  const double res = hypot(g[j + 1].x, g[j + 1].y);
  resid[r] = res;
  if (res <= target[r] || inv[r] == 0.0) active[r] = 0;
}

// end of a step: the step index advances (when given) and any_active = OR of
// the masks
__global__ void k_step_end(int* jdev, const int* active, int R, int* any_active) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (jdev) *jdev += 1;
  int a = 0;
  for (int r = 0; r < R; ++r) a |= active[r];
  *any_active = a;
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

// Arnoldi steps each RHS took in the current cycle
__global__ void k_read_iters(double* small, int m, int R, int* out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  Small S{m};
  out[r] = static_cast<int>(S.scal(small, r)[2]);
}

// ---- TFQMR per-RHS state ------------------------------------------------------
// Transpose-free QMR (Freund, SIAM J. Sci. Comput. 14, 1993) on the
// right-preconditioned system A M^{-1} u = r: two half steps per iteration,
// each one product with A M^{-1}; the quasi-residual bound after half step
// m is tau_m sqrt(m + 1).
struct TqState {
  cd alpha, beta, rho, eta;
  double theta, tau, target, scale;
  int active, done, halfsteps, iters;
};

__global__ void k_tq_start(TqState* S, int R, const cd* nrm2, const double* target, double* inv, double* resid,
                           int* active) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const double beta = sqrt(max(0.0, nrm2[r].x));
  const int act = (beta > target[r]) && isfinite(beta) ? 1 : 0;
  TqState& q = S[r];
  q.alpha = cd{0, 0};
  q.beta = cd{0, 0};
  q.rho = cd{1, 0};
  q.eta = cd{0, 0};
  q.theta = 0;
  q.tau = 1;  // the cycle works on r / ||r||
  q.target = act ? target[r] / beta : 0;
  q.scale = beta;
  q.active = act;
  q.done = 0;
  q.halfsteps = 0;
  q.iters = 0;
  active[r] = act;
  inv[r] = act ? 1.0 / beta : 0.0;
  resid[r] = beta;
}

// rho = <rt, w> at the start of a cycle
__global__ void k_tq_rho0(TqState* S, int R, const cd* dot) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  S[r].rho = dot[r];
}

// alpha = rho / <rt, v>
__global__ void k_tq_alpha(TqState* S, int R, const cd* sigma, int* active) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  TqState& q = S[r];
  if (!q.active) return;
  const cd s = sigma[r];
  if (!(s.x * s.x + s.y * s.y > 0.0) || !(q.rho.x * q.rho.x + q.rho.y * q.rho.y > 0.0)) {
    q.active = 0;  // breakdown: keep the iterate reached so far
    active[r] = 0;
    return;
  }
  q.alpha = cdiv(q.rho, s);
}

// one half step's scalars after w -= alpha u: theta, c, tau, eta; when the
// quasi-residual bound reaches the target the RHS is marked done (the half
// step's update of xhat still applies)
__global__ void k_tq_half(TqState* S, int R, const cd* wnrm2, double* resid) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  TqState& q = S[r];
  if (!q.active) return;
  const double wn = sqrt(max(0.0, wnrm2[r].x));
  q.theta = wn / q.tau;
  const double c = 1.0 / sqrt(1.0 + q.theta * q.theta);
  q.tau = q.tau * q.theta * c;
  q.eta = cd{c * c * q.alpha.x, c * c * q.alpha.y};
  q.halfsteps += 1;
  const double bound = q.tau * sqrt(static_cast<double>(q.halfsteps + 1));
  resid[r] = bound * q.scale;
  if (bound <= q.target || !isfinite(bound)) q.done = 1;
}

// masks after a half step's update of xhat
__global__ void k_tq_commit(TqState* S, int R, int* active) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  TqState& q = S[r];
  if (q.active && q.done) {
    q.active = 0;
    active[r] = 0;
  }
}

// end of an iteration: beta = <rt, w> / rho; rho = <rt, w>
__global__ void k_tq_beta(TqState* S, int R, const cd* rhonew, int* active) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  TqState& q = S[r];
  if (!q.active) return;
  q.iters += 1;
  const cd rn = rhonew[r];
  q.beta = cdiv(rn, q.rho);
  q.rho = rn;
}

__global__ void k_tq_scales(const TqState* S, int R, double* f) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < R) f[r] = S[r].scale;
}
__global__ void k_tq_iters(const TqState* S, int R, int* out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < R) out[r] = S[r].iters;
}

// Elementwise TFQMR updates; right-hand sides that are no longer active are
// left alone.  d is updated with f = theta^2 eta / alpha, theta and eta of
// the previous half step and alpha of the current iteration (zero at the
// start of a cycle).
__device__ __forceinline__ cd tq_dfac(const TqState& q) {
  const double al2 = q.alpha.x * q.alpha.x + q.alpha.y * q.alpha.y;
  if (!(al2 > 0)) return cd{0, 0};
  const cd t = cdiv(q.eta, q.alpha);
  return cd{q.theta * q.theta * t.x, q.theta * q.theta * t.y};
}
// first half step: y2 = y - alpha v; w -= alpha u; d = y + f d
template <class T>
__global__ void k_tq_e1(const TqState* S, const int* active, cx<T>* y2, const cx<T>* y, const cx<T>* v, cx<T>* w,
                        const cx<T>* u, cx<T>* d, int64_t n, int R) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n * R) return;
  const int r = static_cast<int>(e % R);
  if (!active[r]) return;
  const TqState& q = S[r];
  const cd al = q.alpha;
  const cd yv = ld(y, e), vv = ld(v, e), uv = ld(u, e), wv = ld(w, e), dv = ld(d, e);
  const cd av = cmul(al, vv), au = cmul(al, uv);
  st(y2, e, cd{yv.x - av.x, yv.y - av.y});
  st(w, e, cd{wv.x - au.x, wv.y - au.y});
  const cd fd = cmul(tq_dfac(q), dv);
  st(d, e, cd{yv.x + fd.x, yv.y + fd.y});
}
// second half step: w -= alpha u2; d = y2 + f d (f of the first half step)
template <class T>
__global__ void k_tq_e3(const TqState* S, const int* active, cx<T>* w, const cx<T>* u2, const cx<T>* y2, cx<T>* d,
                        int64_t n, int R) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n * R) return;
  const int r = static_cast<int>(e % R);
  if (!active[r]) return;
  const TqState& q = S[r];
  const cd wv = ld(w, e), uv = ld(u2, e), yv = ld(y2, e), dv = ld(d, e);
  const cd au = cmul(q.alpha, uv);
  st(w, e, cd{wv.x - au.x, wv.y - au.y});
  const cd fd = cmul(tq_dfac(q), dv);
  st(d, e, cd{yv.x + fd.x, yv.y + fd.y});
}
// xhat += eta d
template <class T>
__global__ void k_tq_e2(const TqState* S, const int* active, cx<T>* xh, const cx<T>* d, int64_t n, int R) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n * R) return;
  const int r = static_cast<int>(e % R);
  if (!active[r]) return;
  const cd ed = cmul(S[r].eta, ld(d, e));
  const cd xv = ld(xh, e);
  st(xh, e, cd{xv.x + ed.x, xv.y + ed.y});
}
// y = w + beta y2
template <class T>
__global__ void k_tq_e4(const TqState* S, const int* active, cx<T>* y, const cx<T>* w, const cx<T>* y2, int64_t n,
                        int R) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n * R) return;
  const int r = static_cast<int>(e % R);
  if (!active[r]) return;
  const cd by = cmul(S[r].beta, ld(y2, e));
  const cd wv = ld(w, e);
  st(y, e, cd{wv.x + by.x, wv.y + by.y});
}
// v = u + beta (u2 + beta v)
template <class T>
__global__ void k_tq_e5(const TqState* S, const int* active, cx<T>* v, const cx<T>* u, const cx<T>* u2, int64_t n,
                        int R) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n * R) return;
  const int r = static_cast<int>(e % R);
  if (!active[r]) return;
  const cd b = S[r].beta;
  const cd bv = cmul(b, ld(v, e));
  const cd u2v = ld(u2, e);
  const cd t = cmul(b, cd{u2v.x + bv.x, u2v.y + bv.y});
  const cd uv = ld(u, e);
  st(v, e, cd{uv.x + t.x, uv.y + t.y});
}
// cycle start: w = y = rt = r * inv; d = xhat = 0
template <class S, class T>
__global__ void k_tq_init(const cx<S>* r0, const double* inv, cx<T>* w, cx<T>* y, cx<T>* rt, cx<T>* d, cx<T>* xh,
                          int64_t n, int R) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n * R) return;
  const double f = inv[e % R];
  const cd v = ld(r0, e);
  const cd s{v.x * f, v.y * f};
  st(w, e, s);
  st(y, e, s);
  st(rt, e, s);
  st(d, e, cd{0, 0});
  st(xh, e, cd{0, 0});
}

// grad_z[i] = -sum_r lam[r][i] conj(x[r][i]) over (nrhs, N) external-layout
// vectors: the derivative of A = Z + diag(z) contracted with the adjoint and
// forward solutions.
template <class T>
__global__ void k_impedance_grad(const cx<T>* lam, const cx<T>* x, int64_t n, int R, cx<T>* out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  cd acc{0, 0};
  for (int r = 0; r < R; ++r) {
    const cd a = ld(lam, static_cast<int64_t>(r) * n + i);
    const cd b = ld(x, static_cast<int64_t>(r) * n + i);
    acc.x -= a.x * b.x + a.y * b.y;
    acc.y -= a.y * b.x - a.x * b.y;
  }
  st(out, i, acc);
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

template <class T, int MAXV>
void dots_launch(const dim3& grid, int RT, hipStream_t s, const cx<T>* Vp, int64_t vstride, int nv, const int* jdev,
                 int c0, const cx<T>* wp, int64_t n, int R, cd* partial, int rpb) {
  const dim3 blk(RT, kRows / RT);
  switch (RT) {
    case 64:
      hipLaunchKernelGGL((k_dots<T, MAXV, 64>), grid, blk, 0, s, Vp, vstride, nv, jdev, c0, wp, n, R, partial, rpb);
      break;
    case 16:
      hipLaunchKernelGGL((k_dots<T, MAXV, 16>), grid, blk, 0, s, Vp, vstride, nv, jdev, c0, wp, n, R, partial, rpb);
      break;
    case 4:
      hipLaunchKernelGGL((k_dots<T, MAXV, 4>), grid, blk, 0, s, Vp, vstride, nv, jdev, c0, wp, n, R, partial, rpb);
      break;
    default:
      hipLaunchKernelGGL((k_dots<T, MAXV, 1>), grid, blk, 0, s, Vp, vstride, nv, jdev, c0, wp, n, R, partial, rpb);
      break;
  }
}

template <class T>
hipError_t dots_impl(const void* V, int64_t vstride, int nv, const int* jdev, int c0, const void* w, int64_t n, int R,
                     cd* partial, size_t partial_len, cd* out, hipStream_t s) {
  const int RT = R >= 64 ? 64 : (R >= 16 ? 16 : (R >= 4 ? 4 : 1));
  int64_t nb = std::min<int64_t>(1024, (n + 255) / 256);
  while (nb > 1 && static_cast<size_t>(nb) * nv * R > partial_len) nb /= 2;
  const int rpb = static_cast<int>((n + nb - 1) / nb);
  const dim3 grid(static_cast<unsigned>(nb), static_cast<unsigned>((R + RT - 1) / RT));
  const cx<T>* Vp = static_cast<const cx<T>*>(V);
  const cx<T>* wp = static_cast<const cx<T>*>(w);
  if (nv <= 1) dots_launch<T, 1>(grid, RT, s, Vp, vstride, nv, jdev, c0, wp, n, R, partial, rpb);
  else if (nv <= 8) dots_launch<T, 8>(grid, RT, s, Vp, vstride, nv, jdev, c0, wp, n, R, partial, rpb);
  else if (nv <= 16) dots_launch<T, 16>(grid, RT, s, Vp, vstride, nv, jdev, c0, wp, n, R, partial, rpb);
  else dots_launch<T, 32>(grid, RT, s, Vp, vstride, nv, jdev, c0, wp, n, R, partial, rpb);
  hipLaunchKernelGGL(k_sum_partials, nblk(static_cast<int64_t>(nv) * R), 256, 0, s, partial, static_cast<int>(nb), nv,
                     jdev, c0, R, out);
  return hipGetLastError();
}

}  // namespace

hipError_t gm_dots(bool c128, const void* V, int64_t vstride, int nv, const void* w, int64_t n, int R, cd* partial,
                   size_t partial_len, cd* out, hipStream_t s) {
  if (nv > 32 || nv < 1) return hipErrorInvalidValue;
  return c128 ? dots_impl<double>(V, vstride, nv, nullptr, 0, w, n, R, partial, partial_len, out, s)
              : dots_impl<float>(V, vstride, nv, nullptr, 0, w, n, R, partial, partial_len, out, s);
}

hipError_t gm_dots_dev(bool c128, const void* V, int64_t vstride, int m, const int* jdev, const void* w, int64_t n,
                       int R, cd* partial, size_t partial_len, cd* out, hipStream_t s) {
  // chunks of up to 32 basis vectors; the kernels of chunks past j exit at once
  for (int c0 = 0; c0 < m; c0 += 32) {
    const int nv = std::min(32, m - c0);
    const hipError_t e =
        c128 ? dots_impl<double>(V, vstride, nv, jdev, c0, w, n, R, partial, partial_len, out, s)
             : dots_impl<float>(V, vstride, nv, jdev, c0, w, n, R, partial, partial_len, out, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t gm_sub_combo(bool c128, const void* V, int64_t vstride, int nv, const int* jdev, const cd* h, void* w,
                        int64_t n, int R, hipStream_t s) {
  if (c128)
    hipLaunchKernelGGL((k_sub_combo<double>), nblk(n * R), 256, 0, s, (const cd*)V, vstride, nv, jdev, h, (cd*)w, n,
                       R);
  else
    hipLaunchKernelGGL((k_sub_combo<float>), nblk(n * R), 256, 0, s, (const cf*)V, vstride, nv, jdev, h, (cf*)w, n,
                       R);
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

hipError_t gm_scale(bool src128, const void* src, const double* f, bool dst128, void* dst, int64_t dstride,
                    const int* jdev, int64_t n, int R, hipStream_t s) {
  const unsigned nb = nblk(n * R);
  if (src128 && dst128)
    hipLaunchKernelGGL((k_scale<double, double>), nb, 256, 0, s, (const cd*)src, f, (cd*)dst, dstride, jdev, n, R);
  else if (src128)
    hipLaunchKernelGGL((k_scale<double, float>), nb, 256, 0, s, (const cd*)src, f, (cf*)dst, dstride, jdev, n, R);
  else if (dst128)
    hipLaunchKernelGGL((k_scale<float, double>), nb, 256, 0, s, (const cf*)src, f, (cd*)dst, dstride, jdev, n, R);
  else
    hipLaunchKernelGGL((k_scale<float, float>), nb, 256, 0, s, (const cf*)src, f, (cf*)dst, dstride, jdev, n, R);
  return hipGetLastError();
}

hipError_t gm_copy_basis(bool c128, const void* V, int64_t vstride, const int* jdev, void* dst, int64_t m,
                         hipStream_t s) {
  if (c128) hipLaunchKernelGGL((k_copy_basis<double>), nblk(m), 256, 0, s, (const cd*)V, vstride, jdev, (cd*)dst, m);
  else hipLaunchKernelGGL((k_copy_basis<float>), nblk(m), 256, 0, s, (const cf*)V, vstride, jdev, (cf*)dst, m);
  return hipGetLastError();
}

hipError_t gm_copy(bool c128, const void* src, void* dst, int64_t m, hipStream_t s) {
  if (c128) hipLaunchKernelGGL((k_copy<double>), nblk(m), 256, 0, s, (const cd*)src, (cd*)dst, m);
  else hipLaunchKernelGGL((k_copy<float>), nblk(m), 256, 0, s, (const cf*)src, (cf*)dst, m);
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

hipError_t gm_set_int(int* p, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_int, 1, 64, 0, s, p, v);
  return hipGetLastError();
}

hipError_t gm_impedance_grad(bool c128, const void* lam, const void* x, int64_t n, int R, void* out, hipStream_t s) {
  if (c128)
    hipLaunchKernelGGL((k_impedance_grad<double>), nblk(n), 256, 0, s, (const cd*)lam, (const cd*)x, n, R, (cd*)out);
  else
    hipLaunchKernelGGL((k_impedance_grad<float>), nblk(n), 256, 0, s, (const cf*)lam, (const cf*)x, n, R, (cf*)out);
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

hipError_t gm_h_accum(double* small, int m, int R, int j, const int* jdev, const cd* h, hipStream_t s) {
  hipLaunchKernelGGL(k_h_accum, nblk(R, 64), 64, 0, s, small, m, R, j, jdev, h);
  return hipGetLastError();
}

hipError_t gm_givens(double* small, int m, int R, int j, const int* jdev, const cd* nrm2, double* inv, double* resid,
                     const double* target, int* active, hipStream_t s) {
  hipLaunchKernelGGL(k_givens, nblk(R, 64), 64, 0, s, small, m, R, j, jdev, nrm2, inv, resid, target, active);
  return hipGetLastError();
}

hipError_t gm_step_end(int* jdev, const int* active, int R, int* any_active, hipStream_t s) {
  hipLaunchKernelGGL(k_step_end, 1, 64, 0, s, jdev, active, R, any_active);
  return hipGetLastError();
}

hipError_t gm_lsq(double* small, int m, int R, cd* y, hipStream_t s) {
  hipLaunchKernelGGL(k_lsq, nblk(R, 64), 64, 0, s, small, m, R, y);
  return hipGetLastError();
}

hipError_t gm_read_iters(double* small, int m, int R, int* out, hipStream_t s) {
  hipLaunchKernelGGL(k_read_iters, nblk(R, 64), 64, 0, s, small, m, R, out);
  return hipGetLastError();
}

// ---- TFQMR ----------------------------------------------------------------------

size_t tq_state_bytes(int R) { return static_cast<size_t>(R) * sizeof(TqState); }

hipError_t tq_start(void* S, int R, const cd* nrm2, const double* target, double* inv, double* resid, int* active,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_tq_start, nblk(R, 64), 64, 0, s, static_cast<TqState*>(S), R, nrm2, target, inv, resid, active);
  return hipGetLastError();
}
hipError_t tq_rho0(void* S, int R, const cd* dot, hipStream_t s) {
  hipLaunchKernelGGL(k_tq_rho0, nblk(R, 64), 64, 0, s, static_cast<TqState*>(S), R, dot);
  return hipGetLastError();
}
hipError_t tq_alpha(void* S, int R, const cd* sigma, int* active, hipStream_t s) {
  hipLaunchKernelGGL(k_tq_alpha, nblk(R, 64), 64, 0, s, static_cast<TqState*>(S), R, sigma, active);
  return hipGetLastError();
}
hipError_t tq_half(void* S, int R, const cd* wnrm2, double* resid, hipStream_t s) {
  hipLaunchKernelGGL(k_tq_half, nblk(R, 64), 64, 0, s, static_cast<TqState*>(S), R, wnrm2, resid);
  return hipGetLastError();
}
hipError_t tq_commit(void* S, int R, int* active, hipStream_t s) {
  hipLaunchKernelGGL(k_tq_commit, nblk(R, 64), 64, 0, s, static_cast<TqState*>(S), R, active);
  return hipGetLastError();
}
hipError_t tq_beta(void* S, int R, const cd* rhonew, int* active, hipStream_t s) {
  hipLaunchKernelGGL(k_tq_beta, nblk(R, 64), 64, 0, s, static_cast<TqState*>(S), R, rhonew, active);
  return hipGetLastError();
}
hipError_t tq_scales(const void* S, int R, double* f, hipStream_t s) {
  hipLaunchKernelGGL(k_tq_scales, nblk(R, 64), 64, 0, s, static_cast<const TqState*>(S), R, f);
  return hipGetLastError();
}
hipError_t tq_iters(const void* S, int R, int* out, hipStream_t s) {
  hipLaunchKernelGGL(k_tq_iters, nblk(R, 64), 64, 0, s, static_cast<const TqState*>(S), R, out);
  return hipGetLastError();
}

hipError_t tq_e1(bool c128, const void* S, const int* active, void* y2, const void* y, const void* v, void* w,
                 const void* u, void* d, int64_t n, int R, hipStream_t s) {
  const TqState* q = static_cast<const TqState*>(S);
  if (c128)
    hipLaunchKernelGGL((k_tq_e1<double>), nblk(n * R), 256, 0, s, q, active, (cd*)y2, (const cd*)y, (const cd*)v,
                       (cd*)w, (const cd*)u, (cd*)d, n, R);
  else
    hipLaunchKernelGGL((k_tq_e1<float>), nblk(n * R), 256, 0, s, q, active, (cf*)y2, (const cf*)y, (const cf*)v,
                       (cf*)w, (const cf*)u, (cf*)d, n, R);
  return hipGetLastError();
}
hipError_t tq_e2(bool c128, const void* S, const int* active, void* xh, const void* d, int64_t n, int R,
                 hipStream_t s) {
  const TqState* q = static_cast<const TqState*>(S);
  if (c128) hipLaunchKernelGGL((k_tq_e2<double>), nblk(n * R), 256, 0, s, q, active, (cd*)xh, (const cd*)d, n, R);
  else hipLaunchKernelGGL((k_tq_e2<float>), nblk(n * R), 256, 0, s, q, active, (cf*)xh, (const cf*)d, n, R);
  return hipGetLastError();
}
hipError_t tq_e3(bool c128, const void* S, const int* active, void* w, const void* u2, const void* y2, void* d,
                 int64_t n, int R, hipStream_t s) {
  const TqState* q = static_cast<const TqState*>(S);
  if (c128)
    hipLaunchKernelGGL((k_tq_e3<double>), nblk(n * R), 256, 0, s, q, active, (cd*)w, (const cd*)u2, (const cd*)y2,
                       (cd*)d, n, R);
  else
    hipLaunchKernelGGL((k_tq_e3<float>), nblk(n * R), 256, 0, s, q, active, (cf*)w, (const cf*)u2, (const cf*)y2,
                       (cf*)d, n, R);
  return hipGetLastError();
}
hipError_t tq_e4(bool c128, const void* S, const int* active, void* y, const void* w, const void* y2, int64_t n,
                 int R, hipStream_t s) {
  const TqState* q = static_cast<const TqState*>(S);
  if (c128)
    hipLaunchKernelGGL((k_tq_e4<double>), nblk(n * R), 256, 0, s, q, active, (cd*)y, (const cd*)w, (const cd*)y2, n,
                       R);
  else
    hipLaunchKernelGGL((k_tq_e4<float>), nblk(n * R), 256, 0, s, q, active, (cf*)y, (const cf*)w, (const cf*)y2, n,
                       R);
  return hipGetLastError();
}
hipError_t tq_e5(bool c128, const void* S, const int* active, void* v, const void* u, const void* u2, int64_t n,
                 int R, hipStream_t s) {
  const TqState* q = static_cast<const TqState*>(S);
  if (c128)
    hipLaunchKernelGGL((k_tq_e5<double>), nblk(n * R), 256, 0, s, q, active, (cd*)v, (const cd*)u, (const cd*)u2, n,
                       R);
  else
    hipLaunchKernelGGL((k_tq_e5<float>), nblk(n * R), 256, 0, s, q, active, (cf*)v, (const cf*)u, (const cf*)u2, n,
                       R);
  return hipGetLastError();
}
hipError_t tq_init(bool src128, const void* r0, const double* inv, bool c128, void* w, void* y, void* rt, void* d,
                   void* xh, int64_t n, int R, hipStream_t s) {
  const unsigned nb = nblk(n * R);
  if (src128 && c128)
    hipLaunchKernelGGL((k_tq_init<double, double>), nb, 256, 0, s, (const cd*)r0, inv, (cd*)w, (cd*)y, (cd*)rt,
                       (cd*)d, (cd*)xh, n, R);
  else if (src128)
    hipLaunchKernelGGL((k_tq_init<double, float>), nb, 256, 0, s, (const cd*)r0, inv, (cf*)w, (cf*)y, (cf*)rt,
                       (cf*)d, (cf*)xh, n, R);
  else if (c128)
    hipLaunchKernelGGL((k_tq_init<float, double>), nb, 256, 0, s, (const cf*)r0, inv, (cd*)w, (cd*)y, (cd*)rt,
                       (cd*)d, (cd*)xh, n, R);
  else
    hipLaunchKernelGGL((k_tq_init<float, float>), nb, 256, 0, s, (const cf*)r0, inv, (cf*)w, (cf*)y, (cf*)rt,
                       (cf*)d, (cf*)xh, n, R);
  return hipGetLastError();
}

}  // namespace hbf
