// Kernel entries of A = Z + diag(z) (Sec. 3.1) evaluated on the device for the
// construction: the sample and probe matrices of a batch of IDs, the dense
// leaf blocks, the middle couplings and the super-leaf blocks, one workgroup
// per index-set product.  Off-diagonal entries are evaluated here; the
// diagonal is the host's own evaluation, uploaded once.
//
// H0^(2)(x) = J0(x) - i Y0(x) in FP64 from the classical formulas (the same
// ones the host evaluation uses): below x = 25 Miller's backward recurrence
// for J_n normalised by 1 = J0 + 2 sum J_2k, with Y0 from the Neumann series
// (Abramowitz & Stegun 9.1.88); from x = 25 on Hankel's asymptotic expansion
// (A&S 9.2.8), summed until its terms fall below 1e-17.
#include <hip/hip_runtime.h>

#include <cstring>
#include <stdexcept>
#include <string>

#include "hbf_internal.h"

namespace hbf {

namespace {

constexpr double kPiD = 3.14159265358979323846;
constexpr double kEulerGammaD = 0.57721566490153286061;

__device__ double2 h0_asym(double x) {
  const double inv = 1.0 / x;
  double P = 0.0, Q = 0.0, p = 1.0, c = 1.0;
  for (int k = 0; k < 40; ++k) {
    const double term = c * p;
    switch (k & 3) {
      case 0: P += term; break;
      case 1: Q += term; break;
      case 2: P -= term; break;
      default: Q -= term; break;
    }
    if (term < 1e-17 && k > 2) break;
    p *= inv;
    const double t = 2.0 * (k + 1) - 1.0;
    c = c * t * t / (8.0 * (k + 1));
  }
  double s, co;
  sincos(x, &s, &co);
  const double r = sqrt(2.0 / (kPiD * x)) * 0.70710678118654752440;
  const double er = (co + s) * r, ei = (co - s) * r;
  return make_double2(er * P - ei * Q, er * Q + ei * P);
}

__device__ double2 h0_miller(double x) {
  int M = static_cast<int>(x + 12.0 * cbrt(x) + 24.0);
  M += (M & 1);
  const double two_over_x = 2.0 / x;
  double jp1 = 0.0, j = 1e-30;
  double norm = 0.0, neu = 0.0;
  for (int n = M; n >= 1; --n) {
    if ((n & 1) == 0) {
      norm += 2.0 * j;
      const int k = n / 2;
      neu += ((k & 1) ? -j : j) / k;
    }
    const double jm1 = n * two_over_x * j - jp1;
    jp1 = j;
    j = jm1;
    if (fabs(j) > 1e250) {
      j *= 1e-250; jp1 *= 1e-250; norm *= 1e-250; neu *= 1e-250;
    }
  }
  norm += j;
  const double J0 = j / norm;
  const double Y0 = (2.0 / kPiD) * (log(0.5 * x) + kEulerGammaD) * J0 - (4.0 / kPiD) * (neu / norm);
  return make_double2(J0, -Y0);
}

__device__ double2 h0(double x) { return x >= 25.0 ? h0_asym(x) : h0_miller(x); }

struct Geom {
  const double* cx;
  const double* cy;
  const double* w;
  const double2* self;    // the diagonal A[i, i] as the host evaluates it (self term + z; 1 on padding)
  const uint8_t* ghost;   // null: no padding
  double kappa, eta0;
};

__device__ double2 entry(const Geom& g, int i, int j) {
  if (i == j) return g.self[i];
  if (g.ghost && (g.ghost[i] || g.ghost[j])) return make_double2(0.0, 0.0);
  const double r = hypot(g.cx[i] - g.cx[j], g.cy[i] - g.cy[j]);
  const double2 h = h0(g.kappa * r);
  const double f = g.kappa * g.eta0 * g.w[j] / 4.0;
  return make_double2(f * h.x, f * h.y);
}

struct JobDev {
  int64_t rows, cols, out;  // offsets into the index and output arrays
  int32_t nr, nc, swap, pad;
};

__global__ void __launch_bounds__(256) k_entries(Geom g, const JobDev* jobs, const int32_t* idx, double2* out) {
  const JobDev jb = jobs[blockIdx.x];
  const int total = jb.nr * jb.nc;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    const int c = e / jb.nr, a = e - c * jb.nr;
    const int row = idx[jb.rows + a], col = idx[jb.cols + c];
    out[jb.out + e] = jb.swap ? entry(g, col, row) : entry(g, row, col);
  }
}

// ---- column ID of one sample matrix per workgroup (the host column_id's
// steps: pivoted Householder QR stopped at |R_kk| <= eps |R_11|, then
// T = R11^{-1} R12 by back substitution); thread j owns column j ----
struct IdDev {
  int32_t job, kmax;
  double eps;
  int64_t perm, T;  // output offsets (bytes of perm, entries of T)
};

constexpr int kIdThreads = 256;  // >= columns of any ID (candidates <= 255)
constexpr int kIdMaxRows = 256;  // >= rows of a first sample

__device__ __forceinline__ double norm2(double2 a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ double2 cmul2(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cdiv2(double2 a, double2 b) {
  const double d = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

__device__ double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int off = kIdThreads / 2; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(kIdThreads) k_column_id(const JobDev* jobs, const IdDev* ids, double2* mats,
                                                          int* kout, uint8_t* pout, double2* tout) {
  __shared__ double nrm[kIdThreads], nrm0[kIdThreads], red[kIdThreads];
  __shared__ int piv[kIdThreads], redi[kIdThreads];
  __shared__ double2 v[kIdMaxRows];
  const IdDev d = ids[blockIdx.x];
  const JobDev jb = jobs[d.job];
  double2* M = mats + jb.out;  // column-major s x n
  const int s = jb.nr, n = jb.nc;
  const int tid = threadIdx.x;
  if (tid < n) {
    piv[tid] = tid;
    double a = 0.0;
    for (int r = 0; r < s; ++r) a += norm2(M[static_cast<int64_t>(tid) * s + r]);
    nrm[tid] = nrm0[tid] = a;
  }
  __syncthreads();
  const int kcap = min(min(s, n), d.kmax);
  double ref = 0.0;
  int k = 0;
  for (int i = 0; i < kcap; ++i) {
    // norms that lost their accuracy to the downdates are recomputed on the remaining rows
    if (tid >= i && tid < n && nrm[tid] < 1e-4 * nrm0[tid]) {
      double a = 0.0;
      for (int r = i; r < s; ++r) a += norm2(M[static_cast<int64_t>(tid) * s + r]);
      nrm[tid] = nrm0[tid] = a;
    }
    __syncthreads();
    // pivot: the largest norm, the lowest column on ties
    red[tid] = (tid >= i && tid < n) ? nrm[tid] : -1.0;
    redi[tid] = tid;
    __syncthreads();
    for (int off = kIdThreads / 2; off > 0; off >>= 1) {
      if (tid < off) {
        const double o = red[tid + off];
        const int oi = redi[tid + off];
        if (o > red[tid] || (o == red[tid] && oi < redi[tid])) {
          red[tid] = o;
          redi[tid] = oi;
        }
      }
      __syncthreads();
    }
    const int p = redi[0];
    __syncthreads();
    // the exact norm of the pivot column on the remaining rows
    double part = 0.0;
    for (int r = i + tid; r < s; r += kIdThreads) part += norm2(M[static_cast<int64_t>(p) * s + r]);
    const double pn = sqrt(block_sum(part, red));
    if (i == 0) {
      ref = pn;
      if (ref == 0.0) break;
    } else if (pn <= d.eps * ref) {
      break;
    }
    if (p != i) {
      for (int r = tid; r < s; r += kIdThreads) {
        const double2 t = M[static_cast<int64_t>(i) * s + r];
        M[static_cast<int64_t>(i) * s + r] = M[static_cast<int64_t>(p) * s + r];
        M[static_cast<int64_t>(p) * s + r] = t;
      }
      if (tid == 0) {
        const int tp = piv[i]; piv[i] = piv[p]; piv[p] = tp;
        const double t1 = nrm[i]; nrm[i] = nrm[p]; nrm[p] = t1;
        const double t0 = nrm0[i]; nrm0[i] = nrm0[p]; nrm0[p] = t0;
      }
      __syncthreads();
    }
    // Householder vector of column i below the diagonal
    const double2 ci = M[static_cast<int64_t>(i) * s + i];
    const double a0 = sqrt(norm2(ci));
    const double2 ph = a0 > 0.0 ? make_double2(ci.x / a0, ci.y / a0) : make_double2(1.0, 0.0);
    const double2 alpha = make_double2(-ph.x * pn, -ph.y * pn);
    double vp = 0.0;
    for (int r = i + tid; r < s; r += kIdThreads) {
      double2 x = M[static_cast<int64_t>(i) * s + r];
      if (r == i) x = make_double2(x.x - alpha.x, x.y - alpha.y);
      v[r] = x;
      vp += norm2(x);
    }
    const double vn2 = block_sum(vp, red);  // (its barriers also publish v)
    for (int r = i + tid; r < s; r += kIdThreads)
      M[static_cast<int64_t>(i) * s + r] = r == i ? alpha : make_double2(0.0, 0.0);
    if (vn2 > 0.0 && tid > i && tid < n) {
      const double inv = 2.0 / vn2;
      double2* cj = M + static_cast<int64_t>(tid) * s;
      double2 dot = make_double2(0.0, 0.0);
      for (int r = i; r < s; ++r) {
        const double2 vr = v[r], x = cj[r];
        dot.x += vr.x * x.x + vr.y * x.y;  // conj(v) x
        dot.y += vr.x * x.y - vr.y * x.x;
      }
      dot.x *= inv;
      dot.y *= inv;
      for (int r = i; r < s; ++r) {
        const double2 t = cmul2(dot, v[r]);
        cj[r] = make_double2(cj[r].x - t.x, cj[r].y - t.y);
      }
      nrm[tid] = fmax(0.0, nrm[tid] - norm2(cj[i]));
    }
    k = i + 1;
    __syncthreads();
  }
  if (tid == 0) kout[blockIdx.x] = k;
  if (tid < n) pout[d.perm + tid] = static_cast<uint8_t>(piv[tid]);
  // T (k x r, row-major): column c of R12 solved against R11, thread c
  const int r = n - k;
  if (tid < r) {
    double2* T = tout + d.T;
    const double2* rc = M + static_cast<int64_t>(k + tid) * s;
    for (int ii = k - 1; ii >= 0; --ii) {
      double2 acc = rc[ii];
      for (int j = ii + 1; j < k; ++j) {
        const double2 t = cmul2(M[static_cast<int64_t>(j) * s + ii], T[static_cast<int64_t>(j) * r + tid]);
        acc = make_double2(acc.x - t.x, acc.y - t.y);
      }
      T[static_cast<int64_t>(ii) * r + tid] = cdiv2(acc, M[static_cast<int64_t>(ii) * s + ii]);
    }
  }
}

void check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw std::runtime_error(std::string("device entries: ") + what + ": " + hipGetErrorString(e));
}

class DeviceEntries final : public EntryEval {
 public:
  explicit DeviceEntries(int device) : device_(device) {}
  ~DeviceEntries() override {
    for (void* p : {geo_, idx_, jobs_, out_}) if (p) (void)hipFree(p);
    if (host_) (void)hipHostFree(host_);
    if (stream_) (void)hipStreamDestroy(stream_);
  }

  void prepare(const Plan& P) override {
    check(hipSetDevice(device_), "hipSetDevice");
    if (!stream_) check(hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking), "stream");
    const size_t n = static_cast<size_t>(P.n);
    const size_t bytes = 3 * n * sizeof(double) + n * 16 + (P.ghost.empty() ? 0 : n) + 64;
    if (geo_) (void)hipFree(geo_);
    geo_ = nullptr;
    check(hipMalloc(&geo_, bytes), "geometry");
    char* p = static_cast<char*>(geo_);
    g_.cx = reinterpret_cast<const double*>(p);
    check(hipMemcpy(p, P.cx.data(), n * sizeof(double), hipMemcpyHostToDevice), "geometry");
    p += n * sizeof(double);
    g_.cy = reinterpret_cast<const double*>(p);
    check(hipMemcpy(p, P.cy.data(), n * sizeof(double), hipMemcpyHostToDevice), "geometry");
    p += n * sizeof(double);
    g_.w = reinterpret_cast<const double*>(p);
    check(hipMemcpy(p, P.w.data(), n * sizeof(double), hipMemcpyHostToDevice), "geometry");
    p += n * sizeof(double);
    // the diagonal from the host's own evaluation, so that it is bit for bit
    // the one every other part of the library uses (an exactly singular leaf
    // stays exactly singular)
    std::vector<cplx> self(n);
    for (size_t i = 0; i < n; ++i) self[i] = P.self_entry(static_cast<int64_t>(i));
    g_.self = reinterpret_cast<const double2*>(p);
    check(hipMemcpy(p, self.data(), n * 16, hipMemcpyHostToDevice), "diagonal");
    p += n * 16;
    g_.ghost = nullptr;
    if (!P.ghost.empty()) {
      g_.ghost = reinterpret_cast<const uint8_t*>(p);
      check(hipMemcpy(p, P.ghost.data(), n, hipMemcpyHostToDevice), "padding");
    }
    g_.kappa = P.kappa;
    g_.eta0 = P.eta0;
  }

  void eval(const std::vector<EntryJob>& jobs, const std::vector<IdJob>& ids) override {
    if (jobs.empty()) return;
    check(hipSetDevice(device_), "hipSetDevice");
    // matrices with an output pointer first (one download), then those that
    // only feed an ID
    std::vector<JobDev> jd(jobs.size());
    int64_t ni = 0, no = 0;
    for (int pass = 0; pass < 2; ++pass)
      for (size_t q = 0; q < jobs.size(); ++q) {
        if ((jobs[q].out != nullptr) != (pass == 0)) continue;
        jd[q] = JobDev{0, 0, no, jobs[q].nrows, jobs[q].ncols, jobs[q].swap, 0};
        no += static_cast<int64_t>(jobs[q].nrows) * jobs[q].ncols;
      }
    int64_t kept = 0;
    for (size_t q = 0; q < jobs.size(); ++q)
      if (jobs[q].out) kept += static_cast<int64_t>(jobs[q].nrows) * jobs[q].ncols;
    for (size_t q = 0; q < jobs.size(); ++q) {
      jd[q].rows = ni;
      jd[q].cols = ni + jobs[q].nrows;
      ni += jobs[q].nrows + jobs[q].ncols;
    }
    std::vector<int32_t> idx(static_cast<size_t>(ni));
    for (size_t q = 0; q < jobs.size(); ++q) {
      std::memcpy(&idx[jd[q].rows], jobs[q].rows, sizeof(int32_t) * jobs[q].nrows);
      std::memcpy(&idx[jd[q].cols], jobs[q].cols, sizeof(int32_t) * jobs[q].ncols);
    }
    // ID outputs: pivot bytes and interpolation matrices at offsets
    std::vector<IdDev> idd(ids.size());
    int64_t npb = 0, nT = 0;
    for (size_t q = 0; q < ids.size(); ++q) {
      const int nc = jobs[ids[q].job].ncols;
      if (jobs[ids[q].job].nrows > kIdMaxRows || nc > kIdThreads)
        throw std::runtime_error("device entries: ID matrix larger than the kernel's limits");
      idd[q] = IdDev{ids[q].job, ids[q].kmax, ids[q].eps, npb, nT};
      npb += nc;
      nT += static_cast<int64_t>(nc) * nc / 4 + 1;
    }
    const size_t b_out = static_cast<size_t>(no) * 16, b_kept = static_cast<size_t>(kept) * 16;
    const size_t b_k = ids.size() * sizeof(int), b_p = static_cast<size_t>(npb), b_T = static_cast<size_t>(nT) * 16;
    grow(&idx_, idx_cap_, idx.size() * sizeof(int32_t));
    grow(&jobs_, jobs_cap_, jd.size() * sizeof(JobDev) + idd.size() * sizeof(IdDev));
    grow(&out_, out_cap_, b_out + b_T + b_k + b_p + 64);
    // pinned staging: kept matrices, then T, k, pivot bytes
    const size_t b_host = b_kept + b_T + b_k + b_p + 64;
    if (b_host > host_cap_) {
      if (host_) (void)hipHostFree(host_);
      host_ = nullptr;
      host_cap_ = b_host + b_host / 4;
      check(hipHostMalloc(&host_, host_cap_, hipHostMallocDefault), "pinned staging");
    }
    char* dev = static_cast<char*>(out_);
    double2* d_mats = reinterpret_cast<double2*>(dev);
    double2* d_T = reinterpret_cast<double2*>(dev + b_out);
    int* d_k = reinterpret_cast<int*>(dev + b_out + b_T);
    uint8_t* d_p = reinterpret_cast<uint8_t*>(dev + b_out + b_T + b_k);
    JobDev* d_jobs = static_cast<JobDev*>(jobs_);
    IdDev* d_ids = reinterpret_cast<IdDev*>(d_jobs + jd.size());
    check(hipMemcpyAsync(idx_, idx.data(), idx.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream_), "upload");
    check(hipMemcpyAsync(d_jobs, jd.data(), jd.size() * sizeof(JobDev), hipMemcpyHostToDevice, stream_), "upload");
    if (!idd.empty())
      check(hipMemcpyAsync(d_ids, idd.data(), idd.size() * sizeof(IdDev), hipMemcpyHostToDevice, stream_), "upload");
    hipLaunchKernelGGL(k_entries, dim3(static_cast<unsigned>(jd.size())), dim3(256), 0, stream_, g_,
                       static_cast<const JobDev*>(d_jobs), static_cast<const int32_t*>(idx_), d_mats);
    check(hipGetLastError(), "launch");
    if (!idd.empty()) {
      hipLaunchKernelGGL(k_column_id, dim3(static_cast<unsigned>(idd.size())), dim3(kIdThreads), 0, stream_,
                         static_cast<const JobDev*>(d_jobs), static_cast<const IdDev*>(d_ids), d_mats, d_k, d_p, d_T);
      check(hipGetLastError(), "launch");
    }
    char* h = static_cast<char*>(host_);
    if (b_kept) check(hipMemcpyAsync(h, d_mats, b_kept, hipMemcpyDeviceToHost, stream_), "download");
    if (!idd.empty())
      check(hipMemcpyAsync(h + b_kept, d_T, b_T + b_k + b_p, hipMemcpyDeviceToHost, stream_), "download");
    check(hipStreamSynchronize(stream_), "sync");
    for (size_t q = 0; q < jobs.size(); ++q)
      if (jobs[q].out)
        std::memcpy(jobs[q].out, h + jd[q].out * 16, sizeof(cplx) * static_cast<size_t>(jd[q].nr) * jd[q].nc);
    const cplx* hT = reinterpret_cast<const cplx*>(h + b_kept);
    const int* hk = reinterpret_cast<const int*>(h + b_kept + b_T);
    const uint8_t* hp = reinterpret_cast<const uint8_t*>(h + b_kept + b_T + b_k);
    for (size_t q = 0; q < ids.size(); ++q) {
      const int nc = jobs[ids[q].job].ncols;
      const int k = hk[q];
      *ids[q].k = k;
      std::memcpy(ids[q].perm, hp + idd[q].perm, static_cast<size_t>(nc));
      std::memcpy(ids[q].T, hT + idd[q].T, sizeof(cplx) * static_cast<size_t>(k) * (nc - k));
    }
  }

 private:
  void grow(void** p, size_t& cap, size_t need) {
    if (need <= cap) return;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    cap = need + need / 4;
    check(hipMalloc(p, cap), "workspace");
  }
  int device_;
  hipStream_t stream_ = nullptr;
  void* geo_ = nullptr;
  void* idx_ = nullptr;
  void* jobs_ = nullptr;
  void* out_ = nullptr;
  void* host_ = nullptr;
  size_t idx_cap_ = 0, jobs_cap_ = 0, out_cap_ = 0, host_cap_ = 0;
  Geom g_{};
};

}  // namespace

std::unique_ptr<EntryEval> make_device_entry_eval(int device) {
  return std::unique_ptr<EntryEval>(new DeviceEntries(device));
}

}  // namespace hbf
