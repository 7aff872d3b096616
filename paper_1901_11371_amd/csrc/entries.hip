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

  void eval(const std::vector<EntryJob>& jobs) override {
    if (jobs.empty()) return;
    check(hipSetDevice(device_), "hipSetDevice");
    std::vector<JobDev> jd(jobs.size());
    int64_t ni = 0, no = 0;
    for (size_t q = 0; q < jobs.size(); ++q) {
      jd[q] = JobDev{ni, ni + jobs[q].nrows, no, jobs[q].nrows, jobs[q].ncols, jobs[q].swap, 0};
      ni += jobs[q].nrows + jobs[q].ncols;
      no += static_cast<int64_t>(jobs[q].nrows) * jobs[q].ncols;
    }
    std::vector<int32_t> idx(static_cast<size_t>(ni));
    for (size_t q = 0; q < jobs.size(); ++q) {
      std::memcpy(&idx[jd[q].rows], jobs[q].rows, sizeof(int32_t) * jobs[q].nrows);
      std::memcpy(&idx[jd[q].cols], jobs[q].cols, sizeof(int32_t) * jobs[q].ncols);
    }
    grow(&idx_, idx_cap_, idx.size() * sizeof(int32_t));
    grow(&jobs_, jobs_cap_, jd.size() * sizeof(JobDev));
    grow(&out_, out_cap_, static_cast<size_t>(no) * 16);
    if (static_cast<size_t>(no) * 16 > host_cap_) {
      if (host_) (void)hipHostFree(host_);
      host_ = nullptr;
      host_cap_ = static_cast<size_t>(no) * 16;
      check(hipHostMalloc(&host_, host_cap_, hipHostMallocDefault), "pinned staging");
    }
    check(hipMemcpyAsync(idx_, idx.data(), idx.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream_), "upload");
    check(hipMemcpyAsync(jobs_, jd.data(), jd.size() * sizeof(JobDev), hipMemcpyHostToDevice, stream_), "upload");
    hipLaunchKernelGGL(k_entries, dim3(static_cast<unsigned>(jd.size())), dim3(256), 0, stream_, g_,
                       static_cast<const JobDev*>(jobs_), static_cast<const int32_t*>(idx_),
                       static_cast<double2*>(out_));
    check(hipGetLastError(), "launch");
    check(hipMemcpyAsync(host_, out_, static_cast<size_t>(no) * 16, hipMemcpyDeviceToHost, stream_), "download");
    check(hipStreamSynchronize(stream_), "sync");
    const cplx* h = static_cast<const cplx*>(host_);
    for (size_t q = 0; q < jobs.size(); ++q)
      std::memcpy(jobs[q].out, h + jd[q].out, sizeof(cplx) * static_cast<size_t>(jd[q].nr) * jd[q].nc);
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
