// Host construction under AddressSanitizer / UndefinedBehaviorSanitizer:
// builds the H-IDBF of a small arc and a two-curve layout with both
// preconditioner readings, both super-leaf sizes and both storage dtypes'
// schedules, and evaluates matvec and preconditioner (forward and adjoint,
// three right-hand sides) with the host FP64 executor.  Compiled by
// tests/test_host_asan.py with g++ (no GPU code); any memory error aborts.
#include <cmath>
#include <cstdio>
#include <vector>

#include "../../include/hbf.h"

namespace hbf {
// The device program kernel's LDS row budget (defined next to the kernel in
// the library): 160 KiB less 16 (complex64) or 12 (complex128) waves of
// staging, the descriptor ring and the step window, in vector rows.
int prog_lds_rows_budget(int elt_fac, int elt_vec) {
  const int waves = elt_fac == 8 ? 16 : 12;
  const int base = (1024 + 256 * 16) * waves + 3 * 64 * 64 + 5 * 4 * 128 + 16;
  return (160 * 1024 - base) / elt_vec;
}
}  // namespace hbf

static int run(const hbf_curve& c, int n, int dtype, int prec, int sl) {
  hbf_build_opts o{};
  o.dtype = static_cast<hbf_dtype>(dtype);
  o.prec = static_cast<hbf_prec>(prec);
  o.superleaf = sl;
  o.nthreads = 2;
  hbf_plan* p = nullptr;
  if (hbf_plan_build(&c, 2 * M_PI, 64, 1e-6, &o, &p) != HBF_OK) {
    std::printf("build failed: %s\n", hbf_last_error());
    return 1;
  }
  const int R = 3;
  std::vector<double> x(2 * n * R), y(2 * n * R), z(2 * n * R);
  for (size_t i = 0; i < x.size(); ++i) x[i] = std::sin(0.37 * static_cast<double>(i));
  for (int adj = 0; adj < 2; ++adj) {
    if (hbf_plan_apply(p, x.data(), y.data(), R, adj) != HBF_OK) return 2;
    if (hbf_plan_precond(p, x.data(), z.data(), R, adj) != HBF_OK) return 3;
  }
  double s = 0;
  for (double v : z) s += std::fabs(v);
  std::printf("n %d dtype %d prec %d superleaf %d: ok (|z|_1 %.6e)\n", n, dtype, prec, sl, s);
  hbf_plan_free(p);
  return 0;
}

int main() {
  const int n = 2048;
  std::vector<double> xy(2 * (n + 1));
  const double L = n / 10.0, rad = L / (M_PI / 2);
  for (int i = 0; i <= n; ++i) {
    const double t = (M_PI / 2) * i / n;
    xy[2 * i] = rad * std::cos(t);
    xy[2 * i + 1] = rad * std::sin(t);
  }
  int64_t off1[2] = {0, n + 1};
  const hbf_curve arc{1, off1, xy.data()};
  // two strips of 512 segments, 5 wavelengths apart
  const int m = 512;
  std::vector<double> xy2(2 * 2 * (m + 1));
  for (int k = 0; k < 2; ++k)
    for (int i = 0; i <= m; ++i) {
      xy2[2 * (k * (m + 1) + i)] = 0.1 * i;
      xy2[2 * (k * (m + 1) + i) + 1] = 5.0 * k;
    }
  int64_t off2[3] = {0, m + 1, 2 * (m + 1)};
  const hbf_curve two{2, off2, xy2.data()};
  for (int dtype = 0; dtype < 2; ++dtype)
    for (int prec = 0; prec < 2; ++prec)
      for (int sl = 2; sl <= 3; ++sl) {
        if (int e = run(arc, n, dtype, prec, sl)) return e;
      }
  if (int e = run(two, 2 * m, 0, 0, 2)) return e;
  // invalid input is rejected without touching memory
  hbf_build_opts o{};
  o.superleaf = 1;
  hbf_plan* p = nullptr;
  if (hbf_plan_build(&arc, 2 * M_PI, 64, 1e-6, &o, &p) != HBF_EINVAL || p) return 4;
  std::printf("all host checks passed\n");
  return 0;
}
