// FP64 evaluation of the zeroth-order Hankel function of the second kind,
// H0^(2)(x) = J0(x) - i Y0(x), x > 0 -- the kernel of the TM_z EFIE impedance
// matrix (paper Sec. 3.1).  The paper names no evaluation method; this one is
// written from the classical formulas:
//
//  * x < 25: J_n(x) by Miller's backward recurrence J_{n-1} = (2n/x) J_n - J_{n+1}
//    from a start index well above x, normalised with 1 = J_0 + 2 sum_k J_{2k};
//    Y0 from the Neumann series
//      Y0(x) = (2/pi)(ln(x/2) + gamma_E) J0(x) - (4/pi) sum_{k>=1} (-1)^k J_{2k}(x)/k
//    (Abramowitz & Stegun 9.1.88), using the same recurrence values.
//  * x >= 25: Hankel's asymptotic expansion (A&S 9.2.8 / DLMF 10.17.4)
//      H0^(2)(x) ~ sqrt(2/(pi x)) e^{-i(x - pi/4)} sum_k i^k c_k x^{-k},
//      c_k = prod_{j=1..k} (2j-1)^2 / (k! 8^k),
//    summed until the terms fall below 1e-17 (at x >= 25 the smallest term of
//    the divergent series is far below double precision).
#include "hbf_internal.h"

#include <cmath>

namespace hbf {

namespace {
constexpr double kPi = 3.14159265358979323846;
constexpr double kEulerGamma = 0.57721566490153286061;
constexpr double kAsymX = 25.0;
constexpr int kAsymTerms = 40;

struct AsymCoef {
  double c[kAsymTerms];
  AsymCoef() {
    c[0] = 1.0;
    for (int k = 1; k < kAsymTerms; ++k) {
      const double t = 2.0 * k - 1.0;
      c[k] = c[k - 1] * t * t / (8.0 * k);
    }
  }
};
const AsymCoef kCoef;

inline cplx hankel_asym(double x) {
  // sum_k i^k c_k / x^k = P + i Q
  const double inv = 1.0 / x;
  double P = 0.0, Q = 0.0, p = 1.0;
  for (int k = 0; k < kAsymTerms; ++k) {
    const double term = kCoef.c[k] * p;
    switch (k & 3) {
      case 0: P += term; break;
      case 1: Q += term; break;
      case 2: P -= term; break;
      default: Q -= term; break;
    }
    if (term < 1e-17 && k > 2) break;
    p *= inv;
  }
  double s, c;
  sincos(x, &s, &c);
  // e^{-i(x - pi/4)} = (cos x - i sin x)(1 + i)/sqrt(2)
  const double r = std::sqrt(2.0 / (kPi * x)) * 0.70710678118654752440;
  const double er = (c + s) * r, ei = (c - s) * r;
  return cplx(er * P - ei * Q, er * Q + ei * P);
}

inline cplx hankel_miller(double x) {
  // start index: even, comfortably above x so that J_M / J_0 is negligible
  int M = static_cast<int>(x + 12.0 * std::cbrt(x) + 24.0);
  M += (M & 1);
  const double two_over_x = 2.0 / x;
  double jp1 = 0.0, j = 1e-30;  // J_{M+1}, J_M (arbitrary scale)
  double norm = 0.0;     // J_0 + 2 sum J_{2k}
  double neu = 0.0;      // sum_{k>=1} (-1)^k J_{2k} / k
  for (int n = M; n >= 1; --n) {
    // j holds J_n; account for it when n is even
    if ((n & 1) == 0) {
      norm += 2.0 * j;
      const int k = n / 2;
      neu += ((k & 1) ? -j : j) / k;
    }
    const double jm1 = n * two_over_x * j - jp1;
    jp1 = j;
    j = jm1;
    if (std::fabs(j) > 1e250) {  // rescale to avoid overflow at small x
      j *= 1e-250; jp1 *= 1e-250; norm *= 1e-250; neu *= 1e-250;
    }
  }
  norm += j;  // J_0
  const double J0 = j / norm;
  const double Y0 = (2.0 / kPi) * (std::log(0.5 * x) + kEulerGamma) * J0 - (4.0 / kPi) * (neu / norm);
  return cplx(J0, -Y0);
}
}  // namespace

cplx hankel2_0(double x) {
  if (x >= kAsymX) return hankel_asym(x);
  return hankel_miller(x);
}

}  // namespace hbf
