// FP64 Hankel functions of the first kind, orders 0 and 1, for complex
// argument z with Re z > 0 and Im z >= 0 (the k0 r of an absorbing medium).
//
// Used by the Green's-function tabulation: the 2D free-space Green's function
// is (i/4) H0(k0 r) and the disk self-cell integral needs H1(k0 a).  The C++
// standard library has real-argument Bessel functions only, so both regimes
// are written out here:
//
//  * |z| <= 2: the ascending power series of J0, J1, Y0, Y1
//    (Abramowitz & Stegun 9.1.10, 9.1.11 / 9.1.13), H = J + iY.
//  * |z| >  2: Hankel's integral (Watson, Theory of Bessel Functions, ch. 7)
//        H_nu(z) = sqrt(2/(pi z)) e^{i(z - nu pi/2 - pi/4)} / Gamma(nu+1/2)
//                  * int_0^inf e^{-u} u^{nu-1/2} (1 + iu/(2z))^{nu-1/2} du,
//    with u = t^2 so the integrand is smooth and Gaussian-decaying, evaluated
//    by the trapezoidal rule (step 0.2, |t| <= 6.6).  The integrand's nearest
//    singularity sits sqrt(|z|) off the real t axis, so the rule's error is
//    about exp(-2 pi sqrt(|z|) / 0.2) < 1e-30 for |z| > 2.
//
// hankel1_1_reg returns H1(z) + 2i/(pi z), the part of H1 that stays finite as
// z -> 0; the disk self-cell integral subtracts exactly the singular part, so
// computing the remainder directly avoids the cancellation.
//
// Plain C++ when not compiled by hipcc, so the host code and a host-only test
// build share it.
#pragma once

#include <cmath>

#ifndef __HIPCC__
#ifndef __host__
#define __host__
#endif
#ifndef __device__
#define __device__
#endif
#endif

namespace tbs {

struct zd {
  double re, im;
};

__host__ __device__ inline zd zmake(double r, double i) { return zd{r, i}; }
__host__ __device__ inline zd zadd(zd a, zd b) { return zd{a.re + b.re, a.im + b.im}; }
__host__ __device__ inline zd zsub(zd a, zd b) { return zd{a.re - b.re, a.im - b.im}; }
__host__ __device__ inline zd zmul(zd a, zd b) {
  return zd{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__host__ __device__ inline zd zscale(zd a, double s) { return zd{a.re * s, a.im * s}; }
__host__ __device__ inline zd zdiv(zd a, zd b) {
  // Smith's algorithm
  if (fabs(b.re) >= fabs(b.im)) {
    double r = b.im / b.re, d = b.re + b.im * r;
    return zd{(a.re + a.im * r) / d, (a.im - a.re * r) / d};
  }
  double r = b.re / b.im, d = b.re * r + b.im;
  return zd{(a.re * r + a.im) / d, (a.im * r - a.re) / d};
}
__host__ __device__ inline double zabs(zd a) { return hypot(a.re, a.im); }
__host__ __device__ inline zd zexp(zd a) {
  double e = exp(a.re);
  return zd{e * cos(a.im), e * sin(a.im)};
}
__host__ __device__ inline zd zlog(zd a) { return zd{log(zabs(a)), atan2(a.im, a.re)}; }
// principal square root
__host__ __device__ inline zd zsqrt(zd a) {
  double m = zabs(a);
  if (m == 0.0) return zd{0.0, 0.0};
  if (a.re >= 0.0) {
    double t = sqrt(0.5 * (m + a.re));
    return zd{t, a.im / (2.0 * t)};
  }
  double t = sqrt(0.5 * (m - a.re));
  return zd{fabs(a.im) / (2.0 * t), copysign(t, a.im)};
}

constexpr double kPi = 3.14159265358979323846;
constexpr double kEulerGamma = 0.57721566490153286061;

// Power series, |z| <= 2.  h0 = H0(z); h1r = H1(z) + 2i/(pi z).
__host__ __device__ inline void hankel01_series(zd z, zd* h0, zd* h1r) {
  const zd q = zscale(zmul(z, z), -0.25);  // -z^2/4
  zd term0 = zd{1.0, 0.0};                 // (-z^2/4)^k / (k!)^2
  zd term1 = zd{1.0, 0.0};                 // (-z^2/4)^k / (k! (k+1)!)
  zd j0 = term0, j1s = term1;
  zd s0 = zd{0.0, 0.0};                    // sum_{k>=1} (-1)^{k+1} H_k (z^2/4)^k/(k!)^2
  zd s1 = zd{0.0, 0.0};                    // sum_{k>=0} (psi(k+1)+psi(k+2)) (-z^2/4)^k/(k!(k+1)!)
  double hk = 0.0;                         // harmonic number H_k
  s1 = zscale(term1, (-kEulerGamma) + (1.0 - kEulerGamma));
  for (int k = 1; k <= 40; ++k) {
    term0 = zscale(zmul(term0, q), 1.0 / ((double)k * (double)k));
    term1 = zscale(zmul(term1, q), 1.0 / ((double)k * (double)(k + 1)));
    hk += 1.0 / k;
    j0 = zadd(j0, term0);
    j1s = zadd(j1s, term1);
    // (-1)^{k+1} (z^2/4)^k = -( -z^2/4 )^k
    s0 = zsub(s0, zscale(term0, hk));
    // psi(k+1) + psi(k+2) = 2(H_k - gamma) + 1/(k+1)
    s1 = zadd(s1, zscale(term1, 2.0 * (hk - kEulerGamma) + 1.0 / (k + 1)));
  }
  const zd zh = zscale(z, 0.5);
  const zd lg = zlog(zh);
  const zd j1 = zmul(zh, j1s);
  // Y0 = (2/pi)(ln(z/2)+gamma) J0 + (2/pi) s0
  zd y0 = zscale(zadd(zmul(zadd(lg, zd{kEulerGamma, 0.0}), j0), s0), 2.0 / kPi);
  // Y1 + 2/(pi z) = (2/pi) ln(z/2) J1 - (1/pi)(z/2) s1
  zd y1r = zsub(zscale(zmul(lg, j1), 2.0 / kPi), zscale(zmul(zh, s1), 1.0 / kPi));
  *h0 = zd{j0.re - y0.im, j0.im + y0.re};
  *h1r = zd{j1.re - y1r.im, j1.im + y1r.re};
}

// Integral representation, |z| > 2.
__host__ __device__ inline void hankel01_integral(zd z, zd* h0, zd* h1) {
  const double h = 0.2;
  const zd inv2z = zdiv(zd{0.0, 0.5}, z);  // i/(2z)
  zd a0 = zd{0.0, 0.0}, a1 = zd{0.0, 0.0};
  for (int n = 0; n <= 33; ++n) {
    const double t = n * h;
    const double t2 = t * t;
    const double w = (n == 0 ? 0.5 : 1.0) * exp(-t2);
    const zd b = zadd(zd{1.0, 0.0}, zscale(inv2z, t2));   // 1 + i t^2/(2z)
    const zd rs = zsqrt(b);
    const zd ir = zdiv(zd{1.0, 0.0}, rs);                  // b^{-1/2}
    a0 = zadd(a0, zscale(ir, w));
    a1 = zadd(a1, zscale(rs, w * t2));                     // t^2 b^{1/2}
  }
  // integrals: 2 h sum; Gamma(1/2) = sqrt(pi), Gamma(3/2) = sqrt(pi)/2
  a0 = zscale(a0, 2.0 * h / sqrt(kPi));
  a1 = zscale(a1, 4.0 * h / sqrt(kPi));
  // prefactor sqrt(2/(pi z)) e^{i(z - nu pi/2 - pi/4)}; e^{iz} and e^{-i pi/4}
  // are formed separately so that no rounding enters the large phase Re z.
  const double r2 = 0.70710678118654752440;
  const zd pre = zmul(zmul(zsqrt(zdiv(zd{2.0 / kPi, 0.0}, z)), zexp(zd{-z.im, z.re})), zd{r2, -r2});
  *h0 = zmul(pre, a0);
  *h1 = zmul(zmul(pre, zd{0.0, -1.0}), a1);   // e^{-i pi/2} = -i
}

__host__ __device__ inline void hankel01(zd z, zd* h0, zd* h1) {
  if (zabs(z) <= 2.0) {
    zd h1r;
    hankel01_series(z, h0, &h1r);
    const zd sing = zdiv(zd{0.0, 2.0 / kPi}, z);  // 2i/(pi z)
    *h1 = zsub(h1r, sing);
  } else {
    hankel01_integral(z, h0, h1);
  }
}

// H1(z) + 2i/(pi z)
__host__ __device__ inline zd hankel1_1_reg(zd z) {
  zd h0, h1;
  if (zabs(z) <= 2.0) {
    hankel01_series(z, &h0, &h1);
    return h1;
  }
  hankel01_integral(z, &h0, &h1);
  return zadd(h1, zdiv(zd{0.0, 2.0 / kPi}, z));
}

// W(0) for the 2D disk cell of area dx^2: (i pi a/(2 k0)) H1(k0 a) - 1/k0^2
// = (i pi a/(2 k0)) (H1(k0 a) + 2i/(pi k0 a)).
__host__ __device__ inline zd self_cell_2d(zd k0, double dx) {
  const double a = dx / sqrt(kPi);
  const zd z = zscale(k0, a);
  const zd pre = zdiv(zd{0.0, 0.5 * kPi * a}, k0);
  return zmul(pre, hankel1_1_reg(z));
}

// W(0) for the 3D ball cell of volume dx^3: ((1 - i k0 a) e^{i k0 a} - 1)/k0^2.
__host__ __device__ inline zd self_cell_3d(zd k0, double dx) {
  const double a = dx * cbrt(3.0 / (4.0 * kPi));
  const zd x = zscale(k0, a);
  zd num;
  if (zabs(x) < 0.5) {
    // series of (1 - ix) e^{ix} - 1 = sum_{n>=2} (ix)^n (1/n! - 1/(n-1)!) ... = sum_{n>=2} (ix)^n (1-n)/n!
    zd ix = zd{-x.im, x.re};
    zd pw = zmul(ix, ix);  // (ix)^2
    double fact = 2.0;
    num = zd{0.0, 0.0};
    for (int n = 2; n <= 24; ++n) {
      num = zadd(num, zscale(pw, (1.0 - n) / fact));
      pw = zmul(pw, ix);
      fact *= (n + 1);
    }
  } else {
    const zd e = zexp(zd{-x.im, x.re});
    num = zsub(zmul(zd{1.0 + x.im, -x.re}, e), zd{1.0, 0.0});
  }
  return zdiv(num, zmul(k0, k0));
}

}  // namespace tbs
