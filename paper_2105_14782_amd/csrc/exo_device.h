// Device-side building blocks shared by the exohip kernels (gfx950).
//
// Physical model: Kawahara et al., arXiv:2105.14782 (see include/exohip.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace exo {

// ---- constants (cgs; exact SI definitions of h, c, k_B; CODATA 2018 m_u) ----
constexpr double kH = 6.62607015e-27;      // erg s
constexpr double kC = 2.99792458e10;       // cm s^-1
constexpr double kKB = 1.380649e-16;       // erg K^-1
constexpr double kMU = 1.66053906660e-24;  // g
constexpr double kC2 = kH * kC / kKB;      // cm K, second radiation constant
constexpr double kTref = 296.0;            // K
constexpr double kBar = 1.0e6;             // dyn cm^-2
constexpr double kCkms = 2.99792458e5;     // km s^-1
constexpr double kPi = 3.14159265358979323846;
constexpr double kSqrtPi = 1.77245385090551602730;
constexpr double kSqrt2 = 1.41421356237309504880;
constexpr double kLn10 = 2.30258509299404568402;

// Voigt-Hjerting branch switch of the paper's hjert: core (the series in the
// paper) for x^2 + a^2 < 111, asymptotic w_2 otherwise (Sec. 2.1.1).
constexpr double kHjertSwitch = 111.0;
constexpr int kM916 = 27;                  // series length M (plain FP64 form)
// Core branch of the FP32 sum: Weideman's rational approximation of w with
// 20-32 terms by the pair's a (Weideman 1994, SIAM J. Numer. Anal. 31, 1497)
// at z for a >= kWeidAmin (H within 2.3e-7 relative over x^2 + a^2 < 111
// there), and on the real axis, continued to first order in a, below.
constexpr double kWeidAmin = 1e-5;

// Records written by the line-parameter kernel for one (line, layer) and read
// uniformly (staged per wave through LDS) by the Voigt-sum kernel.  Wing branch in physical
// variables: with D = dnu^2 + gamma^2 and r = 1/D, the real part of the
// asymptotic w_2 (Eq. asywofz, n = 2) divided by sqrt(2 pi) beta is exactly
//   (gamma/pi) r [1 + 3b r + (15b^2 - 4bg) r^2 + (105b^3 - 60b^2 g) r^3
//                 + (48b^2g^2 - 840b^3 g) r^4 + 1680 b^3 g^2 r^5 - 960 b^3 g^3 r^6]
// with b = beta^2, g = gamma^2 (expand Re[i/zeta (1 + b/zeta^2 + 3b^2/zeta^4
// + 15 b^3/zeta^6)], zeta = dnu + i gamma, in powers of r).  e_k below are
// those coefficients times the line amplitude.
struct LineRec {
  float e[7];     // wing polynomial, amplitude included
  float gam2;     // gamma^2
  float thr;      // 2 beta^2 * 111: core branch iff D < thr
  float winv;     // 1 / (sqrt2 beta)
  float a;        // gamma / (sqrt2 beta)
  float acore;    // amplitude / (sqrt(2 pi) beta): contribution = acore * H(x, a)
  float pad[4];
};
static_assert(sizeof(LineRec) == 64, "LineRec layout");

// d/dT of the same contribution (tangent mode).
struct LineRecT {
  float t[8];     // wing: d f/dT = r * sum_k t_k r^k
  float kA;       // d ln(acore)/dT
  float kw;       // d ln(winv)/dT = -1/(2T)
  float da;       // da/dT
  float pad[5];
};
static_assert(sizeof(LineRecT) == 64, "LineRecT layout");

// Plain FP64 form: per (line, layer) amplitude, beta, gamma, erfcx(a).
struct LineRec64 {
  double A, beta, gam, erfcxa;
};

// Tiled FP64 form: the fields of LineRec (and LineRecT) in double precision,
// with the full wing polynomial (no tier truncation).
struct LineRec64T {
  double e[7];    // wing polynomial, amplitude included
  double gam2;    // gamma^2
  double thr;     // 2 beta^2 * 111: core branch iff D < thr
  double winv;    // 1 / (sqrt2 beta)
  double a;       // gamma / (sqrt2 beta)
  double acore;   // amplitude / (sqrt(2 pi) beta)
};
static_assert(sizeof(LineRec64T) == 96, "LineRec64T layout");

struct LineRec64TT {
  double t[8];    // wing: d f/dT = r * sum_k t_k r^k
  double kA;      // d ln(acore)/dT
  double kw;      // d ln(winv)/dT
  double da;      // da/dT
  double pad;
};
static_assert(sizeof(LineRec64TT) == 96, "LineRec64TT layout");

// Temperature tangent of the record (FP64): the wing polynomial's T-derivative
// coefficients tk[0..7] and the core-branch factors d ln(acore)/dT,
// d ln(winv)/dT, da/dT, from the amplitude, widths and their T-derivatives.
__device__ inline void record_tangent(double A, double beta, double gam, double dlnA, double dbeta,
                                      double dgam, double (&tk)[8], double* kA, double* kw, double* da) {
  const double b = beta * beta, g = gam * gam;
  const double E0 = A * gam / kPi;
  double c[7];
  c[0] = 1.0;
  c[1] = 3.0 * b;
  c[2] = 15.0 * b * b - 4.0 * b * g;
  c[3] = 105.0 * b * b * b - 60.0 * b * b * g;
  c[4] = 48.0 * b * b * g * g - 840.0 * b * b * b * g;
  c[5] = 1680.0 * b * b * b * g * g;
  c[6] = -960.0 * b * b * b * g * g * g;
  // db/dT, dg/dT
  const double db = 2.0 * beta * dbeta, dg = 2.0 * gam * dgam;
  // dc_k/dT = dc_k/db * db + dc_k/dg * dg
  double dc[7];
  dc[0] = 0.0;
  dc[1] = 3.0 * db;
  dc[2] = (30.0 * b - 4.0 * g) * db - 4.0 * b * dg;
  dc[3] = (315.0 * b * b - 120.0 * b * g) * db - 60.0 * b * b * dg;
  dc[4] = (96.0 * b * g * g - 2520.0 * b * b * g) * db + (96.0 * b * b * g - 840.0 * b * b * b) * dg;
  dc[5] = 5040.0 * b * b * g * g * db + 3360.0 * b * b * b * g * dg;
  dc[6] = -2880.0 * b * b * g * g * g * db - 2880.0 * b * b * b * g * g * dg;
  // E0 = A gam / pi  ->  dE0 = E0 (dlnA) + A dgam / pi
  const double dE0 = E0 * dlnA + A * dgam / kPi;
  // f = sum_k e_k r^{k+1}, r = 1/(s + g):  df/dT = sum_k e'_k r^{k+1} - g' sum_k (k+1) e_k r^{k+2}
  for (int k = 0; k < 8; ++k) tk[k] = 0.0;
  for (int k = 0; k < 7; ++k) {
    tk[k] += dE0 * c[k] + E0 * dc[k];
    tk[k + 1] += -dg * (double)(k + 1) * E0 * c[k];
  }
  const double winv = 1.0 / (kSqrt2 * beta);
  *kA = dlnA - dbeta / beta;
  *kw = -dbeta / beta;
  *da = winv * (dgam - gam * dbeta / beta);
}

// ---------------------------------------------------------------------------
// Record construction (FP64) from the line state at one layer.
//   A      amplitude (cross-section: S(T) [* column factor] [* scale])
//   beta   Gaussian standard deviation, gam Lorentz HWHM
//   dlnA, dbeta, dgam : d/dT of ln A, beta, gamma (tangent records only)
// ---------------------------------------------------------------------------
__device__ inline void make_line_record(double A, double beta, double gam, double T,
                                        double dlnA, double dbeta, double dgam,
                                        LineRec* R, LineRecT* RT) {
  const double b = beta * beta, g = gam * gam;
  const double E0 = A * gam / kPi;
  double c[7];
  c[0] = 1.0;
  c[1] = 3.0 * b;
  c[2] = 15.0 * b * b - 4.0 * b * g;
  c[3] = 105.0 * b * b * b - 60.0 * b * b * g;
  c[4] = 48.0 * b * b * g * g - 840.0 * b * b * b * g;
  c[5] = 1680.0 * b * b * b * g * g;
  c[6] = -960.0 * b * b * b * g * g * g;
  LineRec r;
#pragma unroll
  for (int k = 0; k < 7; ++k) r.e[k] = (float)(E0 * c[k]);
  r.gam2 = (float)g;
  r.thr = (float)(2.0 * kHjertSwitch * b);
  const double winv = 1.0 / (kSqrt2 * beta);
  r.winv = (float)winv;
  r.a = (float)(gam * winv);
  r.acore = (float)(A * winv / kSqrtPi);
  for (int k = 0; k < 4; ++k) r.pad[k] = 0.f;
  *R = r;
  if (RT) {
    LineRecT t;
    double tk[8], kA, kw, da;
    record_tangent(A, beta, gam, dlnA, dbeta, dgam, tk, &kA, &kw, &da);
#pragma unroll
    for (int k = 0; k < 8; ++k) t.t[k] = (float)tk[k];
    t.kA = (float)kA;
    t.kw = (float)kw;
    t.da = (float)da;
    for (int k = 0; k < 5; ++k) t.pad[k] = 0.f;
    *RT = t;
  }
}

// The same records in FP64 for the tiled FP64 form; RT (tangent mode) may be
// nullptr.
__device__ inline void make_line_record64t(double A, double beta, double gam, double dlnA, double dbeta,
                                           double dgam, LineRec64T* R, LineRec64TT* RT) {
  if (RT) {
    LineRec64TT t;
    record_tangent(A, beta, gam, dlnA, dbeta, dgam, t.t, &t.kA, &t.kw, &t.da);
    t.pad = 0.0;
    *RT = t;
  }
  const double b = beta * beta, g = gam * gam;
  const double E0 = A * gam / kPi;
  LineRec64T r;
  r.e[0] = E0;
  r.e[1] = E0 * (3.0 * b);
  r.e[2] = E0 * (15.0 * b * b - 4.0 * b * g);
  r.e[3] = E0 * (105.0 * b * b * b - 60.0 * b * b * g);
  r.e[4] = E0 * (48.0 * b * b * g * g - 840.0 * b * b * b * g);
  r.e[5] = E0 * (1680.0 * b * b * b * g * g);
  r.e[6] = E0 * (-960.0 * b * b * b * g * g * g);
  r.gam2 = g;
  r.thr = 2.0 * kHjertSwitch * b;
  r.winv = 1.0 / (kSqrt2 * beta);
  r.a = gam * r.winv;
  r.acore = A * r.winv / kSqrtPi;
  *R = r;
}

// ---------------------------------------------------------------------------
// e^t for the core branch's arguments (|t| <= 112, far from over- and
// underflow): t = k ln2 + r with |r| <= ln2/2 (Cody-Waite reduction with a
// two-part ln2), e^r by its Taylor series to r^9 (truncation below 1.1e-11
// relative), times 2^k.
__device__ __forceinline__ double exp_core(double t) {
  constexpr double kLog2e = 1.4426950408889634, kLn2Hi = 0.6931471805599453, kLn2Lo = 2.3190468138462996e-17;
  const double k = rint(t * kLog2e);
  double r = fma(-k, kLn2Hi, t);
  r = fma(-k, kLn2Lo, r);
  double p = 1.0 / 362880.0;
  p = fma(p, r, 1.0 / 40320.0);
  p = fma(p, r, 1.0 / 5040.0);
  p = fma(p, r, 1.0 / 720.0);
  p = fma(p, r, 1.0 / 120.0);
  p = fma(p, r, 1.0 / 24.0);
  p = fma(p, r, 1.0 / 6.0);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return ldexp(p, (int)k);
}

// Asymptotic branch Re/Im of w_2^asy(x + i a) in FP32 (diagnostics).
__device__ inline float hjert_asy_f32(float x, float a, float* L) {
  // 1/z, alpha~ = 1/(2 z^2); w = i/(z sqrt(pi)) (1 + al (1 + al (3 + 15 al)))
  const float d = x * x + a * a;
  const float zr = x / d, zi = -a / d;                    // 1/z
  const float u2r = zr * zr - zi * zi, u2i = 2.f * zr * zi;  // 1/z^2
  const float alr = 0.5f * u2r, ali = 0.5f * u2i;
  float pr = 3.f + 15.f * alr, pi_ = 15.f * ali;
  float qr = 1.f + (alr * pr - ali * pi_), qi = alr * pi_ + ali * pr;
  pr = 1.f + (alr * qr - ali * qi);
  pi_ = alr * qi + ali * qr;
  // (1/z) * p
  const float mr = zr * pr - zi * pi_, mi = zr * pi_ + zi * pr;
  const float is = 0.56418958354775628f;  // 1/sqrt(pi)
  if (L) *L = mr * is;
  return -mi * is;
}

// ---------------------------------------------------------------------------
// Plain FP64 hjert: the paper's two branches written out in double.
// ---------------------------------------------------------------------------
__device__ inline double hjert_f64(double x, double a, double erfcxa) {
  if (x * x + a * a < kHjertSwitch) {
    const double eta = 0.5;
    const double ex2 = exp(-x * x);
    double S1 = 0.0, S2 = 0.0, S3 = 0.0;
    for (int n = 1; n <= kM916; ++n) {
      const double en = eta * n;
      const double v0 = 1.0 / (en * en + a * a);
      S1 += v0 * exp(-(en * en + x * x));
      S2 += v0 * exp(-(en + x) * (en + x));
      S3 += v0 * exp(-(en - x) * (en - x));
    }
    const double ax = a * x;
    const double sinc = (ax != 0.0) ? sin(ax) / ax : 1.0;
    return ex2 * erfcxa * cos(2.0 * x * a) + 2.0 * eta * x * sin(ax) / kPi * ex2 * sinc +
           2.0 * eta / kPi * (-a * cos(2.0 * a * x) * S1 + 0.5 * a * S2 + 0.5 * a * S3);
  }
  // w_2^asy(z) = i/(z sqrt pi) * (1 + al (1 + al (3 + 15 al))), al = 1/(2 z^2)
  const double zr = x, zi = a;
  const double z2r = zr * zr - zi * zi, z2i = 2.0 * zr * zi;
  // al = 1 / (2 z^2)
  const double den = 2.0 * (z2r * z2r + z2i * z2i);
  const double alr = z2r / den, ali = -z2i / den;
  double pr = 3.0 + 15.0 * alr, pi_ = 15.0 * ali;
  double qr = 1.0 + (alr * pr - ali * pi_), qi = alr * pi_ + ali * pr;
  pr = 1.0 + (alr * qr - ali * qi);
  pi_ = alr * qi + ali * qr;
  // w = i p / (z sqrt pi): divide p by z
  const double dz = zr * zr + zi * zi;
  const double wr = (pr * zr + pi_ * zi) / dz, wi = (pi_ * zr - pr * zi) / dz;
  // times i/sqrt(pi): Re = -wi/sqrt(pi)
  return -wi / kSqrtPi;
}

// ---------------------------------------------------------------------------
// Transmission T = 2 E3(x) = (1 - x) e^{-x} + x^2 E1(x) with the Abramowitz &
// Stegun (1964) fits 5.1.53 (x <= 1) and 5.1.56 (x > 1) for E1 (Eq. transco),
// and dT/dx = -2 E2(x) = -2 (e^{-x} - x E1(x)).
// ---------------------------------------------------------------------------
__device__ inline void trans2e3(double x, double* T, double* dT) {
  if (x <= 0.0) {
    *T = 1.0;
    if (dT) *dT = -2.0;
    return;
  }
  if (x > 700.0) {  // e^{-x} underflows: the layer is opaque
    *T = 0.0;
    if (dT) *dT = 0.0;
    return;
  }
  const double ex = exp(-x);
  double E1;
  if (x <= 1.0) {
    E1 = -log(x) + (-0.57721566 + x * (0.99999193 + x * (-0.24991055 +
                    x * (0.05519968 + x * (-0.00976004 + x * 0.00107857)))));
  } else {
    const double num = (((x + 8.5733287401) * x + 18.0590169730) * x + 8.6347608925) * x + 0.2677737343;
    const double den = (((x + 9.5733223454) * x + 25.6329561486) * x + 21.0996530827) * x + 3.9584969228;
    E1 = ex / x * num / den;
  }
  *T = (1.0 - x) * ex + x * x * E1;
  if (dT) *dT = -2.0 * (ex - x * E1);
}

// pi B_nu(T) with nu in cm^-1 (Eq. sourcepla) and its T-derivative.
__device__ inline double planck_pi(double T, double nu, double* dBdT) {
  const double x = kC2 * nu / T;
  const double em1 = expm1(x);
  const double B = kPi * 2.0 * kH * kC * kC * nu * nu * nu / em1;
  if (dBdT) *dBdT = B * (x / T) * (em1 + 1.0) / em1;
  return B;
}

// ---------------------------------------------------------------------------
// Wave/block reductions (wave64) in FP64, fixed order => deterministic.
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over a 256-thread block; result valid in thread 0. `sm` holds >= 4 doubles.
__device__ inline double block_sum256(double v, double* sm) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sm[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = (sm[0] + sm[1]) + (sm[2] + sm[3]);
  return r;
}

}  // namespace exo
