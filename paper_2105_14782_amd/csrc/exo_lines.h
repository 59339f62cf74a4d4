// Per-line state at one (T, P): strength, widths and their T-derivatives,
// shared by the Voigt-sum records and the MODIT lineshape density.
#pragma once
#include "exo_device.h"
#include "exo_launch.h"

namespace exo {

// ---------------------------------------------------------------------------
// Line state at one layer (Sec. 2.2 Eq. Slog, Eq. thermal, Eq. gammaexomol,
// Eq. naturalgamma, Sec. 2.3 partition function), FP64.
// ---------------------------------------------------------------------------
__device__ inline void qr_eval(int kind, const double* __restrict__ p, int nq, double T,
                               double* qr, double* dlnqr) {
  if (kind == 0) {
    *qr = pow(T / kTref, p[0]);
    *dlnqr = p[0] / T;
    return;
  }
  const int n = nq / 2;
  const double* tn = p;
  const double* qn = p + n;
  auto interp = [&](double t, double* slope) {
    int i = 0;
    if (t <= tn[0]) i = 0;
    else if (t >= tn[n - 1]) i = n - 2;
    else {
      int lo = 0, hi = n - 1;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tn[mid] <= t) lo = mid; else hi = mid;
      }
      i = lo;
    }
    const double s = (qn[i + 1] - qn[i]) / (tn[i + 1] - tn[i]);
    if (slope) *slope = s;
    // constant extrapolation outside the table, like np.interp; the slope is
    // the derivative from the right (zero where the end value is held)
    if (t < tn[0]) { if (slope) *slope = 0.0; return qn[0]; }
    if (t >= tn[n - 1]) { if (slope) *slope = 0.0; return qn[n - 1]; }
    return qn[i] + s * (t - tn[i]);
  };
  double s;
  const double qT = interp(T, &s);
  const double q0 = interp(kTref, nullptr);
  *qr = qT / q0;
  *dlnqr = s / qT;
}

struct LineState {
  double S, beta, gam, dlnS, dbeta, dgam;
};

__device__ inline LineState line_state(const LinesDev& L, int64_t l, double T, double P) {
  LineState s;
  const double nu = L.nu_c[l];
  double qr, dlnqr;
  qr_eval(L.qr_kind, L.qr_params, L.n_qr, T, &qr, &dlnqr);
  const double E = L.E_low[l];
  const double eT = exp(-kC2 * nu / T), eR = exp(-kC2 * nu / kTref);
  s.S = L.S0[l] / qr * exp(-kC2 * E * (1.0 / T - 1.0 / kTref)) * (1.0 - eT) / (1.0 - eR);
  s.dlnS = -dlnqr + kC2 * E / (T * T) - (kC2 * nu / (T * T)) * eT / (1.0 - eT);
  s.beta = sqrt(kKB * T / (L.mass * kMU)) * nu / kC;
  s.dbeta = s.beta / (2.0 * T);
  const double n = L.n_texp[l];
  const double gp = L.alpha_ref[l] * pow(T / kTref, -n) * P;
  s.gam = gp + (L.gamma_nat ? L.gamma_nat[l] : 0.0);
  s.dgam = -n * gp / T;
  return s;
}

}  // namespace exo
