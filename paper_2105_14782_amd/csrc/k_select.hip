// Weak-line pre-selection (App. G): a line is kept when the layer where its
// line-centre contribution function peaks is no deeper than the layer where
// the H2-H2 continuum's peaks at the same wavenumber, plus a margin.
//
// Isothermal atmosphere at T_atm; the line's strength is its largest over a
// list of temperatures; in layer n the line-centre optical depth of the line
// alone is col_n S/(sqrt(2 pi) beta) erfcx(gamma_n/(sqrt2 beta)) with
// gamma_n = alpha_ref (T_atm/296)^-n P_n + gamma_nat; tau_n includes layer n;
// the contribution function is e^{-tau_n} dtau_n P_n/dP_n (the Planck factor
// is common to all layers), and its argmax is the first maximum.  FP64.
#include "exo_device.h"
#include "exo_launch.h"
#include "exo_lines.h"

namespace exo {

__global__ __launch_bounds__(256) void k_select_lines(SelectArgs A) {
  __shared__ double sm[4];
  const int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double kept = 0.0;
  if (l < A.L.n) {
    double S = 0.0;
    for (int t = 0; t < A.n_T; ++t) S = fmax(S, line_state(A.L, l, A.T_strength[t], 0.0).S);
    const double beta = sqrt(kKB * A.T_atm / (A.L.mass * kMU)) * A.L.nu_c[l] / kC;
    const double amp = S / (sqrt(2.0 * kPi) * beta);
    const double g1 = A.L.alpha_ref[l] * pow(A.T_atm / kTref, -A.L.n_texp[l]);
    const double gnat = A.L.gamma_nat ? A.L.gamma_nat[l] : 0.0;
    const double ciaf = exp(A.cia_slope * (A.L.nu_c[l] - A.cia_nu_c) / 40.0);
    double tau = 0.0, tauc = 0.0, best = -1.0, bestc = -1.0;
    int nl = 0, nc = 0;
    for (int n = 0; n < A.nlay; ++n) {
      const double r = A.P[n] / A.dP[n];
      const double gam = g1 * A.P[n] + gnat;
      const double dt = A.col[n] * amp * erfcx(gam / (kSqrt2 * beta));
      tau += dt;
      const double psi = exp(-tau) * dt * r;
      if (psi > best) {
        best = psi;
        nl = n;
      }
      const double dc = A.cia[n] * ciaf;
      tauc += dc;
      const double psic = exp(-tauc) * dc * r;
      if (psic > bestc) {
        bestc = psic;
        nc = n;
      }
    }
    const bool keep = nl <= nc + A.margin;
    A.keep[A.perm[l]] = keep ? 1 : 0;
    kept = keep ? 1.0 : 0.0;
  }
  const double s = block_sum256(kept, sm);
  if (threadIdx.x == 0 && s > 0.0) atomicAdd(A.n_kept, (unsigned long long)s);
}

__global__ void k_clear_count(unsigned long long* c) {
  if (threadIdx.x == 0) *c = 0ull;
}

hipError_t launch_select_lines(const SelectArgs& A, hipStream_t st) {
  hipLaunchKernelGGL(k_clear_count, dim3(1), dim3(64), 0, st, A.n_kept);
  hipLaunchKernelGGL(k_select_lines, dim3((unsigned)((A.L.n + 255) / 256)), dim3(256), 0, st, A);
  return hipGetLastError();
}

}  // namespace exo
