// Atmosphere set-up, layer radiative transfer (Sec. 3), response (Sec. 4)
// and their adjoints.
#include "exo_device.h"
#include "exo_launch.h"

namespace exo {

// Response convolutions: taps per LDS chunk and the input window they reach
// from a block of 256 consecutive outputs.
constexpr int kTapChunk = 512;
constexpr int kWin = 256 + kTapChunk - 1;

// win[m] = src[lo + m] for m < n, 0 where lo + m lies outside [vlo, vhi]
// (every index a valid output reads lies inside).  Block-wide; the caller
// synchronises.
template <typename T>
__device__ __forceinline__ void stage_window(double* __restrict__ win, const T* __restrict__ src, int64_t lo,
                                             int n, int64_t vlo, int64_t vhi) {
  for (int m = threadIdx.x; m < n; m += 256) {
    const int64_t idx = lo + m;
    win[m] = (idx >= vlo && idx <= vhi) ? (double)src[idx] : 0.0;
  }
}

// ---------------------------------------------------------------------------
// Per-layer quantities: T_n = T0 (P_n/1 bar)^alpha (Sec. 5.2), dP_n, the
// column factor dP/(m_u g) X_m/M_m of Eq. dtau_line2, and the layer factor of
// the CIA optical depth (Eq. taucont with Eq. scaleheight):
//   xi^2 P dP alpha0 (T/1000)^p / (k_B T mu m_u g)   [times exp(s (nu-nu_c)/40)]
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_atmos(AtmosDev A) {
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= A.nlay) return;
  const double P = A.P[n];
  const double Pprev = n > 0 ? A.P[n - 1] : A.P[0] * A.P[0] / A.P[1];
  const double dP = P - Pprev;
  const double lnP = log(P);
  const double T = A.T_in ? A.T_in[n] : A.T0 * exp(A.alpha * lnP);
  A.T[n] = T;
  A.dP[n] = dP;
  A.lnP[n] = lnP;
  for (int m = 0; m < A.nspec; ++m) {
    const double X = exp(kLn10 * A.logx[m]);
    A.col[m * A.nlay + n] = dP * kBar / (kMU * A.g) * X / A.mass[m];
  }
  const double c = A.vmr_h2 * A.vmr_h2 * (P * kBar) * (dP * kBar) * A.cia_alpha0 *
                   pow(T / 1000.0, A.cia_Tpow) / (kKB * T * A.mmw * kMU * A.g);
  A.cia[n] = c;
  A.dcia[n] = c * (A.cia_Tpow - 1.0) / T;
}

template <typename TT>
__device__ inline double tau_sum(const RtArgs& R, int n, int64_t j, double ciaf) {
  const TT* tau = (const TT*)R.tau;
  double t = 0.0;
  for (int m = 0; m < R.nspec; ++m) t += (double)tau[((int64_t)m * R.nlay + n) * R.ng + j];
  return t + R.cia[n] * ciaf;
}

// ---------------------------------------------------------------------------
// Forward transfer per grid point, top to bottom (the closed form of Eq. rerr,
// F0 = sum_n Phi_n (1 - T_n) S_n + Phi_N F_B with Phi_n = prod_{k<n} T_k).
// ---------------------------------------------------------------------------
template <typename TT>
__global__ __launch_bounds__(256) void k_rt_forward(RtArgs R) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= R.ng) return;
  const double nu = R.nu[j];
  const double ciaf = exp(R.cia_slope * (nu - R.cia_nu_c) / 40.0);
  double Phi = 1.0, F0 = 0.0;
  for (int n = 0; n < R.nlay; ++n) {
    const double tau = tau_sum<TT>(R, n, j, ciaf);
    double Tr;
    trans2e3(tau, &Tr, nullptr);
    const double S = planck_pi(R.T[n], nu, nullptr);
    F0 += Phi * (1.0 - Tr) * S;
    Phi *= Tr;
  }
  if (R.bottom == 0) F0 += Phi * planck_pi(R.T[R.nlay - 1], nu, nullptr);
  R.F0[j] = F0;
}

// ---------------------------------------------------------------------------
// Reverse transfer.  With F_n the upward flux entering layer n from below:
//   dF0/dT_n    = Phi_n (F_{n+1} - S_n),  dT_n/dtau_n = -2 E2(tau_n)
//   dF0/dS_n    = Phi_n (1 - T_n),        dF0/dF_B = Phi_N.
// Pass 1 (bottom-up) stores F_{n+1}; pass 2 (top-down) forms the adjoints,
// the per-layer temperature gradient (block partial sums, fixed order) and
// tau-bar for the mixing-ratio gradient.
// ---------------------------------------------------------------------------
template <typename TT>
__global__ __launch_bounds__(256) void k_rt_adjoint(RtArgs R) {
  __shared__ double sm[4];
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool live = j < R.ng;
  const int64_t jc = live ? j : R.ng - 1;
  const double nu = R.nu[jc];
  const double ciaf = exp(R.cia_slope * (nu - R.cia_nu_c) / 40.0);
  const double Fbar = live ? R.F0bar[jc] : 0.0;
  const TT* taut = (const TT*)R.taut;

  double F = R.bottom == 0 ? planck_pi(R.T[R.nlay - 1], nu, nullptr) : 0.0;
  for (int n = R.nlay - 1; n >= 0; --n) {
    const double tau = tau_sum<TT>(R, n, jc, ciaf);
    double Tr;
    trans2e3(tau, &Tr, nullptr);
    const double S = planck_pi(R.T[n], nu, nullptr);
    if (live) R.Fup[(int64_t)n * R.ng + j] = F;
    F = Tr * F + (1.0 - Tr) * S;
  }
  double Phi = 1.0;
  for (int n = 0; n < R.nlay; ++n) {
    const double tau = tau_sum<TT>(R, n, jc, ciaf);
    double Tr, dTr;
    trans2e3(tau, &Tr, &dTr);
    double dS;
    const double S = planck_pi(R.T[n], nu, &dS);
    const double Fn1 = live ? R.Fup[(int64_t)n * R.ng + j] : 0.0;
    const double tbar = Fbar * Phi * (Fn1 - S) * dTr;
    const double Sbar = Fbar * Phi * (1.0 - Tr);
    double dtau = R.dcia[n] * ciaf;
    for (int m = 0; m < R.nspec; ++m) dtau += (double)taut[((int64_t)m * R.nlay + n) * R.ng + jc];
    double gT = tbar * dtau + Sbar * dS;
    Phi *= Tr;
    if (n == R.nlay - 1 && R.bottom == 0) {
      double dB;
      planck_pi(R.T[n], nu, &dB);
      gT += Fbar * Phi * dB;
    }
    if (live) R.taubar[(int64_t)n * R.ng + j] = tbar;
    const double s = block_sum256(live ? gT : 0.0, sm);
    if (threadIdx.x == 0) R.partT[(int64_t)blockIdx.x * R.nlay + n] = s;
  }
}

// ---------------------------------------------------------------------------
// Forward-mode transfer (App. D): with dT_n the layer temperature tangent and
// dtau_n = sum_m (dtau^m_n/dT_n dT_n + ln10 tau^m_n dlog10 X_m)
//          + dtau^CIA_n/dT_n dT_n,
// the tangent of F0 = sum_n Phi_n (1 - T_n) S_n + Phi_N F_B, top to bottom:
//   dPhi_{n+1} = dPhi_n T_n + Phi_n dT_n,  dT_n = -2 E2(tau_n) dtau_n,
//   dS_n = pi dB/dT(T_n) dT_n,  dF_B = pi dB/dT(T_{N-1}) dT_{N-1}.
// ---------------------------------------------------------------------------
template <typename TT>
__global__ __launch_bounds__(256) void k_rt_jvp(RtArgs R, JvpArgs J) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= R.ng) return;
  const double nu = R.nu[j];
  const double ciaf = exp(R.cia_slope * (nu - R.cia_nu_c) / 40.0);
  const TT* tau = (const TT*)R.tau;
  const TT* taut = (const TT*)R.taut;
  double Phi = 1.0, dPhi = 0.0, dF0 = 0.0, dTlast = 0.0;
  for (int n = 0; n < R.nlay; ++n) {
    const double dT = (J.powerlaw ? R.T[n] * (J.dT0_rel + J.dalpha * J.lnP[n]) : 0.0) +
                      (J.dTl ? J.dTl[n] : 0.0);
    double t = R.cia[n] * ciaf, dt = R.dcia[n] * ciaf * dT;
    for (int m = 0; m < R.nspec; ++m) {
      const int64_t o = ((int64_t)m * R.nlay + n) * R.ng + j;
      const double tm = (double)tau[o];
      t += tm;
      dt += (double)taut[o] * dT + kLn10 * J.dlogx[m] * tm;
    }
    double Tr, dTr;
    trans2e3(t, &Tr, &dTr);
    double dB;
    const double S = planck_pi(R.T[n], nu, &dB);
    const double dTrn = dTr * dt;
    dF0 += dPhi * (1.0 - Tr) * S - Phi * dTrn * S + Phi * (1.0 - Tr) * dB * dT;
    dPhi = dPhi * Tr + Phi * dTrn;
    Phi *= Tr;
    dTlast = dT;
  }
  if (R.bottom == 0) {
    double dB;
    const double FB = planck_pi(R.T[R.nlay - 1], nu, &dB);
    dF0 += dPhi * FB + Phi * dB * dTlast;
  }
  J.dF0[j] = dF0;
}

// Tangent of the rotation stage: dmid[p] = sum_k rot_k dF0_{i - dlo - k}
//   + (drot_rv_k dRV + drot_vs_k dvsini) F0_{i - dlo - k}
__global__ __launch_bounds__(256) void k_conv_rot_jvp(RespDev R, const double* __restrict__ F0,
                                                      const double* __restrict__ dF0, double d_rv,
                                                      double d_vs, double* __restrict__ dmid,
                                                      int64_t nmid) {
  __shared__ double tap[kTapChunk], tap2[kTapChunk];
  __shared__ double win[kWin], dwin[kWin];
  const int t = threadIdx.x;
  const int64_t p0 = (int64_t)blockIdx.x * 256, p = p0 + t;
  // F0 indices the valid outputs read: [ob - K - dlo - (nrot - 1), ob - K + nmid - 1 - dlo]
  const int64_t vlo = R.ob - R.K - R.dlo - (R.nrot - 1), vhi = R.ob - R.K + nmid - 1 - R.dlo;
  double acc = 0.0;
  for (int64_t k0 = 0; k0 < R.nrot; k0 += kTapChunk) {
    const int nk = (int)min((int64_t)kTapChunk, R.nrot - k0);
    const int64_t lo = R.ob - R.K + p0 - R.dlo - (k0 + nk - 1);
    __syncthreads();
    for (int m = t; m < nk; m += 256) {
      tap[m] = R.rot[k0 + m];
      tap2[m] = fma(R.drot_rv[k0 + m], d_rv, R.drot_vs[k0 + m] * d_vs);
    }
    stage_window(win, F0, lo, 255 + nk, vlo, vhi);
    stage_window(dwin, dF0, lo, 255 + nk, vlo, vhi);
    __syncthreads();
    for (int kk = 0; kk < nk; ++kk) {
      acc = fma(tap[kk], dwin[t + nk - 1 - kk], acc);
      acc = fma(tap2[kk], win[t + nk - 1 - kk], acc);
    }
  }
  if (p < nmid) dmid[p] = acc;
}

// sum_{n,j} taubar_nj tau^m_nj per block (fixed order), for every species m.
template <typename TT>
__global__ __launch_bounds__(256) void k_grad_x(const double* __restrict__ taubar,
                                                const TT* __restrict__ tau, int nspec, int nlay,
                                                int64_t ng, double* __restrict__ partX) {
  __shared__ double sm[4];
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (int m = 0; m < nspec; ++m) {
    double acc = 0.0;
    if (j < ng)
      for (int n = 0; n < nlay; ++n)
        acc += taubar[(int64_t)n * ng + j] * (double)tau[((int64_t)m * nlay + n) * ng + j];
    const double s = block_sum256(acc, sm);
    if (threadIdx.x == 0) partX[(int64_t)blockIdx.x * nspec + m] = s;
  }
}

// Final fixed-order reductions and the chain rule to (T0, alpha) of the
// power-law profile:  dT_n/dT0 = T_n/T0,  dT_n/dalpha = T_n ln(P_n / 1 bar).
// out = {dT0, dalpha, dlog10X_1..M, dRV, dvsini, dT_0..dT_{N-1}}
__global__ void k_grad_final(const double* __restrict__ partT, int64_t nbT,
                             const double* __restrict__ partX, int64_t nbX,
                             const double* __restrict__ partR, int64_t nbR,
                             const double* __restrict__ T, const double* __restrict__ lnP, int nlay,
                             int nspec, double T0, int powerlaw, double* __restrict__ out) {
  const int t = threadIdx.x;
  double* gT = out + 2 + nspec + 2;
  for (int n = t; n < nlay; n += blockDim.x) {
    double s = 0.0;
    for (int64_t b = 0; b < nbT; ++b) s += partT[b * nlay + n];
    gT[n] = s;
  }
  __threadfence_block();
  __syncthreads();
  if (t == 0) {
    double g0 = 0.0, ga = 0.0;
    for (int n = 0; n < nlay; ++n) {
      g0 += gT[n] * T[n] / T0;
      ga += gT[n] * T[n] * lnP[n];
    }
    // a layer-by-layer profile does not depend on (T0, alpha)
    out[0] = powerlaw ? g0 : 0.0;
    out[1] = powerlaw ? ga : 0.0;
    for (int m = 0; m < nspec; ++m) {
      double s = 0.0;
      for (int64_t b = 0; b < nbX; ++b) s += partX[b * nspec + m];
      out[2 + m] = kLn10 * s;
    }
    double r0 = 0.0, r1 = 0.0;
    for (int64_t b = 0; b < nbR; ++b) {
      r0 += partR[2 * b];
      r1 += partR[2 * b + 1];
    }
    out[2 + nspec] = r0;
    out[2 + nspec + 1] = r1;
  }
}

// ---------------------------------------------------------------------------
// Response taps (Sec. 4).  Rotation kernel: closed form of the quadratic
// limb-darkened disk integral along the rotation axis,
//   zeta(x) = [2s(1-u1-u2) + pi/2 (u1+2u2) s^2 - 4/3 u2 s^3] / [pi (1-u1/3-u2/6)],
//   s = sqrt(1-x^2), zero for |x| >= 1,
// evaluated at x = (d dv + RV)/vsini for grid offsets d = i - j (Eq. responsenu
// with c ln(nu_i/nu_j) = d dv on the log-uniform grid).  Taps are normalised
// by their own sum; derivatives of the normalised taps w.r.t. RV and vsini
// are kept for the adjoint.  IP: exp(-(d dv)^2 / (2 beta_IP^2)), |d dv| <= 6
// beta_IP, normalised.
// ---------------------------------------------------------------------------
__device__ inline void zeta_eval(double x, double u1, double u2, double* z, double* dz) {
  if (fabs(x) >= 1.0) {
    *z = 0.0;
    *dz = 0.0;
    return;
  }
  const double s = sqrt(1.0 - x * x);
  const double norm = kPi * (1.0 - u1 / 3.0 - u2 / 6.0);
  *z = (2.0 * s * (1.0 - u1 - u2) + 0.5 * kPi * (u1 + 2.0 * u2) * s * s - (4.0 / 3.0) * u2 * s * s * s) / norm;
  const double dnum = 2.0 * (1.0 - u1 - u2) + kPi * (u1 + 2.0 * u2) * s - 4.0 * u2 * s * s;
  *dz = dnum * (-x / s) / norm;
}

__global__ __launch_bounds__(256) void k_taps(RespDev R) {
  __shared__ double sm[4];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int64_t k = threadIdx.x; k < R.nrot; k += 256) {
    const double x = ((double)(R.dlo + k) * R.dv + R.rv) / R.vsini;
    double z, dz;
    zeta_eval(x, R.u1, R.u2, &z, &dz);
    R.rot[k] = z;
    R.drot_rv[k] = dz / R.vsini;
    R.drot_vs[k] = -dz * x / R.vsini;
    s0 += z;
    s1 += dz / R.vsini;
    s2 += -dz * x / R.vsini;
  }
  double tot = block_sum256(s0, sm);
  __shared__ double tots[3];
  if (threadIdx.x == 0) tots[0] = tot;
  tot = block_sum256(s1, sm);
  if (threadIdx.x == 0) tots[1] = tot;
  tot = block_sum256(s2, sm);
  if (threadIdx.x == 0) tots[2] = tot;
  __syncthreads();
  const double St = tots[0], Srv = tots[1], Svs = tots[2];
  for (int64_t k = threadIdx.x; k < R.nrot; k += 256) {
    const double tn = R.rot[k] / St;
    R.rot[k] = tn;
    R.drot_rv[k] = (R.drot_rv[k] - tn * Srv) / St;
    R.drot_vs[k] = (R.drot_vs[k] - tn * Svs) / St;
  }
  // IP
  double si = 0.0;
  for (int64_t k = threadIdx.x; k < 2 * R.K + 1; k += 256) {
    const double v = (double)(k - R.K) * R.dv;
    const double g = exp(-0.5 * (v / R.beta_ip) * (v / R.beta_ip));
    R.ip[k] = g;
    si += g;
  }
  tot = block_sum256(si, sm);
  if (threadIdx.x == 0) tots[0] = tot;
  __syncthreads();
  for (int64_t k = threadIdx.x; k < 2 * R.K + 1; k += 256) R.ip[k] /= tots[0];
}

// The response convolutions below are 1-D sums over a few hundred taps on
// the log-uniform grid.  A block of 256 consecutive outputs stages the taps,
// in chunks of kTapChunk, and the input window those taps reach (255 + chunk
// points) in LDS, so every tap and input point is read from memory once per
// block; each thread then sums its output over the chunk from LDS, taps in
// increasing order (the same order as a plain per-output loop).

// mid[p] = G at model index i = ob - K + p:  G_i = sum_k rot_k F0_{i - dlo - k}
__global__ __launch_bounds__(256) void k_conv_rot(RespDev R, const double* __restrict__ F0,
                                                  double* __restrict__ mid, int64_t nmid) {
  __shared__ double tap[kTapChunk];
  __shared__ double win[kWin];
  const int t = threadIdx.x;
  const int64_t p0 = (int64_t)blockIdx.x * 256, p = p0 + t;
  const int64_t vlo = R.ob - R.K - R.dlo - (R.nrot - 1), vhi = R.ob - R.K + nmid - 1 - R.dlo;
  double acc = 0.0;
  for (int64_t k0 = 0; k0 < R.nrot; k0 += kTapChunk) {
    const int nk = (int)min((int64_t)kTapChunk, R.nrot - k0);
    const int64_t lo = R.ob - R.K + p0 - R.dlo - (k0 + nk - 1);   // F0 index of win[0]
    __syncthreads();
    for (int m = t; m < nk; m += 256) tap[m] = R.rot[k0 + m];
    stage_window(win, F0, lo, 255 + nk, vlo, vhi);
    __syncthreads();
    for (int kk = 0; kk < nk; ++kk) acc = fma(tap[kk], win[t + nk - 1 - kk], acc);
  }
  if (p < nmid) mid[p] = acc;
}

// out[o] = F at model index ob + o = sum_{d=-K..K} ip_{d+K} G_{ob + o - d}
//        = sum_k ip_k mid[o + 2K - k]
template <typename TO>
__global__ __launch_bounds__(256) void k_conv_ip(RespDev R, const double* __restrict__ mid,
                                                 TO* __restrict__ out) {
  __shared__ double tap[kTapChunk];
  __shared__ double win[kWin];
  const int t = threadIdx.x;
  const int64_t o0 = (int64_t)blockIdx.x * 256, o = o0 + t;
  const int64_t ntap = 2 * R.K + 1, nmid = R.ol + 2 * R.K;
  double acc = 0.0;
  for (int64_t k0 = 0; k0 < ntap; k0 += kTapChunk) {
    const int nk = (int)min((int64_t)kTapChunk, ntap - k0);
    const int64_t lo = o0 + 2 * R.K - (k0 + nk - 1);
    __syncthreads();
    for (int m = t; m < nk; m += 256) tap[m] = R.ip[k0 + m];
    stage_window(win, mid, lo, 255 + nk, 0, nmid - 1);
    __syncthreads();
    for (int kk = 0; kk < nk; ++kk) acc = fma(tap[kk], win[t + nk - 1 - kk], acc);
  }
  if (o < R.ol) out[o] = (TO)acc;
}

// Transpose of the IP stage: midbar[p] = sum_d ip_{d+K} cot[o = p - K + d]
//                                      = sum_k ip_k cot[p - 2K + k], 0 <= o < ol
template <typename TC>
__global__ __launch_bounds__(256) void k_convT_ip(RespDev R, const TC* __restrict__ cot,
                                                  double* __restrict__ midbar, int64_t nmid) {
  __shared__ double tap[kTapChunk];
  __shared__ double win[kWin];
  const int t = threadIdx.x;
  const int64_t p0 = (int64_t)blockIdx.x * 256, p = p0 + t;
  const int64_t ntap = 2 * R.K + 1;
  double acc = 0.0;
  for (int64_t k0 = 0; k0 < ntap; k0 += kTapChunk) {
    const int nk = (int)min((int64_t)kTapChunk, ntap - k0);
    const int64_t lo = p0 - 2 * R.K + k0;   // cot index of win[0]
    __syncthreads();
    for (int m = t; m < nk; m += 256) tap[m] = R.ip[k0 + m];
    stage_window(win, cot, lo, 255 + nk, 0, R.ol - 1);   // outside [0, ol): 0
    __syncthreads();
    for (int kk = 0; kk < nk; ++kk) acc = fma(tap[kk], win[t + kk], acc);
  }
  if (p < nmid) midbar[p] = acc;
}

// Transpose of the rotation stage: F0bar[j] = sum_k rot_k midbar[p(i = j + dlo + k)]
__global__ __launch_bounds__(256) void k_convT_rot(RespDev R, const double* __restrict__ midbar,
                                                   int64_t nmid, double* __restrict__ F0bar,
                                                   int64_t ng) {
  __shared__ double tap[kTapChunk];
  __shared__ double win[kWin];
  const int t = threadIdx.x;
  const int64_t j0 = (int64_t)blockIdx.x * 256, j = j0 + t;
  double acc = 0.0;
  for (int64_t k0 = 0; k0 < R.nrot; k0 += kTapChunk) {
    const int nk = (int)min((int64_t)kTapChunk, R.nrot - k0);
    const int64_t lo = j0 + R.dlo - (R.ob - R.K) + k0;   // midbar index of win[0]
    __syncthreads();
    for (int m = t; m < nk; m += 256) tap[m] = R.rot[k0 + m];
    stage_window(win, midbar, lo, 255 + nk, 0, nmid - 1);   // outside [0, nmid): 0
    __syncthreads();
    for (int kk = 0; kk < nk; ++kk) acc = fma(tap[kk], win[t + kk], acc);
  }
  if (j < ng) F0bar[j] = acc;
}

// RV / vsini: sum_p midbar[p] * sum_k drot_k F0_{i - dlo - k}; block partials.
__global__ __launch_bounds__(256) void k_rot_param_grad(RespDev R, const double* __restrict__ F0,
                                                        const double* __restrict__ midbar,
                                                        int64_t nmid, double* __restrict__ partR) {
  __shared__ double sm[4];
  __shared__ double tap_rv[kTapChunk], tap_vs[kTapChunk];
  __shared__ double win[kWin];
  const int t = threadIdx.x;
  const int64_t p0 = (int64_t)blockIdx.x * 256, p = p0 + t;
  const int64_t vlo = R.ob - R.K - R.dlo - (R.nrot - 1), vhi = R.ob - R.K + nmid - 1 - R.dlo;
  double a = 0.0, b = 0.0;
  for (int64_t k0 = 0; k0 < R.nrot; k0 += kTapChunk) {
    const int nk = (int)min((int64_t)kTapChunk, R.nrot - k0);
    const int64_t lo = R.ob - R.K + p0 - R.dlo - (k0 + nk - 1);
    __syncthreads();
    for (int m = t; m < nk; m += 256) {
      tap_rv[m] = R.drot_rv[k0 + m];
      tap_vs[m] = R.drot_vs[k0 + m];
    }
    stage_window(win, F0, lo, 255 + nk, vlo, vhi);
    __syncthreads();
    for (int kk = 0; kk < nk; ++kk) {
      const double f = win[t + nk - 1 - kk];
      a = fma(tap_rv[kk], f, a);
      b = fma(tap_vs[kk], f, b);
    }
  }
  if (p < nmid) {
    a *= midbar[p];
    b *= midbar[p];
  } else {
    a = b = 0.0;
  }
  const double sa = block_sum256(a, sm);
  const double sb = block_sum256(b, sm);
  if (threadIdx.x == 0) {
    partR[2 * blockIdx.x] = sa;
    partR[2 * blockIdx.x + 1] = sb;
  }
}

// Gaussian likelihood on the output spectrum: cot_j = dL/dF_j = (F_j - d_j)/s_j^2
// and block partials of L = 1/2 sum_j ((d_j - F_j)/s_j)^2 (fixed order).
__global__ __launch_bounds__(256) void k_gauss_cot(const float* __restrict__ F, const float* __restrict__ d,
                                                   const float* __restrict__ sg, int64_t n,
                                                   float* __restrict__ cot, double* __restrict__ part) {
  __shared__ double sm[4];
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double l = 0.0;
  if (j < n) {
    const double r = ((double)F[j] - (double)d[j]) / (double)sg[j];
    cot[j] = (float)(r / (double)sg[j]);
    l = 0.5 * r * r;
  }
  const double t = block_sum256(l, sm);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

template <typename TO>
__global__ __launch_bounds__(256) void k_cast(const double* __restrict__ s, TO* __restrict__ d, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) d[i] = (TO)s[i];
}

template <typename TI>
__global__ __launch_bounds__(256) void k_to_double(const TI* __restrict__ s, double* __restrict__ d, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) d[i] = (double)s[i];
}

__global__ __launch_bounds__(256) void k_trans2e3(int64_t n, const double* __restrict__ x,
                                                  double* __restrict__ T, double* __restrict__ dT) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double t, d;
  trans2e3(x[i], &t, &d);
  T[i] = t;
  if (dT) dT[i] = d;
}

// ---------------------------------------------------------------------------
static inline unsigned nb(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_atmos(const AtmosDev& A, hipStream_t st) {
  hipLaunchKernelGGL(k_atmos, dim3(nb(A.nlay)), dim3(256), 0, st, A);
  return hipGetLastError();
}

hipError_t launch_rt_forward(const RtArgs& R, bool tau64, hipStream_t st) {
  if (tau64) hipLaunchKernelGGL(k_rt_forward<double>, dim3(nb(R.ng)), dim3(256), 0, st, R);
  else hipLaunchKernelGGL(k_rt_forward<float>, dim3(nb(R.ng)), dim3(256), 0, st, R);
  return hipGetLastError();
}

hipError_t launch_rt_adjoint(const RtArgs& R, bool tau64, int64_t nblocks, hipStream_t st) {
  if (tau64) hipLaunchKernelGGL(k_rt_adjoint<double>, dim3((unsigned)nblocks), dim3(256), 0, st, R);
  else hipLaunchKernelGGL(k_rt_adjoint<float>, dim3((unsigned)nblocks), dim3(256), 0, st, R);
  return hipGetLastError();
}

hipError_t launch_grad_x(const double* taubar, const void* tau, bool tau64, int nspec, int nlay,
                         int64_t ng, double* partX, int64_t nblocks, hipStream_t st) {
  if (tau64)
    hipLaunchKernelGGL(k_grad_x<double>, dim3((unsigned)nblocks), dim3(256), 0, st, taubar,
                       (const double*)tau, nspec, nlay, ng, partX);
  else
    hipLaunchKernelGGL(k_grad_x<float>, dim3((unsigned)nblocks), dim3(256), 0, st, taubar,
                       (const float*)tau, nspec, nlay, ng, partX);
  return hipGetLastError();
}

hipError_t launch_grad_final(const double* partT, int64_t nbT, const double* partX, int64_t nbX,
                             const double* partR, int64_t nbR, const double* T, const double* lnP,
                             int nlay, int nspec, double T0, int powerlaw, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_grad_final, dim3(1), dim3(256), 0, st, partT, nbT, partX, nbX, partR, nbR,
                     T, lnP, nlay, nspec, T0, powerlaw, out);
  return hipGetLastError();
}

hipError_t launch_rt_jvp(const RtArgs& R, const JvpArgs& J, hipStream_t st) {
  hipLaunchKernelGGL(k_rt_jvp<float>, dim3(nb(R.ng)), dim3(256), 0, st, R, J);
  return hipGetLastError();
}

hipError_t launch_response_jvp(const RespDev& R, const double* F0, const double* dF0, double d_rv,
                               double d_vsini, double* dmid, float* dout, hipStream_t st) {
  const int64_t nmid = R.ol + 2 * R.K;
  hipLaunchKernelGGL(k_conv_rot_jvp, dim3(nb(nmid)), dim3(256), 0, st, R, F0, dF0, d_rv, d_vsini,
                     dmid, nmid);
  hipLaunchKernelGGL(k_conv_ip<float>, dim3(nb(R.ol)), dim3(256), 0, st, R, dmid, dout);
  return hipGetLastError();
}

hipError_t launch_trans2e3(int64_t n, const double* x, double* T, double* dT, hipStream_t st) {
  hipLaunchKernelGGL(k_trans2e3, dim3(nb(n)), dim3(256), 0, st, n, x, T, dT);
  return hipGetLastError();
}

hipError_t launch_taps(const RespDev& R, hipStream_t st) {
  hipLaunchKernelGGL(k_taps, dim3(1), dim3(256), 0, st, R);
  return hipGetLastError();
}

hipError_t launch_response(const RespDev& R, const double* F0, double* mid, void* out, bool out64,
                           hipStream_t st) {
  const int64_t nmid = R.ol + 2 * R.K;
  hipLaunchKernelGGL(k_conv_rot, dim3(nb(nmid)), dim3(256), 0, st, R, F0, mid, nmid);
  if (out64) hipLaunchKernelGGL(k_conv_ip<double>, dim3(nb(R.ol)), dim3(256), 0, st, R, mid, (double*)out);
  else hipLaunchKernelGGL(k_conv_ip<float>, dim3(nb(R.ol)), dim3(256), 0, st, R, mid, (float*)out);
  return hipGetLastError();
}

hipError_t launch_response_vjp(const RespDev& R, const double* F0, const void* cot, bool cot64,
                               double* midbar, double* F0bar, int64_t ng, double* partR,
                               int64_t nblocks_mid, hipStream_t st) {
  const int64_t nmid = R.ol + 2 * R.K;
  if (cot64) hipLaunchKernelGGL(k_convT_ip<double>, dim3(nb(nmid)), dim3(256), 0, st, R, (const double*)cot, midbar, nmid);
  else hipLaunchKernelGGL(k_convT_ip<float>, dim3(nb(nmid)), dim3(256), 0, st, R, (const float*)cot, midbar, nmid);
  hipLaunchKernelGGL(k_convT_rot, dim3(nb(ng)), dim3(256), 0, st, R, midbar, nmid, F0bar, ng);
  hipLaunchKernelGGL(k_rot_param_grad, dim3((unsigned)nblocks_mid), dim3(256), 0, st, R, F0, midbar, nmid, partR);
  return hipGetLastError();
}

hipError_t launch_gauss_cot(const float* F, const float* d, const float* sg, int64_t n, float* cot,
                            double* part, hipStream_t st) {
  hipLaunchKernelGGL(k_gauss_cot, dim3(nb(n)), dim3(256), 0, st, F, d, sg, n, cot, part);
  return hipGetLastError();
}

hipError_t launch_cast_copy(const double* src, void* dst, bool dst64, int64_t n, hipStream_t st) {
  if (dst64) hipLaunchKernelGGL(k_cast<double>, dim3(nb(n)), dim3(256), 0, st, src, (double*)dst, n);
  else hipLaunchKernelGGL(k_cast<float>, dim3(nb(n)), dim3(256), 0, st, src, (float*)dst, n);
  return hipGetLastError();
}

hipError_t launch_to_double(const void* src, bool src64, double* dst, int64_t n, hipStream_t st) {
  if (src64) hipLaunchKernelGGL(k_to_double<double>, dim3(nb(n)), dim3(256), 0, st, (const double*)src, dst, n);
  else hipLaunchKernelGGL(k_to_double<float>, dim3(nb(n)), dim3(256), 0, st, (const float*)src, dst, n);
  return hipGetLastError();
}

}  // namespace exo
