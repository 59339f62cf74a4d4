// Kernel argument blocks and launchers shared between the kernels and the
// host library (internal; not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "exo_device.h"

namespace exo {

constexpr int kMaxSpecies = 64;
#ifndef EXO_VOIGT_G
#define EXO_VOIGT_G 4
#endif
constexpr int kVoigtG = EXO_VOIGT_G;  // grid points per thread in the FP32 Voigt sum

struct LinesDev {
  const double *nu_c, *S0, *E_low, *alpha_ref, *n_texp, *gamma_nat;
  int64_t n;
  double mass;
  int qr_kind;
  const double* qr_params;
  int n_qr;
};

struct VoigtArgs {
  const double* nu;   // model grid (already offset to the model range)
  int64_t ng;
  const double* nu_c;
  int64_t n_lines;
  const LineRec* rec;
  const LineRecT* rect;
  const LineRec64* rec64;
  const LineRec64T* rec64t;  // tiled FP64 form
  const LineRec64TT* rect64t;  // tiled FP64 form, tangent mode
  int64_t lines_per_split;
  int ksplit;
  int nlay;
  float out_scale;
  const float* out_scale_dev;  // if set, the output scale is read from here (adaptive cross-section scale)
  double out_scale64;
  float* out;
  float* out_t;
  double* out64;
  double* out_t64;   // tiled FP64 tangent output (or nullptr)
  int64_t ld_out;
  float2* part;
  float2* part_t;
  double* part64;
  double* part_t64;
  const float* far_reach2;         // [nlay] squared far-tier reach of each layer (cm^-2)
  const int* far_t3;               // [nlay] tangent mode: 1 if far pairs keep the tangent's r^4 term
  const float* far_outer2;         // [nlay] squared outer reach (>= far_reach2; FLT_MAX: none)
  unsigned long long* near_pairs;  // profiling only: [0] pairs summed by the near tier,
                                   // [1] far pairs whose tangent stops at r^3, [2] outer pairs
};

// Per-layer quantities of one atmosphere.
struct AtmosDev {
  int nlay, nspec, bottom;
  const double* P;                 // [nlay] bar
  const double* T_in;              // [nlay] K, or nullptr: T = T0 (P / 1 bar)^alpha
  double T0, alpha, g, mmw;
  double cia_alpha0, cia_Tpow, cia_slope, cia_nu_c, vmr_h2;
  double logx[kMaxSpecies];
  double mass[kMaxSpecies];
  // outputs
  double *T, *dP, *lnP, *col, *cia, *dcia;   // col: [nspec][nlay]
};

// Radiative transfer on the model grid.
struct RtArgs {
  const double* nu;      // model grid
  int64_t ng;
  int nlay, nspec, bottom;
  const double *T, *cia, *dcia;
  double cia_slope, cia_nu_c;
  const void* tau;       // [nspec][nlay][ng] float or double
  const void* taut;      // tangent d tau^m / dT_n, same layout (adjoint only)
  double* F0;            // [ng]
  // adjoint
  const double* F0bar;   // [ng]
  double* Fup;           // scratch [nlay][ng]
  double* taubar;        // [nlay][ng]
  double* partT;         // [nblocks][nlay]
};

// Forward-mode tangent of the transfer: per-layer dT_n =
// [powerlaw] T_n (dT0/T0 + dalpha ln P_n) + dTl[n], per-species dlog10 X_m.
struct JvpArgs {
  const double* lnP;     // [nlay]
  const double* dTl;     // [nlay] or nullptr
  const double* dlogx;   // [nspec]
  double dT0_rel, dalpha;
  int powerlaw;
  double* dF0;           // [ng] output
};

// MODIT (Sec. 2.1.2) of one species on a batch of layers (blockIdx.y).
constexpr int kModitMaxBins = 32;   // width bins of the lineshape density
// The width rows are real: rows 2p and 2p + 1 travel as the real and the
// imaginary part of one complex DFT row.
constexpr int kModitRows = kModitMaxBins / 2;
struct ModitBins {
  double lng0, d;   // ln gamma~_k = lng0 + k d
  int K;
  int yexp;         // FP32: the layer's strength exponent (largest block exponent), 0 in FP64
};
// Per-layer constants of the MODIT line pass.
struct ModitLayer {
  double T, invT, lnTr, P, inv_qr, ln_inv_qr, lng_floor;   // lnTr = ln(T / T_ref); floor = ln(1e-3 beta~)
};
struct ModitArgs {
  LinesDev L;
  const double* T;         // device [nl] layer temperatures
  const double* P;         // device [nl] layer pressures
  const double* col;       // device [nl] column factors, or NULL: when given the output is
                           // col[n] sigma clamped at zero (an optical depth)
  double mass, R0, dlng;
  int amp_exp;             // FP32: a layer's largest strength is held at about 2^amp_exp (0 in FP64)
  const double* nu;        // grid [ng] (log-uniform)
  int64_t ng, n_fft;
  const double* nu_c;      // sorted centres (= L.nu_c)
  int64_t l0, n_in;        // lines inside the grid: [l0, l0 + n_in)
  int nl;                  // layers of this launch
  bool want_pos;           // compute f and cell (they depend on the grid only)
  void* f;                 // [n_in] R: position of the line in its cell, in [0, 1]
  int64_t* cell;           // [ng + 1]: lines of cell j are [cell[j], cell[j + 1]) (window-relative)
  ModitLayer* lay;         // [nl]
  void* rec;               // [nl][n_in] {ln gamma~, S} as R pairs (FP32: S 2^(amp_exp - block exponent))
  double* part;            // [nl][3 n_part] per line block: min and max of ln gamma~, and (FP32)
                           // the block's strength exponent
  int64_t n_part;
  ModitBins* bins;         // device [nl]
  void *rows0, *rows1;     // [nl][kModitRows][n_fft] complex (float2 or double2), bins in pairs
  void* out;               // [nl][ng] float or double
  bool out64;
};
// Largest batch of layers per MODIT launch (the forward DFT grid has
// nl * kModitRows rows in blockIdx.y).
constexpr int kModitMaxLayersPerLaunch = 65535 / kModitRows;

// Weak-line pre-selection (App. G) of one species in an isothermal atmosphere.
struct SelectArgs {
  LinesDev L;
  const int64_t* perm;       // caller index of sorted line i
  const double* T_strength;  // [n_T] temperatures scanned for the largest strength
  int n_T;
  double T_atm;
  int nlay, margin;
  const double *P, *dP, *col, *cia;   // per layer (col, cia at T_atm)
  double cia_slope, cia_nu_c;
  unsigned char* keep;       // [n] by caller index
  unsigned long long* n_kept;
};

// Response (rotation + IP) on the model grid.
struct RespDev {
  int64_t dlo, nrot;     // rotation taps for d = dlo .. dlo + nrot - 1, d = i - j
  int64_t K;             // IP taps for d' = -K .. K
  double dv, rv, vsini, u1, u2, beta_ip;
  double *rot, *drot_rv, *drot_vs, *ip;   // normalised taps / derivatives
  int64_t ob, ol;        // output range on the model grid
};

// T_lay == nullptr: one layer at (T_one, P_one).
// g2max_bits (FP32 records only, else nullptr): [nlay] running maximum of
// gamma^2 over the lines as FP32 bit patterns, raised by atomicMax.
// amax (FP32 single-layer records only, else nullptr): a zeroed word that
// receives the largest S(T) of the call; the records then carry the adaptive
// power-of-two amplitude scale it implies and write its inverse to *oscale.
// rec64t (tiled FP64 form, else nullptr): FP64 records with the full wing
// polynomial, and their tangents in rect64t (tangent mode, else nullptr);
// rec, rect, rec64 and g2max_bits are then unused.
hipError_t launch_line_records(const LinesDev& L, const double* T_lay, const double* P_lay,
                               const double* col_lay, double T_one, double P_one, double amp_scale,
                               const unsigned long long* amax, float* oscale, int layer0, int nlay,
                               LineRec* rec, LineRecT* rect, LineRec64* rec64, unsigned int* g2max_bits,
                               hipStream_t st, LineRec64T* rec64t = nullptr, LineRec64TT* rect64t = nullptr);
// Squared far-tier and outer reaches of each layer from its records and
// g2max_bits, which it resets to zero for the next chunk (and *amax, if given).
hipError_t launch_far_reach(const LineRec* rec, int64_t n_lines, int nlay, bool tangent,
                            unsigned int* g2max_bits, float* reach2, int* t3, float* outer2,
                            unsigned long long* amax, hipStream_t st);
// fp64 && tiled: the tiled FP64 form (A.rec64t; tangent mode with A.rect64t,
// A.out_t64 and A.part_t64).
hipError_t launch_voigt(const VoigtArgs& A, bool fp64, bool tangent, hipStream_t st, bool tiled = false);
// Zeroes bytes (a multiple of 4) at p with a kernel (no memset node).
hipError_t launch_zero_words(void* p, size_t bytes, hipStream_t st);
// Fills the coefficient table of the core branch's rational approximation on
// the current device (once per process and device; synchronises the device).
hipError_t ensure_weideman();
hipError_t launch_modit(const ModitArgs& M, bool fp64, hipStream_t st);
hipError_t launch_select_lines(const SelectArgs& A, hipStream_t st);
hipError_t launch_hjert_f32(int64_t n, const float* x, const float* a, float* H, float* L,
                            hipStream_t st);
hipError_t launch_hjert_f64(int64_t n, const double* x, const double* a, double* H, hipStream_t st);

hipError_t launch_atmos(const AtmosDev& A, hipStream_t st);
hipError_t launch_rt_forward(const RtArgs& R, bool tau64, hipStream_t st);
hipError_t launch_rt_adjoint(const RtArgs& R, bool tau64, int64_t nblocks, hipStream_t st);
hipError_t launch_grad_x(const double* taubar, const void* tau, bool tau64, int nspec, int nlay,
                         int64_t ng, double* partX, int64_t nblocks, hipStream_t st);
hipError_t launch_trans2e3(int64_t n, const double* x, double* T, double* dT, hipStream_t st);

hipError_t launch_taps(const RespDev& R, hipStream_t st);
hipError_t launch_response(const RespDev& R, const double* F0, double* mid, void* out, bool out64,
                           hipStream_t st);
// Transpose of the response: F0bar[ng] from cot[ol]; RV / vsini partials.
hipError_t launch_response_vjp(const RespDev& R, const double* F0, const void* cot, bool cot64,
                               double* midbar, double* F0bar, int64_t ng, double* partR,
                               int64_t nblocks_mid, hipStream_t st);
hipError_t launch_cast_copy(const double* src, void* dst, bool dst64, int64_t n, hipStream_t st);
// cot = (F - d)/s^2 and ceil(n/256) block partials of 1/2 sum ((d - F)/s)^2
hipError_t launch_gauss_cot(const float* F, const float* d, const float* sg, int64_t n, float* cot,
                            double* part, hipStream_t st);
hipError_t launch_to_double(const void* src, bool src64, double* dst, int64_t n, hipStream_t st);
hipError_t launch_grad_final(const double* partT, int64_t nbT, const double* partX, int64_t nbX,
                             const double* partR, int64_t nbR, const double* T, const double* lnP,
                             int nlay, int nspec, double T0, int powerlaw, double* out, hipStream_t st);
hipError_t launch_rt_jvp(const RtArgs& R, const JvpArgs& J, hipStream_t st);
// dF = IP * (rot * dF0 + (drot/dRV dRV + drot/dvsini dvsini) * F0), float output
hipError_t launch_response_jvp(const RespDev& R, const double* F0, const double* dF0, double d_rv,
                               double d_vsini, double* dmid, float* dout, hipStream_t st);

}  // namespace exo
