/*
 * exohip -- direct line-by-line opacity, emission radiative transfer and
 * broadening response on AMD Instinct MI355X (gfx950), with hand-written
 * adjoints.  C ABI.
 *
 * The model is the "direct LPF" spectrum model of Kawahara et al.,
 * arXiv:2105.14782:
 *   - line strength S(T) (Sec. 2.2, Eq. Slog), thermal Doppler width
 *     (Sec. 2.1.1, Eq. thermal), pressure + natural Lorentz width
 *     (Eq. gammaexomol, Eq. naturalgamma);
 *   - Voigt profile through the Voigt-Hjerting function H = Re w(x+ia),
 *     with the branches of the paper's "hjert" (Sec. 2.1.1): the asymptotic
 *     w_2 for x^2 + a^2 >= 111 (Eq. asywofz); inside, the plain FP64 form
 *     takes the Algorithm-916 series (eta = 0.5, M = 27, Eq. algo916) and the
 *     FP32 form a rational approximation of w (Weideman 1994), continued to
 *     first order in a from the real axis for a < 1e-5; the FP32 form drops,
 *     for lines far from a group of grid points, the terms of w_2 that a
 *     per-layer bound keeps below FP32 rounding (two distance tiers);
 *   - cross-section sum over lines (Eq. crosssec), layer optical depth
 *     (Sec. 3, Eq. dtau_line2) plus H2-H2 CIA (Sec. 2.4, Eq. taucont);
 *   - pure-absorption two-stream transfer F_n = T_n F_{n+1} + (1-T_n) S_n
 *     with T = 2 E3(dtau) (Eq. rerr, Eq. trans, AS70 E1 of Eq. transco) and
 *     S = pi B(T_n) (Eq. sourcepla);
 *   - rotation (rigid-body limb-darkened kernel, Sec. 4.1) with radial
 *     velocity, then Gaussian instrumental profile (Sec. 4.2), as the
 *     normalised response of Eq. responsenu on a log-uniform grid.
 *
 * Conventions (all functions):
 *   - Return value: EXO_OK (0) or a negative exo_status.  Nothing aborts or
 *     throws across this boundary.  exo_last_error() gives a message for the
 *     calling thread's last failure.
 *   - Validation failures return before any device work is enqueued.
 *   - "dev" pointers are device memory owned by the caller; "host" pointers
 *     are host memory read (or written) before the call returns, unless said
 *     otherwise.  The library never frees caller memory.
 *   - `stream` is a hipStream_t (NULL = default stream).  Device work is
 *     asynchronous on that stream unless a host output is produced.
 *   - Units: wavenumber cm^-1, temperature K, pressure bar, velocities km/s,
 *     cross-sections cm^2/molecule, fluxes erg s^-1 cm^-2 (cm^-1)^-1.
 */
#ifndef EXOHIP_H
#define EXOHIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct exo_ctx exo_ctx;

typedef enum {
  EXO_OK = 0,
  EXO_EINVAL = -1,   /* invalid argument (nothing was launched) */
  EXO_ENOMEM = -2,   /* device or host allocation failed / over budget */
  EXO_ENOTSET = -3,  /* species or grid not registered */
  EXO_EDEVICE = -4   /* HIP runtime error */
} exo_status;

typedef enum {
  /* FP64 line parameters and FP64 line-centre offset, FP32 Voigt
   * evaluation with compensated (Neumaier) accumulation over lines. */
  EXO_FP32_KAHAN = 0,
  /* The plain FP64 form: the paper's hjert written out in double precision
   * per (line, grid point) with IEEE divisions; plain FP64 accumulation. */
  EXO_FP64 = 1,
  /* The FP32 form's algorithm in double precision: the same thread
   * mapping, per-wave record staging, near/far split and core branch (the
   * rational approximation of w), with the full asymptotic polynomial on
   * every wing pair and plain FP64 accumulation.  For measuring the cost of
   * precision alone.  Taken by exo_cross_section, exo_emission_flux and
   * exo_flux_vjp (whose FP64 gradient always runs this form, through its
   * tangent mode); outputs are double. */
  EXO_FP64_TILED = 2
} exo_precision;

typedef enum {
  EXO_QR_POWER = 0, /* q_r(T) = (T/296)^k, qr_params = {k}, n_qr = 1      */
  EXO_QR_TABLE = 1  /* linear interpolation of Q on T nodes:
                       qr_params = {T_0..T_{n-1}, Q_0..Q_{n-1}}, n_qr = 2n,
                       nodes ascending, n >= 2; q_r = Q(T)/Q(296);
                       outside [T_0, T_{n-1}] the end value is held, and
                       d ln q_r/dT is the derivative from the right (zero
                       for T < T_0 and T >= T_{n-1}) (Sec. 2.3)           */
} exo_qr_kind;

typedef enum {
  EXO_FB_PLANCK_BOTTOM = 0, /* F_B = pi B(T of the deepest layer)          */
  EXO_FB_ZERO = 1           /* F_B = 0                                      */
} exo_bottom;

/* Line optical depths of the emission model (exo_atmos.opacity). */
typedef enum {
  EXO_OPACITY_LPF = 0,      /* direct sum of the line profiles (Sec. 2.1.1)  */
  EXO_OPACITY_MODIT = 1     /* MODIT (Sec. 2.1.2) on the model grid, which must be
                               log-uniform: only the lines inside the model grid
                               contribute; the cross-section is clamped at zero
                               before it becomes an optical depth.  Forward only:
                               the derivative entry points reject it. */
} exo_opacity;

#define EXO_MAX_SPECIES 64

/* Message describing the calling thread's most recent failure ("" if none).
 * The pointer stays valid until the next exo_* call on the same thread. */
const char* exo_last_error(void);

/* Library version string. */
const char* exo_version(void);

/* Create a context on HIP device `device`.  The context owns the resident
 * line lists, the wavenumber grid and a grow-only device workspace.
 * Errors: EXO_EINVAL (bad device), EXO_EDEVICE. */
int exo_create(int device, exo_ctx** out);

/* Release every device buffer of the context.  Waits for outstanding work. */
int exo_destroy(exo_ctx* ctx);

/* Register (or replace) the line list of species slot s (0 <= s < 64),
 * Table 1 quantities in ExoMol broadening form (Sec. 2.2.2):
 *   nu_c      [n_lines] line centres, cm^-1, > 0
 *   S0        [n_lines] strength at T_ref = 296 K, cm/molecule, >= 0
 *   E_low     [n_lines] lower-state energy, cm^-1, >= 0
 *   alpha_ref [n_lines] Lorentz HWHM at 296 K and 1 bar, cm^-1 bar^-1, >= 0
 *   n_texp    [n_lines] temperature exponent of alpha_ref
 *   gamma_nat [n_lines] natural HWHM A/(4 pi c), cm^-1 (Eq. naturalgamma);
 *             may be NULL (zero)
 *   mass_amu  molecular mass in atomic mass units, > 0
 *   qr_kind, qr_params, n_qr: partition-function ratio (exo_qr_kind).
 * All arrays are host memory, copied before return (the caller may free
 * them).  Lines are sorted by centre internally; results do not depend on
 * the input order beyond floating-point summation order.
 * Errors: EXO_EINVAL (n_lines < 1, NaN, negative widths...), EXO_ENOMEM,
 * EXO_EDEVICE. */
int exo_set_lines(exo_ctx* ctx, int s, int64_t n_lines, const double* nu_c,
                  const double* S0, const double* E_low, const double* alpha_ref,
                  const double* n_texp, const double* gamma_nat, double mass_amu,
                  int qr_kind, const double* qr_params, int n_qr);

/* Register the wavenumber grid nu_j (host, [n_nu], strictly ascending,
 * n_nu >= 2), copied before return.  The library detects whether the grid
 * is log-uniform (relative spread of ln(nu_{j+1}/nu_j) below 1e-6); the
 * response of Sec. 4 requires such a grid (Eq. response2).
 * Errors: EXO_EINVAL, EXO_ENOMEM, EXO_EDEVICE. */
int exo_set_grid(exo_ctx* ctx, int64_t n_nu, const double* nu);

/* Single-layer cross-section of species s at (T_K, P_bar) on the whole grid
 * (Eq. crosssec summed over lines):
 *   sigma(nu_j) = sum_l S_l(T) V(nu_j - nu_l; beta_l(T), gamma_l(T, P)).
 * sigma_dev: device, [n_nu] float (EXO_FP32_KAHAN) or double (EXO_FP64,
 * EXO_FP64_TILED).  A float cross-section beyond the FP32 range comes back
 * as +inf.
 * Errors: EXO_ENOTSET, EXO_EINVAL (T <= 0, P < 0, bad precision),
 * EXO_ENOMEM, EXO_EDEVICE. */
int exo_cross_section(exo_ctx* ctx, int s, double T_K, double P_bar, int precision,
                      void* sigma_dev, void* stream);

/* exo_cross_section for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, kernels and result (bitwise) as
 * exo_cross_section; no hipMalloc, hipFree, memset or event is issued.  Its
 * scratch (line records, the far-tier table and split partial sums) is not
 * the context's workspace but a fixed 128 MiB array per GPU, held from the
 * first exo_create on that GPU until the process ends.  Every call on a GPU
 * shares that GPU's array and it keeps the last call's contents (each call
 * clears what must start at zero, with a kernel): calls that overlap on one
 * GPU (other streams, threads or contexts) race, and the caller must
 * serialise them.
 * precision: EXO_FP32_KAHAN or EXO_FP64.
 * Errors: as exo_cross_section, and EXO_ENOMEM (nothing launched) when the
 * call would need more than 128 MiB of scratch: 64 B (FP32) or 32 B (FP64)
 * per line, 64 KiB, and 8 B per grid point and line split (the splits bring
 * the workgroups of one launch to about 8192). */
int exo_cross_section_noalloc(exo_ctx* ctx, int s, double T_K, double P_bar, int precision,
                              void* sigma_dev, void* stream);

/* The same cross-section by MODIT (Sec. 2.1.2), the paper's method for many
 * lines: a lineshape density on the log-uniform grid (q = R0 ln nu, every
 * line split over the neighbouring grid points and log-spaced Lorentz-width
 * bins with linear weights) convolved with the Voigt profile through its
 * Fourier transform exp(-2 pi^2 beta~^2 f^2 - 2 pi gamma~ |f|), with the
 * common Doppler width beta~ = sqrt(k_B T/(M m_u)) R0/c in grid steps.
 *   dln_gamma  step of the width bins in ln(gamma R0/nu) (>= 1e-3; the bins
 *              widen when more than 32 would be needed)
 * Needs a log-uniform grid.  Only lines with nu_0 <= nu_l <= nu_{N-1} enter
 * the density; the transform length is the smallest power of two >= 2N (the
 * aliasing correction the paper mentions is unpublished and not applied).
 * FP32: the strengths are carried with exact power-of-two scales per block
 * of lines and per layer, so no intermediate sum overflows; a result beyond
 * the FP32 range comes back infinite, and values far below the layer's
 * largest lose precision to the transform's rounding (App. B).
 * sigma_dev as exo_cross_section.  Errors: EXO_EINVAL, EXO_ENOTSET,
 * EXO_ENOMEM, EXO_EDEVICE. */
int exo_cross_section_modit(exo_ctx* ctx, int species, double T_K, double P_bar, int precision,
                            double dln_gamma, void* sigma_dev, void* stream);

/* Atmosphere of Sec. 3 with the power-law T-P profile of Sec. 5.2:
 * T_n = T0 (P_n / 1 bar)^alpha, layer 0 at the top (lowest pressure).
 * dP_n = P_n - P_{n-1} with P_{-1} = P_0^2/P_1.  Molecular optical depth of
 * Eq. dtau_line2 with mass mixing ratio X_m = 10^log10_mmr[m]; CIA of
 * Eq. taucont with the smooth coefficient
 *   alpha_CIA(T, nu) = cia_alpha0 (T/1000)^cia_Tpow exp(cia_slope (nu - cia_nu_c)/40)
 * [cm^5] and H2 volume mixing ratio vmr_h2. */
typedef struct {
  int32_t n_layers;          /* 2..4096 */
  const double* P_bar;       /* host [n_layers], strictly ascending, > 0 */
  double T0_K, alpha;
  int32_t n_species;         /* 1..EXO_MAX_SPECIES */
  const int32_t* species;    /* host [n_species] registered species slots */
  const double* log10_mmr;   /* host [n_species] */
  double g_cgs;              /* gravity, cm s^-2 */
  double mmw;                /* mean molecular weight mu */
  double cia_alpha0, cia_Tpow, cia_slope, cia_nu_c, vmr_h2;
  int32_t bottom;            /* exo_bottom */
  int64_t grid_begin;        /* model grid = context grid [grid_begin, grid_begin+grid_len) */
  int64_t grid_len;          /* 0 = the whole context grid */
  const double* T_layers;    /* host [n_layers] K (each > 1, finite) or NULL: the
                                layer-by-layer temperature model of Sec. 6.1; when
                                given, T0_K and alpha are not used */
  int32_t opacity;           /* exo_opacity: how the line optical depths are formed */
  double modit_dln_gamma;    /* EXO_OPACITY_MODIT: width-grid step in ln gamma~ (>= 1e-3) */
} exo_atmos;

/* Response of Sec. 4 on the (log-uniform) model grid: rotation with
 * quadratic limb darkening (u1, u2) and radial velocity in the kernel
 * argument, then a Gaussian IP of standard deviation c/(2 sqrt(2 ln 2) R),
 * truncated at 6 sigma.  Each stage is normalised by the sum of its own
 * (shifted) taps.  The output grid is model-grid indices
 * [out_begin, out_begin + out_len); every tap they need must lie inside the
 * model grid (else EXO_EINVAL). */
typedef struct {
  double rv_kms;     /* radial velocity; > 0 shifts lines to lower nu */
  double vsini_kms;  /* > 0, and at least two grid spacings */
  double u1, u2;     /* limb darkening */
  double R_inst;     /* resolving power, > 0 */
  int64_t out_begin, out_len;
} exo_response;

/* Emission spectrum F = k_G * k_R * F0 (Eq. model without the photometric
 * normalisation), or F0 on the whole model grid when `resp` is NULL.
 * flux_dev: device [out_len] (or [model grid length]) float for
 * EXO_FP32_KAHAN, double for EXO_FP64 and EXO_FP64_TILED.
 * Errors: EXO_ENOTSET, EXO_EINVAL, EXO_ENOMEM, EXO_EDEVICE. */
int exo_emission_flux(exo_ctx* ctx, const exo_atmos* atm, const exo_response* resp,
                      int precision, void* flux_dev, void* stream);

/* Vector-Jacobian product of the emission spectrum (the paper provides
 * forward-mode JVPs, App. D; this is the reverse-mode counterpart).
 *   precision EXO_FP32_KAHAN, or EXO_FP64 / EXO_FP64_TILED: both run the
 *             tiled FP64 form, which has a tangent mode (the plain FP64 form
 *             has none), for the forward pass and the gradient
 *   cot_dev   device [out_len] (or model grid length when resp == NULL),
 *             dL/dF, float (EXO_FP32_KAHAN) or double (FP64)
 *   grad_host host [2 + n_species + 2] doubles, written on return:
 *             {dL/dT0, dL/dalpha, dL/dlog10X_1..S, dL/dRV, dL/dvsini}
 *             (RV, vsini entries are 0 when resp == NULL; T0, alpha
 *             entries are 0 with atm->T_layers, whose gradient is
 *             dL_dT_layers)
 *   dL_dT_layers host [n_layers] or NULL: dL/dT_n of every layer
 *   flux_dev  device or NULL: if given, the forward spectrum F is written
 *             there as by exo_emission_flux (one pass gives F and gradient;
 *             float or double as cot_dev)
 * The forward model is re-evaluated internally.  Blocks until the gradient
 * is on the host.  Errors as exo_emission_flux. */
int exo_flux_vjp(exo_ctx* ctx, const exo_atmos* atm, const exo_response* resp,
                 int precision, const void* cot_dev, double* grad_host,
                 double* dL_dT_layers, void* flux_dev, void* stream);

/* Gaussian log-likelihood and its gradient in one pass (what a Hamiltonian
 * sampler needs at every leapfrog step, Sec. 5.2):
 *   loss = 1/2 sum_j ((data_j - F_j) / sigma_j)^2
 * with F the spectrum of (atm, resp) as exo_emission_flux computes it.
 *   data_dev, sigma_dev  device [out_len] float (sigma > 0)
 *   loss_host            host double, written on return
 *   grad_host, dL_dT_layers, flux_dev as exo_flux_vjp (the gradient of loss)
 * One forward pass: the cotangent (F - data)/sigma^2 is formed on the device
 * from this pass's F.  EXO_FP32_KAHAN only.  Blocks until loss and gradient
 * are on the host.  Errors as exo_flux_vjp. */
int exo_loss_grad(exo_ctx* ctx, const exo_atmos* atm, const exo_response* resp, int precision,
                  const void* data_dev, const void* sigma_dev, double* loss_host, double* grad_host,
                  double* dL_dT_layers, void* flux_dev, void* stream);

/* Jacobian-vector product of the emission spectrum (forward mode, App. D):
 * dF = J dtheta along the parameter tangent
 *   dtheta_host   host [2 + n_species + 2] doubles
 *                 {dT0, dalpha, dlog10X_1..S, dRV, dvsini}; dT0 and dalpha
 *                 are not used with atm->T_layers, dRV and dvsini not when
 *                 resp == NULL
 *   dT_layers_host host [n_layers] or NULL: a per-layer temperature tangent
 *                 dT_n, added to the one (dT0, dalpha) induce
 *   flux_dev      device [out_len] float or NULL: the spectrum F, as
 *                 exo_emission_flux writes it
 *   dflux_dev     device [out_len] float: J dtheta
 * (out_len: resp->out_len, or the model grid length when resp == NULL.)
 * EXO_FP32_KAHAN only (the tangents are those of the FP32 Voigt sum; the
 * transfer and the response run in FP64).  Host arrays are copied before
 * the call returns; the work is asynchronous on `stream`.
 * Errors: EXO_ENOTSET, EXO_EINVAL, EXO_ENOMEM, EXO_EDEVICE. */
int exo_flux_jvp(exo_ctx* ctx, const exo_atmos* atm, const exo_response* resp,
                 int precision, const double* dtheta_host, const double* dT_layers_host,
                 void* flux_dev, void* dflux_dev, void* stream);

/* Weak-line pre-selection (App. G): which lines of species `species` can
 * shape the emission spectrum.  In an isothermal atmosphere at T_atm_K on
 * the pressure grid of `atm` (its n_layers, P_bar, g_cgs, mmw and CIA fields
 * are used; T0/alpha/T_layers, species and grid fields are not), every line
 * gets its largest strength over T_strength_host[n_T] (n_T = 0: T_atm alone),
 * its line-centre optical depth per layer
 * dP_n/(m_u g) 10^log10_mmr/M S/(sqrt(2 pi) beta) erfcx(gamma_n/(sqrt2 beta))
 * and the contribution function e^{-tau_n} dtau_n P_n/dP_n (tau_n including
 * layer n).  The line is kept iff the layer where that peaks (the first
 * maximum) is at most `margin_layers` deeper than where the H2-H2
 * continuum's peaks at the line centre (the paper uses 2).
 *   keep_dev     device [n_lines] uint8, in the caller's order of exo_set_lines:
 *                1 = kept, 0 = shielded by the continuum
 *   n_kept_host  NULL, or the number kept (then the call blocks until done)
 * FP64 throughout.  Errors: EXO_EINVAL, EXO_ENOTSET, EXO_ENOMEM, EXO_EDEVICE. */
int exo_select_lines(exo_ctx* ctx, int species, double log10_mmr, const exo_atmos* atm,
                     double T_atm_K, const double* T_strength_host, int n_T, int margin_layers,
                     uint8_t* keep_dev, int64_t* n_kept_host, void* stream);

/* Response alone (Sec. 4) applied to a caller spectrum F0 on the model grid
 * [grid_begin, grid_begin + grid_len) of the context grid (grid_len 0 = all):
 * F0_dev device [grid_len] double, out_dev device [resp->out_len] double.
 * Errors: EXO_ENOTSET, EXO_EINVAL, EXO_EDEVICE. */
int exo_broaden(exo_ctx* ctx, int64_t grid_begin, int64_t grid_len,
                const exo_response* resp, const void* F0_dev, void* out_dev,
                void* stream);

/* The Voigt-Hjerting function exactly as the FP32 hot kernel evaluates it
 * (Sec. 2.1.1 hjert branches; the core as described at the top of this file):
 * x_dev, a_dev device [n] float (a >= 0); H_dev device [n] float;
 * L_dev device [n] float or NULL (Im w).  Errors: EXO_EINVAL, EXO_EDEVICE. */
int exo_hjert_f32(int64_t n, const float* x_dev, const float* a_dev, float* H_dev,
                  float* L_dev, void* stream);

/* Same in the plain FP64 form (double arrays; L not provided). */
int exo_hjert_f64(int64_t n, const double* x_dev, const double* a_dev, double* H_dev,
                  void* stream);

/* Transmission T = 2 E3(x) with the AS70 E1 fit (Eq. trans, Eq. transco) and
 * its derivative dT/dx = -2 E2(x), as the transfer kernels evaluate them.
 * x_dev device [n] double (>= 0); T_dev, dT_dev device [n] double (dT may be
 * NULL).  Errors: EXO_EINVAL, EXO_EDEVICE. */
int exo_trans2e3(int64_t n, const double* x_dev, double* T_dev, double* dT_dev, void* stream);

/* ---- timing of the Voigt-sum kernel (for roofline reporting) ----------- */
/* Enable (1) / disable (0) HIP-event timing of every Voigt-sum launch on the
 * stream it is launched on; enabling clears previous records. */
int exo_profile_enable(exo_ctx* ctx, int on);
/* Synchronises on the recorded events and returns the number of Voigt-sum
 * launches, their summed duration in ms and the summed pair evaluations
 * (lines x grid points x layers) they performed. */
int exo_profile_read(exo_ctx* ctx, int64_t* n_launches, double* total_ms,
                     double* total_evals);
/* Of those evaluations, the number the FP32 launches summed with the full
 * wing polynomial and the core test (the near tier); the rest used the
 * truncated far-tier polynomial.  Synchronises like exo_profile_read.
 * Errors: EXO_EINVAL, EXO_EDEVICE. */
int exo_profile_read_near(exo_ctx* ctx, double* near_evals);
/* Of the far-tier evaluations of the profiled tangent-mode launches inside
 * the outer reach, the number whose T-derivative polynomial stops at r^3
 * (layers whose truncation bound allows it; the others keep the r^4 term).
 * Synchronises like exo_profile_read.  Errors: EXO_EINVAL, EXO_EDEVICE. */
int exo_profile_read_far_cut(exo_ctx* ctx, double* far_cut_evals);
/* Of the far-tier evaluations of the profiled FP32 launches, the number
 * beyond the layer's outer reach, summed with the value (and tangent)
 * polynomial cut after r^2.  Synchronises like exo_profile_read.
 * Errors: EXO_EINVAL, EXO_EDEVICE. */
int exo_profile_read_far_outer(exo_ctx* ctx, double* outer_evals);

#ifdef __cplusplus
}
#endif
#endif /* EXOHIP_H */
