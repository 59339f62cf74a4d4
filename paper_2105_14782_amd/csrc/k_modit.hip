// MODIT (Sec. 2.1.2): the cross-section of many lines as the discrete
// convolution of a lineshape density with the Voigt profile, on a
// log-uniform grid where q = R0 ln(nu) is the grid index and the Doppler
// width in q, beta~ = sqrt(k_B T / (M m_u)) R0 / c, is common to all lines.
//
//   1. per line: fractional grid index x (linear in ln nu between grid
//      points), ln gamma~ with gamma~ = R0 gamma / nu (floored at 1e-3 beta~),
//      strength S(T) (FP32: scaled by powers of two, below);
//   2. width grid ln gamma~_k = lng0 + k d from the lines' range;
//   3. lineshape density S_{jk}: every line split over the four neighbouring
//      (j, k) nodes with linear weights, gathered per grid cell (the lines are
//      sorted by centre, so a cell's lines are one contiguous range and the
//      sum order is fixed);
//   4. DFT of every width row (length n_fft, zero padded; the rows are real,
//      so rows 2p and 2p + 1 share one complex DFT as its real and imaginary
//      parts), the product with the Voigt transform
//      exp(-2 pi^2 beta~^2 f^2 - 2 pi gamma~_k |f|) summed over k, inverse DFT;
//   5. sigma(nu_i) = sigma(q_i) R0 / nu_i.
// The DFTs are radix-4 / radix-2 Stockham passes through global memory.
// FP32 range: strengths of one layer can span more decades than FP32 holds
// (S(T) grows as exp(c2 E_low (1/T_ref - 1/T))), and every sum below is
// bounded by n_fft times the sum of the strengths.  So each block of 256
// lines stores S 2^(A - e_b), e_b = ceil(log2 of the block's largest S), the
// density scales a line by 2^(e_b - e_n) with e_n the layer's largest e_b
// (exact powers of two), and the output multiplies by 2^(e_n - A).  With
// A = 126 - log2(n_fft) - log2(lines) - 2 no sum can overflow; strengths more
// than ~2^(A + 126) below the layer's largest fall below FP32 and drop out.
// Every kernel takes a batch of layers in blockIdx.y (the line positions x
// are common to all of them); used as an opacity, the output of layer n is
// col_n sigma, clamped at zero where the Nyquist-truncated transform rings
// below it next to lines whose Doppler width is about one grid step.
#include <algorithm>
#include <type_traits>
#include <utility>

#include "exo_device.h"
#include "exo_launch.h"
#include "exo_lines.h"

namespace exo {

template <typename R> struct Cplx;
template <> struct Cplx<float> { using T = float2; };
template <> struct Cplx<double> { using T = double2; };

// -------------------------------------------------------------------------- 1
template <typename R> struct Pair;
template <> struct Pair<float> { using T = float2; };
template <> struct Pair<double> { using T = double2; };

__device__ inline double modit_beta_t(double T, double mass, double R0) {
  return sqrt(kKB * T / (mass * kMU)) * R0 / kC;
}

// first index in [lo, hi) with a[i] >= v (STRICT: a[i] > v)
template <bool STRICT>
__device__ inline int64_t lower_index(const double* __restrict__ a, int64_t lo, int64_t hi, double v) {
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (STRICT ? a[mid] <= v : a[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Per layer: 1/T, ln(T/T_ref), P, 1/q_r(T) and ln(1e-3 beta~).
__global__ __launch_bounds__(256) void k_modit_layers(const double* __restrict__ T, const double* __restrict__ P,
                                                      int nl, double mass, double R0, int qr_kind,
                                                      const double* __restrict__ qr_params, int n_qr,
                                                      ModitLayer* __restrict__ lay) {
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= nl) return;
  const double Tn = T[n];
  double qr, dlnqr;
  qr_eval(qr_kind, qr_params, n_qr, Tn, &qr, &dlnqr);
  ModitLayer c;
  c.T = Tn;
  c.invT = 1.0 / Tn;
  c.lnTr = log(Tn / kTref);
  c.P = P[n];
  c.inv_qr = 1.0 / qr;
  c.ln_inv_qr = -log(qr);
  c.lng_floor = log(1e-3 * modit_beta_t(Tn, mass, R0));
  lay[n] = c;
}

// Line position in its cell (grid only): for nu_j <= nu_l < nu_{j+1} the
// line belongs to cell j with f = (ln nu_l - ln nu_j) / (ln nu_{j+1} - ln nu_j);
// a line at nu_{ng-1} belongs to the last cell with f = 0.
template <typename R>
__global__ __launch_bounds__(256) void k_modit_pos(const double* __restrict__ nu_c, int64_t l0,
                                                   int64_t n_in, const double* __restrict__ nu,
                                                   int64_t ng, R* __restrict__ f) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n_in) return;
  const double nl = nu_c[l0 + i];
  if (nl >= nu[ng - 1]) {
    f[i] = (R)0;
    return;
  }
  int64_t lo = 0, hi = ng - 1;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (nu[mid] <= nl) lo = mid;
    else hi = mid;
  }
  const double lj = log(nu[lo]);
  f[i] = (R)((log(nl) - lj) / (log(nu[lo + 1]) - lj));
}

// cell[j] = first window line with nu_l >= nu_j (j < ng); cell[ng] = n_in
__global__ __launch_bounds__(256) void k_modit_cells(const double* __restrict__ nu_c, int64_t l0,
                                                     int64_t n_in, const double* __restrict__ nu,
                                                     int64_t ng, int64_t* __restrict__ cell) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j > ng) return;
  cell[j] = (j < ng ? lower_index<false>(nu_c, l0, l0 + n_in, nu[j]) : l0 + n_in) - l0;
}

// -------------------------------------------------------------------------- 2
// min/max of ln gamma~ and max of the strength exponent over a block of 256
__device__ inline void block_reduce3_256(double& mn, double& mx, double& ym, double* sm) {
  for (int o = 32; o > 0; o >>= 1) {
    mn = fmin(mn, __shfl_xor(mn, o));
    mx = fmax(mx, __shfl_xor(mx, o));
    ym = fmax(ym, __shfl_xor(ym, o));
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) {
    sm[w] = mn;
    sm[4 + w] = mx;
    sm[8 + w] = ym;
  }
  __syncthreads();
  mn = fmin(fmin(sm[0], sm[1]), fmin(sm[2], sm[3]));
  mx = fmax(fmax(sm[4], sm[5]), fmax(sm[6], sm[7]));
  ym = fmax(fmax(sm[8], sm[9]), fmax(sm[10], sm[11]));
}

// {ln gamma~, S} of one line at one layer.  FP64: the formulas as
// written.  FP32 records: ln S = a - c2 E / T - ln q_r + ln(1 - e^{-c2 nu / T})
// with a = ln(S0 / (1 - e^{-c2 nu / T_ref})) + c2 E / T_ref; y = log2 of the
// first three terms (whose parts nearly cancel) in FP64 (modit_log2core),
// then 2^(y + shift) as 2^m exp2(y + shift - m) with the integer m exact and
// exp2 in FP32 (relative error ~1e-7), the remaining factor and ln gamma~ in
// FP32.
struct ModitLine {
  double nu, S0, E, alpha, nt, gnat;
  double sfac;      // FP64 form: S0 / (1 - e^{-c2 nu / T_ref})
  double a, c2E;    // FP32 form
  float c2nu, R0nu;
};

__device__ inline ModitLine modit_line(const LinesDev& L, int64_t l, double R0) {
  ModitLine m;
  m.nu = L.nu_c[l];
  m.S0 = L.S0[l];
  m.E = L.E_low[l];
  m.alpha = L.alpha_ref[l];
  m.nt = L.n_texp[l];
  m.gnat = L.gamma_nat ? L.gamma_nat[l] : 0.0;
  const double eR = exp(-kC2 * m.nu / kTref);
  m.sfac = m.S0 / (1.0 - eR);
  m.c2E = kC2 * m.E;
  m.a = log(m.sfac) + m.c2E / kTref;
  m.c2nu = (float)(kC2 * m.nu);
  m.R0nu = (float)(R0 / m.nu);
  return m;
}

// log2 of S(T) without the stimulated-emission factor (<= 1); -2000 for S0 = 0
__device__ inline double modit_log2core(const ModitLine& m, const ModitLayer& c) {
  return fmax((fma(-m.c2E, c.invT, m.a) + c.ln_inv_qr) * 1.4426950408889634, -2000.0);
}

__device__ inline double2 modit_line_layer64(const ModitLine& m, const ModitLayer& c, double R0) {
  const double eT = exp(-kC2 * m.nu * c.invT);
  const double S = m.sfac * c.inv_qr * exp(-m.c2E * (c.invT - 1.0 / kTref)) * (1.0 - eT);
  const double g = m.alpha * exp(-m.nt * c.lnTr) * c.P + m.gnat;
  return make_double2(fmax(log(R0 * g / m.nu), c.lng_floor), S);
}

__device__ inline float modit_lng32(const ModitLine& m, const ModitLayer& c) {
  const float g = (float)m.alpha * expf(-(float)m.nt * (float)c.lnTr) * (float)c.P + (float)m.gnat;
  return fmaxf(logf(m.R0nu * g), (float)c.lng_floor);
}

// S 2^shift from y = modit_log2core, clamped so that the exponent stays a
// small integer (S0 = 0 and strengths below 2^-200 of the scale give
// 2^-200, zero in FP32)
__device__ inline float modit_strength32(const ModitLine& m, const ModitLayer& c, double y_raw, double shift) {
  const double y = fmin(fmax(y_raw + shift, -200.0), 200.0);
  const double mi = rint(y);
  const float core = ldexpf(exp2f((float)(y - mi)), (int)mi);
  return core * (1.0f - expf(-m.c2nu * (float)c.invT));
}

// One thread per line, looping over the layers of the launch (the line's
// parameters are read once): rec[n][i] = {ln gamma~, S(T_n)} with gamma~ =
// R0 gamma / nu_l floored at 1e-3 beta~, and per block the min/max of
// ln gamma~ (as stored) and the block's strength exponent into
// part[n][3 blockIdx.x ..].  FP32: S is stored as S 2^(amp_exp - e_b) with
// e_b = ceil(log2 of the block's largest S) (at least -1000); FP64: as is,
// e_b = 0.
template <typename R>
__global__ __launch_bounds__(256) void k_modit_lines(LinesDev L, const ModitLayer* __restrict__ lay, int nl,
                                                     double R0, int amp_exp, int64_t l0, int64_t n_in,
                                                     typename Pair<R>::T* __restrict__ rec,
                                                     double* __restrict__ part, int64_t n_part) {
  using P2 = typename Pair<R>::T;
  constexpr bool kF32 = std::is_same<R, float>::value;
  __shared__ double sm[12];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool ok = i < n_in;
  const ModitLine m = modit_line(L, l0 + (ok ? i : 0), R0);
  for (int n = 0; n < nl; ++n) {
    const ModitLayer c = lay[n];
    P2 v;
    double y = 0.0;
    if constexpr (kF32) {
      v.x = modit_lng32(m, c);
      y = modit_log2core(m, c);
    } else {
      v = modit_line_layer64(m, c, R0);
    }
    double mn = INFINITY, mx = -INFINITY, ym = -INFINITY;
    if (ok) {
      mn = mx = (double)v.x;
      ym = y;
    }
    block_reduce3_256(mn, mx, ym, sm);
    const double eb = kF32 ? fmax(ceil(ym), -1000.0) : 0.0;
    if constexpr (kF32) v.y = modit_strength32(m, c, y, (double)amp_exp - eb);
    if (ok) rec[(int64_t)n * n_in + i] = v;
    if (threadIdx.x == 0) {
      part[(int64_t)n * 3 * n_part + 3 * blockIdx.x] = mn;
      part[(int64_t)n * 3 * n_part + 3 * blockIdx.x + 1] = mx;
      part[(int64_t)n * 3 * n_part + 3 * blockIdx.x + 2] = eb;
    }
  }
}

// K = floor(range / d) + 2, at most kModitMaxBins (the step widens to range / (max - 2))
// and the layer's strength exponent, the largest block exponent
__global__ __launch_bounds__(256) void k_modit_bins(const double* __restrict__ part, int64_t nb,
                                                    double dlng, ModitBins* __restrict__ bins) {
  __shared__ double sm[12];
  part += (int64_t)blockIdx.y * 3 * nb;
  double mn = INFINITY, mx = -INFINITY, ym = -INFINITY;
  for (int64_t b = threadIdx.x; b < nb; b += 256) {
    mn = fmin(mn, part[3 * b]);
    mx = fmax(mx, part[3 * b + 1]);
    ym = fmax(ym, part[3 * b + 2]);
  }
  block_reduce3_256(mn, mx, ym, sm);
  if (threadIdx.x == 0) {
    // in doubles, so that a non-finite range still ends with 2 <= K <= max
    const double range = mx - mn;
    double d = dlng;
    double Kd = floor(range / d) + 2.0;
    if (!(Kd <= (double)kModitMaxBins)) {
      d = range / (kModitMaxBins - 2);
      Kd = fmin(floor(range / d) + 2.0, (double)kModitMaxBins);
    }
    bins[blockIdx.y].lng0 = mn;
    bins[blockIdx.y].d = d;
    bins[blockIdx.y].K = (int)fmax(2.0, fmin(Kd, (double)kModitMaxBins));
    bins[blockIdx.y].yexp = (int)ym;
  }
}

// -------------------------------------------------------------------------- 3
// Lineshape density of layer n = blockIdx.y: width rows 2p and 2p + 1 into
// the real and imaginary parts of rows[(n kModitRows + p) n_fft + j].
// Cell j gathers the lines of cell j - 1 (weight f) and of cell j (weight
// 1 - f).  A group of G = 2^lgG lanes shares a cell: lane g takes the lines
// g, g + G, ... of each range (consecutive lanes read consecutive lines, so
// the loads coalesce), accumulates them in its own LDS column, and the group
// then sums its G columns in lane order: a fixed summation order.  The first
// ceil(ng G / 256) blocks do the cells; the rest write the zero padding
// j = ng .. n_fft - 1.
// FP32: the line's strength times 2^(e_b - e_n) (e_b of its block of 256,
// e_n of the layer), an exact power of two <= 1
template <typename R>
__device__ inline R lsd_strength(typename Pair<R>::T r, const double* __restrict__ part, int64_t l, int yexp) {
  if constexpr (std::is_same<R, float>::value) return ldexpf(r.y, (int)part[3 * (l >> 8) + 2] - yexp);
  else return r.y;
}

template <typename R>
__device__ inline void lsd_add(R (*acc)[256], typename Pair<R>::T r, R S, R w, R lng0, R dinv, int K) {
  const R t = (r.x - lng0) * dinv;
  const int k0 = min(max((int)floor(t), 0), K - 2);   // 0 <= t by construction; clamp all the same
  const R fk = t - (R)k0;
  const R sw = S * w;
  acc[k0][threadIdx.x] += sw * ((R)1 - fk);
  acc[k0 + 1][threadIdx.x] += sw * fk;
}

template <typename R>
__global__ __launch_bounds__(256) void k_modit_lsd(const int64_t* __restrict__ cell, int64_t ng, int64_t n_fft,
                                                   int lgG, const R* __restrict__ f,
                                                   const typename Pair<R>::T* __restrict__ rec, int64_t n_in,
                                                   const ModitBins* __restrict__ bins,
                                                   const double* __restrict__ part, int64_t n_part,
                                                   typename Cplx<R>::T* __restrict__ rows) {
  using C = typename Cplx<R>::T;
  __shared__ R acc[kModitMaxBins][256];
  const int n = blockIdx.y;
  rec += (int64_t)n * n_in;
  part += (int64_t)n * 3 * n_part;
  rows += (int64_t)n * kModitRows * n_fft;
  const ModitBins b = bins[n];
  const int Kp = (b.K + 1) / 2;
  const int G = 1 << lgG;
  const int64_t cell_blocks = ((ng << lgG) + 255) / 256;
  if ((int64_t)blockIdx.x >= cell_blocks) {   // zero padding (whole block)
    const int64_t j = ng + ((int64_t)blockIdx.x - cell_blocks) * 256 + threadIdx.x;
    if (j < n_fft) {
      C z;
      z.x = (R)0;
      z.y = (R)0;
      for (int p = 0; p < Kp; ++p) rows[(int64_t)p * n_fft + j] = z;
    }
    return;
  }
  const R lng0 = (R)b.lng0, dinv = (R)(1.0 / b.d);
  const int g = threadIdx.x & (G - 1);
  const int64_t j = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> lgG;
  for (int k = 0; k < 2 * Kp; ++k) acc[k][threadIdx.x] = (R)0;   // an odd K pairs with a zero row
  if (j < ng) {
    const int64_t a1 = cell[j], a2 = cell[j + 1];
    const int64_t a0 = j > 0 ? cell[j - 1] : a1;
    for (int64_t l = a0 + g; l < a1; l += G) {
      const typename Pair<R>::T r = rec[l];
      lsd_add<R>(acc, r, lsd_strength<R>(r, part, l, b.yexp), f[l], lng0, dinv, b.K);
    }
    for (int64_t l = a1 + g; l < a2; l += G) {
      const typename Pair<R>::T r = rec[l];
      lsd_add<R>(acc, r, lsd_strength<R>(r, part, l, b.yexp), (R)1 - f[l], lng0, dinv, b.K);
    }
  }
  __syncthreads();
  if (j < ng) {
    const int base = threadIdx.x & ~(G - 1);
    for (int p = g; p < Kp; p += G) {
      C v;
      v.x = (R)0;
      v.y = (R)0;
      for (int q = 0; q < G; ++q) {
        v.x += acc[2 * p][base + q];
        v.y += acc[2 * p + 1][base + q];
      }
      rows[(int64_t)p * n_fft + j] = v;
    }
  }
}

// -------------------------------------------------------------------------- 4
__device__ inline void twiddle(double num, double den, double* c, double* s) {
  sincospi(2.0 * num / den, s, c);   // e^{-2 pi i num/den} = (c, -s)
}
__device__ inline void twiddle(float num, float den, float* c, float* s) {
  sincospif(2.0f * num / den, s, c);
}

template <typename C>
__device__ inline C cmul(C a, decltype(a.x) c, decltype(a.x) s) {
  // a * (c - i s)
  C r;
  r.x = a.x * c + a.y * s;
  r.y = a.y * c - a.x * s;
  return r;
}

// One Stockham pass of radix RADIX over rows of length n: the sub-transforms
// of length L become transforms of length RADIX * L.  With bins, row
// y = n kModitRows + p holds width rows 2p, 2p + 1 of layer n and is skipped
// when 2p >= K_n.
template <typename R, int RADIX>
__global__ __launch_bounds__(256) void k_fft_pass(const typename Cplx<R>::T* __restrict__ in,
                                                  typename Cplx<R>::T* __restrict__ out, int64_t n,
                                                  int64_t L, const ModitBins* __restrict__ bins) {
  using C = typename Cplx<R>::T;
  if (bins && (int)(blockIdx.y % kModitRows) >= (bins[blockIdx.y / kModitRows].K + 1) / 2) return;
  const int64_t q = n / RADIX;
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= q) return;
  const C* __restrict__ a = in + (int64_t)blockIdx.y * n;
  C* __restrict__ b = out + (int64_t)blockIdx.y * n;
  const int64_t k = j & (L - 1);
  const int64_t o = (j - k) * RADIX + k;
  C d[RADIX];
#pragma unroll
  for (int r = 0; r < RADIX; ++r) {
    d[r] = a[j + r * q];
    if (r > 0) {
      R c, s;
      twiddle((R)(r * k), (R)(RADIX * L), &c, &s);
      d[r] = cmul(d[r], c, s);
    }
  }
  if (RADIX == 2) {
    C y0, y1;
    y0.x = d[0].x + d[1].x;
    y0.y = d[0].y + d[1].y;
    y1.x = d[0].x - d[1].x;
    y1.y = d[0].y - d[1].y;
    b[o] = y0;
    b[o + L] = y1;
  } else {
    // 4-point DFT with e^{-2 pi i r s / 4}
    const R s02x = d[0].x + d[2].x, s02y = d[0].y + d[2].y;
    const R d02x = d[0].x - d[2].x, d02y = d[0].y - d[2].y;
    const R s13x = d[1].x + d[3].x, s13y = d[1].y + d[3].y;
    const R d13x = d[1].x - d[3].x, d13y = d[1].y - d[3].y;
    C y;
    y.x = s02x + s13x;
    y.y = s02y + s13y;
    b[o] = y;
    y.x = d02x + d13y;   // d0 - i d1 - d2 + i d3
    y.y = d02y - d13x;
    b[o + L] = y;
    y.x = s02x - s13x;
    y.y = s02y - s13y;
    b[o + 2 * L] = y;
    y.x = d02x - d13y;   // d0 + i d1 - d2 - i d3
    y.y = d02y + d13x;
    b[o + 3 * L] = y;
  }
}

// -------------------------------------------------------------------------- 4 (LDS)
// The same DFT in two passes through global memory (n = P Q, both powers of
// two, 32 <= P, Q <= 512).  With S = n / P transforms of length P:
//   pass A: B[t][k] = sum_i a[t + S i] W_P^{ik}, written to b[t P + k];
//   pass B: X[k + P u] = sum_t W_n^{tk} B[t][k] W_Q^{tu}.
// A block does C transforms side by side (C consecutive t in A, C consecutive
// k in B, so every gather and scatter moves C contiguous samples = 128 bytes),
// held in LDS as element (i, c) at i (C + 1) + c, and runs the radix-4/2
// Stockham stages of the global pass above in LDS, its twiddles from a table
// of W_N^e, e < N.
constexpr int kFftMaxLds = 512;

template <typename R> struct FftCols;
template <> struct FftCols<float> { static constexpr int C = 16; };
template <> struct FftCols<double> { static constexpr int C = 8; };

template <typename R, int RADIX>
__device__ __forceinline__ void lds_stage(typename Cplx<R>::T* lds, const typename Cplx<R>::T* tw, int N, int L) {
  using Cx = typename Cplx<R>::T;
  constexpr int C = FftCols<R>::C, Cp = C + 1;
  constexpr int MAXB = C * kFftMaxLds / (RADIX * 256);
  const int q = N / RADIX;
  const int nb = C * q;
  const int step = N / (RADIX * L);   // W_{RADIX L}^{e} = W_N^{e step}
  Cx d[MAXB][RADIX];
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int w = threadIdx.x + 256 * b;
    if (w < nb) {
      const int c = w & (C - 1), j = w / C, k = j & (L - 1);
#pragma unroll
      for (int r = 0; r < RADIX; ++r) {
        Cx v = lds[(j + r * q) * Cp + c];
        if (r > 0) {
          const Cx t = tw[r * k * step];   // W_N^{e} = (cos, -sin) stored as (c, s)
          v = cmul(v, t.x, t.y);
        }
        d[b][r] = v;
      }
      if (RADIX == 2) {
        const Cx a0 = d[b][0], a1 = d[b][1];
        d[b][0].x = a0.x + a1.x; d[b][0].y = a0.y + a1.y;
        d[b][1].x = a0.x - a1.x; d[b][1].y = a0.y - a1.y;
      } else {
        const R s02x = d[b][0].x + d[b][2].x, s02y = d[b][0].y + d[b][2].y;
        const R d02x = d[b][0].x - d[b][2].x, d02y = d[b][0].y - d[b][2].y;
        const R s13x = d[b][1].x + d[b][3].x, s13y = d[b][1].y + d[b][3].y;
        const R d13x = d[b][1].x - d[b][3].x, d13y = d[b][1].y - d[b][3].y;
        d[b][0].x = s02x + s13x; d[b][0].y = s02y + s13y;
        d[b][1].x = d02x + d13y; d[b][1].y = d02y - d13x;
        d[b][2].x = s02x - s13x; d[b][2].y = s02y - s13y;
        d[b][3].x = d02x - d13y; d[b][3].y = d02y + d13x;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int w = threadIdx.x + 256 * b;
    if (w < nb) {
      const int c = w & (C - 1), j = w / C, k = j & (L - 1);
      const int o = (j - k) * RADIX + k;
#pragma unroll
      for (int r = 0; r < RADIX; ++r) lds[(o + r * L) * Cp + c] = d[b][r];
    }
  }
  __syncthreads();
}

// twiddle table W_N^e = (cos, sin)(2 pi e / N), e < N, then the Stockham stages
template <typename R>
__device__ __forceinline__ void lds_fft(typename Cplx<R>::T* lds, typename Cplx<R>::T* tw, int N) {
  for (int e = threadIdx.x; e < N; e += 256) {
    R c, s;
    twiddle((R)e, (R)N, &c, &s);
    tw[e].x = c;
    tw[e].y = s;
  }
  __syncthreads();
  for (int L = 1; L < N;) {
    if (N / L >= 4) {
      lds_stage<R, 4>(lds, tw, N, L);
      L *= 4;
    } else {
      lds_stage<R, 2>(lds, tw, N, L);
      L *= 2;
    }
  }
}

// LDS holds two blocks per CU: ask for the registers of two waves per SIMD
template <typename R>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_fft_lds_a(const typename Cplx<R>::T* __restrict__ in,
                                                   typename Cplx<R>::T* __restrict__ out, int64_t n, int lgP,
                                                   const ModitBins* __restrict__ bins) {
  using Cx = typename Cplx<R>::T;
  constexpr int C = FftCols<R>::C, Cp = C + 1;
  __shared__ Cx lds[kFftMaxLds * Cp];
  __shared__ Cx tw[kFftMaxLds];
  if (bins && (int)(blockIdx.y % kModitRows) >= (bins[blockIdx.y / kModitRows].K + 1) / 2) return;
  const int P = 1 << lgP;
  const int64_t S = n >> lgP;
  const int64_t t0 = (int64_t)blockIdx.x * C;
  const Cx* __restrict__ a = in + (int64_t)blockIdx.y * n;
  Cx* __restrict__ b = out + (int64_t)blockIdx.y * n;
  for (int e = threadIdx.x; e < C * P; e += 256) {
    const int c = e & (C - 1), i = e / C;
    lds[i * Cp + c] = a[t0 + c + S * i];
  }
  __syncthreads();
  lds_fft<R>(lds, tw, P);
  for (int e = threadIdx.x; e < C * P; e += 256) {
    const int k = e & (P - 1), c = e >> lgP;
    b[(t0 + c) * P + k] = lds[k * Cp + c];
  }
}

// LDS holds two blocks per CU: ask for the registers of two waves per SIMD
template <typename R>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_fft_lds_b(const typename Cplx<R>::T* __restrict__ in,
                                                   typename Cplx<R>::T* __restrict__ out, int64_t n, int lgP,
                                                   const ModitBins* __restrict__ bins) {
  using Cx = typename Cplx<R>::T;
  constexpr int C = FftCols<R>::C, Cp = C + 1;
  __shared__ Cx lds[kFftMaxLds * Cp];
  __shared__ Cx tw[kFftMaxLds];
  if (bins && (int)(blockIdx.y % kModitRows) >= (bins[blockIdx.y / kModitRows].K + 1) / 2) return;
  const int64_t P = (int64_t)1 << lgP;
  const int Q = (int)(n >> lgP);
  const int64_t k0 = (int64_t)blockIdx.x * C;
  const Cx* __restrict__ a = in + (int64_t)blockIdx.y * n;
  Cx* __restrict__ b = out + (int64_t)blockIdx.y * n;
  for (int e = threadIdx.x; e < C * Q; e += 256) {
    const int c = e & (C - 1), t = e / C;
    const int64_t kk = k0 + c;
    R cs, sn;
    twiddle((R)(((int64_t)t * kk) & (n - 1)), (R)n, &cs, &sn);
    lds[t * Cp + c] = cmul(a[(int64_t)t * P + kk], cs, sn);
  }
  __syncthreads();
  lds_fft<R>(lds, tw, Q);
  for (int e = threadIdx.x; e < C * Q; e += 256) {
    const int c = e & (C - 1), u = e / C;
    b[k0 + c + P * u] = lds[u * Cp + c];
  }
}

// -------------------------------------------------------------------------- 4'
// Layer n = blockIdx.y:
// Y_n = conj( sum_k X_nk exp(-2 pi^2 beta~_n^2 f^2 - 2 pi gamma~_nk |f|) ), f
// the signed DFT frequency in cycles per grid step.  The DFT Z of row p packs
// the real rows 2p and 2p + 1: with A = Z[m], B = conj(Z[-m]),
// X_2p[m] = (A + B)/2 and X_2p+1[m] = (A - B)/(2i).  (The inverse DFT is then
// a forward DFT of Y, conjugated and divided by n_fft.)
template <typename R>
__global__ __launch_bounds__(256) void k_modit_product(const typename Cplx<R>::T* __restrict__ X,
                                                       int64_t n_fft, const ModitBins* __restrict__ bins,
                                                       const double* __restrict__ T, double mass,
                                                       double R0, typename Cplx<R>::T* __restrict__ Y) {
  using C = typename Cplx<R>::T;
  const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (m >= n_fft) return;
  const int n = blockIdx.y;
  X += (int64_t)n * kModitRows * n_fft;
  const int64_t mr = (n_fft - m) & (n_fft - 1);   // -m mod n_fft
  const double beta_t = modit_beta_t(T[n], mass, R0);
  const double f = (double)(m <= n_fft / 2 ? m : m - n_fft) / (double)n_fft;
  const double g = -2.0 * kPi * kPi * beta_t * beta_t * f * f;
  const double h = -2.0 * kPi * fabs(f);
  const ModitBins b = bins[n];
  double sx = 0.0, sy = 0.0;
  for (int k = 0; k < b.K; k += 2) {
    const C A = X[(int64_t)(k / 2) * n_fft + m];
    const C Bc = X[(int64_t)(k / 2) * n_fft + mr];   // B = conj(Bc)
    const double we = exp(g + h * exp(b.lng0 + b.d * k));
    // (A + B)/2
    sx += we * 0.5 * ((double)A.x + (double)Bc.x);
    sy += we * 0.5 * ((double)A.y - (double)Bc.y);
    if (k + 1 < b.K) {
      const double wo = exp(g + h * exp(b.lng0 + b.d * (k + 1)));
      // (A - B)/(2i) = -i (A - B)/2
      sx += wo * 0.5 * ((double)A.y + (double)Bc.y);
      sy -= wo * 0.5 * ((double)A.x - (double)Bc.x);
    }
  }
  C y;
  y.x = (R)sx;
  y.y = (R)-sy;
  Y[(int64_t)n * n_fft + m] = y;
}

// -------------------------------------------------------------------------- 5
// out[n][i] = Re Z_n[i] / n_fft * R0 / nu_i * 2^(e_n - amp_exp), times col[n]
// and clamped at zero when col is given (and, for FP32 optical depths, at
// 1e30: a layer that deep is opaque either way)
template <typename R, typename TO>
__global__ __launch_bounds__(256) void k_modit_out(const typename Cplx<R>::T* __restrict__ Z,
                                                   int64_t ng, int64_t n_fft, double R0,
                                                   const double* __restrict__ nu, int amp_exp,
                                                   const ModitBins* __restrict__ bins,
                                                   const double* __restrict__ col, TO* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= ng) return;
  const int n = blockIdx.y;
  double v = ldexp((double)Z[(int64_t)n * n_fft + i].x / (double)n_fft * R0 / nu[i], bins[n].yexp - amp_exp);
  if (col) {
    v = fmax(v * col[n], 0.0);
    if (sizeof(TO) == 4) v = fmin(v, 1e30);
  }
  out[(int64_t)n * ng + i] = (TO)v;
}

template <typename TO>
__global__ __launch_bounds__(256) void k_zero(TO* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = (TO)0;
}

// -------------------------------------------------------------------------- launch
static inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

// Stockham passes over `rows` rows of length n (a power of two); returns the
// buffer holding the result (a or b).
template <typename R>
static void* fft_rows(void* a, void* b, int64_t n, int rows, const ModitBins* bins, hipStream_t st) {
  using C = typename Cplx<R>::T;
  int m = 0;
  while (((int64_t)1 << m) < n) ++m;
  if (m >= 10 && m <= 18) {
    constexpr int NC = FftCols<R>::C;
    const int lgP = m / 2;
    hipLaunchKernelGGL(k_fft_lds_a<R>, dim3((unsigned)((n >> lgP) / NC), (unsigned)rows), dim3(256), 0, st,
                       (const C*)a, (C*)b, n, lgP, bins);
    hipLaunchKernelGGL(k_fft_lds_b<R>, dim3((unsigned)(((int64_t)1 << lgP) / NC), (unsigned)rows), dim3(256), 0,
                       st, (const C*)b, (C*)a, n, lgP, bins);
    return a;
  }
  C* src = (C*)a;
  C* dst = (C*)b;
  for (int64_t L = 1; L < n;) {
    const int radix = n / L >= 4 ? 4 : 2;
    dim3 grid(nblk(n / radix), (unsigned)rows);
    if (radix == 4) hipLaunchKernelGGL((k_fft_pass<R, 4>), grid, dim3(256), 0, st, src, dst, n, L, bins);
    else hipLaunchKernelGGL((k_fft_pass<R, 2>), grid, dim3(256), 0, st, src, dst, n, L, bins);
    std::swap(src, dst);
    L *= radix;
  }
  return src;
}

template <typename R>
static hipError_t modit_impl(const ModitArgs& M, hipStream_t st) {
  using C = typename Cplx<R>::T;
  using P2 = typename Pair<R>::T;
  const unsigned nl = (unsigned)M.nl;
  const int64_t nbl = nblk(M.n_in);
  if (M.want_pos) {
    hipLaunchKernelGGL(k_modit_pos<R>, dim3((unsigned)nbl), dim3(256), 0, st, M.nu_c, M.l0, M.n_in, M.nu, M.ng,
                       (R*)M.f);
    hipLaunchKernelGGL(k_modit_cells, dim3(nblk(M.ng + 1)), dim3(256), 0, st, M.nu_c, M.l0, M.n_in, M.nu, M.ng,
                       M.cell);
  }
  hipLaunchKernelGGL(k_modit_layers, dim3(nblk(M.nl)), dim3(256), 0, st, M.T, M.P, M.nl, M.mass, M.R0,
                     M.L.qr_kind, M.L.qr_params, M.L.n_qr, M.lay);
  hipLaunchKernelGGL(k_modit_lines<R>, dim3((unsigned)nbl), dim3(256), 0, st, M.L, (const ModitLayer*)M.lay,
                     M.nl, M.R0, M.amp_exp, M.l0, M.n_in, (P2*)M.rec, M.part, M.n_part);
  hipLaunchKernelGGL(k_modit_bins, dim3(1, nl), dim3(256), 0, st, M.part, M.n_part, M.dlng, M.bins);
  // lanes per cell: about a quarter of the mean lines per cell, a power of two in [1, 64]
  int lgG = 0;
  while (lgG < 6 && ((int64_t)4 << lgG) * 2 <= M.n_in / M.ng) ++lgG;
  const int64_t lsd_blocks = ((M.ng << lgG) + 255) / 256 + nblk(M.n_fft - M.ng);
  hipLaunchKernelGGL(k_modit_lsd<R>, dim3((unsigned)lsd_blocks, nl), dim3(256), 0, st, M.cell, M.ng, M.n_fft,
                     lgG, (const R*)M.f, (const P2*)M.rec, M.n_in, M.bins, M.part, M.n_part, (C*)M.rows0);
  void* X = fft_rows<R>(M.rows0, M.rows1, M.n_fft, M.nl * kModitRows, M.bins, st);
  void* Y = X == M.rows0 ? M.rows1 : M.rows0;
  hipLaunchKernelGGL(k_modit_product<R>, dim3(nblk(M.n_fft), nl), dim3(256), 0, st, (const C*)X, M.n_fft,
                     M.bins, M.T, M.mass, M.R0, (C*)Y);
  void* Z = fft_rows<R>(Y, X, M.n_fft, M.nl, nullptr, st);
  if (M.out64)
    hipLaunchKernelGGL((k_modit_out<R, double>), dim3(nblk(M.ng), nl), dim3(256), 0, st, (const C*)Z, M.ng,
                       M.n_fft, M.R0, M.nu, M.amp_exp, M.bins, M.col, (double*)M.out);
  else
    hipLaunchKernelGGL((k_modit_out<R, float>), dim3(nblk(M.ng), nl), dim3(256), 0, st, (const C*)Z, M.ng,
                       M.n_fft, M.R0, M.nu, M.amp_exp, M.bins, M.col, (float*)M.out);
  return hipGetLastError();
}

hipError_t launch_modit(const ModitArgs& M, bool fp64, hipStream_t st) {
  if (M.nl < 1 || M.nl > kModitMaxLayersPerLaunch) return hipErrorInvalidValue;
  if (M.n_in == 0) {
    const int64_t n = (int64_t)M.nl * M.ng;
    if (M.out64) hipLaunchKernelGGL(k_zero<double>, dim3(nblk(n)), dim3(256), 0, st, (double*)M.out, n);
    else hipLaunchKernelGGL(k_zero<float>, dim3(nblk(n)), dim3(256), 0, st, (float*)M.out, n);
    return hipGetLastError();
  }
  return fp64 ? modit_impl<double>(M, st) : modit_impl<float>(M, st);
}

}  // namespace exo
