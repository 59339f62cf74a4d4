// MODIT (Sec. 2.1.2): the cross-section of many lines as the discrete
// convolution of a lineshape density with the Voigt profile, on a
// log-uniform grid where q = R0 ln(nu) is the grid index and the Doppler
// width in q, beta~ = sqrt(k_B T / (M m_u)) R0 / c, is common to all lines.
//
//   1. per line: fractional grid index x (linear in ln nu between grid
//      points), ln gamma~ with gamma~ = R0 gamma / nu (floored at 1e-3 beta~),
//      strength S(T);
//   2. width grid ln gamma~_k = lng0 + k d from the lines' range;
//   3. lineshape density S_{jk}: every line split over the four neighbouring
//      (j, k) nodes with linear weights, gathered per grid cell (the lines are
//      sorted by centre, so a cell's lines are one contiguous range and the
//      sum order is fixed);
//   4. DFT of every width row (length n_fft, zero padded), the product with
//      the Voigt transform exp(-2 pi^2 beta~^2 f^2 - 2 pi gamma~_k |f|) summed
//      over k, inverse DFT;
//   5. sigma(nu_i) = sigma(q_i) R0 / nu_i.
// The DFTs are radix-4 / radix-2 Stockham passes through global memory.
#include <algorithm>
#include <utility>

#include "exo_device.h"
#include "exo_launch.h"
#include "exo_lines.h"

namespace exo {

template <typename R> struct Cplx;
template <> struct Cplx<float> { using T = float2; };
template <> struct Cplx<double> { using T = double2; };

// -------------------------------------------------------------------------- 1
__global__ __launch_bounds__(256) void k_modit_lines(LinesDev L, double T, double P, double R0,
                                                     double beta_t, double amp_scale,
                                                     const double* __restrict__ nu, int64_t ng,
                                                     int64_t l0, int64_t n_in, double* __restrict__ x,
                                                     double* __restrict__ lng, double* __restrict__ S) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n_in) return;
  const int64_t l = l0 + i;
  const LineState st = line_state(L, l, T, P);
  const double nl = L.nu_c[l];
  // j: the largest grid index <= ng - 2 with nu_j <= nl  (nu_0 <= nl <= nu_{ng-1})
  int64_t lo = 0, hi = ng - 1;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (nu[mid] <= nl) lo = mid;
    else hi = mid;
  }
  const double lj = log(nu[lo]);
  x[i] = (double)lo + (log(nl) - lj) / (log(nu[lo + 1]) - lj);
  lng[i] = log(fmax(R0 * st.gam / nl, 1e-3 * beta_t));
  S[i] = st.S * amp_scale;
}

// -------------------------------------------------------------------------- 2
__device__ inline void block_minmax256(double& mn, double& mx, double* sm) {
  for (int o = 32; o > 0; o >>= 1) {
    mn = fmin(mn, __shfl_xor(mn, o));
    mx = fmax(mx, __shfl_xor(mx, o));
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) {
    sm[w] = mn;
    sm[4 + w] = mx;
  }
  __syncthreads();
  mn = fmin(fmin(sm[0], sm[1]), fmin(sm[2], sm[3]));
  mx = fmax(fmax(sm[4], sm[5]), fmax(sm[6], sm[7]));
}

__global__ __launch_bounds__(256) void k_modit_minmax(const double* __restrict__ v, int64_t n,
                                                      double* __restrict__ part) {
  __shared__ double sm[8];
  double mn = INFINITY, mx = -INFINITY;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    mn = fmin(mn, v[i]);
    mx = fmax(mx, v[i]);
  }
  block_minmax256(mn, mx, sm);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = mn;
    part[2 * blockIdx.x + 1] = mx;
  }
}

// K = floor(range / d) + 2, at most kModitMaxBins (the step widens to range / (max - 2))
__global__ __launch_bounds__(256) void k_modit_bins(const double* __restrict__ part, int nb, double dlng,
                                                    ModitBins* __restrict__ bins) {
  __shared__ double sm[8];
  double mn = INFINITY, mx = -INFINITY;
  for (int b = threadIdx.x; b < nb; b += 256) {
    mn = fmin(mn, part[2 * b]);
    mx = fmax(mx, part[2 * b + 1]);
  }
  block_minmax256(mn, mx, sm);
  if (threadIdx.x == 0) {
    const double range = mx - mn;
    double d = dlng;
    int K = (int)floor(range / d) + 2;
    if (K > kModitMaxBins) {
      d = range / (kModitMaxBins - 2);
      K = min((int)floor(range / d) + 2, kModitMaxBins);
    }
    bins->lng0 = mn;
    bins->d = d;
    bins->K = K;
  }
}

// -------------------------------------------------------------------------- 3
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

// One thread per DFT sample j of every width row: rows[k * n_fft + j].  For
// j < ng the cell gathers the lines with nu_{j-1} <= nu_l < nu_j (weight
// x - (j - 1)) and nu_j <= nu_l < nu_{j+1} (weight 1 - (x - j)); the last
// cell's second range is the lines exactly at nu_{ng-1}.  Samples j >= ng are
// the zero padding.
template <typename R>
__global__ __launch_bounds__(256) void k_modit_lsd(const double* __restrict__ nu_c, int64_t l0,
                                                   int64_t n_in, const double* __restrict__ nu,
                                                   int64_t ng, int64_t n_fft, const double* __restrict__ x,
                                                   const double* __restrict__ lng,
                                                   const double* __restrict__ S,
                                                   const ModitBins* __restrict__ bins,
                                                   typename Cplx<R>::T* __restrict__ rows) {
  using C = typename Cplx<R>::T;
  __shared__ R acc[kModitMaxBins][256];
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int K = bins->K;
  const double lng0 = bins->lng0, dinv = 1.0 / bins->d;
  for (int k = 0; k < K; ++k) acc[k][threadIdx.x] = (R)0;
  if (j < ng) {
    const int64_t le = l0 + n_in;
    const int64_t a0 = j > 0 ? lower_index<false>(nu_c, l0, le, nu[j - 1]) : l0;
    const int64_t a1 = lower_index<false>(nu_c, a0, le, nu[j]);
    const int64_t a2 = j + 1 < ng ? lower_index<false>(nu_c, a1, le, nu[j + 1])
                                  : lower_index<true>(nu_c, a1, le, nu[ng - 1]);
    for (int64_t l = (j > 0 ? a0 : a1); l < a2; ++l) {
      const int64_t i = l - l0;
      const double w = l < a1 ? x[i] - (double)(j - 1) : 1.0 - (x[i] - (double)j);
      const double t = (lng[i] - lng0) * dinv;
      const int k0 = min((int)floor(t), K - 2);
      const double fk = t - (double)k0;
      const double sw = S[i] * w;
      acc[k0][threadIdx.x] += (R)(sw * (1.0 - fk));
      acc[k0 + 1][threadIdx.x] += (R)(sw * fk);
    }
  }
  if (j < n_fft) {
    for (int k = 0; k < K; ++k) {
      C v;
      v.x = acc[k][threadIdx.x];
      v.y = (R)0;
      rows[(int64_t)k * n_fft + j] = v;
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
// of length L become transforms of length RADIX * L.  Rows >= bins->K (when
// bins is given) are skipped.
template <typename R, int RADIX>
__global__ __launch_bounds__(256) void k_fft_pass(const typename Cplx<R>::T* __restrict__ in,
                                                  typename Cplx<R>::T* __restrict__ out, int64_t n,
                                                  int64_t L, const ModitBins* __restrict__ bins) {
  using C = typename Cplx<R>::T;
  if (bins && (int)blockIdx.y >= bins->K) return;
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

// -------------------------------------------------------------------------- 4'
// Y = conj( sum_k X_k exp(-2 pi^2 beta~^2 f^2 - 2 pi gamma~_k |f|) ), f the
// signed DFT frequency in cycles per grid step.  (The inverse DFT is then a
// forward DFT of Y, conjugated and divided by n.)
template <typename R>
__global__ __launch_bounds__(256) void k_modit_product(const typename Cplx<R>::T* __restrict__ X,
                                                       int64_t n, const ModitBins* __restrict__ bins,
                                                       double beta_t, typename Cplx<R>::T* __restrict__ Y) {
  using C = typename Cplx<R>::T;
  const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (m >= n) return;
  const double f = (double)(m <= n / 2 ? m : m - n) / (double)n;
  const double g = -2.0 * kPi * kPi * beta_t * beta_t * f * f;
  const double h = -2.0 * kPi * fabs(f);
  const int K = bins->K;
  double sx = 0.0, sy = 0.0;
  for (int k = 0; k < K; ++k) {
    const double gk = exp(bins->lng0 + bins->d * k);
    const R w = (R)exp(g + h * gk);
    const C v = X[(int64_t)k * n + m];
    sx += (double)(v.x * w);
    sy += (double)(v.y * w);
  }
  C y;
  y.x = (R)sx;
  y.y = (R)-sy;
  Y[m] = y;
}

// -------------------------------------------------------------------------- 5
template <typename R, typename TO>
__global__ __launch_bounds__(256) void k_modit_out(const typename Cplx<R>::T* __restrict__ Z,
                                                   int64_t ng, int64_t n_fft, double R0,
                                                   const double* __restrict__ nu, double scale,
                                                   TO* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= ng) return;
  out[i] = (TO)((double)Z[i].x / (double)n_fft * R0 / nu[i] * scale);
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
  const int64_t nbl = nblk(M.n_in);
  hipLaunchKernelGGL(k_modit_lines, dim3((unsigned)nbl), dim3(256), 0, st, M.L, M.T, M.P, M.R0,
                     M.beta_t, M.amp_scale, M.nu, M.ng, M.l0, M.n_in, M.x, M.lng, M.S);
  const int nb = (int)std::min<int64_t>(M.n_part, nbl);
  hipLaunchKernelGGL(k_modit_minmax, dim3((unsigned)nb), dim3(256), 0, st, M.lng, M.n_in, M.part);
  hipLaunchKernelGGL(k_modit_bins, dim3(1), dim3(256), 0, st, M.part, nb, M.dlng, M.bins);
  hipLaunchKernelGGL(k_modit_lsd<R>, dim3(nblk(M.n_fft)), dim3(256), 0, st, M.nu_c, M.l0, M.n_in, M.nu,
                     M.ng, M.n_fft, M.x, M.lng, M.S, M.bins, (C*)M.rows0);
  void* X = fft_rows<R>(M.rows0, M.rows1, M.n_fft, kModitMaxBins, M.bins, st);
  void* Y = X == M.rows0 ? M.rows1 : M.rows0;
  hipLaunchKernelGGL(k_modit_product<R>, dim3(nblk(M.n_fft)), dim3(256), 0, st, (const C*)X, M.n_fft,
                     M.bins, M.beta_t, (C*)Y);
  void* Z = fft_rows<R>(Y, X, M.n_fft, 1, nullptr, st);
  if (M.out64)
    hipLaunchKernelGGL((k_modit_out<R, double>), dim3(nblk(M.ng)), dim3(256), 0, st, (const C*)Z, M.ng,
                       M.n_fft, M.R0, M.nu, 1.0 / M.amp_scale, (double*)M.out);
  else
    hipLaunchKernelGGL((k_modit_out<R, float>), dim3(nblk(M.ng)), dim3(256), 0, st, (const C*)Z, M.ng,
                       M.n_fft, M.R0, M.nu, 1.0 / M.amp_scale, (float*)M.out);
  return hipGetLastError();
}

hipError_t launch_modit(const ModitArgs& M, bool fp64, hipStream_t st) {
  if (M.n_in == 0) {
    if (M.out64) hipLaunchKernelGGL(k_zero<double>, dim3(nblk(M.ng)), dim3(256), 0, st, (double*)M.out, M.ng);
    else hipLaunchKernelGGL(k_zero<float>, dim3(nblk(M.ng)), dim3(256), 0, st, (float*)M.out, M.ng);
    return hipGetLastError();
  }
  return fp64 ? modit_impl<double>(M, st) : modit_impl<float>(M, st);
}

}  // namespace exo
