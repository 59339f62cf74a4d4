// Line-parameter precompute and tiled Voigt sums (direct LPF, Sec. 2.1.1).
#include "exo_device.h"
#include "exo_launch.h"
#include "exo_lines.h"

#include <mutex>
#include <type_traits>
#include <vector>

namespace exo {

// Largest FP32 line amplitude (see k_line_records).
constexpr double kAmpMax = 1e25;

// Adaptive amplitude scale of a single-layer FP32 cross-section: a power of
// two (exact) that brings the call's largest line strength to [2^80, 2^81),
// far below kAmpMax (so no line is clipped) while lines 1e60 times weaker
// than the strongest still sit above FP32's subnormal range.  The exponent is
// clamped so that its inverse, the output scale, is a normal FP32 number.
constexpr int kAmpExp = 80;

__device__ inline double amp_scale_of(unsigned long long bits) {
  const double m = __longlong_as_double((long long)bits);
  if (!(m > 0.0) || !isfinite(m)) return 18446744073709551616.0;  // no strength: 2^64
  const int e = min(126, max(-126, kAmpExp - ilogb(m)));
  return ldexp(1.0, e);
}

// Largest S(T) over the lines at (T, P), raised into *amax as its FP64 bit
// pattern (non-negative doubles order like their bit patterns).  *amax is
// zero on entry; k_far_reach clears it after the records have used it.
__global__ __launch_bounds__(256) void k_amp_max(LinesDev L, double T, double P,
                                                 unsigned long long* __restrict__ amax) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double S = 0.0;
  if (l < L.n) S = line_state(L, l, T, P).S;
#pragma unroll
  for (int k = 32; k > 0; k >>= 1) S = fmax(S, __shfl_xor(S, k, 64));
  if ((threadIdx.x & 63) == 0 && S > 0.0) atomicMax(amax, (unsigned long long)__double_as_longlong(S));
}

// grid: x over lines, y over layers of the chunk.  col == nullptr: column
// factor 1 (single-layer cross-section).  T_lay == nullptr: one layer at
// (T_one, P_one), passed by value.  FP32 records also raise g2max_bits[y] to
// the layer's largest gamma^2 (one atomic per wave).  amax != nullptr: the
// amplitude scale is amp_scale_of(*amax) instead of amp_scale, and its
// inverse goes to *oscale for the Voigt sum's output.
__global__ __launch_bounds__(256) void k_line_records(LinesDev L, const double* __restrict__ T_lay,
                                                      const double* __restrict__ P_lay,
                                                      const double* __restrict__ col_lay,
                                                      double T_one, double P_one,
                                                      double amp_scale, int layer0,
                                                      const unsigned long long* __restrict__ amax,
                                                      float* __restrict__ oscale,
                                                      LineRec* __restrict__ rec,
                                                      LineRecT* __restrict__ rect,
                                                      LineRec64* __restrict__ rec64,
                                                      unsigned int* __restrict__ g2max_bits,
                                                      LineRec64T* __restrict__ rec64t,
                                                      LineRec64TT* __restrict__ rect64t) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = l < L.n;
  const int y = blockIdx.y;
  const int n = layer0 + y;
  if (amax) {
    amp_scale = amp_scale_of(*amax);
    if (oscale && l == 0 && y == 0) *oscale = (float)(1.0 / amp_scale);
  }
  const double T = T_lay ? T_lay[n] : T_one, P = T_lay ? P_lay[n] : P_one;
  const double col = col_lay ? col_lay[n] : 1.0;
  const int64_t o = (int64_t)y * L.n + l;
  if (rec64t) {
    if (!in) return;
    const LineState s = line_state(L, l, T, P);
    make_line_record64t(s.S * col * amp_scale, s.beta, s.gam, s.dlnS, s.dbeta, s.dgam, rec64t + o,
                        rect64t ? rect64t + o : nullptr);
    return;
  }
  if (rec64) {
    if (!in) return;
    const LineState s = line_state(L, l, T, P);
    LineRec64 r;
    r.A = s.S * col * amp_scale;
    r.beta = s.beta;
    r.gam = s.gam;
    r.erfcxa = erfcx(s.gam / (kSqrt2 * s.beta));
    rec64[o] = r;
    return;
  }
  float g2 = 0.f;
  if (in) {
    const LineState s = line_state(L, l, T, P);
    double A = s.S * col * amp_scale;
    double dlnA = s.dlnS;
    // FP32 range guard: an amplitude above kAmpMax makes every grid point of
    // the window optically thick (dtau >> 700, T = 0) whether or not it is
    // clipped, so clipping it changes no flux; it keeps FP32 sums finite.
    if (A > kAmpMax) {
      A = kAmpMax;
      dlnA = 0.0;
    }
    make_line_record(A, s.beta, s.gam, T, dlnA, s.dbeta, s.dgam, rec + o, rect ? rect + o : nullptr);
    g2 = (float)(s.gam * s.gam);
  }
  if (g2max_bits) {
    // every lane of the wave takes part (none has returned on this path)
#pragma unroll
    for (int k = 32; k > 0; k >>= 1) g2 = fmaxf(g2, __shfl_xor(g2, k, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(g2max_bits + y, __float_as_uint(g2));
  }
}

// ---------------------------------------------------------------------------
// FP32 Voigt sum with compensated accumulation.
//
// Block = 256 threads = 4 waves; thread (wave w, lane) owns grid points
// j = tile0 + (w*G + g)*64 + lane, g < G.  All lanes walk the same line
// sequence, so line records are wave-uniform (LDS broadcasts).  A near pair's offset nu_j - nu_l is
// one FP64 subtraction, rounded once to FP32: an FP32 offset would carry an
// absolute error of ulp(nu) ~ 5e-4 cm^-1, a few percent of a Doppler width.
// Contributions of a block of lines (64 far, kChunk near) are summed in plain
// FP32, and every block sum enters a Neumaier-compensated accumulator.
// ---------------------------------------------------------------------------
constexpr int kChunk = 32;

// ---------------------------------------------------------------------------
// Far tier.  In the asymptotic branch the contribution is E0 r sum_k c_k r^k
// (make_line_record) with r = 1/D, D = dnu^2 + gamma^2.  With u = beta^2 r
// and v = gamma^2 r, c_k r^k is a homogeneous polynomial of degree k in
// (u, v): 1, 3u, 15u^2 - 4uv, 105u^3 - 60u^2 v, 48u^2 v^2 - 840u^3 v,
// 1680u^3 v^2, -960u^3 v^3.  A far pair keeps k <= 2 of the value and k <= 3
// of the tangent (k <= 1 of both beyond the outer reach), and skips the core
// test.
//
// A line farther than `reach` from every grid point of a wave has, at each
// of them, D >= reach^2 + gamma^2, so every monomial obeys
//   u^p v^q <= U^p max_{g <= g_max} (g/R)^q / (1 + g/R)^(p+q),   R = reach^2,
// U = beta_max^2 / R, g_max = the layer's largest gamma^2; the maximum sits
// at g/R = min(g_max/R, q/p).  Summing these bounds over the dropped terms
// bounds the dropped value relative to E0 r, and the dropped tangent relative
// to E0 r (|d ln E0| + |d ln beta^2| + |d ln gamma^2|) (k-th derivative
// terms are at most k times the term, and d/dT of r adds a factor (k+1) v).
// k_far_reach picks, per layer, the smallest R (a search in ln R) at which
// the two bounds stay below kFarEpsV and kFarEpsT: the largest values the
// same bounds take for U = 2e-5 at any g_max, so no layer is treated more
// loosely than with that fixed U, and R never exceeds beta_max^2 / 2e-5.
// Layers with narrow lines (low pressure) get a reach several times smaller.
// R >= 2 * 111 beta_max^2 keeps every far pair out of the core branch.
// In tangent mode it also tries a tangent cut after r^3 (one FMA less per
// far pair; its dropped terms add 3 A_3 and 3 A_2 v to the tangent bound)
// and takes it where the reach that bound needs is at most twice R: a few
// more near pairs against fewer FMAs on every far pair.  Where the Lorentz
// widths are small (v ~ 0) the two reaches nearly coincide.
//
// Farther out the c_2 term itself falls below the same targets: beyond a
// second, per-layer distance (the outer reach, searched the same way over
// R .. 1e4 R with c_2 and t_2 added to the dropped terms) the value and the
// tangent both stop at r^2, two FMAs less per pair.  The bound per pair is
// the same in every tier, so the error of the sum does not grow.  With a
// band a few tens of cm^-1 wide and Doppler widths ~0.01 cm^-1 most pairs
// are outer ones; layers whose Lorentz widths are wide (high pressure) may
// have none (outer reach FLT_MAX).
//
// The Doppler width is proportional to the line centre (Eq. thermal) and the
// lines are sorted by centre, so the last line of a layer has the largest
// beta^2.  The far (and, within them, the outer) lines of a wave are a
// prefix and a suffix of the sorted list, found by binary search.
// ---------------------------------------------------------------------------
constexpr double kFarU = 2e-5;
constexpr double kFarEpsV = 4.8e-9;
constexpr double kFarEpsT = 1.42e-8;
constexpr double kFarOuterSpan = 9.210340371976184;  // ln 1e4: outer reach <= 1e4 R

// bound of u^p v^q over the far pairs of a layer (gr = g_max / R)
__device__ inline double far_monomial(int p, int q, double U, double gr) {
  double m = 1.0;
  for (int i = 0; i < p; ++i) m *= U;
  if (q == 0) return m;
  const double t = fmin(gr, (double)q / (double)p);
  double den = 1.0;
  for (int i = 0; i < q; ++i) m *= t;
  for (int i = 0; i < p + q; ++i) den *= 1.0 + t;
  return m / den;
}

// Bound of the wing terms a tier drops: the value keeps c_0 .. c_(kv-1), the
// tangent t_0 .. t_(kt-1) (kt = 8: no tangent).  A_k bounds |c_k r^k| (in
// units of E0 r) by the monomials u^p v^q (u = beta^2 r, v = gamma^2 r) of
// c_k; Av_k is the same with one more factor v.  Dropping t_k costs at most
// k (A_k + Av_(k-1)): the T-derivative of the c_k term (degree k in u, v) and
// the gamma^2-derivative of r in the c_(k-1) term.
__device__ inline bool far_bound_holds(double U, double gr, int kv, int kt) {
  auto M = [&](int p, int q) { return far_monomial(p, q, U, gr); };
  const double A[8] = {0.0,
                       3.0 * M(1, 0),
                       15.0 * M(2, 0) + 4.0 * M(1, 1),
                       105.0 * M(3, 0) + 60.0 * M(2, 1),
                       48.0 * M(2, 2) + 840.0 * M(3, 1),
                       1680.0 * M(3, 2),
                       960.0 * M(3, 3),
                       0.0};
  const double Av[7] = {0.0,  // t_0 is always kept
                        3.0 * M(1, 1),
                        15.0 * M(2, 1) + 4.0 * M(1, 2),
                        105.0 * M(3, 1) + 60.0 * M(2, 2),
                        48.0 * M(2, 3) + 840.0 * M(3, 2),
                        1680.0 * M(3, 3),
                        960.0 * M(3, 4)};
  double ev = 0.0, et = 0.0;
  for (int k = kv; k < 7; ++k) ev += A[k];
  for (int k = kt; k < 8; ++k) et += (double)k * (A[k] + Av[k - 1]);
  return ev <= kFarEpsV && et <= kFarEpsT;
}

// Two-level search on ln R in [lo, hi] by the 64 lanes of a wave: the
// smallest candidate (to (hi - lo)/4096) at which the bound holds; fails if
// it does not hold at hi.
__device__ inline bool far_search(double bmax, double gmax, double lo, double hi, int kv, int kt, int k,
                                  double* x) {
  double a = lo, b = hi;
  bool found = false;
  for (int level = 0; level < 2; ++level) {
    const double xk = a + (b - a) * (double)(k + 1) * (1.0 / 64.0);
    const double R = exp(xk);
    const unsigned long long ok = __ballot(far_bound_holds(bmax / R, gmax / R, kv, kt));
    if (ok == 0ull) break;
    const int k1 = __builtin_ctzll(ok);
    const double bn = a + (b - a) * (double)(k1 + 1) * (1.0 / 64.0);
    a = k1 == 0 ? a : a + (b - a) * (double)k1 * (1.0 / 64.0);
    b = bn;
    found = true;
  }
  *x = b;
  return found;
}

// One 64-lane block per layer of the chunk.  reach2[y]: squared distance
// beyond which a line is summed with the value polynomial cut after r^3;
// t3[y] (tangent mode): 1 if those pairs keep the tangent's r^4 term;
// outer2[y] (>= reach2[y]; FLT_MAX if none): squared distance beyond which
// the value and the tangent both stop at r^2 (the value alone in forward
// mode).
__global__ __launch_bounds__(64) void k_far_reach(const LineRec* __restrict__ rec, int64_t n_lines,
                                                  int tangent, unsigned int* __restrict__ g2max_bits,
                                                  float* __restrict__ reach2, int* __restrict__ t3,
                                                  float* __restrict__ outer2,
                                                  unsigned long long* __restrict__ amax) {
  const int y = blockIdx.x, k = threadIdx.x;
  // the records are written: clear the strength maximum for the next call
  if (amax && y == 0 && k == 0) *amax = 0ull;
  // beta_max^2 from the threshold 2 * 111 beta^2, with margin for its rounding
  const double bmax = (double)rec[(int64_t)y * n_lines + n_lines - 1].thr * (1.001 / (2.0 * kHjertSwitch));
  const unsigned int bits = g2max_bits[y];
  __syncthreads();  // every lane has read the maximum before lane 0 clears it
  const double lo = log(2.0 * kHjertSwitch * bmax), hi = log(bmax / kFarU);
  double x = hi;
  int keep3 = 1;
  float ro = __FLT_MAX__;
  // an unknown maximum (not a finite non-negative float) keeps the fixed-U
  // reach and no outer zone
  if (bits <= 0x7f7fffffu && lo < hi) {
    const double gmax = (double)__uint_as_float(bits) * 1.001;
    double x3, x2, xo;
    if (far_search(bmax, gmax, lo, hi, 3, 4, k, &x3)) x = x3;
    if (tangent && far_search(bmax, gmax, lo, hi, 3, 3, k, &x2) && x2 <= x + 0.6931471805599453) {
      x = x2;
      keep3 = 0;
    }
    if (far_search(bmax, gmax, x, x + kFarOuterSpan, 2, tangent ? 2 : 8, k, &xo))
      ro = (float)(exp(xo) * (1.0 + 1e-6));
  }
  if (k == 0) {
    g2max_bits[y] = 0u;
    // rounded up so that the FP32 value does not undercut the bound
    const float r = (float)(exp(x) * (1.0 + 1e-6));
    reach2[y] = r;
    t3[y] = keep3;
    outer2[y] = fmaxf(ro, r);
  }
}

// first index i in [lo, hi) with a[i] >= v (strict: a[i] > v); hi if none
template <bool STRICT>
__device__ inline int search_sorted(const double* __restrict__ a, int lo, int hi, double v) {
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const bool left = STRICT ? a[mid] <= v : a[mid] < v;
    if (left) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__device__ inline void neumaier(float& s, float& c, float v) {
  const float t = s + v;
  if (fabsf(s) >= fabsf(v)) c += (s - t) + v;
  else c += (v - t) + s;
  s = t;
}

// ---------------------------------------------------------------------------
// Rational approximation of w for the core branch (Weideman 1994):
//   w(z) ~ u/sqrt(pi) + 2 u^2 sum_{n=1..N} c_n Z^(n-1), with
// u = 1/(L - iz), Z = (L + iz)/(L - iz), L = (N/sqrt2)^(1/2), and
// c_n = (1/2M) sum_{|k|<M} f(t_k) cos(n theta_k), theta_k = k pi/M,
// t_k = L tan(theta_k/2), f(t) = e^{-t^2} (L^2 + t^2), M = 2N.  About 2N + 20
// FP64 operations, a fraction of the paper's Algorithm-916 series (no
// exponentials, no sine), with H and L = Im w from the same evaluation.  Its absolute error is a
// small fraction of |w| that falls exponentially with N; near the real axis
// far from the centre (small a) |w| is much larger than H, so the N a pair
// needs grows as a falls (core_w below).  The coefficients of every N used
// live back to back in one table.
// ---------------------------------------------------------------------------
constexpr int kWeidNs[4] = {20, 24, 28, 32};
constexpr int kWeidOff[4] = {0, 20, 44, 72};
constexpr int kWeidTab = 104;
__device__ double g_weid[kWeidTab];  // c_1 .. c_N of each N, filled once per device

__global__ __launch_bounds__(64) void k_weid_init() {
  const int n = threadIdx.x + 1;
  for (int t = 0; t < 4; ++t) {
    const int N = kWeidNs[t];
    if (n > N) continue;
    const int M = 2 * N;
    const double L = sqrt((double)N / kSqrt2);
    double s = 0.0;
    for (int k = -M + 1; k <= M - 1; ++k) {
      const double th = k * (kPi / M);
      const double tt = L * tan(0.5 * th);
      s += exp(-tt * tt) * (L * L + tt * tt) * cos(n * th);
    }
    g_weid[kWeidOff[t] + n - 1] = s / (2.0 * M);
  }
}

// Re w and Im w at z = x + ia (a >= 0) in FP64 from the N coefficients c.
template <int N>
__device__ inline void weideman_w(double x, double a, const double __attribute__((address_space(4)))* c,
                                  double* re, double* im) {
  const double L = sqrt((double)N / kSqrt2);
  // u = 1/(L - iz) = 1/((L + a) - ix) = ((L + a) + ix)/den
  const double p = L + a;
  const double den = fma(p, p, x * x);
  double inv = __builtin_amdgcn_rcp(den);
  inv = fma(inv, fma(-den, inv, 1.0), inv);
  inv = fma(inv, fma(-den, inv, 1.0), inv);
  const double ur = p * inv, ui = x * inv;
  // Z = (L + iz) u = ((L - a) + ix) u
  const double q = L - a;
  const double zr = fma(q, ur, -x * ui), zi = fma(q, ui, x * ur);
  // s = sum_{n<N} c_n Z^n with real c_n, by dividing the polynomial by the
  // real quadratic t^2 - 2 Re(Z) t + |Z|^2, which vanishes at Z: the
  // remainder alpha t + beta gives s = alpha Z + beta (Goertzel's method;
  // Knuth, TAOCP vol. 2, 4.6.4).  Two real FMAs per coefficient instead of
  // the four of complex Horner steps.  |Z| <= 1 for a >= 0, so the
  // recurrence does not amplify rounding.
  const double r = 2.0 * zr, m = -fma(zr, zr, zi * zi);
  double e2 = 0.0, e1 = c[N - 1];
#pragma unroll 8
  for (int k = N - 3; k >= 1; --k) {
    const double e = fma(r, e1, fma(m, e2, c[k + 1]));
    e2 = e1;
    e1 = e;
  }
  const double al = fma(r, e1, fma(m, e2, c[1]));
  const double sr = fma(al, zr, fma(m, e1, c[0])), si = al * zi;
  // w = u (1/sqrt(pi) + 2 u s)
  const double vr = 0.56418958354775628 + 2.0 * fma(ur, sr, -ui * si);
  const double vi = 2.0 * fma(ur, si, ui * sr);
  *re = fma(ur, vr, -ui * vi);
  *im = fma(ur, vi, ui * vr);
}

template <int T>
__device__ inline const double __attribute__((address_space(4)))* weid_coeffs() {
  return (const double __attribute__((address_space(4)))*)((const double*)g_weid + kWeidOff[T]);
}

// H = Re w and L = Im w at z = x + ia in the core branch, with the shortest
// rational approximation that keeps H within 2.3e-7 relative over
// x^2 + a^2 < 111 for the pair's a (measured against wofz on a dense grid:
// N = 32 for 1e-5 <= a < 1e-3, 28 up to 3e-2, 24 up to 1, 20 beyond, where
// the relative error of H falls about as 1/a).  For a < kWeidAmin, w to first
// order in a about the real axis, where w(x) = e^{-x^2} + i Im w(x) and
// w'(z) = -2z w(z) + 2i/sqrt(pi):
//   H = e^{-x^2} + 2a (x Im w(x) - 1/sqrt(pi)),  L = Im w(x) - 2ax e^{-x^2},
// with Im w(x) from the rational approximation (N = 28: accurate there
// relative to |w| ~ Im w) and e^{-x^2} exact.  The neglected terms are
// O(a^2 x^2) relative (2e-9 at a = 1e-5 over the core); the rational form's
// own error in H never enters, since H is mostly e^{-x^2} or the small
// difference x Im w - 1/sqrt(pi), both formed from accurate parts.  a is
// uniform per line, so the branches do not diverge.
__device__ inline void core_w(double x, double a, double* H, double* L) {
  if (a >= kWeidAmin) {
    if (a < 1e-3) weideman_w<32>(x, a, weid_coeffs<3>(), H, L);
    else if (a < 3e-2) weideman_w<28>(x, a, weid_coeffs<2>(), H, L);
    else if (a < 1.0) weideman_w<24>(x, a, weid_coeffs<1>(), H, L);
    else weideman_w<20>(x, a, weid_coeffs<0>(), H, L);
    return;
  }
  double re, im;
  weideman_w<28>(x, 0.0, weid_coeffs<2>(), &re, &im);
  const double ex2 = exp_core(-x * x);
  *H = ex2 + 2.0 * a * fma(x, im, -0.56418958354775628);
  *L = im - 2.0 * a * x * ex2;
}

// Core evaluations are out-of-line calls: their FP64 temporaries would
// otherwise set the register budget of the line loops and cut occupancy.
__device__ __attribute__((noinline)) float core_value(float x, float a) {
  double H, L;
  core_w((double)x, (double)a, &H, &L);
  return (float)H;
}

__device__ __attribute__((noinline)) float2 core_value_tan(float x, float a) {
  double H, L;
  core_w((double)x, (double)a, &H, &L);
  return make_float2((float)H, (float)L);
}

// Grid points of thread (wave w, lane): j = tile0 + (w*G + g)*64 + lane.
// Points past the end repeat the last one (their sums are not stored).
template <int G>
__device__ __forceinline__ void load_points(const VoigtArgs& A, int64_t tile0, int w, int lane,
                                            double (&nuj)[G]) {
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int64_t j = tile0 + (int64_t)(w * G + g) * 64 + lane;
    nuj[g] = A.nu[j < A.ng ? j : A.ng - 1];
  }
}

// Line ranges of wave w within [lb, le): near [i0, i1), far [o0, i0) and
// [i1, o1), outer [lb, o0) and [o1, le).
template <int G>
__device__ __forceinline__ void tier_ranges(const VoigtArgs& A, int64_t tile0, int w, int lb, int le, int& o0,
                                            int& i0, int& i1, int& o1) {
  const int64_t jw = tile0 + (int64_t)w * G * 64, jlast = A.ng - 1;
  const double lo = A.nu[jw < jlast ? jw : jlast];
  const double hi = A.nu[jw + G * 64 - 1 < jlast ? jw + G * 64 - 1 : jlast];
  const double reach = sqrt((double)A.far_reach2[blockIdx.y]);
  const double outer = sqrt((double)A.far_outer2[blockIdx.y]);  // >= reach
  o0 = __builtin_amdgcn_readfirstlane(search_sorted<false>(A.nu_c, lb, le, lo - outer));
  i0 = __builtin_amdgcn_readfirstlane(search_sorted<false>(A.nu_c, o0, le, lo - reach));
  i1 = __builtin_amdgcn_readfirstlane(search_sorted<true>(A.nu_c, i0, le, hi + reach));
  o1 = __builtin_amdgcn_readfirstlane(search_sorted<true>(A.nu_c, i1, le, hi + outer));
}

// Far lines [sb, se): truncated wing polynomial, no core branch.
// Offsets in FP32 from the wave's first point nu_w: d = (nu_j - nu_w) -
// (nu_l - nu_w), each difference formed in FP64 and rounded once (the line's
// once per wave, the points' once per chunk); for a far line (|d| >= the near
// reach) this errs by ~1e-7 relative, like rounding the FP64 offset.  One
// reciprocal serves two points: r0 = D1 / (D0 D1), r1 = D0 / (D0 D1) (D >= the
// squared reach, so the product stays a normal FP32 number for any physical
// width).  KT: terms the tangent keeps (4: up to r^4; 3: up to r^3 where the
// layer's bound allows; 2: up to r^2, outer lines, where the value also stops
// at r^2).  The forward sum ignores KT except for KT = 2.
//
// Each chunk of 64 far lines passes through a slice of LDS private to the
// wave: lane i loads line i's value and tangent coefficients and gamma^2 with
// vector loads and forms its offset nu_l - nu_w (one FP64 subtraction for the
// 64 lines); the line loop reads them back as wave-uniform LDS broadcasts
// into vector registers, and sums the chunk in plain FP32 before it enters
// the compensated accumulator.  Per-line scalar
// loads of the same records were slower (their latency stalled the loop), and
// coefficients in vector registers need no copies to get round the one-scalar
// operand limit of a VALU instruction.  The stage needs no workgroup barrier:
// LDS operations of one wave complete in order.
constexpr int kFarChunk = 64;
struct FarStage {
  float4 eg[kFarChunk];  // e0, e1, e2, gamma^2
  float4 t[kFarChunk];   // tangent t0..t3
  float dl[kFarChunk];   // (float)(nu_l - nu_w)
};
// The near tier stages its lines the same way (full polynomials, the core
// threshold and the FP64 centre; lanes 0..31 the value side, 32..63 the
// tangent side of 32 lines), and walks them one line per iteration (two
// lines in flight spilled inside the loop at 64 registers per lane).
struct NearStage {
  float4 e03[kChunk];  // e0..e3
  float4 e4g[kChunk];  // e4, e5, e6, gamma^2
  float4 t03[kChunk];  // tangent t0..t3
  float4 t47[kChunk];  // tangent t4..t7
  double nu[kChunk];   // line centre
  float thr[kChunk];   // core threshold
};
union LineStage {
  FarStage far;
  NearStage near;
};

// Orders one wave's LDS writes before its later reads of another lane's
// data, and its reads before later overwrites.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool TAN, int KT, int G>
__device__ __forceinline__ void far_lines(int sb, int se, const LineRec* __restrict__ R,
                                          const LineRecT* __restrict__ RT,
                                          const double* __restrict__ nuc, const double (&nuj)[G], double nuw,
                                          FarStage* __restrict__ st, int lane,
                                          float (&s)[G], float (&c)[G], float (&ts)[G],
                                          float (&tc)[G]) {
  static_assert(G % 2 == 0, "points go in pairs");
  float dj[G];
#pragma unroll
  for (int g = 0; g < G; ++g) dj[g] = (float)(nuj[g] - nuw);
  for (int l0 = sb; l0 < se; l0 += kFarChunk) {
    const int l1 = min(l0 + kFarChunk, se);
    // stage the chunk: lane i holds line l0 + i
    const int li = l0 + lane;
    if (li < l1) {
      const float4 e = *reinterpret_cast<const float4*>(R[li].e);
      st->eg[lane] = make_float4(e.x, e.y, e.z, R[li].gam2);
      st->dl[lane] = (float)(nuc[li] - nuw);
      if (TAN) st->t[lane] = *reinterpret_cast<const float4*>(RT[li].t);
    }
    wave_lds_sync();
    float blk[G], tblk[G];
#pragma unroll
    for (int g = 0; g < G; ++g) blk[g] = tblk[g] = 0.f;
    const int n = l1 - l0;
#pragma unroll 2
    for (int i = 0; i < n; ++i) {
      const float4 e = st->eg[i];
      const float dl = st->dl[i];
      float4 t;
      if (TAN) t = st->t[i];
      float D[G], r[G];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const float d = dj[g] - dl;
        D[g] = fmaf(d, d, e.w);
      }
#pragma unroll
      for (int g = 0; g < G; g += 2) {
        const float inv = __builtin_amdgcn_rcpf(D[g] * D[g + 1]);
        r[g] = D[g + 1] * inv;
        r[g + 1] = D[g] * inv;
      }
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const float h = KT == 2 ? fmaf(e.y, r[g], e.x) : fmaf(fmaf(e.z, r[g], e.y), r[g], e.x);
        blk[g] = fmaf(h, r[g], blk[g]);
        if (TAN) {
          const float ht = KT == 4   ? fmaf(fmaf(fmaf(t.w, r[g], t.z), r[g], t.y), r[g], t.x)
                           : KT == 3 ? fmaf(fmaf(t.z, r[g], t.y), r[g], t.x)
                                     : fmaf(t.y, r[g], t.x);
          tblk[g] = fmaf(ht, r[g], tblk[g]);
        }
      }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      neumaier(s[g], c[g], blk[g]);
      if (TAN) neumaier(ts[g], tc[g], tblk[g]);
    }
    // the next chunk overwrites the stage only after these reads
    wave_lds_sync();
  }
}

// Near lines [sb, se): full wing polynomial, core_w in the core.
// The line loop evaluates the wing and only marks the pairs inside the core
// (x^2 + a^2 < 111), one bit per line of the chunk per point; the marked
// pairs are evaluated after the loop, line by line in chunk order, with less
// state live across the out-of-line core call than inside the loop.
template <bool TAN, int G>
__device__ __forceinline__ void near_lines(int sb, int se, const LineRec* __restrict__ R,
                                           const LineRecT* __restrict__ RT,
                                           const double* __restrict__ nuc, const double (&nuj)[G],
                                           NearStage* __restrict__ st, int lane,
                                           float (&s)[G], float (&c)[G], float (&ts)[G],
                                           float (&tc)[G]) {
  static_assert(kChunk == 32, "one mask bit per line of the chunk");
  const int half = lane & 31;
  for (int l0 = sb; l0 < se; l0 += kChunk) {
    const int l1 = min(l0 + kChunk, se);
    const int li = l0 + half;
    if (li < l1) {
      if (lane < 32) {
        st->e03[half] = *reinterpret_cast<const float4*>(R[li].e);
        st->e4g[half] = *reinterpret_cast<const float4*>(R[li].e + 4);
        st->thr[half] = R[li].thr;
        st->nu[half] = nuc[li];
      } else if (TAN) {
        st->t03[half] = *reinterpret_cast<const float4*>(RT[li].t);
        st->t47[half] = *reinterpret_cast<const float4*>(RT[li].t + 4);
      }
    }
    wave_lds_sync();
    float blk[G], tblk[G];
    uint32_t cm[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      blk[g] = tblk[g] = 0.f;
      cm[g] = 0u;
    }
    const int n = l1 - l0;
#pragma unroll 1
    for (int i = 0; i < n; ++i) {
      const float4 e03 = st->e03[i], e4g = st->e4g[i];
      const float thr = st->thr[i];
      const double nul = st->nu[i];
      float4 t03, t47;
      if (TAN) {
        t03 = st->t03[i];
        t47 = st->t47[i];
      }
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const float dd = (float)(nuj[g] - nul);  // FP64 offset, rounded once
        const float D = fmaf(dd, dd, e4g.w);
        // core pairs (marked here, evaluated after the loop) take r = 0, so
        // the wing terms add exactly nothing for them (and never overflow)
        const bool in_core = D < thr;
        cm[g] |= (uint32_t)in_core << i;
        const float r = in_core ? 0.f : __builtin_amdgcn_rcpf(D);
        float h = fmaf(e4g.z, r, e4g.y);
        h = fmaf(h, r, e4g.x);
        h = fmaf(h, r, e03.w);
        h = fmaf(h, r, e03.z);
        h = fmaf(h, r, e03.y);
        h = fmaf(h, r, e03.x);
        blk[g] = fmaf(h, r, blk[g]);
        if (TAN) {
          float ht = fmaf(t47.w, r, t47.z);
          ht = fmaf(ht, r, t47.y);
          ht = fmaf(ht, r, t47.x);
          ht = fmaf(ht, r, t03.w);
          ht = fmaf(ht, r, t03.z);
          ht = fmaf(ht, r, t03.y);
          ht = fmaf(ht, r, t03.x);
          tblk[g] = fmaf(ht, r, tblk[g]);
        }
      }
    }
    wave_lds_sync();
    // lines of the chunk with a core pair at any point of the wave
    uint32_t u = 0u;
#pragma unroll
    for (int g = 0; g < G; ++g) u |= cm[g];
    for (int o = 32; o > 0; o >>= 1) u |= (uint32_t)__shfl_xor((int)u, o);
    u = __builtin_amdgcn_readfirstlane(u);
    while (u) {
      const int i = __builtin_ctz(u);
      u &= u - 1u;
      const int l = l0 + i;
      const LineRec q = R[l];
      const double nul = nuc[l];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        if ((cm[g] >> i) & 1u) {
          const float x = (float)(nuj[g] - nul) * q.winv;
          if (TAN) {
            const LineRecT qt = RT[l];
            const float2 HL = core_value_tan(x, q.a);
            const float H = HL.x, L = HL.y;
            // custom derivatives of Sec. 2.1.1:
            //   dH/dx = 2aL - 2xH,  dH/da = 2xL + 2aH - 2/sqrt(pi)
            const float Hx = 2.0f * (q.a * L - x * H);
            const float Ha = 2.0f * (x * L + q.a * H) - 1.1283791670955126f;
            blk[g] += q.acore * H;
            tblk[g] += q.acore * (qt.kA * H + Hx * x * qt.kw + Ha * qt.da);
          } else {
            blk[g] += q.acore * core_value(x, q.a);
          }
        }
      }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      neumaier(s[g], c[g], blk[g]);
      if (TAN) neumaier(ts[g], tc[g], tblk[g]);
    }
  }
}

// One (tile, layer, split): far prefix, near lines, far suffix, each summed
// in blocks of kChunk lines into the compensated accumulator.
template <bool TAN, int G>
__device__ __forceinline__ void voigt_body(const VoigtArgs& A) {
  const int y = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  __shared__ LineStage stage[4];
  const int64_t tile0 = (int64_t)blockIdx.x * (256 * G);
  double nuj[G];
  load_points<G>(A, tile0, w, lane, nuj);
  // line range of this split (n_lines < 2^31 is checked on the host)
  const int lb = (int)blockIdx.z * (int)A.lines_per_split;
  const int le = min(lb + (int)A.lines_per_split, (int)A.n_lines);
  const LineRec* __restrict__ R = A.rec + (int64_t)y * A.n_lines;
  const LineRecT* __restrict__ RT = TAN ? A.rect + (int64_t)y * A.n_lines : nullptr;
  int o0, i0, i1, o1;
  tier_ranges<G>(A, tile0, w, lb, le, o0, i0, i1, o1);
  // base of the far tier's FP32 offsets: the wave's first point (uniform)
  const int64_t jw = tile0 + (int64_t)w * G * 64;
  const double nuw = A.nu[jw < A.ng ? jw : A.ng - 1];

  float s[G], c[G], ts[G], tc[G];
#pragma unroll
  for (int g = 0; g < G; ++g) s[g] = c[g] = ts[g] = tc[g] = 0.f;
#pragma unroll 1
  for (int seg = 0; seg < 2; ++seg) {
    // outer lines [lb, o0) and [o1, le); far lines [o0, i0) and [i1, o1)
    const int ob = seg == 0 ? lb : o1, oe = seg == 0 ? o0 : le;
    const int sb = seg == 0 ? o0 : i1, se = seg == 0 ? i0 : o1;
    far_lines<TAN, 2, G>(ob, oe, R, RT, A.nu_c, nuj, nuw, &stage[w].far, lane, s, c, ts, tc);
    if (!TAN || A.far_t3[y]) far_lines<TAN, 4, G>(sb, se, R, RT, A.nu_c, nuj, nuw, &stage[w].far, lane, s, c, ts, tc);
    else far_lines<TAN, 3, G>(sb, se, R, RT, A.nu_c, nuj, nuw, &stage[w].far, lane, s, c, ts, tc);
    if (seg == 0) near_lines<TAN, G>(i0, i1, R, RT, A.nu_c, nuj, &stage[w].near, lane, s, c, ts, tc);
  }
  if (A.near_pairs && lane == 0) {
    const int64_t npts = min((int64_t)G * 64, A.ng - (tile0 + (int64_t)w * G * 64));
    if (npts > 0) {
      atomicAdd(A.near_pairs, (unsigned long long)(i1 - i0) * (unsigned long long)npts);
      if (TAN && !A.far_t3[y])
        atomicAdd(A.near_pairs + 1, (unsigned long long)((o1 - o0) - (i1 - i0)) * (unsigned long long)npts);
      atomicAdd(A.near_pairs + 2, (unsigned long long)((le - lb) - (o1 - o0)) * (unsigned long long)npts);
    }
  }

#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int64_t j = tile0 + (int64_t)(w * G + g) * 64 + lane;
    if (j >= A.ng) continue;
    if (A.ksplit == 1) {
      const int64_t o = (int64_t)y * A.ld_out + j;
      const float os = A.out_scale_dev ? *A.out_scale_dev : A.out_scale;
      A.out[o] = (s[g] + c[g]) * os;
      if (TAN) A.out_t[o] = (ts[g] + tc[g]) * os;
    } else {
      const int64_t p = ((int64_t)blockIdx.z * A.nlay + y) * A.ng + j;
      A.part[p] = make_float2(s[g], c[g]);
      if (TAN) A.part_t[p] = make_float2(ts[g], tc[g]);
    }
  }
}

// The kernels.  The tangent kernel asks for 5 waves per SIMD (96 registers
// per lane), where nothing spills around the out-of-line core call; the
// forward kernel for 6 (80 registers).  With the records staged through LDS
// and the core's polynomial evaluated by Goertzel's method, the tangent
// kernel measured 4.5 % faster at 5 waves than at 8 (64 registers, spills
// around the call), 1.7 % faster than at 4 and 1 % faster than at 6; the
// forward kernel 1.5 % faster at 6 than at 8.
template <bool TAN, int G>
__global__ void k_voigt_f32(VoigtArgs A);
template <>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 6))) void k_voigt_f32<false, kVoigtG>(
    VoigtArgs A) {
  voigt_body<false, kVoigtG>(A);
}
template <>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 5))) void k_voigt_f32<true, kVoigtG>(
    VoigtArgs A) {
  voigt_body<true, kVoigtG>(A);
}

// Fixed-order combine of split-K partials.
template <bool TAN>
__global__ __launch_bounds__(256) void k_voigt_combine(VoigtArgs A) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int y = blockIdx.y;
  if (j >= A.ng) return;
  float s = 0.f, c = 0.f, ts = 0.f, tc = 0.f;
  for (int z = 0; z < A.ksplit; ++z) {
    const int64_t p = ((int64_t)z * A.nlay + y) * A.ng + j;
    const float2 v = A.part[p];
    neumaier(s, c, v.x);
    c += v.y;
    if (TAN) {
      const float2 t = A.part_t[p];
      neumaier(ts, tc, t.x);
      tc += t.y;
    }
  }
  const int64_t o = (int64_t)y * A.ld_out + j;
  const float os = A.out_scale_dev ? *A.out_scale_dev : A.out_scale;
  A.out[o] = (s + c) * os;
  if (TAN) A.out_t[o] = (ts + tc) * os;
}

// ---------------------------------------------------------------------------
// The tiled FP64 form: the FP32 sum's thread mapping, per-wave record
// staging and core branch (core_w) in double precision, with the full
// asymptotic polynomial on every wing pair (no far/outer truncation) and
// plain FP64 accumulation.  Next to the FP32 sum it isolates the cost of
// precision; next to the plain FP64 form, the cost of the paper's per-pair
// evaluation.  Lines farther than the core reach sqrt(222) beta_max from
// every point of a wave cannot have a core pair there: a prefix and a
// suffix of the sorted list, summed without the core test.  Forward only.
// ---------------------------------------------------------------------------
constexpr int kChunk64 = 32;
struct Stage64 {
  double e[7][kChunk64];  // wing coefficients, one row per power of r
  double gam2[kChunk64];
  double nu[kChunk64];
  double thr[kChunk64];
  double winv[kChunk64];
  double a[kChunk64];
  double acore[kChunk64];
};
struct Stage64T : Stage64 {   // tangent mode
  double t[8][kChunk64];
  double kA[kChunk64], kw[kChunk64], da[kChunk64];
};

// 1/D in FP64: the hardware reciprocal and two Newton steps (each doubles
// the number of correct bits of the ~23-bit estimate).
__device__ __forceinline__ double rcp64(double D) {
  double inv = __builtin_amdgcn_rcp(D);
  inv = fma(inv, fma(-D, inv, 1.0), inv);
  return fma(inv, fma(-D, inv, 1.0), inv);
}

template <bool NEAR, bool TAN, int G, class ST>
__device__ __forceinline__ void lines64(int sb, int se, const LineRec64T* __restrict__ R,
                                        const LineRec64TT* __restrict__ RT,
                                        const double* __restrict__ nuc, const double (&nuj)[G],
                                        ST* __restrict__ st, int lane, double (&acc)[G], double (&tacc)[G]) {
  for (int l0 = sb; l0 < se; l0 += kChunk64) {
    const int l1 = min(l0 + kChunk64, se);
    const int h = lane & 31;
    const int li = l0 + h;
    if (li < l1) {
      const LineRec64T& q = R[li];
      if (lane < 32) {
#pragma unroll
        for (int k = 0; k < 7; ++k) st->e[k][h] = q.e[k];
        st->gam2[h] = q.gam2;
      } else {
        st->nu[h] = nuc[li];
        st->thr[h] = q.thr;
        st->winv[h] = q.winv;
        st->a[h] = q.a;
        st->acore[h] = q.acore;
      }
      if constexpr (TAN) {
        const LineRec64TT& qt = RT[li];
        if (lane < 32) {
#pragma unroll
          for (int k = 0; k < 8; ++k) st->t[k][h] = qt.t[k];
        } else {
          st->kA[h] = qt.kA;
          st->kw[h] = qt.kw;
          st->da[h] = qt.da;
        }
      }
    }
    wave_lds_sync();
    const int n = l1 - l0;
#pragma unroll 1
    for (int i = 0; i < n; ++i) {
      double e[7];
#pragma unroll
      for (int k = 0; k < 7; ++k) e[k] = st->e[k][i];
      const double g2 = st->gam2[i], nul = st->nu[i];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const double d = nuj[g] - nul;
        const double D = fma(d, d, g2);
        if (NEAR && D < st->thr[i]) {
          const double x = d * st->winv[i], a = st->a[i];
          double H, L;
          core_w(x, a, &H, &L);
          acc[g] = fma(st->acore[i], H, acc[g]);
          if constexpr (TAN) {
            // custom derivatives of Sec. 2.1.1:
            //   dH/dx = 2aL - 2xH,  dH/da = 2xL + 2aH - 2/sqrt(pi)
            const double Hx = 2.0 * (a * L - x * H);
            const double Ha = 2.0 * (x * L + a * H) - 1.1283791670955126;
            tacc[g] = fma(st->acore[i], st->kA[i] * H + Hx * x * st->kw[i] + Ha * st->da[i], tacc[g]);
          }
        } else {
          const double r = rcp64(D);
          double hv = fma(e[6], r, e[5]);
          hv = fma(hv, r, e[4]);
          hv = fma(hv, r, e[3]);
          hv = fma(hv, r, e[2]);
          hv = fma(hv, r, e[1]);
          hv = fma(hv, r, e[0]);
          acc[g] = fma(hv, r, acc[g]);
          if constexpr (TAN) {
            double ht = fma(st->t[7][i], r, st->t[6][i]);
#pragma unroll
            for (int k = 5; k >= 0; --k) ht = fma(ht, r, st->t[k][i]);
            tacc[g] = fma(ht, r, tacc[g]);
          }
        }
      }
    }
    wave_lds_sync();
  }
}

template <bool TAN, int G>
__global__ __launch_bounds__(256) void k_voigt_f64t(VoigtArgs A) {
  using ST = typename std::conditional<TAN, Stage64T, Stage64>::type;
  const int y = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  __shared__ ST stage[4];
  const int64_t tile0 = (int64_t)blockIdx.x * (256 * G);
  double nuj[G];
  load_points<G>(A, tile0, w, lane, nuj);
  const int lb = (int)blockIdx.z * (int)A.lines_per_split;
  const int le = min(lb + (int)A.lines_per_split, (int)A.n_lines);
  const LineRec64T* __restrict__ R = A.rec64t + (int64_t)y * A.n_lines;
  const LineRec64TT* __restrict__ RT = TAN ? A.rect64t + (int64_t)y * A.n_lines : nullptr;
  // the last line (largest centre) has the largest Doppler width, hence the
  // largest core threshold of the layer
  const double reach = sqrt(R[A.n_lines - 1].thr) * (1.0 + 1e-12);
  const int64_t jw = tile0 + (int64_t)w * G * 64, jlast = A.ng - 1;
  const double lo = A.nu[jw < jlast ? jw : jlast];
  const double hi = A.nu[jw + G * 64 - 1 < jlast ? jw + G * 64 - 1 : jlast];
  const int i0 = __builtin_amdgcn_readfirstlane(search_sorted<false>(A.nu_c, lb, le, lo - reach));
  const int i1 = __builtin_amdgcn_readfirstlane(search_sorted<true>(A.nu_c, i0, le, hi + reach));
  double acc[G], tacc[G];
#pragma unroll
  for (int g = 0; g < G; ++g) acc[g] = tacc[g] = 0.0;
  lines64<false, TAN, G>(lb, i0, R, RT, A.nu_c, nuj, &stage[w], lane, acc, tacc);
  lines64<true, TAN, G>(i0, i1, R, RT, A.nu_c, nuj, &stage[w], lane, acc, tacc);
  lines64<false, TAN, G>(i1, le, R, RT, A.nu_c, nuj, &stage[w], lane, acc, tacc);
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int64_t j = tile0 + (int64_t)(w * G + g) * 64 + lane;
    if (j >= A.ng) continue;
    if (A.ksplit == 1) {
      const int64_t o = (int64_t)y * A.ld_out + j;
      A.out64[o] = acc[g] * A.out_scale64;
      if (TAN) A.out_t64[o] = tacc[g] * A.out_scale64;
    } else {
      const int64_t p = ((int64_t)blockIdx.z * A.nlay + y) * A.ng + j;
      A.part64[p] = acc[g];
      if (TAN) A.part_t64[p] = tacc[g];
    }
  }
}

// ---------------------------------------------------------------------------
// The plain FP64 form: per pair x = dnu/(sqrt2 beta), a = gamma/(sqrt2 beta),
// H from hjert_f64, contribution A/(sqrt(2 pi) beta) H; plain accumulation.
// Same thread-to-grid mapping as the FP32 kernel (G = 1).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_voigt_f64(VoigtArgs A) {
  const int y = blockIdx.y;
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const double nuj = A.nu[j < A.ng ? j : A.ng - 1];
  const int64_t lb = (int64_t)blockIdx.z * A.lines_per_split;
  const int64_t le = lb + A.lines_per_split < A.n_lines ? lb + A.lines_per_split : A.n_lines;
  const LineRec64* __restrict__ R = A.rec64 + (int64_t)y * A.n_lines;
  double acc = 0.0;
  for (int64_t l = lb; l < le; ++l) {
    const LineRec64 q = R[l];
    const double dn = nuj - A.nu_c[l];
    const double x = dn / (kSqrt2 * q.beta);
    const double a = q.gam / (kSqrt2 * q.beta);
    acc += q.A / (sqrt(2.0 * kPi) * q.beta) * hjert_f64(x, a, q.erfcxa);
  }
  if (j >= A.ng) return;
  if (A.ksplit == 1) {
    A.out64[(int64_t)y * A.ld_out + j] = acc * A.out_scale64;
  } else {
    A.part64[((int64_t)blockIdx.z * A.nlay + y) * A.ng + j] = acc;
  }
}

__global__ __launch_bounds__(256) void k_voigt_combine64(VoigtArgs A) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int y = blockIdx.y;
  if (j >= A.ng) return;
  double s = 0.0, t = 0.0;
  for (int z = 0; z < A.ksplit; ++z) {
    const int64_t p = ((int64_t)z * A.nlay + y) * A.ng + j;
    s += A.part64[p];
    if (A.out_t64) t += A.part_t64[p];
  }
  A.out64[(int64_t)y * A.ld_out + j] = s * A.out_scale64;
  if (A.out_t64) A.out_t64[(int64_t)y * A.ld_out + j] = t * A.out_scale64;
}

// ---------------------------------------------------------------------------
// Diagnostics: H (and L) of the FP32 path through the same record and pair
// arithmetic as the Voigt sum (beta = 1/sqrt2, so dnu = x, gamma = a and the
// contribution with amplitude sqrt(pi) equals H).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_hjert_f32(int64_t n, const float* __restrict__ x,
                                                   const float* __restrict__ a, float* __restrict__ H,
                                                   float* __restrict__ L) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double beta = 1.0 / kSqrt2;
  LineRec q;
  make_line_record(kSqrtPi, beta, (double)a[i], 1.0, 0.0, 0.0, 0.0, &q, nullptr);
  const float d = x[i];
  const float D = fmaf(d, d, q.gam2);
  const float r = __builtin_amdgcn_rcpf(D);
  float h = fmaf(q.e[6], r, q.e[5]);
  h = fmaf(h, r, q.e[4]);
  h = fmaf(h, r, q.e[3]);
  h = fmaf(h, r, q.e[2]);
  h = fmaf(h, r, q.e[1]);
  h = fmaf(h, r, q.e[0]);
  float f = h * r;
  float l = 0.f;
  if (D < q.thr) {
    double Hc, Lc;
    core_w((double)(d * q.winv), (double)q.a, &Hc, &Lc);
    f = q.acore * (float)Hc;
    l = (float)Lc;
  } else if (L) {
    hjert_asy_f32(d, q.a, &l);
  }
  H[i] = f;
  if (L) L[i] = l;
}

__global__ __launch_bounds__(256) void k_hjert_f64(int64_t n, const double* __restrict__ x,
                                                   const double* __restrict__ a, double* __restrict__ H) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  H[i] = hjert_f64(x[i], a[i], erfcx(a[i]));
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_line_records(const LinesDev& L, const double* T_lay, const double* P_lay,
                               const double* col_lay, double T_one, double P_one, double amp_scale,
                               const unsigned long long* amax, float* oscale, int layer0, int nlay,
                               LineRec* rec, LineRecT* rect, LineRec64* rec64, unsigned int* g2max_bits,
                               hipStream_t st, LineRec64T* rec64t, LineRec64TT* rect64t) {
  dim3 grid((unsigned)((L.n + 255) / 256), (unsigned)nlay);
  if (amax) {
    // the scale needs the largest strength of the call: one layer at (T_one, P_one)
    if (T_lay || nlay != 1 || rec64 || rec64t) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_amp_max, dim3((unsigned)((L.n + 255) / 256)), dim3(256), 0, st, L, T_one, P_one,
                       const_cast<unsigned long long*>(amax));
  }
  hipLaunchKernelGGL(k_line_records, grid, dim3(256), 0, st, L, T_lay, P_lay, col_lay, T_one, P_one,
                     amp_scale, layer0, amax, oscale, rec, rect, rec64, (rec64 || rec64t) ? nullptr : g2max_bits,
                     rec64t, rec64t ? rect64t : nullptr);
  return hipGetLastError();
}

hipError_t launch_far_reach(const LineRec* rec, int64_t n_lines, int nlay, bool tangent,
                            unsigned int* g2max_bits, float* reach2, int* t3, float* outer2,
                            unsigned long long* amax, hipStream_t st) {
  hipLaunchKernelGGL(k_far_reach, dim3((unsigned)nlay), dim3(64), 0, st, rec, n_lines, tangent ? 1 : 0, g2max_bits,
                     reach2, t3, outer2, amax);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_zero_words(unsigned int* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0u;
}

hipError_t launch_zero_words(void* p, size_t bytes, hipStream_t st) {
  const int64_t n = (int64_t)(bytes / sizeof(unsigned int));
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_words, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (unsigned int*)p, n);
  return hipGetLastError();
}

hipError_t launch_voigt(const VoigtArgs& A, bool fp64, bool tangent, hipStream_t st, bool tiled) {
  if (fp64 && tiled) {
    if (tangent && (!A.rect64t || !A.out_t64 || (A.ksplit > 1 && !A.part_t64))) return hipErrorInvalidValue;
    constexpr int G = kVoigtG;
    dim3 grid((unsigned)((A.ng + 256 * G - 1) / (256 * G)), (unsigned)A.nlay, (unsigned)A.ksplit);
    if (tangent) hipLaunchKernelGGL((k_voigt_f64t<true, G>), grid, dim3(256), 0, st, A);
    else hipLaunchKernelGGL((k_voigt_f64t<false, G>), grid, dim3(256), 0, st, A);
    if (A.ksplit > 1) {
      dim3 g2((unsigned)((A.ng + 255) / 256), (unsigned)A.nlay);
      hipLaunchKernelGGL(k_voigt_combine64, g2, dim3(256), 0, st, A);
    }
    return hipGetLastError();
  }
  if (fp64) {
    dim3 grid((unsigned)((A.ng + 255) / 256), (unsigned)A.nlay, (unsigned)A.ksplit);
    hipLaunchKernelGGL(k_voigt_f64, grid, dim3(256), 0, st, A);
    if (A.ksplit > 1) {
      dim3 g2((unsigned)((A.ng + 255) / 256), (unsigned)A.nlay);
      hipLaunchKernelGGL(k_voigt_combine64, g2, dim3(256), 0, st, A);
    }
    return hipGetLastError();
  }
  constexpr int G = kVoigtG;
  dim3 grid((unsigned)((A.ng + 256 * G - 1) / (256 * G)), (unsigned)A.nlay, (unsigned)A.ksplit);
  if (tangent) hipLaunchKernelGGL((k_voigt_f32<true, G>), grid, dim3(256), 0, st, A);
  else hipLaunchKernelGGL((k_voigt_f32<false, G>), grid, dim3(256), 0, st, A);
  if (A.ksplit > 1) {
    dim3 g2((unsigned)((A.ng + 255) / 256), (unsigned)A.nlay);
    if (tangent) hipLaunchKernelGGL(k_voigt_combine<true>, g2, dim3(256), 0, st, A);
    else hipLaunchKernelGGL(k_voigt_combine<false>, g2, dim3(256), 0, st, A);
  }
  return hipGetLastError();
}

hipError_t ensure_weideman() {
  static std::mutex mu;
  static std::vector<char> done;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> g(mu);
  if ((int)done.size() <= dev) done.resize(dev + 1, 0);
  if (done[dev]) return hipSuccess;
  hipLaunchKernelGGL(k_weid_init, dim3(1), dim3(64), 0, 0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipDeviceSynchronize()) != hipSuccess) return e;
  done[dev] = 1;
  return hipSuccess;
}

hipError_t launch_hjert_f32(int64_t n, const float* x, const float* a, float* H, float* L,
                            hipStream_t st) {
  const hipError_t e = ensure_weideman();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_hjert_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, x, a, H, L);
  return hipGetLastError();
}

hipError_t launch_hjert_f64(int64_t n, const double* x, const double* a, double* H, hipStream_t st) {
  hipLaunchKernelGGL(k_hjert_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, x, a, H);
  return hipGetLastError();
}

}  // namespace exo
