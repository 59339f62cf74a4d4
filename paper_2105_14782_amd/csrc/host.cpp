// exohip host library: context, validation, device memory, launch sequencing.
// C ABI in include/exohip.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/exohip.h"
#include "exo_host.h"
#include "exo_launch.h"

using namespace exo;

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

int exo::set_err(int code, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                 \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return set_err(EXO_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));      \
  } while (0)

extern "C" const char* exo_last_error(void) { return g_err.c_str(); }
extern "C" const char* exo_version(void) { return "exohip 0.1 (gfx950)"; }

// ---------------------------------------------------------------------------
// Device buffers
// ---------------------------------------------------------------------------
int exo::DevBuf::reserve(size_t bytes) {
  if (bytes <= cap) return EXO_OK;
  if (p) {
    // the old buffer may still be read by queued work
    (void)hipDeviceSynchronize();
    (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
  size_t want = bytes + bytes / 8 + 256;
  if (fail_alloc_hook()) return set_err(EXO_ENOMEM, "allocation of %zu bytes failed (test hook)", want);
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    return set_err(EXO_ENOMEM, "hipMalloc(%zu) failed: %s", want, hipGetErrorString(e));
  }
  cap = want;
  return EXO_OK;
}

void exo::DevBuf::release() {
  if (p && owned) (void)hipFree(p);
  p = nullptr;
  cap = 0;
  owned = true;
}

// EXO_TEST_FAIL_ALLOC=n makes the n-th subsequent device allocation fail.
bool exo::fail_alloc_hook() {
  static std::mutex mu;
  static long countdown = -2;
  std::lock_guard<std::mutex> g(mu);
  if (countdown == -2) {
    const char* s = getenv("EXO_TEST_FAIL_ALLOC");
    countdown = s ? atol(s) : -1;
  }
  if (countdown < 0) return false;
  if (countdown == 0) {
    countdown = -1;
    return true;
  }
  --countdown;
  return false;
}

Workspace::~Workspace() { release(); }

void Workspace::release() {
  for (DevBuf* b : bufs()) b->release();
  arena = nullptr;
  arena_cap = arena_used = 0;
  if (h_stage) (void)hipHostFree(h_stage);
  h_stage = nullptr;
  if (stage_ev) (void)hipEventDestroy(stage_ev);
  stage_ev = nullptr;
  if (done_ev) (void)hipEventDestroy(done_ev);
  done_ev = nullptr;
}

int Workspace::reserve(DevBuf& b, size_t bytes) {
  if (bytes <= b.cap) return EXO_OK;
  if (!arena) return b.reserve(bytes);
  const size_t need = (bytes + 255) & ~size_t(255);
  if (arena_used + need > arena_cap)
    return set_err(EXO_ENOMEM, "request needs more than its %zu-byte memory region", arena_cap);
  b.p = arena + arena_used;
  b.cap = need;
  b.owned = false;
  arena_used += need;
  return EXO_OK;
}

void Workspace::bind_arena(char* base, size_t cap) {
  for (DevBuf* b : bufs()) {
    if (b->owned) b->release();
    b->p = nullptr;
    b->cap = 0;
    b->owned = false;
  }
  arena = base;
  arena_cap = cap;
  arena_used = 0;
  tier_zeroed = nullptr;
}

int Workspace::begin(hipStream_t st) {
  if (done_ev && last_st != st) HIP_TRY(hipStreamWaitEvent(st, done_ev, 0));
  return EXO_OK;
}

int Workspace::end(hipStream_t st) {
  if (!done_ev) HIP_TRY(hipEventCreateWithFlags(&done_ev, hipEventDisableTiming));
  HIP_TRY(hipEventRecord(done_ev, st));
  last_st = st;
  return EXO_OK;
}

// Runs f(ws, st) between ws.begin and ws.end.
template <class F>
static int with_ws(Workspace& ws, hipStream_t st, F&& f) {
  int rc = ws.begin(st);
  if (rc) return rc;
  rc = f();
  const int rc2 = ws.end(st);
  return rc ? rc : rc2;
}

int Workspace::stage_params(const double* host, size_t n, double* dev, hipStream_t st) {
  if (!h_stage) {
    HIP_TRY(hipHostMalloc((void**)&h_stage, kStageDoubles * sizeof(double), hipHostMallocDefault));
    HIP_TRY(hipEventCreateWithFlags(&stage_ev, hipEventDisableTiming));
  } else {
    HIP_TRY(hipEventSynchronize(stage_ev));
  }
  if (n > kStageDoubles) return set_err(EXO_EINVAL, "parameter block too large (%zu doubles)", n);
  memcpy(h_stage, host, n * sizeof(double));
  HIP_TRY(hipMemcpyAsync(dev, h_stage, n * sizeof(double), hipMemcpyHostToDevice, st));
  HIP_TRY(hipEventRecord(stage_ev, st));
  return EXO_OK;
}

// ---------------------------------------------------------------------------
// Scratch of the cross-section that allocates nothing
// ---------------------------------------------------------------------------
// exo_cross_section_noalloc keeps its line records, far-tier table and split
// partial sums in this fixed array, one copy per device for the life of the
// process.  In host code `scratch` names a host-side stand-in, not device
// memory: its device address on each device comes from hipGetSymbolAddress
// (at exo_create, with that device current) and only that address is used.
static constexpr size_t kNoAllocScratchBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
static std::mutex g_scratch_mu;
static std::vector<void*> g_scratch_dev;   // [device] address of `scratch`

// With `device` current: look up and keep the device's scratch address.
static int bind_scratch(int device) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if ((int)g_scratch_dev.size() <= device) g_scratch_dev.resize(device + 1, nullptr);
  if (g_scratch_dev[device]) return EXO_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return set_err(EXO_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", device,
                   hipGetErrorString(e));
  g_scratch_dev[device] = p;
  return EXO_OK;
}

static void* scratch_of(int device) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  return device < (int)g_scratch_dev.size() ? g_scratch_dev[device] : nullptr;
}

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
extern "C" int exo_create(int device, exo_ctx** out) {
  if (!out) return set_err(EXO_EINVAL, "out is NULL");
  *out = nullptr;
  int n = 0;
  HIP_TRY(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return set_err(EXO_EINVAL, "device %d out of range (%d devices)", device, n);
  HIP_TRY(hipSetDevice(device));
  HIP_TRY(ensure_weideman());
  const int rc = bind_scratch(device);
  if (rc) return rc;
  exo_ctx* c = new exo_ctx();
  c->device = device;
  *out = c;
  return EXO_OK;
}

extern "C" int exo_destroy(exo_ctx* c) {
  if (!c) return EXO_OK;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  for (auto& s : c->sp) s.release();
  c->d_nu.release();
  c->ws.release();
  c->prof_near.release();
  for (auto& p : c->prof) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  delete c;
  return EXO_OK;
}

void Species::release() {
  for (DevBuf* b : {&nu_c, &S0, &E_low, &alpha_ref, &n_texp, &gamma_nat, &qr, &perm}) b->release();
  h_nu_c.clear();
  h_nu_c.shrink_to_fit();
  set = false;
  n = 0;
}

static bool finite_all(const double* a, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

extern "C" int exo_set_lines(exo_ctx* c, int s, int64_t n, const double* nu_c, const double* S0,
                             const double* E_low, const double* alpha_ref, const double* n_texp,
                             const double* gamma_nat, double mass_amu, int qr_kind,
                             const double* qr_params, int n_qr) {
  if (!c) return set_err(EXO_EINVAL, "ctx is NULL");
  if (s < 0 || s >= EXO_MAX_SPECIES) return set_err(EXO_EINVAL, "species slot %d out of range", s);
  if (n < 1 || n >= ((int64_t)1 << 31)) return set_err(EXO_EINVAL, "n_lines must be in [1, 2^31)");
  if (!nu_c || !S0 || !E_low || !alpha_ref || !n_texp) return set_err(EXO_EINVAL, "NULL line array");
  if (!(mass_amu > 0) || !std::isfinite(mass_amu)) return set_err(EXO_EINVAL, "mass must be > 0");
  if (!finite_all(nu_c, n) || !finite_all(S0, n) || !finite_all(E_low, n) ||
      !finite_all(alpha_ref, n) || !finite_all(n_texp, n) || (gamma_nat && !finite_all(gamma_nat, n)))
    return set_err(EXO_EINVAL, "non-finite line parameter");
  for (int64_t i = 0; i < n; ++i) {
    if (!(nu_c[i] > 0)) return set_err(EXO_EINVAL, "line %lld: nu_c must be > 0", (long long)i);
    if (S0[i] < 0 || E_low[i] < 0 || alpha_ref[i] < 0 || (gamma_nat && gamma_nat[i] < 0))
      return set_err(EXO_EINVAL, "line %lld: negative strength/energy/width", (long long)i);
  }
  if (qr_kind == EXO_QR_POWER) {
    if (n_qr != 1 || !qr_params || !std::isfinite(qr_params[0]))
      return set_err(EXO_EINVAL, "EXO_QR_POWER needs one finite parameter");
  } else if (qr_kind == EXO_QR_TABLE) {
    if (n_qr < 4 || (n_qr & 1) || !qr_params || !finite_all(qr_params, n_qr))
      return set_err(EXO_EINVAL, "EXO_QR_TABLE needs 2n (n >= 2) finite values");
    const int k = n_qr / 2;
    for (int i = 0; i < k; ++i) {
      if (i > 0 && !(qr_params[i] > qr_params[i - 1])) return set_err(EXO_EINVAL, "Q table T nodes must ascend");
      if (!(qr_params[k + i] > 0)) return set_err(EXO_EINVAL, "Q table values must be > 0");
    }
  } else {
    return set_err(EXO_EINVAL, "unknown qr_kind %d", qr_kind);
  }
  HIP_TRY(hipSetDevice(c->device));
  // sort by line centre
  std::vector<int64_t> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return nu_c[a] < nu_c[b]; });
  std::vector<double> tmp(n);
  Species& sp = c->sp[s];
  HIP_TRY(hipDeviceSynchronize());
  sp.release();
  auto up = [&](DevBuf& b, const double* src) -> int {
    for (int64_t i = 0; i < n; ++i) tmp[i] = src ? src[idx[i]] : 0.0;
    int rc = b.reserve(n * sizeof(double));
    if (rc) return rc;
    HIP_TRY(hipMemcpy(b.p, tmp.data(), n * sizeof(double), hipMemcpyHostToDevice));
    return EXO_OK;
  };
  int rc;
  if ((rc = up(sp.nu_c, nu_c)) || (rc = up(sp.S0, S0)) || (rc = up(sp.E_low, E_low)) ||
      (rc = up(sp.alpha_ref, alpha_ref)) || (rc = up(sp.n_texp, n_texp))) {
    sp.release();
    return rc;
  }
  if (gamma_nat && (rc = up(sp.gamma_nat, gamma_nat))) {
    sp.release();
    return rc;
  }
  if ((rc = sp.perm.reserve(n * sizeof(int64_t)))) {
    sp.release();
    return rc;
  }
  HIP_TRY(hipMemcpy(sp.perm.p, idx.data(), n * sizeof(int64_t), hipMemcpyHostToDevice));
  if ((rc = sp.qr.reserve(n_qr * sizeof(double)))) {
    sp.release();
    return rc;
  }
  HIP_TRY(hipMemcpy(sp.qr.p, qr_params, n_qr * sizeof(double), hipMemcpyHostToDevice));
  sp.n = n;
  sp.has_gnat = gamma_nat != nullptr;
  sp.mass = mass_amu;
  sp.qr_kind = qr_kind;
  sp.n_qr = n_qr;
  sp.h_nu_c.resize(n);
  for (int64_t i = 0; i < n; ++i) sp.h_nu_c[i] = nu_c[idx[i]];
  sp.nu_lo = tmp.empty() ? 0 : nu_c[idx.front()];
  sp.nu_hi = nu_c[idx.back()];
  sp.set = true;
  return EXO_OK;
}

extern "C" int exo_set_grid(exo_ctx* c, int64_t n, const double* nu) {
  if (!c) return set_err(EXO_EINVAL, "ctx is NULL");
  if (n < 2 || !nu) return set_err(EXO_EINVAL, "grid needs >= 2 points");
  if (!finite_all(nu, n)) return set_err(EXO_EINVAL, "non-finite grid value");
  if (!(nu[0] > 0)) return set_err(EXO_EINVAL, "grid must be positive");
  for (int64_t i = 1; i < n; ++i)
    if (!(nu[i] > nu[i - 1])) return set_err(EXO_EINVAL, "grid must be strictly ascending (index %lld)", (long long)i);
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipDeviceSynchronize());
  int rc = c->d_nu.reserve(n * sizeof(double));
  if (rc) return rc;
  HIP_TRY(hipMemcpy(c->d_nu.p, nu, n * sizeof(double), hipMemcpyHostToDevice));
  c->n_nu = n;
  c->h_nu.assign(nu, nu + n);
  // log-uniform detection
  const double mean = std::log(nu[n - 1] / nu[0]) / (double)(n - 1);
  double dev = 0.0;
  for (int64_t i = 1; i < n; ++i) dev = std::max(dev, std::fabs(std::log(nu[i] / nu[i - 1]) - mean));
  c->eslog = dev <= 1e-6 * mean + 1e-14;
  c->dv_kms = kCkms * mean;
  return EXO_OK;
}

// ---------------------------------------------------------------------------
// Profiling of the Voigt-sum launches
// ---------------------------------------------------------------------------
extern "C" int exo_profile_enable(exo_ctx* c, int on) {
  if (!c) return set_err(EXO_EINVAL, "ctx is NULL");
  (void)hipSetDevice(c->device);
  for (auto& p : c->prof) {
    (void)hipEventSynchronize(p.b);
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  c->prof.clear();
  if (on) {
    if (c->prof_near.reserve(3 * sizeof(unsigned long long))) return EXO_ENOMEM;
    HIP_TRY(hipMemset(c->prof_near.p, 0, 3 * sizeof(unsigned long long)));
  }
  c->profile = on != 0;
  return EXO_OK;
}

extern "C" int exo_profile_read_near(exo_ctx* c, double* near_evals) {
  if (!c) return set_err(EXO_EINVAL, "ctx is NULL");
  if (!near_evals) return set_err(EXO_EINVAL, "near_evals is NULL");
  HIP_TRY(hipSetDevice(c->device));
  for (auto& p : c->prof) HIP_TRY(hipEventSynchronize(p.b));
  unsigned long long n = 0;
  if (c->prof_near.p) HIP_TRY(hipMemcpy(&n, c->prof_near.p, sizeof(n), hipMemcpyDeviceToHost));
  *near_evals = (double)n;
  return EXO_OK;
}

extern "C" int exo_profile_read_far_cut(exo_ctx* c, double* far_cut_evals) {
  if (!c) return set_err(EXO_EINVAL, "ctx is NULL");
  if (!far_cut_evals) return set_err(EXO_EINVAL, "far_cut_evals is NULL");
  HIP_TRY(hipSetDevice(c->device));
  for (auto& p : c->prof) HIP_TRY(hipEventSynchronize(p.b));
  unsigned long long n[2] = {0, 0};
  if (c->prof_near.p) HIP_TRY(hipMemcpy(n, c->prof_near.p, sizeof(n), hipMemcpyDeviceToHost));
  *far_cut_evals = (double)n[1];
  return EXO_OK;
}

extern "C" int exo_profile_read_far_outer(exo_ctx* c, double* outer_evals) {
  if (!c) return set_err(EXO_EINVAL, "ctx is NULL");
  if (!outer_evals) return set_err(EXO_EINVAL, "outer_evals is NULL");
  HIP_TRY(hipSetDevice(c->device));
  for (auto& p : c->prof) HIP_TRY(hipEventSynchronize(p.b));
  unsigned long long n[3] = {0, 0, 0};
  if (c->prof_near.p) HIP_TRY(hipMemcpy(n, c->prof_near.p, sizeof(n), hipMemcpyDeviceToHost));
  *outer_evals = (double)n[2];
  return EXO_OK;
}

extern "C" int exo_profile_read(exo_ctx* c, int64_t* nl, double* ms, double* evals) {
  if (!c) return set_err(EXO_EINVAL, "ctx is NULL");
  HIP_TRY(hipSetDevice(c->device));
  double tot = 0, ev = 0;
  for (auto& p : c->prof) {
    HIP_TRY(hipEventSynchronize(p.b));
    float t = 0;
    HIP_TRY(hipEventElapsedTime(&t, p.a, p.b));
    tot += t;
    ev += p.evals;
  }
  if (nl) *nl = (int64_t)c->prof.size();
  if (ms) *ms = tot;
  if (evals) *evals = ev;
  return EXO_OK;
}

int exo::voigt_launch_profiled(exo_ctx* c, const VoigtArgs& A, bool fp64, bool tan, hipStream_t st, bool tiled) {
  ProfRec pr{};
  const bool prof = c && c->profile;
  if (prof) {
    HIP_TRY(hipEventCreate(&pr.a));
    HIP_TRY(hipEventCreate(&pr.b));
    HIP_TRY(hipEventRecord(pr.a, st));
  }
  VoigtArgs Ap = A;
  if (prof && !fp64) Ap.near_pairs = (unsigned long long*)c->prof_near.p;
  HIP_TRY(launch_voigt(Ap, fp64, tan, st, tiled));
  if (prof) {
    HIP_TRY(hipEventRecord(pr.b, st));
    pr.evals = (double)A.n_lines * (double)A.ng * (double)A.nlay;
    std::lock_guard<std::mutex> g(c->prof_mu);
    c->prof.push_back(pr);
  }
  return EXO_OK;
}

// ---------------------------------------------------------------------------
// Voigt sum of one species over a layer range into tau[(layer)][ng]
// ---------------------------------------------------------------------------
static LinesDev lines_dev(const Species& sp) {
  LinesDev L;
  L.nu_c = (const double*)sp.nu_c.p;
  L.S0 = (const double*)sp.S0.p;
  L.E_low = (const double*)sp.E_low.p;
  L.alpha_ref = (const double*)sp.alpha_ref.p;
  L.n_texp = (const double*)sp.n_texp.p;
  L.gamma_nat = sp.has_gnat ? (const double*)sp.gamma_nat.p : nullptr;
  L.n = sp.n;
  L.mass = sp.mass;
  L.qr_kind = sp.qr_kind;
  L.qr_params = (const double*)sp.qr.p;
  L.n_qr = sp.n_qr;
  return L;
}

// Record-buffer budget per workspace (bytes); layers are processed in chunks
// that fit it.
static constexpr size_t kRecBudget = size_t(4) << 30;

// Split over lines when the grid x layer tiles of one launch cannot fill the
// device (fixed by the shape only, so results never depend on the load).
// Splits go down to 16 lines: a small problem (a few tiles) is otherwise
// bound by one wave's line-record load latency, line after line.  The target
// is 8192 workgroups, 5-6 per resident slot (1280 of 4 waves at the tangent
// kernel's 5 waves per SIMD, 1536 at the forward kernel's 6): a wave's near
// lines and core pairs fall in one split, so finer splits even out the
// workgroups' run times (config 2: 5 splits instead of 2, 2.8 % faster per
// step; 4096, 6144 and 12288 measured no better).
static void split_plan(int64_t ng, int nl, int64_t n_lines, bool one_point, int64_t* ks_out,
                       int64_t* lps_out) {
  // one_point: the plain FP64 form (one grid point per thread)
  const int64_t G = one_point ? 1 : kVoigtG;
  const int64_t tiles = (ng + 256 * G - 1) / (256 * G);
  const int64_t blocks = tiles * nl;
  int64_t ks = 1;
  if (blocks < 8192) ks = std::min<int64_t>((8192 + blocks - 1) / blocks, std::max<int64_t>(1, n_lines / 16));
  const int64_t lps = (n_lines + ks - 1) / ks;
  ks = (n_lines + lps - 1) / lps;
  *ks_out = ks;
  *lps_out = lps;
}

OpacityPlan exo::plan_opacity(int64_t n_lines, int nlay, int64_t ng, bool fp64, bool tangent, bool tiled64) {
  OpacityPlan P{};
  tiled64 = tiled64 && fp64;
  tangent = tangent && (!fp64 || tiled64);   // the plain FP64 form has no tangent mode
  const size_t rec64_size = tiled64 ? sizeof(LineRec64T) : sizeof(LineRec64);
  const size_t per_layer =
      (size_t)n_lines * (fp64 ? rec64_size + (tangent ? sizeof(LineRec64TT) : 0)
                              : sizeof(LineRec) + (tangent ? sizeof(LineRecT) : 0));
  P.nlc = (int)std::max<size_t>(1, std::min<size_t>((size_t)nlay, kRecBudget / per_layer));
  if (fp64) {
    // the tiled FP64 records share the plain form's buffers
    P.rec64 = (size_t)P.nlc * n_lines * rec64_size;
    if (tangent) P.rect = (size_t)P.nlc * n_lines * sizeof(LineRec64TT);
  } else {
    P.rec = (size_t)P.nlc * n_lines * sizeof(LineRec);
    P.tier = kTierBytes;
    if (tangent) P.rect = (size_t)P.nlc * n_lines * sizeof(LineRecT);
  }
  // partial sums (the FP32 sum always passes its far-line state through
  // them): the largest over the chunk sizes that occur
  for (int nl : {P.nlc, nlay % P.nlc}) {
    if (nl <= 0) continue;
    int64_t ks, lps;
    split_plan(ng, nl, n_lines, fp64 && !tiled64, &ks, &lps);
    if (ks > 1 || !fp64) {
      const size_t pb = (size_t)ks * nl * ng * (fp64 ? sizeof(double) : sizeof(float2));
      P.part = std::max(P.part, pb);
      if (tangent) P.part_t = std::max(P.part_t, pb);
    }
  }
  return P;
}

OpacityPlan exo::plan_opacity_all(const exo_ctx* c, const exo_atmos* a, int64_t gl, bool fp64,
                                  bool tangent, bool tiled64) {
  OpacityPlan P{};
  for (int m = 0; m < a->n_species; ++m) {
    const OpacityPlan Q = plan_opacity(c->sp[a->species[m]].n, a->n_layers, gl, fp64, tangent, tiled64);
    P.rec = std::max(P.rec, Q.rec);
    P.rect = std::max(P.rect, Q.rect);
    P.rec64 = std::max(P.rec64, Q.rec64);
    P.tier = std::max(P.tier, Q.tier);
    P.part = std::max(P.part, Q.part);
    P.part_t = std::max(P.part_t, Q.part_t);
  }
  return P;
}

int exo::reserve_opacity(Workspace& ws, const OpacityPlan& P) {
  int rc;
  if (P.rec64 && (rc = ws.reserve(ws.rec64, P.rec64))) return rc;
  if (P.rec && (rc = ws.reserve(ws.rec, P.rec))) return rc;
  if (P.tier && (rc = ws.reserve(ws.tier, P.tier))) return rc;
  if (P.rect && (rc = ws.reserve(ws.rect, P.rect))) return rc;
  if (P.part && (rc = ws.reserve(ws.part, P.part))) return rc;
  if (P.part_t && (rc = ws.reserve(ws.part_t, P.part_t))) return rc;
  return EXO_OK;
}

int exo::species_opacity(exo_ctx* c, Workspace& ws, const Species& sp, const double* d_T,
                         const double* d_P, const double* d_col, int nlay, double amp_scale,
                         bool fp64, bool tangent, const double* d_nu, int64_t ng, void* out,
                         void* out_t, hipStream_t st, double T_one, double P_one, bool adaptive_scale,
                         bool tiled64) {
  const LinesDev L = lines_dev(sp);
  tiled64 = tiled64 && fp64;
  if (fp64 && !tiled64 && tangent) return set_err(EXO_EINVAL, "the plain FP64 form has no tangent mode");
  const OpacityPlan P = plan_opacity(sp.n, nlay, ng, fp64, tangent, tiled64);
  int rc;
  if ((rc = reserve_opacity(ws, P))) return rc;
  const int nlc = P.nlc;
  // tier buffer: [kMaxLayers] gamma^2 maximum bits, then [kMaxLayers] each
  // squared reach, t3 flag and squared outer reach, then the strength
  // maximum and the output scale of an adaptive cross-section scale;
  // k_far_reach zeroes the maxima of its chunk after use
  unsigned int* g2bits = fp64 ? nullptr : (unsigned int*)ws.tier.p;
  float* reach2 = fp64 ? nullptr : (float*)(g2bits + kMaxLayers);
  int* t3 = fp64 ? nullptr : (int*)(g2bits + 2 * kMaxLayers);
  float* outer2 = fp64 ? nullptr : (float*)(g2bits + 3 * kMaxLayers);
  const bool adaptive = adaptive_scale && !fp64 && d_T == nullptr && nlay == 1;
  unsigned long long* amax = adaptive ? (unsigned long long*)(g2bits + 4 * kMaxLayers) : nullptr;
  float* oscale = adaptive ? (float*)(g2bits + 4 * kMaxLayers + 2) : nullptr;
  // cleared by a kernel, not a memset: the call may be captured in a graph
  if (!fp64 && ws.tier_zeroed != ws.tier.p) HIP_TRY(launch_zero_words(ws.tier.p, kTierBytes, st));
  ws.tier_zeroed = nullptr;
  for (int l0 = 0; l0 < nlay; l0 += nlc) {
    const int nl = std::min(nlc, nlay - l0);
    HIP_TRY(launch_line_records(L, d_T, d_P, d_col, T_one, P_one, amp_scale, amax, oscale, l0, nl,
                                fp64 ? nullptr : (LineRec*)ws.rec.p,
                                (!fp64 && tangent) ? (LineRecT*)ws.rect.p : nullptr,
                                (fp64 && !tiled64) ? (LineRec64*)ws.rec64.p : nullptr, g2bits, st,
                                tiled64 ? (LineRec64T*)ws.rec64.p : nullptr,
                                (tiled64 && tangent) ? (LineRec64TT*)ws.rect.p : nullptr));
    if (!fp64)
      HIP_TRY(launch_far_reach((const LineRec*)ws.rec.p, sp.n, nl, tangent, g2bits, reach2, t3, outer2, amax, st));
    VoigtArgs A{};
    A.nu = d_nu;
    A.ng = ng;
    A.nu_c = L.nu_c;
    A.n_lines = sp.n;
    A.rec = (const LineRec*)ws.rec.p;
    A.rect = (const LineRecT*)ws.rect.p;
    A.rec64 = tiled64 ? nullptr : (const LineRec64*)ws.rec64.p;
    A.rec64t = tiled64 ? (const LineRec64T*)ws.rec64.p : nullptr;
    A.rect64t = (tiled64 && tangent) ? (const LineRec64TT*)ws.rect.p : nullptr;
    A.far_reach2 = reach2;
    A.far_t3 = t3;
    A.far_outer2 = outer2;
    A.nlay = nl;
    A.out_scale = (float)(1.0 / amp_scale);
    A.out_scale_dev = oscale;
    A.out_scale64 = 1.0 / amp_scale;
    A.ld_out = ng;
    if (fp64) {
      A.out64 = (double*)out + (int64_t)l0 * ng;
      A.out_t64 = tangent ? (double*)out_t + (int64_t)l0 * ng : nullptr;
    } else {
      A.out = (float*)out + (int64_t)l0 * ng;
      A.out_t = tangent ? (float*)out_t + (int64_t)l0 * ng : nullptr;
    }
    int64_t ks, lps;
    split_plan(ng, nl, sp.n, fp64 && !tiled64, &ks, &lps);
    A.lines_per_split = lps;
    A.ksplit = (int)ks;
    if (ks > 1 || !fp64) {
      A.part = (float2*)ws.part.p;
      A.part_t = (float2*)ws.part_t.p;
      A.part64 = (double*)ws.part.p;
      A.part_t64 = (double*)ws.part_t.p;
    }
    if ((rc = voigt_launch_profiled(ws.no_alloc ? nullptr : c, A, fp64, tangent, st, tiled64))) return rc;
  }
  if (!fp64) ws.tier_zeroed = ws.tier.p;
  return EXO_OK;
}

extern "C" int exo_select_lines(exo_ctx* c, int s, double log10_mmr, const exo_atmos* a, double T_atm,
                                const double* T_strength, int n_T, int margin, uint8_t* keep,
                                int64_t* n_kept, void* stream) {
  if (!c) return set_err(EXO_EINVAL, "ctx is NULL");
  if (s < 0 || s >= EXO_MAX_SPECIES) return set_err(EXO_EINVAL, "species slot %d out of range", s);
  if (!c->sp[s].set) return set_err(EXO_ENOTSET, "species slot %d not set", s);
  if (!a || !keep) return set_err(EXO_EINVAL, "atmos / keep_dev is NULL");
  if (a->n_layers < 2 || a->n_layers > kMaxLayers || !a->P_bar)
    return set_err(EXO_EINVAL, "need 2..%d layers", kMaxLayers);
  for (int i = 0; i < a->n_layers; ++i) {
    if (!(a->P_bar[i] > 0) || !std::isfinite(a->P_bar[i])) return set_err(EXO_EINVAL, "P must be > 0");
    if (i > 0 && !(a->P_bar[i] > a->P_bar[i - 1])) return set_err(EXO_EINVAL, "P must ascend (top -> bottom)");
  }
  if (!(a->g_cgs > 0) || !(a->mmw > 0)) return set_err(EXO_EINVAL, "need g > 0 and mmw > 0");
  if (!std::isfinite(a->cia_alpha0) || a->cia_alpha0 < 0 || !std::isfinite(a->cia_Tpow) ||
      !std::isfinite(a->cia_slope) || !std::isfinite(a->cia_nu_c) || !(a->vmr_h2 >= 0))
    return set_err(EXO_EINVAL, "bad CIA parameters");
  if (!std::isfinite(log10_mmr) || log10_mmr > 0) return set_err(EXO_EINVAL, "log10_mmr must be finite and <= 0");
  if (!(T_atm > 1.0) || !std::isfinite(T_atm)) return set_err(EXO_EINVAL, "T_atm must exceed 1 K");
  if (n_T < 0 || n_T > 256 || (n_T > 0 && !T_strength)) return set_err(EXO_EINVAL, "bad temperature list");
  for (int t = 0; t < n_T; ++t)
    if (!(T_strength[t] > 1.0) || !std::isfinite(T_strength[t])) return set_err(EXO_EINVAL, "bad temperature list");
  if (margin < 0 || margin > kMaxLayers) return set_err(EXO_EINVAL, "margin must be in [0, %d]", kMaxLayers);
  HIP_TRY(hipSetDevice(c->device));
  std::lock_guard<std::mutex> g(c->mu);
  hipStream_t st = (hipStream_t)stream;
  const Species& sp = c->sp[s];
  const int NL = a->n_layers;
  return with_ws(c->ws, st, [&]() -> int {
    Workspace& ws = c->ws;
    int rc;
    // parameter block: P, the isothermal T, the strength temperatures
    std::vector<double> blk(a->P_bar, a->P_bar + NL);
    blk.insert(blk.end(), NL, T_atm);
    if (n_T > 0) blk.insert(blk.end(), T_strength, T_strength + n_T);
    else blk.push_back(T_atm);
    if ((rc = ws.reserve(ws.params, blk.size() * sizeof(double)))) return rc;
    if ((rc = ws.stage_params(blk.data(), blk.size(), (double*)ws.params.p, st))) return rc;
    if ((rc = ws.reserve(ws.layer, (size_t)6 * NL * sizeof(double)))) return rc;
    if ((rc = ws.reserve(ws.col, (size_t)NL * sizeof(double)))) return rc;
    if ((rc = ws.reserve(ws.gout, 256))) return rc;
    double* lay = (double*)ws.layer.p;
    AtmosDev A{};
    A.nlay = NL;
    A.nspec = 1;
    A.P = (const double*)ws.params.p;
    A.T_in = (const double*)ws.params.p + NL;
    A.g = a->g_cgs;
    A.mmw = a->mmw;
    A.cia_alpha0 = a->cia_alpha0;
    A.cia_Tpow = a->cia_Tpow;
    A.cia_slope = a->cia_slope;
    A.cia_nu_c = a->cia_nu_c;
    A.vmr_h2 = a->vmr_h2;
    A.logx[0] = log10_mmr;
    A.mass[0] = sp.mass;
    A.T = lay;
    A.dP = lay + NL;
    A.lnP = lay + 2 * NL;
    A.cia = lay + 3 * NL;
    A.dcia = lay + 4 * NL;
    A.col = (double*)ws.col.p;
    HIP_TRY(launch_atmos(A, st));
    SelectArgs S{};
    S.L = lines_dev(sp);
    S.perm = (const int64_t*)sp.perm.p;
    S.T_strength = (const double*)ws.params.p + 2 * NL;
    S.n_T = n_T > 0 ? n_T : 1;
    S.T_atm = T_atm;
    S.nlay = NL;
    S.margin = margin;
    S.P = A.P;
    S.dP = A.dP;
    S.col = A.col;
    S.cia = A.cia;
    S.cia_slope = a->cia_slope;
    S.cia_nu_c = a->cia_nu_c;
    S.keep = keep;
    S.n_kept = (unsigned long long*)ws.gout.p;
    HIP_TRY(launch_select_lines(S, st));
    if (n_kept) {
      unsigned long long h = 0;
      HIP_TRY(hipMemcpyAsync(&h, ws.gout.p, sizeof(h), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      *n_kept = (int64_t)h;
    }
    return EXO_OK;
  });
}

// Per-layer device bytes of a MODIT launch; layers go in batches that fit
// kModitBudget.
static constexpr size_t kModitBudget = size_t(4) << 30;

static int64_t modit_fft_len(int64_t ng) {
  int64_t n = 1;
  while (n < 2 * ng) n *= 2;
  return n;
}

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

struct ModitPlan {
  int nb;                 // layers per launch
  int64_t n_fft, nbl;     // transform length, line blocks
  size_t off_cell, off_lay, off_rec, lines_bytes;   // layout of ws.mlines
  size_t part_bytes, rows_bytes;
};

static ModitPlan modit_plan(int64_t n_in, int64_t ng, int nlay, bool fp64) {
  ModitPlan q{};
  const size_t csz = fp64 ? 2 * sizeof(double) : 2 * sizeof(float);   // complex sample
  const size_t psz = csz;                                             // {ln gamma~, S} pair
  const int64_t ni = std::max<int64_t>(n_in, 1);
  q.n_fft = modit_fft_len(ng);
  q.nbl = (ni + 255) / 256;
  const size_t per_layer = 2 * (size_t)kModitRows * q.n_fft * csz + (size_t)ni * psz +
                           3 * (size_t)q.nbl * sizeof(double) + sizeof(ModitBins) + sizeof(ModitLayer);
  const size_t nb = std::max<size_t>(1, kModitBudget / per_layer);
  q.nb = (int)std::min<size_t>({nb, (size_t)nlay, (size_t)kModitMaxLayersPerLaunch});
  q.off_cell = align256((size_t)ni * sizeof(double));
  q.off_lay = q.off_cell + align256((size_t)(ng + 1) * sizeof(int64_t));
  q.off_rec = q.off_lay + align256((size_t)q.nb * sizeof(ModitLayer));
  q.lines_bytes = q.off_rec + (size_t)q.nb * ni * psz;
  q.part_bytes = align256((size_t)q.nb * 3 * q.nbl * sizeof(double)) + (size_t)q.nb * sizeof(ModitBins);
  q.rows_bytes = (size_t)q.nb * kModitRows * q.n_fft * csz;
  return q;
}

// lines of sp with nu_lo <= nu_c <= nu_hi: [l0, l0 + n_in) of the sorted list
static void modit_window(const Species& sp, double nu_lo, double nu_hi, int64_t* l0, int64_t* n_in) {
  const auto& h = sp.h_nu_c;
  *l0 = std::lower_bound(h.begin(), h.end(), nu_lo) - h.begin();
  *n_in = (std::upper_bound(h.begin(), h.end(), nu_hi) - h.begin()) - *l0;
}

size_t exo::modit_workspace(const Species& sp, double nu_lo, double nu_hi, int64_t ng, int nlay,
                            bool fp64) {
  int64_t l0, n_in;
  modit_window(sp, nu_lo, nu_hi, &l0, &n_in);
  const ModitPlan q = modit_plan(n_in, ng, nlay, fp64);
  return align256(q.lines_bytes) + align256(q.part_bytes) + 2 * align256(q.rows_bytes);
}

// MODIT cross-sections (col == NULL) or optical depths col_n sigma clamped
// at zero, of nlay layers (device T, P, col [nlay]) on the log-uniform grid
// d_nu [ng], into out [nlay][ng] (float, or double with fp64).
int exo::modit_opacity(exo_ctx* c, Workspace& ws, const Species& sp, const double* d_T, const double* d_P,
                       const double* d_col, int nlay, double dlng, bool fp64, const double* d_nu,
                       double nu_lo, double nu_hi, int64_t ng, void* out, hipStream_t st) {
  ModitArgs M{};
  M.L = lines_dev(sp);
  M.mass = sp.mass;
  M.R0 = kCkms / c->dv_kms;   // 1 / mean ln spacing
  M.dlng = dlng;
  M.nu = d_nu;
  M.ng = ng;
  M.nu_c = (const double*)sp.nu_c.p;
  modit_window(sp, nu_lo, nu_hi, &M.l0, &M.n_in);
  const ModitPlan q = modit_plan(M.n_in, ng, nlay, fp64);
  M.n_fft = q.n_fft;
  // FP32: a layer's largest strength goes to ~2^amp_exp, so that n_fft times
  // the sum of all strengths stays below 2^124
  if (!fp64) {
    int lf = 0, ll = 0;
    while (((int64_t)1 << lf) < q.n_fft) ++lf;
    while (((int64_t)1 << ll) < std::max<int64_t>(M.n_in, 1)) ++ll;
    M.amp_exp = 124 - lf - ll;
  }
  M.n_part = q.nbl;
  M.out64 = fp64;
  const size_t esz = fp64 ? sizeof(double) : sizeof(float);
  int rc;
  if ((rc = ws.reserve(ws.mlines, q.lines_bytes))) return rc;
  if ((rc = ws.reserve(ws.mpart, q.part_bytes))) return rc;
  if ((rc = ws.reserve(ws.mrows0, q.rows_bytes))) return rc;
  if ((rc = ws.reserve(ws.mrows1, q.rows_bytes))) return rc;
  char* base = (char*)ws.mlines.p;
  M.f = base;
  M.cell = (int64_t*)(base + q.off_cell);
  M.lay = (ModitLayer*)(base + q.off_lay);
  M.rec = base + q.off_rec;
  M.part = (double*)ws.mpart.p;
  M.bins = (ModitBins*)((char*)ws.mpart.p + align256((size_t)q.nb * 3 * q.nbl * sizeof(double)));
  M.rows0 = ws.mrows0.p;
  M.rows1 = ws.mrows1.p;
  for (int n0 = 0; n0 < nlay; n0 += q.nb) {
    M.nl = std::min(q.nb, nlay - n0);
    M.want_pos = n0 == 0;
    M.T = d_T + n0;
    M.P = d_P + n0;
    M.col = d_col ? d_col + n0 : nullptr;
    M.out = (char*)out + (size_t)n0 * ng * esz;
    HIP_TRY(launch_modit(M, fp64, st));
  }
  return EXO_OK;
}

extern "C" int exo_cross_section_modit(exo_ctx* c, int s, double T, double P, int precision,
                                       double dln_gamma, void* sigma, void* stream) {
  if (!c) return set_err(EXO_EINVAL, "ctx is NULL");
  if (s < 0 || s >= EXO_MAX_SPECIES) return set_err(EXO_EINVAL, "species slot %d out of range", s);
  if (!c->sp[s].set) return set_err(EXO_ENOTSET, "species slot %d not set", s);
  if (c->n_nu < 2) return set_err(EXO_ENOTSET, "grid not set");
  if (!c->eslog) return set_err(EXO_EINVAL, "MODIT needs a log-uniform grid");
  if (!(T > 0) || !(P >= 0) || !std::isfinite(T) || !std::isfinite(P))
    return set_err(EXO_EINVAL, "need T > 0 and P >= 0");
  if (precision != EXO_FP32_KAHAN && precision != EXO_FP64) return set_err(EXO_EINVAL, "bad precision");
  if (!(dln_gamma >= 1e-3) || !std::isfinite(dln_gamma)) return set_err(EXO_EINVAL, "dln_gamma must be >= 1e-3");
  if (!sigma) return set_err(EXO_EINVAL, "sigma_dev is NULL");
  HIP_TRY(hipSetDevice(c->device));
  std::lock_guard<std::mutex> g(c->mu);
  hipStream_t st = (hipStream_t)stream;
  Workspace& ws = c->ws;
  return with_ws(ws, st, [&]() -> int {
    int rc;
    if ((rc = ws.reserve(ws.params, 16 * sizeof(double)))) return rc;
    const double hp[2] = {T, P};
    double* dp = (double*)ws.params.p;
    if ((rc = ws.stage_params(hp, 2, dp, st))) return rc;
    return modit_opacity(c, ws, c->sp[s], dp, dp + 1, nullptr, 1, dln_gamma, precision == EXO_FP64,
                         (const double*)c->d_nu.p, c->h_nu.front(), c->h_nu.back(), c->n_nu, sigma, st);
  });
}

extern "C" int exo_cross_section(exo_ctx* c, int s, double T, double P, int precision, void* sigma,
                                 void* stream) {
  if (!c) return set_err(EXO_EINVAL, "ctx is NULL");
  if (s < 0 || s >= EXO_MAX_SPECIES || !c->sp[s].set) return set_err(EXO_ENOTSET, "species %d not set", s);
  if (c->n_nu < 2) return set_err(EXO_ENOTSET, "grid not set");
  if (!(T > 0) || !std::isfinite(T) || !(P >= 0) || !std::isfinite(P))
    return set_err(EXO_EINVAL, "need T > 0 and P >= 0");
  if (precision != EXO_FP32_KAHAN && precision != EXO_FP64 && precision != EXO_FP64_TILED)
    return set_err(EXO_EINVAL, "bad precision");
  if (!sigma) return set_err(EXO_EINVAL, "sigma_dev is NULL");
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> g(c->mu);
  Workspace& ws = c->ws;
  const bool fp64 = precision != EXO_FP32_KAHAN;
  const bool tiled64 = precision == EXO_FP64_TILED;
  // FP32 records carry the amplitude times a power of two chosen on the
  // device from the call's largest line strength, so that single-molecule
  // strengths (1e-30 .. 1e8 cm/molecule) stay far from both ends of the
  // FP32 range.
  // (T, P) go to the record kernel by value: no staging copy on this path
  return with_ws(ws, st, [&] {
    return species_opacity(c, ws, c->sp[s], nullptr, nullptr, nullptr, 1, 1.0, fp64, false,
                           (const double*)c->d_nu.p, c->n_nu, sigma, nullptr, st, T, P, !fp64, tiled64);
  });
}

// Bytes of scratch a plan carves (256-byte aligned pieces).
static size_t plan_bytes(const OpacityPlan& P) {
  size_t t = 0;
  for (size_t b : {P.rec, P.rect, P.rec64, P.tier, P.part, P.part_t}) t += (b + 255) & ~size_t(255);
  return t;
}

extern "C" int exo_cross_section_noalloc(exo_ctx* c, int s, double T, double P, int precision,
                                         void* sigma, void* stream) {
  if (!c) return set_err(EXO_EINVAL, "ctx is NULL");
  if (s < 0 || s >= EXO_MAX_SPECIES || !c->sp[s].set) return set_err(EXO_ENOTSET, "species %d not set", s);
  if (c->n_nu < 2) return set_err(EXO_ENOTSET, "grid not set");
  if (!(T > 0) || !std::isfinite(T) || !(P >= 0) || !std::isfinite(P))
    return set_err(EXO_EINVAL, "need T > 0 and P >= 0");
  if (precision != EXO_FP32_KAHAN && precision != EXO_FP64) return set_err(EXO_EINVAL, "bad precision");
  if (!sigma) return set_err(EXO_EINVAL, "sigma_dev is NULL");
  char* base = (char*)scratch_of(c->device);
  if (!base) return set_err(EXO_EDEVICE, "no scratch address on device %d", c->device);
  const bool fp64 = precision == EXO_FP64;
  const Species& sp = c->sp[s];
  const size_t need = plan_bytes(plan_opacity(sp.n, 1, c->n_nu, fp64, false));
  if (need > kNoAllocScratchBytes)
    return set_err(EXO_ENOMEM, "this cross-section needs %zu bytes of scratch; the no-allocation scratch holds %zu",
                   need, kNoAllocScratchBytes);
  HIP_TRY(hipSetDevice(c->device));
  std::lock_guard<std::mutex> g(c->mu);
  Workspace ws;   // carved from the scratch: reserves allocate nothing
  ws.no_alloc = true;
  ws.bind_arena(base, kNoAllocScratchBytes);
  return species_opacity(c, ws, sp, nullptr, nullptr, nullptr, 1, 1.0, fp64, false, (const double*)c->d_nu.p,
                         c->n_nu, sigma, nullptr, (hipStream_t)stream, T, P, !fp64);
}

// ---------------------------------------------------------------------------
// Emission
// ---------------------------------------------------------------------------
int exo::validate_atmos(const exo_ctx* c, const exo_atmos* a, int64_t* gb, int64_t* gl) {
  if (!a) return set_err(EXO_EINVAL, "atmos is NULL");
  if (c->n_nu < 2) return set_err(EXO_ENOTSET, "grid not set");
  if (a->n_layers < 2 || a->n_layers > kMaxLayers || !a->P_bar)
    return set_err(EXO_EINVAL, "need 2..%d layers", kMaxLayers);
  for (int i = 0; i < a->n_layers; ++i) {
    if (!(a->P_bar[i] > 0) || !std::isfinite(a->P_bar[i])) return set_err(EXO_EINVAL, "P must be > 0");
    if (i > 0 && !(a->P_bar[i] > a->P_bar[i - 1])) return set_err(EXO_EINVAL, "P must ascend (top -> bottom)");
  }
  if (a->T_layers) {
    for (int i = 0; i < a->n_layers; ++i)
      if (!(a->T_layers[i] > 1.0) || !std::isfinite(a->T_layers[i]))
        return set_err(EXO_EINVAL, "layer temperatures must be finite and exceed 1 K");
  } else if (!(a->T0_K > 0) || !std::isfinite(a->T0_K) || !std::isfinite(a->alpha)) {
    return set_err(EXO_EINVAL, "bad T0/alpha");
  }
  if (a->n_species < 1 || a->n_species > EXO_MAX_SPECIES || !a->species || !a->log10_mmr)
    return set_err(EXO_EINVAL, "bad species list");
  for (int m = 0; m < a->n_species; ++m) {
    const int s = a->species[m];
    if (s < 0 || s >= EXO_MAX_SPECIES || !c->sp[s].set) return set_err(EXO_ENOTSET, "species slot %d not set", s);
    if (!std::isfinite(a->log10_mmr[m]) || a->log10_mmr[m] > 0) return set_err(EXO_EINVAL, "log10_mmr must be finite and <= 0");
  }
  if (!(a->g_cgs > 0) || !(a->mmw > 0)) return set_err(EXO_EINVAL, "need g > 0 and mmw > 0");
  if (!std::isfinite(a->cia_alpha0) || a->cia_alpha0 < 0 || !std::isfinite(a->cia_Tpow) ||
      !std::isfinite(a->cia_slope) || !std::isfinite(a->cia_nu_c) || !(a->vmr_h2 >= 0))
    return set_err(EXO_EINVAL, "bad CIA parameters");
  if (a->bottom != EXO_FB_PLANCK_BOTTOM && a->bottom != EXO_FB_ZERO) return set_err(EXO_EINVAL, "bad bottom");
  if (a->opacity != EXO_OPACITY_LPF && a->opacity != EXO_OPACITY_MODIT) return set_err(EXO_EINVAL, "bad opacity");
  if (a->opacity == EXO_OPACITY_MODIT) {
    if (!c->eslog) return set_err(EXO_EINVAL, "MODIT needs a log-uniform grid");
    if (!(a->modit_dln_gamma >= 1e-3) || !std::isfinite(a->modit_dln_gamma))
      return set_err(EXO_EINVAL, "modit_dln_gamma must be >= 1e-3");
  }
  if (!a->T_layers) {
    const double Tmin = std::min(a->T0_K * std::pow(a->P_bar[0], a->alpha),
                                 a->T0_K * std::pow(a->P_bar[a->n_layers - 1], a->alpha));
    if (!(Tmin > 1.0) || !std::isfinite(Tmin)) return set_err(EXO_EINVAL, "layer temperatures must exceed 1 K");
  }
  int64_t b = a->grid_begin, l = a->grid_len;
  if (l == 0) {
    if (b != 0) return set_err(EXO_EINVAL, "grid_len 0 requires grid_begin 0");
    l = c->n_nu;
  }
  if (b < 0 || l < 2 || b + l > c->n_nu) return set_err(EXO_EINVAL, "model grid range outside the grid");
  *gb = b;
  *gl = l;
  return EXO_OK;
}

int exo::prepare_response(const exo_ctx* c, const exo_response* r, int64_t gl, RespDev* R) {
  if (!c->eslog) return set_err(EXO_EINVAL, "the response needs a log-uniform grid");
  if (!std::isfinite(r->rv_kms) || !std::isfinite(r->vsini_kms) || !std::isfinite(r->u1) ||
      !std::isfinite(r->u2) || !(r->R_inst > 0))
    return set_err(EXO_EINVAL, "bad response parameters");
  const double dv = c->dv_kms;
  if (!(r->vsini_kms >= 2.0 * dv)) return set_err(EXO_EINVAL, "vsini must span at least two grid spacings");
  if (1.0 - r->u1 / 3.0 - r->u2 / 6.0 <= 0) return set_err(EXO_EINVAL, "limb darkening gives a non-positive disk flux");
  const int64_t dmin = (int64_t)std::ceil((-r->vsini_kms - r->rv_kms) / dv) - 1;
  const int64_t dmax = (int64_t)std::floor((r->vsini_kms - r->rv_kms) / dv) + 1;
  R->dlo = dmin;
  R->nrot = dmax - dmin + 1;
  R->beta_ip = kCkms / (2.0 * std::sqrt(2.0 * std::log(2.0)) * r->R_inst);
  R->K = (int64_t)std::floor(6.0 * R->beta_ip / dv);
  R->dv = dv;
  R->rv = r->rv_kms;
  R->vsini = r->vsini_kms;
  R->u1 = r->u1;
  R->u2 = r->u2;
  R->ob = r->out_begin;
  R->ol = r->out_len;
  if (r->out_len < 1) return set_err(EXO_EINVAL, "out_len must be >= 1");
  const int64_t imin = r->out_begin - R->K, imax = r->out_begin + r->out_len - 1 + R->K;
  if (imin - dmax < 0 || imax - dmin > gl - 1)
    return set_err(EXO_EINVAL,
                   "output range [%lld, %lld) needs model points [%lld, %lld] outside [0, %lld)",
                   (long long)r->out_begin, (long long)(r->out_begin + r->out_len),
                   (long long)(imin - dmax), (long long)(imax - dmin), (long long)gl);
  return EXO_OK;
}

// Forward model into ws.tau (and ws.taut), then F0 into ws.F0.
int exo::forward_core(exo_ctx* c, Workspace& ws, const exo_atmos* a, int64_t gb, int64_t gl,
                      bool fp64, bool tangent, hipStream_t st, bool tiled64) {
  const int NL = a->n_layers, M = a->n_species;
  int rc;
  // parameter block: P, then the layer temperatures when the atmosphere gives them
  if ((rc = ws.reserve(ws.params, (size_t)2 * NL * sizeof(double)))) return rc;
  {
    std::vector<double> blk(a->P_bar, a->P_bar + NL);
    if (a->T_layers) blk.insert(blk.end(), a->T_layers, a->T_layers + NL);
    if ((rc = ws.stage_params(blk.data(), blk.size(), (double*)ws.params.p, st))) return rc;
  }
  if ((rc = ws.reserve(ws.layer, (size_t)6 * NL * sizeof(double)))) return rc;
  if ((rc = ws.reserve(ws.col, (size_t)M * NL * sizeof(double)))) return rc;
  double* lay = (double*)ws.layer.p;
  AtmosDev A{};
  A.nlay = NL;
  A.nspec = M;
  A.bottom = a->bottom;
  A.P = (const double*)ws.params.p;
  A.T_in = a->T_layers ? (const double*)ws.params.p + NL : nullptr;
  A.T0 = a->T0_K;
  A.alpha = a->alpha;
  A.g = a->g_cgs;
  A.mmw = a->mmw;
  A.cia_alpha0 = a->cia_alpha0;
  A.cia_Tpow = a->cia_Tpow;
  A.cia_slope = a->cia_slope;
  A.cia_nu_c = a->cia_nu_c;
  A.vmr_h2 = a->vmr_h2;
  for (int m = 0; m < M; ++m) {
    A.logx[m] = a->log10_mmr[m];
    A.mass[m] = c->sp[a->species[m]].mass;
  }
  A.T = lay;
  A.dP = lay + NL;
  A.lnP = lay + 2 * NL;
  A.cia = lay + 3 * NL;
  A.dcia = lay + 4 * NL;
  A.col = (double*)ws.col.p;
  HIP_TRY(launch_atmos(A, st));

  const size_t esz = fp64 ? sizeof(double) : sizeof(float);
  if ((rc = ws.reserve(ws.tau, (size_t)M * NL * gl * esz))) return rc;
  if (tangent && (rc = ws.reserve(ws.taut, (size_t)M * NL * gl * esz))) return rc;
  const bool modit = a->opacity == EXO_OPACITY_MODIT;
  if (modit && tangent) return set_err(EXO_EINVAL, "the MODIT opacity has no tangents");
  // every species' buffers fit in the largest plan, reserved once up front
  if (!modit && (rc = reserve_opacity(ws, plan_opacity_all(c, a, gl, fp64, tangent, tiled64)))) return rc;
  const double* d_nu = (const double*)c->d_nu.p + gb;
  for (int m = 0; m < M; ++m) {
    const Species& sp = c->sp[a->species[m]];
    char* out = (char*)ws.tau.p + (size_t)m * NL * gl * esz;
    void* out_t = tangent ? (char*)ws.taut.p + (size_t)m * NL * gl * esz : nullptr;
    if (modit)
      rc = modit_opacity(c, ws, sp, A.T, A.P, A.col + (size_t)m * NL, NL, a->modit_dln_gamma, fp64, d_nu,
                         c->h_nu[gb], c->h_nu[gb + gl - 1], gl, out, st);
    else
      rc = species_opacity(c, ws, sp, A.T, A.P, A.col + (size_t)m * NL, NL, 1.0, fp64, tangent, d_nu, gl,
                           out, out_t, st, 0.0, 0.0, false, tiled64);
    if (rc) return rc;
  }
  if ((rc = ws.reserve(ws.F0, (size_t)gl * sizeof(double)))) return rc;
  RtArgs R{};
  R.nu = d_nu;
  R.ng = gl;
  R.nlay = NL;
  R.nspec = M;
  R.bottom = a->bottom;
  R.T = A.T;
  R.cia = A.cia;
  R.dcia = A.dcia;
  R.cia_slope = a->cia_slope;
  R.cia_nu_c = a->cia_nu_c;
  R.tau = ws.tau.p;
  R.taut = ws.taut.p;
  R.F0 = (double*)ws.F0.p;
  HIP_TRY(launch_rt_forward(R, fp64, st));
  ws.last_rt = R;
  return EXO_OK;
}

int exo::apply_response(Workspace& ws, RespDev& R, const double* F0, void* out, bool out64,
                        hipStream_t st) {
  int rc;
  if ((rc = ws.reserve(ws.taps, (size_t)(3 * R.nrot + 2 * R.K + 1) * sizeof(double)))) return rc;
  double* t = (double*)ws.taps.p;
  R.rot = t;
  R.drot_rv = t + R.nrot;
  R.drot_vs = t + 2 * R.nrot;
  R.ip = t + 3 * R.nrot;
  HIP_TRY(launch_taps(R, st));
  if (!out) return EXO_OK;  // taps only (the adjoint needs them without a forward output)
  if ((rc = ws.reserve(ws.mid, (size_t)(R.ol + 2 * R.K) * sizeof(double)))) return rc;
  HIP_TRY(launch_response(R, F0, (double*)ws.mid.p, out, out64, st));
  return EXO_OK;
}

size_t exo::estimate_workspace(const exo_ctx* c, const exo_atmos* a, const exo_response* r,
                               bool fp64, bool vjp) {
  // mirrors the reservations of forward_core, apply_response and vjp_impl
  int64_t gb, gl;
  if (validate_atmos(c, a, &gb, &gl)) return 0;
  auto R = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t NL = a->n_layers, M = a->n_species;
  const size_t esz = fp64 ? sizeof(double) : sizeof(float);
  size_t t = R(2 * NL * 8) + R(6 * NL * 8) + R(M * NL * 8) + R(M * NL * gl * esz) + R(gl * 8);
  if (vjp) t += R(M * NL * gl * sizeof(float));
  if (a->opacity == EXO_OPACITY_MODIT) {
    size_t mb = 0;
    for (int m = 0; m < a->n_species; ++m)
      mb = std::max(mb, modit_workspace(c->sp[a->species[m]], c->h_nu[gb], c->h_nu[gb + gl - 1], gl,
                                        a->n_layers, fp64));
    t += mb;
  } else {
    const OpacityPlan P = plan_opacity_all(c, a, gl, fp64, vjp);
    for (size_t b : {P.rec, P.rect, P.rec64, P.part, P.part_t, P.tier}) t += b ? R(b) : 0;
  }
  int64_t nmid = 0;
  if (r) {
    RespDev RD{};
    if (prepare_response(c, r, gl, &RD)) return 0;
    nmid = RD.ol + 2 * RD.K;
    t += R((3 * RD.nrot + 2 * RD.K + 1) * 8) + R(nmid * 8);
  }
  if (vjp) {
    const size_t nbg = (gl + 255) / 256;
    t += R(gl * 8);
    if (r) t += R(nmid * 8) + R(2 * ((nmid + 255) / 256) * 8);
    t += R(NL * gl * 8) * 2 + R(nbg * NL * 8) + R(nbg * M * 8) + R((4 + M + NL) * 8);
  }
  return t;
}

int exo::emission_impl(exo_ctx* c, Workspace& ws, const exo_atmos* a, const exo_response* r,
                       int precision, void* flux, hipStream_t st) {
  int64_t gb, gl;
  int rc;
  if ((rc = validate_atmos(c, a, &gb, &gl))) return rc;
  if (precision != EXO_FP32_KAHAN && precision != EXO_FP64 && precision != EXO_FP64_TILED)
    return set_err(EXO_EINVAL, "bad precision");
  if (!flux) return set_err(EXO_EINVAL, "flux_dev is NULL");
  RespDev R{};
  if (r && (rc = prepare_response(c, r, gl, &R))) return rc;
  const bool fp64 = precision != EXO_FP32_KAHAN;
  if ((rc = forward_core(c, ws, a, gb, gl, fp64, false, st, precision == EXO_FP64_TILED))) return rc;
  if (r) return apply_response(ws, R, (const double*)ws.F0.p, flux, fp64, st);
  HIP_TRY(launch_cast_copy((const double*)ws.F0.p, flux, fp64, gl, st));
  return EXO_OK;
}

extern "C" int exo_emission_flux(exo_ctx* c, const exo_atmos* a, const exo_response* r, int precision,
                                 void* flux, void* stream) {
  if (!c) return set_err(EXO_EINVAL, "ctx is NULL");
  HIP_TRY(hipSetDevice(c->device));
  std::lock_guard<std::mutex> g(c->mu);
  hipStream_t st = (hipStream_t)stream;
  return with_ws(c->ws, st, [&] { return emission_impl(c, c->ws, a, r, precision, flux, st); });
}

int exo::vjp_impl(exo_ctx* c, Workspace& ws, const exo_atmos* a, const exo_response* r,
                  int precision, const void* cot, double* grad, double* dLdT, void* flux,
                  hipStream_t st, const float* data, const float* sigma, double* loss) {
  int64_t gb, gl;
  int rc;
  if ((rc = validate_atmos(c, a, &gb, &gl))) return rc;
  if (precision != EXO_FP32_KAHAN && precision != EXO_FP64 && precision != EXO_FP64_TILED)
    return set_err(EXO_EINVAL, "bad precision");
  if (a->opacity != EXO_OPACITY_LPF) return set_err(EXO_EINVAL, "the gradient is provided for the direct opacity");
  const bool fused = data != nullptr;
  // FP64 gradients run the tiled FP64 form (the plain form has no tangent mode)
  const bool fp64 = precision != EXO_FP32_KAHAN;
  if (fused && fp64) return set_err(EXO_EINVAL, "the fused likelihood gradient is provided for EXO_FP32_KAHAN");
  if (fused ? (!sigma || !loss || !grad) : (!cot || !grad))
    return set_err(EXO_EINVAL, fused ? "sigma_dev / loss_host / grad_host is NULL" : "cot_dev / grad_host is NULL");
  RespDev R{};
  if (r && (rc = prepare_response(c, r, gl, &R))) return rc;
  const int NL = a->n_layers, M = a->n_species;
  if ((rc = forward_core(c, ws, a, gb, gl, fp64, true, st, fp64))) return rc;
  const double* F0 = (const double*)ws.F0.p;
  const int64_t nbg = (gl + 255) / 256;
  if ((rc = ws.reserve(ws.F0bar, (size_t)gl * sizeof(double)))) return rc;
  double* F0bar = (double*)ws.F0bar.p;
  // Gaussian likelihood: the spectrum (into flux_dev or scratch), then its cotangent
  const int64_t nout = r ? R.ol : gl, nbL = (nout + 255) / 256;
  void* Fout = flux;
  if (fused) {
    if (!Fout) {
      if ((rc = ws.reserve(ws.lossF, (size_t)nout * sizeof(float)))) return rc;
      Fout = ws.lossF.p;
    }
    if ((rc = ws.reserve(ws.lossC, (size_t)nout * sizeof(float)))) return rc;
    if ((rc = ws.reserve(ws.lossP, (size_t)nbL * sizeof(double)))) return rc;
    cot = ws.lossC.p;
  }
  int64_t nbR = 0;
  if (r) {
    if ((rc = apply_response(ws, R, F0, Fout, fp64, st))) return rc;
    if (fused) HIP_TRY(launch_gauss_cot((const float*)Fout, data, sigma, nout, (float*)ws.lossC.p, (double*)ws.lossP.p, st));
    const int64_t nmid = R.ol + 2 * R.K;
    nbR = (nmid + 255) / 256;
    if ((rc = ws.reserve(ws.midbar, (size_t)nmid * sizeof(double)))) return rc;
    if ((rc = ws.reserve(ws.partR, (size_t)2 * nbR * sizeof(double)))) return rc;
    HIP_TRY(launch_response_vjp(R, F0, cot, fp64, (double*)ws.midbar.p, F0bar, gl,
                                (double*)ws.partR.p, nbR, st));
  } else {
    if (Fout) HIP_TRY(launch_cast_copy(F0, Fout, fp64, gl, st));
    if (fused) HIP_TRY(launch_gauss_cot((const float*)Fout, data, sigma, nout, (float*)ws.lossC.p, (double*)ws.lossP.p, st));
    HIP_TRY(launch_to_double(cot, fp64, F0bar, gl, st));
  }
  if ((rc = ws.reserve(ws.Fup, (size_t)NL * gl * sizeof(double)))) return rc;
  if ((rc = ws.reserve(ws.taubar, (size_t)NL * gl * sizeof(double)))) return rc;
  if ((rc = ws.reserve(ws.partT, (size_t)nbg * NL * sizeof(double)))) return rc;
  if ((rc = ws.reserve(ws.partX, (size_t)nbg * M * sizeof(double)))) return rc;
  if ((rc = ws.reserve(ws.gout, (size_t)(4 + M + NL) * sizeof(double)))) return rc;
  RtArgs Rt = ws.last_rt;
  Rt.F0bar = F0bar;
  Rt.Fup = (double*)ws.Fup.p;
  Rt.taubar = (double*)ws.taubar.p;
  Rt.partT = (double*)ws.partT.p;
  HIP_TRY(launch_rt_adjoint(Rt, fp64, nbg, st));
  HIP_TRY(launch_grad_x(Rt.taubar, ws.tau.p, fp64, M, NL, gl, (double*)ws.partX.p, nbg, st));
  const double* lay = (const double*)ws.layer.p;
  HIP_TRY(launch_grad_final(Rt.partT, nbg, (const double*)ws.partX.p, nbg, (const double*)ws.partR.p,
                            nbR, lay, lay + 2 * NL, NL, M, a->T0_K, a->T_layers ? 0 : 1,
                            (double*)ws.gout.p, st));
  std::vector<double> h(4 + M + NL), hl(fused ? nbL : 0);
  HIP_TRY(hipMemcpyAsync(h.data(), ws.gout.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  if (fused) HIP_TRY(hipMemcpyAsync(hl.data(), ws.lossP.p, hl.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (fused) {
    double sum = 0.0;
    for (double v : hl) sum += v;   // fixed order
    *loss = sum;
  }
  for (int k = 0; k < 2 + M + 2; ++k) grad[k] = h[k];
  if (dLdT)
    for (int n = 0; n < NL; ++n) dLdT[n] = h[4 + M + n];
  return EXO_OK;
}

extern "C" int exo_flux_vjp(exo_ctx* c, const exo_atmos* a, const exo_response* r, int precision,
                            const void* cot, double* grad, double* dLdT, void* flux, void* stream) {
  if (!c) return set_err(EXO_EINVAL, "ctx is NULL");
  HIP_TRY(hipSetDevice(c->device));
  std::lock_guard<std::mutex> g(c->mu);
  hipStream_t st = (hipStream_t)stream;
  return with_ws(c->ws, st, [&] { return vjp_impl(c, c->ws, a, r, precision, cot, grad, dLdT, flux, st); });
}

static int jvp_impl(exo_ctx* c, Workspace& ws, const exo_atmos* a, const exo_response* r,
                    int precision, const double* dth, const double* dTl, void* flux, void* dflux,
                    hipStream_t st) {
  int64_t gb, gl;
  int rc;
  if ((rc = validate_atmos(c, a, &gb, &gl))) return rc;
  if (precision != EXO_FP32_KAHAN)
    return set_err(EXO_EINVAL, "flux_jvp is provided for EXO_FP32_KAHAN");
  if (a->opacity != EXO_OPACITY_LPF) return set_err(EXO_EINVAL, "flux_jvp is provided for the direct opacity");
  if (!dth || !dflux) return set_err(EXO_EINVAL, "dtheta_host / dflux_dev is NULL");
  const int NL = a->n_layers, M = a->n_species;
  for (int k = 0; k < 2 + M + 2; ++k)
    if (!std::isfinite(dth[k])) return set_err(EXO_EINVAL, "non-finite dtheta");
  if (dTl)
    for (int n = 0; n < NL; ++n)
      if (!std::isfinite(dTl[n])) return set_err(EXO_EINVAL, "non-finite dT_layers");
  RespDev R{};
  if (r && (rc = prepare_response(c, r, gl, &R))) return rc;
  if ((rc = forward_core(c, ws, a, gb, gl, false, true, st))) return rc;
  // tangent parameter block: dlog10 X, then the per-layer dT
  if ((rc = ws.reserve(ws.gout, (size_t)(M + NL) * sizeof(double)))) return rc;
  {
    std::vector<double> blk(dth + 2, dth + 2 + M);
    if (dTl) blk.insert(blk.end(), dTl, dTl + NL);
    if ((rc = ws.stage_params(blk.data(), blk.size(), (double*)ws.gout.p, st))) return rc;
  }
  if ((rc = ws.reserve(ws.F0bar, (size_t)gl * sizeof(double)))) return rc;
  const double* lay = (const double*)ws.layer.p;
  JvpArgs J{};
  J.lnP = lay + 2 * NL;
  J.dlogx = (const double*)ws.gout.p;
  J.dTl = dTl ? (const double*)ws.gout.p + M : nullptr;
  J.powerlaw = a->T_layers ? 0 : 1;
  J.dT0_rel = a->T_layers ? 0.0 : dth[0] / a->T0_K;
  J.dalpha = a->T_layers ? 0.0 : dth[1];
  J.dF0 = (double*)ws.F0bar.p;
  HIP_TRY(launch_rt_jvp(ws.last_rt, J, st));
  const double* F0 = (const double*)ws.F0.p;
  if (r) {
    // taps (and the spectrum when asked for), then the tangent of both stages
    if ((rc = apply_response(ws, R, F0, flux, false, st))) return rc;
    if ((rc = ws.reserve(ws.midbar, (size_t)(R.ol + 2 * R.K) * sizeof(double)))) return rc;
    HIP_TRY(launch_response_jvp(R, F0, J.dF0, dth[2 + M], dth[2 + M + 1], (double*)ws.midbar.p,
                                (float*)dflux, st));
  } else {
    if (flux) HIP_TRY(launch_cast_copy(F0, flux, false, gl, st));
    HIP_TRY(launch_cast_copy(J.dF0, dflux, false, gl, st));
  }
  return EXO_OK;
}

extern "C" int exo_flux_jvp(exo_ctx* c, const exo_atmos* a, const exo_response* r, int precision,
                            const double* dth, const double* dTl, void* flux, void* dflux,
                            void* stream) {
  if (!c) return set_err(EXO_EINVAL, "ctx is NULL");
  HIP_TRY(hipSetDevice(c->device));
  std::lock_guard<std::mutex> g(c->mu);
  hipStream_t st = (hipStream_t)stream;
  return with_ws(c->ws, st, [&] { return jvp_impl(c, c->ws, a, r, precision, dth, dTl, flux, dflux, st); });
}

extern "C" int exo_loss_grad(exo_ctx* c, const exo_atmos* a, const exo_response* r, int precision,
                             const void* data, const void* sigma, double* loss, double* grad, double* dLdT,
                             void* flux, void* stream) {
  if (!c) return set_err(EXO_EINVAL, "ctx is NULL");
  if (!data) return set_err(EXO_EINVAL, "data_dev is NULL");
  HIP_TRY(hipSetDevice(c->device));
  std::lock_guard<std::mutex> g(c->mu);
  hipStream_t st = (hipStream_t)stream;
  return with_ws(c->ws, st, [&] {
    return vjp_impl(c, c->ws, a, r, precision, nullptr, grad, dLdT, flux, st, (const float*)data,
                    (const float*)sigma, loss);
  });
}

extern "C" int exo_broaden(exo_ctx* c, int64_t gb, int64_t gl, const exo_response* r,
                           const void* F0, void* out, void* stream) {
  if (!c) return set_err(EXO_EINVAL, "ctx is NULL");
  if (c->n_nu < 2) return set_err(EXO_ENOTSET, "grid not set");
  if (!r || !F0 || !out) return set_err(EXO_EINVAL, "NULL argument");
  if (gl == 0) {
    if (gb != 0) return set_err(EXO_EINVAL, "grid_len 0 requires grid_begin 0");
    gl = c->n_nu;
  }
  if (gb < 0 || gl < 2 || gb + gl > c->n_nu) return set_err(EXO_EINVAL, "grid range outside the grid");
  HIP_TRY(hipSetDevice(c->device));
  std::lock_guard<std::mutex> g(c->mu);
  RespDev R{};
  int rc;
  if ((rc = prepare_response(c, r, gl, &R))) return rc;
  hipStream_t st = (hipStream_t)stream;
  return with_ws(c->ws, st, [&] { return apply_response(c->ws, R, (const double*)F0, out, true, st); });
}

// ---------------------------------------------------------------------------
// Diagnostics
// ---------------------------------------------------------------------------
extern "C" int exo_hjert_f32(int64_t n, const float* x, const float* a, float* H, float* L, void* stream) {
  if (n < 0 || (n > 0 && (!x || !a || !H))) return set_err(EXO_EINVAL, "bad arguments");
  if (n == 0) return EXO_OK;
  HIP_TRY(launch_hjert_f32(n, x, a, H, L, (hipStream_t)stream));
  return EXO_OK;
}

extern "C" int exo_hjert_f64(int64_t n, const double* x, const double* a, double* H, void* stream) {
  if (n < 0 || (n > 0 && (!x || !a || !H))) return set_err(EXO_EINVAL, "bad arguments");
  if (n == 0) return EXO_OK;
  HIP_TRY(launch_hjert_f64(n, x, a, H, (hipStream_t)stream));
  return EXO_OK;
}

extern "C" int exo_trans2e3(int64_t n, const double* x, double* T, double* dT, void* stream) {
  if (n < 0 || (n > 0 && (!x || !T))) return set_err(EXO_EINVAL, "bad arguments");
  if (n == 0) return EXO_OK;
  HIP_TRY(launch_trans2e3(n, x, T, dT, (hipStream_t)stream));
  return EXO_OK;
}
