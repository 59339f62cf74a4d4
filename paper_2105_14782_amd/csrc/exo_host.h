// Host-side internals of the exohip library (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/exohip.h"
#include "exo_launch.h"

namespace exo {

// Layers per atmosphere (per-call parameter blocks are staged through a
// fixed pinned buffer).
constexpr int kMaxLayers = 4096;
// FP32 far-tier table of a workspace: per layer the gamma^2 maximum bits,
// squared reach, t3 flag and squared outer reach, then the strength maximum
// (8 B) and output scale (4 B) of an adaptive cross-section scale.
constexpr size_t kTierBytes = (size_t)kMaxLayers * 16 + 16;

int set_err(int code, const char* fmt, ...);
bool fail_alloc_hook();

// Grow-only device allocation.
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  bool owned = true;   // false: carved from a workspace arena
  int reserve(size_t bytes);
  void release();
};

// All scratch of one in-flight evaluation.  One per context for the
// synchronous API; the serving engine owns one per slot.
struct Workspace {
  static constexpr size_t kStageDoubles = 1 << 14;
  DevBuf rec, rect, rec64, tier, tau, taut, part, part_t, F0, F0bar, mid, midbar, Fup, taubar, layer,
      col, taps, partT, partX, partR, gout, params, mlines, mpart, mrows0, mrows1, lossF, lossC, lossP;
  // tier.p when its gamma^2 maximum bits are known to be zero (every FP32
  // Voigt chunk leaves them zero); otherwise they are cleared before use
  void* tier_zeroed = nullptr;
  double* h_stage = nullptr;     // pinned staging for per-call parameters
  hipEvent_t stage_ev = nullptr; // guards h_stage reuse
  RtArgs last_rt{};
  // Arena mode (serving): buffers are carved from [arena, arena + arena_cap)
  // instead of being allocated; no allocation happens while serving.
  char* arena = nullptr;
  // No device work that allocates or records a memset: scratch is cleared by
  // kernels and the Voigt launches are not profiled (events).
  bool no_alloc = false;
  size_t arena_cap = 0, arena_used = 0;
  int reserve(DevBuf& b, size_t bytes);
  void bind_arena(char* base, size_t cap);
  std::vector<DevBuf*> bufs() {
    return {&rec, &rect, &rec64, &tier, &tau, &taut, &part, &part_t, &F0, &F0bar, &mid, &midbar,
            &Fup, &taubar, &layer, &col, &taps, &partT, &partX, &partR, &gout, &params,
            &mlines, &mpart, &mrows0, &mrows1, &lossF, &lossC, &lossP};
  }
  hipEvent_t done_ev = nullptr;  // end of the last evaluation using this workspace
  hipStream_t last_st = nullptr;
  // Order this evaluation after the previous one when it runs on another stream.
  int begin(hipStream_t st);
  int end(hipStream_t st);
  ~Workspace();
  void release();
  int stage_params(const double* host, size_t n, double* dev, hipStream_t st);
  size_t bytes() const {
    size_t b = 0;
    for (const DevBuf* x : {&rec, &rect, &rec64, &tier, &tau, &taut, &part, &part_t, &F0, &F0bar, &mid,
                            &midbar, &Fup, &taubar, &layer, &col, &taps, &partT, &partX, &partR,
                            &gout, &params})
      b += x->cap;
    return b;
  }
};

struct Species {
  bool set = false;
  int64_t n = 0;
  DevBuf nu_c, S0, E_low, alpha_ref, n_texp, gamma_nat, qr, perm;   // perm: caller index of sorted line i
  bool has_gnat = false;
  double mass = 0;
  int qr_kind = 0, n_qr = 0;
  double nu_lo = 0, nu_hi = 0;
  std::vector<double> h_nu_c;   // sorted centres (host copy: window ranges without a device round trip)
  void release();
};

struct ProfRec {
  hipEvent_t a = nullptr, b = nullptr;
  double evals = 0;
};

}  // namespace exo

struct exo_ctx {
  int device = 0;
  exo::Species sp[EXO_MAX_SPECIES];
  exo::DevBuf d_nu;
  std::vector<double> h_nu;
  int64_t n_nu = 0;
  bool eslog = false;
  double dv_kms = 0;
  exo::Workspace ws;
  std::mutex mu;  // serialises the synchronous API on this context
  bool profile = false;
  std::mutex prof_mu;
  std::vector<exo::ProfRec> prof;
  exo::DevBuf prof_near;  // near-tier pair counter of the profiled FP32 launches
};

namespace exo {
struct OpacityPlan {
  int nlc;  // layers per record chunk
  size_t rec, rect, rec64, part, part_t;
  size_t tier;  // FP32 far tier: per layer of a chunk, the gamma^2 maximum bits and the squared reach
};
// tiled64 (with fp64): the tiled FP64 form's records and splits.
OpacityPlan plan_opacity(int64_t n_lines, int nlay, int64_t ng, bool fp64, bool tangent, bool tiled64 = false);
// component-wise largest plan over the species of an atmosphere
OpacityPlan plan_opacity_all(const exo_ctx* c, const exo_atmos* a, int64_t gl, bool fp64, bool tangent,
                             bool tiled64 = false);
int reserve_opacity(Workspace& ws, const OpacityPlan& P);
// Upper bound of the workspace bytes one evaluation reserves (arena sizing).
size_t estimate_workspace(const exo_ctx* c, const exo_atmos* a, const exo_response* r, bool fp64,
                          bool vjp);
int voigt_launch_profiled(exo_ctx* c, const VoigtArgs& A, bool fp64, bool tan, hipStream_t st,
                          bool tiled = false);
// d_T == nullptr: one layer at (T_one, P_one), passed to the kernels by value.
// adaptive_scale (FP32, one layer at (T_one, P_one)): amp_scale is replaced
// by a power of two chosen on the device from the largest line strength.
// tiled64 (with fp64): the tiled FP64 form instead of the plain one.
int species_opacity(exo_ctx* c, Workspace& ws, const Species& sp, const double* d_T,
                    const double* d_P, const double* d_col, int nlay, double amp_scale, bool fp64,
                    bool tangent, const double* d_nu, int64_t ng, void* out, void* out_t,
                    hipStream_t st, double T_one = 0.0, double P_one = 0.0, bool adaptive_scale = false,
                    bool tiled64 = false);
// MODIT cross-sections (d_col == NULL) or optical depths col_n sigma clamped
// at zero, of nlay layers, from the lines with nu_lo <= nu_c <= nu_hi.
int modit_opacity(exo_ctx* c, Workspace& ws, const Species& sp, const double* d_T, const double* d_P,
                  const double* d_col, int nlay, double dlng, bool fp64, const double* d_nu, double nu_lo,
                  double nu_hi, int64_t ng, void* out, hipStream_t st);
size_t modit_workspace(const Species& sp, double nu_lo, double nu_hi, int64_t ng, int nlay, bool fp64);
int validate_atmos(const exo_ctx* c, const exo_atmos* a, int64_t* gb, int64_t* gl);
int prepare_response(const exo_ctx* c, const exo_response* r, int64_t gl, RespDev* R);
int forward_core(exo_ctx* c, Workspace& ws, const exo_atmos* a, int64_t gb, int64_t gl, bool fp64,
                 bool tangent, hipStream_t st, bool tiled64 = false);
int apply_response(Workspace& ws, RespDev& R, const double* F0, void* out, bool out64, hipStream_t st);
int emission_impl(exo_ctx* c, Workspace& ws, const exo_atmos* a, const exo_response* r,
                  int precision, void* flux, hipStream_t st);
// With data != nullptr the cotangent is that of the Gaussian likelihood
// 1/2 sum ((data - F)/sigma)^2, formed on the device from this pass's F;
// its value goes to *loss.
int vjp_impl(exo_ctx* c, Workspace& ws, const exo_atmos* a, const exo_response* r, int precision,
             const void* cot, double* grad, double* dLdT, void* flux, hipStream_t st,
             const float* data = nullptr, const float* sigma = nullptr, double* loss = nullptr);
}  // namespace exo
