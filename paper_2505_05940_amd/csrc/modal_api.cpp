// Host side of libmodal: validation, FP64 scheme coefficients, the work
// partition, device memory, launches and graph capture.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <queue>
#include <atomic>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/modal.h"
#include "kernels.h"

namespace modal {
hipError_t launch_step(const StepParams& P, int gm, int nw, int n_wg, size_t lds_bytes, hipStream_t s);
hipError_t launch_advance(long long* step_base, int n, hipStream_t s);
hipError_t launch_ctr_fill(const InstDev* inst, int batch, const long long* step_base, unsigned int* ctr,
                           hipStream_t s);
hipError_t launch_check(const float* H, const InstDev* inst, int batch, int* out, hipStream_t s);
hipError_t step_occupancy(int* blocks_per_cu, int gm, int nw, size_t lds_bytes, bool res = false);
hipError_t launch_chip(const StepParams& P, int nt_tile, int rows, int n_wg, hipStream_t s);
hipError_t launch_chip_wave(const StepParams& P, int m, int n_wg, hipStream_t s);
bool chip_shape(int max_nt, int max_rows, int& nt_tile, int& rows);
hipError_t launch_grad(const GradParams& P, int gm, bool tangent, int nw, bool split, int n_wg, size_t lds,
                       hipStream_t s);
hipError_t grad_occupancy(int* blocks, int gm, bool tangent, int nw, bool split, size_t lds);
hipError_t launch_restore(const float* ckpt, long long slot, int mode_floats, const InstDev* inst,
                          const UnitDev* unit, int n_units, float* state, int state_floats,
                          long long* step_base, long long step, unsigned int* ctr, hipStream_t s);
hipError_t launch_shared(const SharedParams& P, int kt, int kc, int jt, int n_wg, hipStream_t s);
hipError_t launch_row_sum(const float* rrec, int seg_len, int rows, float* acc, hipStream_t s);
hipError_t launch_tf_response(const float2* coef, const int* mode_off, int batch, const FFc* z, int n_freq,
                              FFc* H, hipStream_t s);
hipError_t launch_tf_grad(const float2* coef, const int* mode_off, int batch, int max_modes, const FFc* z,
                          int n_freq, const FFc* gH, float2* g_coef, hipStream_t s);
hipError_t launch_sym_check(const float* H, int nin, int nt, int* bad, hipStream_t s);
hipError_t launch_tensor_grad(const TGradJob* jobs, int n_jobs, int max_nin, int max_nt, const float* rec_x,
                              const float* urec, const float* trec, int mode_floats, int rows_total,
                              int seg_len, hipStream_t s);
hipError_t launch_lin_sum(const LinMode* modes, const FFc* amp, const FFc* ztab, const LinSeg* segs,
                          int n_segs, long long max_len, float* out, hipStream_t s);
hipError_t launch_lin_sum_ff(const LinMode* modes, const FFc* amp, const FFc* ztab, const LinSeg* segs,
                             int n_segs, long long max_len, float2* out, hipStream_t s);
hipError_t launch_lin_amp(const LinInit* init, const LinMode* modes, int M, const float* e_ext, FFc* amp,
                          FFc* ztab, hipStream_t s);
hipError_t launch_lin_conv(const LinForced* forced, int n_forced, const float2* h, long long h_stride,
                           const float* e_ext, long long base, long long n_steps, long long window,
                           float* y, long long y_stride, hipStream_t s);
}  // namespace modal

using namespace modal;

// Device memory of modal_run_noalloc: the arrival words and partial forces
// of split instances, which modal_run keeps in memory the context allocated.
// One copy per GPU, held until the process ends.  In host code the name is
// only a stand-in; the address of each device's copy comes from
// hipGetSymbolAddress (modal_init, once per device) and is the one passed to
// kernels.
constexpr size_t kScratchBytes = (size_t)16 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

thread_local std::string g_err;

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// Address of the current device's scratch copy, resolved on first use per
// device (with that device current).
hipError_t resolve_scratch(int dev, void** out) {
  *out = nullptr;
  if (dev < 0 || dev >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                               \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return fail(MODAL_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));  \
  } while (0)

bool finite_all(const double* v, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

int round4(int n) { return (n + 3) & ~3; }

// float-float split of an FP64 value
void split(double v, float& hi, float& lo) {
  hi = (float)v;
  lo = (float)(v - (double)hi);
}

// FP64 complex -> float-float complex
FFc ffc(std::complex<double> v) {
  FFc r;
  split(v.real(), r.rh, r.rl);
  split(v.imag(), r.ih, r.il);
  return r;
}

struct Coef {
  double m, p, r;
};

// Per-mode recursion q+ = g q + p q- + r f, returned as (m = g + p - 1, p, r).
// Stormer-Verlet (paper: Sec. 3.2): r = 2T^2/(2 + 2 gamma T),
// g = r (2/T^2 - omega^2), p = r (-1/T^2 + gamma/T); hence
// p = -(1 - gamma T)/(1 + gamma T) and m = -r omega^2 exactly.
// Transfer function (impulse invariance, Sec. 3.2, denominator
// z^2 + a1 z + a2): g = -a1 = 2 e^{-gamma T} cos(w T), p = -a2 = -e^{-2 gamma T},
// r = T e^{-gamma T} sin(w T)/w with w = sqrt(omega^2 - gamma^2) (force per
// unit mass), and m = -(1 - e^{-gamma T})^2 - 4 e^{-gamma T} sin^2(w T/2).
template <class S>
void coefficients_t(int scheme, S omega, S gamma, double T, S& m, S& p, S& r) {
  using std::exp;
  using std::sin;
  using std::sqrt;
  if (scheme == MODAL_SCHEME_SV) {
    r = T * T / (1.0 + gamma * T);
    p = -(1.0 - gamma * T) / (1.0 + gamma * T);
    m = -r * omega * omega;
  } else {
    const S w = sqrt(omega * omega - gamma * gamma);
    const S e = exp(-gamma * T);
    const S em1 = e - 1.0;
    const S sh = sin(0.5 * w * T);
    p = -e * e;
    r = T * e * sin(w * T) / w;
    m = -em1 * em1 - 4.0 * e * sh * sh;
  }
}

Coef coefficients(int scheme, double omega, double gamma, double T) {
  Coef c;
  if (scheme == MODAL_SCHEME_SV) {
    coefficients_t<double>(scheme, omega, gamma, T, c.m, c.p, c.r);
  } else {
    // expm1 keeps m's relative accuracy when gamma T is tiny
    const double w = std::sqrt(omega * omega - gamma * gamma);
    const double e = std::exp(-gamma * T);
    const double em1 = std::expm1(-gamma * T);
    const double sh = std::sin(0.5 * w * T);
    c.p = -e * e;
    c.r = T * e * std::sin(w * T) / w;
    c.m = -em1 * em1 - 4.0 * e * sh * sh;
  }
  return c;
}

// d(m, p, r)/d(omega) and /d(gamma) by the complex step (exact to rounding).
void coefficient_derivs(int scheme, double omega, double gamma, double T, double dw[3], double dg[3]) {
  using C = std::complex<double>;
  const double h = 1e-30;
  C m, p, r;
  coefficients_t<C>(scheme, C(omega, h), C(gamma, 0.0), T, m, p, r);
  dw[0] = m.imag() / h;
  dw[1] = p.imag() / h;
  dw[2] = r.imag() / h;
  coefficients_t<C>(scheme, C(omega, 0.0), C(gamma, h), T, m, p, r);
  dg[0] = m.imag() / h;
  dg[1] = p.imag() / h;
  dg[2] = r.imag() / h;
}

// Schur-Cohn (Jury) test for z^2 - g z - p: both roots in |z| <= 1.
bool stable(const Coef& c) {
  const double g = c.m - c.p + 1.0;
  const double tol = 1e-12;
  return std::fabs(c.p) <= 1.0 + tol && std::fabs(g) <= 1.0 - c.p + tol;
}

struct Unit {
  int inst, row0, row1, slab;
  double cost;
};

}  // namespace

struct modal_ctx {
  int batch = 0, scheme = 0, flags = 0, chunk = 0;
  int device = 0;  // the device current at modal_init
  double fs = 0;
  int n_wg = 0, n_units = 0, n_split = 0, occ = 0, gm = 1, nw = 4;
  int res_stride = 0;  // > 0: LDS-resident state (one unit per workgroup)
  // > 0: the on-chip kernel (one workgroup per instance, tensor in
  // registers), with chip_nt tensor columns per lane and chip_rows rows per
  // wave, and its register layouts (one ChipMap per instance)
  int chip_nt = 0, chip_rows = 0;
  ChipMap* dChip = nullptr;
  // > 0: the on-chip kernel for instances without a tensor, one wave each,
  // with this many modes per lane
  int chip_wave = 0;
  // waves of the reverse kernel without and with a tangent tensor (its
  // reduction space per wave holds two or three reduced vectors per row)
  int nw_grad[2] = {4, 4};
  size_t grad_lds_v[2] = {0, 0};
  double makespan = 0, mean_load = 0;
  size_t lds_bytes = 0;
  long long coupling_bytes = 0, padded_bytes = 0, steps = 0;
  int state_floats = 0, mode_floats = 0;
  std::vector<int> nt, unit_state_of_inst, inst_mode_off;
  std::vector<float> state0;  // x_hi, x_lo, d_hi, d_lo concatenated
  // device
  float* dH = nullptr;
  void* dMeta = nullptr;     // InstDev, UnitDev, wg_begin
  float* dCoef = nullptr;    // 9 per-mode arrays
  float* dState = nullptr;   // 4 per-unit arrays
  float* dPart = nullptr;
  unsigned int* dCtr = nullptr;  // arrival words, n_ctr of them (one per slab)
  int n_ctr = 0;
  int* dFlags = nullptr;
  long long* dStep = nullptr;
  float* dE = nullptr;
  StepParams P{};
  long long h_floats = 0, part_floats = 0;
  int red_floats = 0;
  std::vector<UnitDev> units;
  std::vector<InstDev> inst_host;
  std::vector<double> omega, gamma;  // concatenated over instances
  std::vector<int> kind;
  // gradient buffers (allocated on first modal_grad)
  float *dHd = nullptr, *dCkpt = nullptr, *dRec = nullptr, *dAdj = nullptr, *dAcc = nullptr,
        *dGPart = nullptr;
  unsigned int* dGCtr = nullptr;
  long long ckpt_floats = 0, rec_floats = 0;
  // Checkpoints recorded by the forward runs of a gradient context, every
  // kRunCkpt steps from step 0: valid for the steps [0, ckpt_upto) run with
  // the current tensors unless broken (a gap, or a buffer that had to grow
  // mid-run); modal_grad with the same spacing reuses them instead of running
  // the forward pass again.
  long long ckpt_upto = 0;
  bool ckpt_broken = false;
  bool run_ckpt = false;  // the run being enqueued records checkpoints
  // With them, while it fits kRecAllBytes, the whole trajectory (q and d per
  // step, FP32 high parts, laid out like a segment's record): modal_grad then
  // skips the segment recomputes too.  Valid for [0, rec_upto).
  float* dRecAll = nullptr;
  long long recall_cap = 0;  // steps the buffer holds
  long long rec_upto = 0;
  bool run_rec = false;
  // modal_run_noalloc advanced the steps on arrival words of its own: the
  // context's words must be brought up to date before its next launch
  bool ctr_stale = false;
  bool tangent = false;
  // per-row (in-plane) gradient pools: rows of all VK instances
  int rows_total = 0;
  float *dRrec = nullptr, *dRacc = nullptr;
  long long rrec_floats = 0;
  // full tensor gradient: u and (eta, V.u) records of a segment, job list
  float *dUrec = nullptr, *dTrec = nullptr;
  long long urec_floats = 0, trec_floats = 0;
  TGradJob* dTJobs = nullptr;
  int tjobs_cap = 0;
  // parity-blocked tensors
  int n_blocked = 0;
  long long dense_bytes = 0;
  int4* dJmap = nullptr;
  std::vector<std::vector<int>> mode_slot;  // per instance: caller mode -> internal slot
  // linear closed-form path: per mode roots, amplitude sets [free | post |
  // impulse], and the output-space impulse response of every forced instance
  // over its excitation window; runs are evaluated at absolute steps
  bool linear = false;
  std::vector<std::complex<double>> lz1, lz2, lA, lB, lC;  // per mode (caller order)
  std::vector<double> lc, lb;                               // output and force weights
  std::vector<char> lconj;                                  // complex-conjugate root pair
  std::vector<std::vector<float>> le;                       // excitation per instance
  std::vector<int> lin_moff, lin_mc;  // device mode ranges; [moff, mc) conjugate pairs
  LinMode* dLinModes = nullptr;
  LinInit* dLinInit = nullptr;
  FFc* dLinAmp = nullptr;      // [3 sets][modes][2 roots]
  FFc* dLinTab = nullptr;      // z1^l, l < 64, per mode
  LinSeg* dLinSeg = nullptr;
  LinForced* dLinForced = nullptr;
  float2* dLinH = nullptr;     // float-float impulse responses of forced instances
  int n_forced = 0;
  long long lin_h_stride = 1, lin_max_exc = 0;
  // shared-tensor path
  bool shared = false;
  int sh_kt = 0, sh_kc = 0, sh_jt = 0;
  long long flops = 0;
  float *dShA = nullptr, *dShS2 = nullptr;
  SharedParams SP{};
  hipStream_t cap_stream = nullptr;  // private stream used only for graph capture
  struct Graph {
    int64_t n, stride;
    float* y;
    hipGraphExec_t exec;
  };
  std::vector<Graph> graphs;
};

namespace {

void free_ctx(modal_ctx* c) {
  if (!c) return;
  for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  void* ptrs[] = {c->dH,   c->dMeta, c->dCoef, c->dState, c->dPart, c->dCtr, c->dFlags,
                  c->dStep, c->dE,   c->dHd,   c->dCkpt,  c->dRec,  c->dAdj, c->dAcc,
                  c->dGPart, c->dGCtr, c->dShA, c->dShS2, c->dJmap, c->dRrec, c->dRacc,
                  c->dLinModes, c->dLinInit, c->dLinAmp, c->dLinSeg, c->dLinForced, c->dLinH,
                  c->dLinTab, c->dUrec, c->dTrec, c->dTJobs, c->dRecAll, c->dChip};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete c;
}

template <class T>
int dalloc(T** p, size_t bytes) {
  if (bytes == 0) bytes = 256;
  hipError_t e = hipMalloc((void**)p, bytes);
  if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? MODAL_ENOMEM : MODAL_EHIP,
                                   std::string("hipMalloc: ") + hipGetErrorString(e));
  return MODAL_OK;
}

// Stored rows of a tensor row swept at once: as many as kSweepLoads float4
// loads per lane cover (nc float4 columns each), at most nt.
void choose_sweep(int nt, int nc, int& qs, int& J) {
  J = kSweepLoads;
  qs = std::max(1, std::min(nt, (kWave * J) / nc));
}

int validate(const modal_desc* d) {
  if (!d) return fail(MODAL_EINVAL, "desc is NULL");
  if (d->batch < 1 || !d->inst) return fail(MODAL_EINVAL, "batch < 1 or inst NULL");
  if (!(d->fs > 0) || !std::isfinite(d->fs)) return fail(MODAL_EINVAL, "fs must be > 0");
  if (d->scheme != MODAL_SCHEME_SV && d->scheme != MODAL_SCHEME_TF)
    return fail(MODAL_EINVAL, "unknown scheme");
  if ((d->waves != 0 && d->waves != 1 && d->waves != 4 && d->waves != 8) || d->max_workgroups < 0 ||
      d->chunk_steps < 0 || d->barrier_us < 0 || d->split_cost_kb < 0 || d->split_cost_kb > (1 << 20))
    return fail(MODAL_EINVAL, "waves (0, 1, 4 or 8), max_workgroups, chunk_steps, barrier_us or split_cost_kb");
  const double T = 1.0 / d->fs;
  for (int b = 0; b < d->batch; ++b) {
    const modal_instance& I = d->inst[b];
    const std::string at = " (instance " + std::to_string(b) + ")";
    if (I.kind < MODAL_KIND_LINEAR || I.kind > MODAL_KIND_VK) return fail(MODAL_EINVAL, "kind" + at);
    if (I.n_t < 1 || I.n_t > kMaxModes) return fail(MODAL_EINVAL, "n_t outside 1..1024" + at);
    if (I.reserved != 0) return fail(MODAL_EINVAL, "reserved must be 0" + at);
    if (!I.omega || !I.gamma || !I.x0 || !I.xm1 || !I.c_out)
      return fail(MODAL_EINVAL, "NULL per-mode array" + at);
    if (!finite_all(I.omega, I.n_t) || !finite_all(I.gamma, I.n_t) || !finite_all(I.x0, I.n_t) ||
        !finite_all(I.xm1, I.n_t) || !finite_all(I.c_out, I.n_t))
      return fail(MODAL_EINVAL, "non-finite per-mode input" + at);
    if (I.kind == MODAL_KIND_VK) {
      if (I.n_in < 1 || !I.H) return fail(MODAL_EINVAL, "VK needs n_in >= 1 and H" + at);
      if (I.h_row_scale && !finite_all(I.h_row_scale, I.n_in))
        return fail(MODAL_EINVAL, "non-finite h_row_scale" + at);
      if (I.mode_class)
        for (int k = 0; k < I.n_t; ++k)
          if (I.mode_class[k] > 3) return fail(MODAL_EINVAL, "mode_class outside 0..3" + at);
    } else if (I.n_in != 0 || I.h_row_scale || I.mode_class) {
      return fail(MODAL_EINVAL, "n_in must be 0 and h_row_scale, mode_class NULL unless VK" + at);
    }
    if (I.kind == MODAL_KIND_TENSION) {
      if (!I.lambda || !finite_all(I.lambda, I.n_t) || !std::isfinite(I.kappa))
        return fail(MODAL_EINVAL, "TENSION needs finite lambda and kappa" + at);
    }
    if (I.n_exc < 0 || (I.n_exc > 0 && (!I.e_ext || !I.b_ext)))
      return fail(MODAL_EINVAL, "forcing needs b_ext and e_ext" + at);
    if (I.b_ext && !finite_all(I.b_ext, I.n_t)) return fail(MODAL_EINVAL, "non-finite b_ext" + at);
    for (int64_t i = 0; i < I.n_exc; ++i)
      if (!std::isfinite(I.e_ext[i])) return fail(MODAL_EINVAL, "non-finite e_ext" + at);
    for (int k = 0; k < I.n_t; ++k) {
      // a mode without loss (gamma = 0) is rejected too: every scheme's
      // damping factors then sit on the unit circle, where rounding decides
      // growth or decay
      if (!(I.gamma[k] > 0)) return fail(MODAL_EUNSTABLE, "gamma <= 0" + at);
      if (I.omega[k] < 0) return fail(MODAL_EINVAL, "omega < 0" + at);
      if (d->scheme == MODAL_SCHEME_TF && !(I.omega[k] > I.gamma[k]))
        return fail(MODAL_EUNSTABLE, "TF needs omega > gamma" + at);
      if (!stable(coefficients(d->scheme, I.omega[k], I.gamma[k], T)))
        return fail(MODAL_EUNSTABLE, "mode " + std::to_string(k) + " unstable" + at);
    }
  }
  return MODAL_OK;
}

// Checkpoint spacing of forward runs in gradient contexts (modal_grad's
// default).
constexpr int kRunCkpt = 512;
// Largest whole-trajectory record a gradient context keeps (bytes).
constexpr double kRecAllBytes = 2.0 * 1073741824.0;

// A batch of at most one instance per CU whose dense tensors together stay
// below this many bytes per step is bound by each step's latency, not by
// HBM: it runs dense (no parity blocks), with 8 waves per workgroup, each
// instance cut into slabs of about kLatencyRows in-plane rows (at most
// no more than CUs / batch, and only in batches of at most
// kLatencyMaxSplitBatch instances), one slab per workgroup.
// Measured on single sine-family plates: 100/100 modes step in 11.0 us this
// way (13 slabs), against 82 us blocked on the byte-balanced plan; 50/50 in
// 9.1 us against 39.6 us.  About 8 rows, one per wave, was the best slab size
// of 5, 6, 8 and 10 (100/100: 13.2, 11.8, 11.0, 13.5 us): smaller slabs add
// workgroups to every step's exchange, larger ones give some waves two rows.
// Default limit of a wait for the other slabs of a split instance, in ticks
// of the device's 100 MHz clock (4 s).
constexpr unsigned long long kBarrierTicks = 400000000ull;
constexpr double kLatencyBytes = 64.0 * 1048576.0;
constexpr int kLatencyRows = 8;
constexpr int kLatencyMaxSplitBatch = 16;  // larger latency-bound batches keep instances whole
// A large instance of such a batch is also cut so that no slab streams more
// than about this many tensor bytes per step (the waves of a one-unit
// workgroup share its row blocks, so slabs of fewer rows than waves keep
// every wave busy); half as many for a tensor larger than kLatencyBigTensor,
// which no longer stays in the XCDs' L2 caches, so that more CUs stream it
// from the last-level cache.  Measured on lone sine plates with the partial
// forces exchanged as 16-byte coherent accesses: a 100/100 plate (4 MB)
// steps in 9.0 us with 256 KB slabs (16) against 11.5 us at 128 KB (31) and
// 11.7 us at 384 KB (13); a 200/200 plate (32 MB) steps forward in 14.1 us
// with 128 KB slabs (one in-plane row each, 200) against 16.9 us at 256 KB
// (123) and 21.2 us at 512 KB (62), its forward and reverse step together in
// 32.8 us against 38.4 and 47.0 us.
constexpr double kLatencySlabBytes = 256.0 * 1024.0;
constexpr double kLatencyBigTensor = 16.0 * 1048576.0;

// Per-step cost of the exchange and barrier of one slab of a split instance,
// in streamed-byte units (publishing its partial force, arrival, wait and
// reading every slab's partial).  It steers the packing rather than
// predicting time: on the 256-plate batch, with the exchange as 16-byte
// coherent accesses, 0, 8, 16, 24, 32, 48, 64, 128 and 256 KB gave 231.8,
// 234.7, 235.8, 232.6, 232.9, 240.2, 241.9, 236.7 and 238.1 ms per
// 441-sample launch (runs of one setting differ by about 1 %).
constexpr double kSplitSyncCost = 32768.0;
// the cost a description asks for (its autotuned value), else the default
double split_cost(const modal_desc* d) {
  return d->split_cost_kb > 0 ? 1024.0 * d->split_cost_kb : kSplitSyncCost;
}
// Instances below this cost are never split: their tensors stay L2-resident
// from step to step and a whole-instance workgroup outruns any slab barrier.
constexpr double kMinSplitCost = 4.0 * 1048576.0;

// ------------------------------------------------------ parity-blocked tensors
// Internal layout of an instance whose tensor splits by mode class: modes
// grouped by class (each class padded to a multiple of 4), and for every
// in-plane row n and class i the single class jmap[n][i] of columns that
// holds nonzero entries in the rows of class i (-1: none).
struct BlockPlan {
  bool ok = false;
  int cls[5] = {0, 0, 0, 0, 0};
  int w = 0, rmax = 0;
  std::vector<int> slot_mode, mode_slot, jmap;
  // float offset of block (n, i) from the instance's start (stored blocks
  // only: rows of class i, as wide as its column class), rows laid out in
  // order, and the stored floats in all
  std::vector<int> boff;
  long long floats = 0;
  long long stored_bytes = 0;
};

// Checks that H has the block structure the classes imply, exactly (every
// other entry is 0.0), and that it is finite and symmetric to 1e-6; any
// failure leaves the instance dense, where the device check reports it.
void analyze_blocks(const modal_instance& I, BlockPlan& bp) {
  bp.ok = false;
  const int nt = I.n_t, nin = I.n_in;
  int cnt[4] = {0, 0, 0, 0};
  for (int k = 0; k < nt; ++k) cnt[I.mode_class[k]]++;
  int off = 0;
  for (int i = 0; i < 4; ++i) {
    bp.cls[i] = off;
    const int R = round4(cnt[i]);
    off += R;
    bp.w = std::max(bp.w, R);
  }
  bp.cls[4] = off;
  bp.rmax = bp.w;
  if (off > kMaxModes) return;
  bp.slot_mode.assign(off, -1);
  bp.mode_slot.assign(nt, -1);
  int fill[4] = {0, 0, 0, 0};
  for (int k = 0; k < nt; ++k) {
    const int i = I.mode_class[k];
    const int sl = bp.cls[i] + fill[i]++;
    bp.slot_mode[sl] = k;
    bp.mode_slot[k] = sl;
  }
  bp.jmap.assign((size_t)nin * 4, -1);
  bp.stored_bytes = 0;
  float hmax = 0.f, dmax = 0.f;
  const uint8_t* ck = I.mode_class;
  for (int n = 0; n < nin; ++n) {
    bool nz[4][4] = {};
    const float* Hn = I.H + (size_t)n * nt * nt;
    for (int p = 0; p < nt; ++p) {
      const float* row = Hn + (size_t)p * nt;
      bool* nzp = nz[ck[p]];
      for (int q = 0; q < nt; ++q) {
        const float v = row[q];
        if (!std::isfinite(v)) return;
        if (v != 0.f) {
          nzp[ck[q]] = true;
          hmax = std::max(hmax, std::fabs(v));
        }
      }
      for (int q = p + 1; q < nt; ++q) dmax = std::max(dmax, std::fabs(row[q] - Hn[(size_t)q * nt + p]));
    }
    for (int i = 0; i < 4; ++i) {
      if (cnt[i] == 0) continue;
      int found = -1;
      for (int j = 0; j < 4; ++j)
        if (nz[i][j]) {
          if (found >= 0) return;  // two column classes in one block row
          found = j;
        }
      bp.jmap[(size_t)n * 4 + i] = found;
      if (found >= 0) bp.stored_bytes += 4LL * cnt[i] * cnt[found];
    }
  }
  if (dmax > 1e-6f * hmax) return;
  // An exactly symmetric tensor stores one block of each transposed pair:
  // (i, j) with i < j stands for (j, i) too (flag 8), whose entry becomes -1.
  if (dmax == 0.f) {
    for (int n = 0; n < nin; ++n) {
      int* jm = &bp.jmap[(size_t)n * 4];
      for (int i = 0; i < 4; ++i) {
        const int j = jm[i];
        if (j >= 0 && j < 4 && j > i && jm[j] == i) {
          jm[i] = j | 8;
          jm[j] = -1;
          bp.stored_bytes -= 4LL * cnt[j] * cnt[i];
        }
      }
    }
  }
  bp.boff.assign((size_t)nin * 4, 0);
  long long pos = 0;
  for (int n = 0; n < nin; ++n)
    for (int i = 0; i < 4; ++i) {
      const int je = bp.jmap[(size_t)n * 4 + i];
      const int R = bp.cls[i + 1] - bp.cls[i];
      if (je < 0 || R == 0) continue;
      const int tj = je & 7;
      bp.boff[(size_t)n * 4 + i] = (int)pos;
      pos += (long long)R * (bp.cls[tj + 1] - bp.cls[tj]);
      if (pos > (1LL << 31) - 1) return;  // offsets are 32-bit
    }
  bp.floats = pos;
  bp.ok = true;
}

// Analyses every VK instance that carries mode classes and host tensors, on
// all host threads (largest first).
void plan_blocks(const modal_desc* d, std::vector<BlockPlan>& plans) {
  plans.assign(d->batch, BlockPlan{});
  if (d->flags & (MODAL_FLAG_GRAD | MODAL_FLAG_NO_BLOCK)) return;
  std::vector<int> todo;
  for (int b = 0; b < d->batch; ++b) {
    const modal_instance& I = d->inst[b];
    if (I.kind != MODAL_KIND_VK || !I.mode_class) continue;
    hipPointerAttribute_t attr;
    bool on_device = false;
    if (hipPointerGetAttributes(&attr, I.H) == hipSuccess)
      on_device = attr.type == hipMemoryTypeDevice;
    else
      (void)hipGetLastError();
    if (!on_device) todo.push_back(b);
  }
  std::stable_sort(todo.begin(), todo.end(), [&](int a, int b) {
    return (double)d->inst[a].n_in * d->inst[a].n_t * d->inst[a].n_t >
           (double)d->inst[b].n_in * d->inst[b].n_t * d->inst[b].n_t;
  });
  std::atomic<size_t> next{0};
  auto work = [&]() {
    for (size_t i = next++; i < todo.size(); i = next++) analyze_blocks(d->inst[todo[i]], plans[todo[i]]);
  };
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const unsigned nth = (unsigned)std::min<size_t>(hw, todo.size());
  std::vector<std::thread> th;
  for (unsigned t = 1; t < nth; ++t) th.emplace_back(work);
  work();
  for (auto& t : th) t.join();
}

// On-chip register layout of one instance (see ChipMap), with the columns
// per lane (w_need) and rows per wave (r_need) it takes; false if it does
// not fit one workgroup (more than kWave lanes, or more than kChipMaxRows
// rows on a wave).  A VK tensor with mode classes, on the host, with the
// exact block structure of the classes gets its modes grouped by class, and
// each wave the rows of one column pattern, so a lane holds only the one
// class of columns that can be nonzero against it; any other tensor is
// held whole (all nt columns), its rows dealt to the waves in turn.
bool chip_map(const modal_instance& I, ChipMap& m, int& w_need, int& r_need) {
  const int nt = I.n_t;
  w_need = r_need = 0;
  if (nt > kWave) return false;
  for (int p = 0; p < kWave; ++p) m.perm[p] = (short)(p < nt ? p : -1);
  for (int w = 0; w < kChipWaves; ++w) {
    for (int r = 0; r < kChipMaxRows; ++r) m.row[w][r] = -1;
    for (int p = 0; p < kWave; ++p) {
      m.jb[w][p] = 0;
      m.jl[w][p] = 0;
    }
  }
  if (I.kind != MODAL_KIND_VK) return true;
  BlockPlan bp;
  if (I.mode_class) {
    hipPointerAttribute_t attr;
    bool on_device = false;
    if (hipPointerGetAttributes(&attr, I.H) == hipSuccess)
      on_device = attr.type == hipMemoryTypeDevice;
    else
      (void)hipGetLastError();
    if (!on_device) analyze_blocks(I, bp);
  }
  const int nin = I.n_in;
  if (!bp.ok || bp.cls[4] > kWave) {  // whole tensor, rows dealt in turn
    r_need = (nin + kChipWaves - 1) / kChipWaves;
    if (r_need > kChipMaxRows) return false;
    for (int n = 0; n < nin; ++n) m.row[n % kChipWaves][n / kChipWaves] = (short)n;
    for (int w = 0; w < kChipWaves; ++w)
      for (int p = 0; p < nt; ++p) m.jl[w][p] = (unsigned char)nt;
    w_need = nt;
    return true;
  }
  // modes grouped by class; the column class partnering each class of a
  // row, with a stored transposed pair counted for both of its blocks
  for (int p = 0; p < kWave; ++p) m.perm[p] = (short)(p < bp.cls[4] ? bp.slot_mode[p] : -1);
  int real[4] = {0, 0, 0, 0};
  for (int c = 0; c < 4; ++c)
    for (int p = bp.cls[c]; p < bp.cls[c + 1]; ++p) real[c] += bp.slot_mode[p] >= 0;
  std::map<std::array<int, 4>, std::vector<int>> by_pattern;
  for (int n = 0; n < nin; ++n) {
    std::array<int, 4> part = {-1, -1, -1, -1};
    for (int i = 0; i < 4; ++i) {
      const int je = bp.jmap[(size_t)n * 4 + i];
      if (je < 0) continue;
      part[i] = je & 7;
      if (je & 8) part[je & 7] = i;
    }
    if (part[0] < 0 && part[1] < 0 && part[2] < 0 && part[3] < 0) continue;  // a zero row
    by_pattern[part].push_back(n);
  }
  const int npat = (int)by_pattern.size();
  if (npat > kChipWaves) return false;
  std::vector<const std::array<int, 4>*> pats;
  std::vector<const std::vector<int>*> rows;
  for (auto& kv : by_pattern) {
    pats.push_back(&kv.first);
    rows.push_back(&kv.second);
  }
  // one wave per pattern, the rest where the most rows per wave remain
  std::vector<int> waves(npat, 1);
  for (int left = kChipWaves - npat; left > 0; --left) {
    int best = -1;
    double most = -1;
    for (int i = 0; i < npat; ++i) {
      const double per = (double)rows[i]->size() / waves[i];
      if (per > most) {
        most = per;
        best = i;
      }
    }
    if (best < 0) break;
    waves[best]++;
  }
  int w0 = 0;
  for (int i = 0; i < npat; ++i) {
    const std::vector<int>& rs = *rows[i];
    const int per = ((int)rs.size() + waves[i] - 1) / waves[i];
    if (per > kChipMaxRows) return false;
    r_need = std::max(r_need, per);
    for (size_t t = 0; t < rs.size(); ++t) m.row[w0 + (int)(t % waves[i])][t / waves[i]] = (short)rs[t];
    for (int w = w0; w < w0 + waves[i]; ++w)
      for (int c = 0; c < 4; ++c) {
        const int cj = (*pats[i])[c];
        if (cj < 0) continue;
        for (int p = bp.cls[c]; p < bp.cls[c + 1]; ++p) {
          m.jb[w][p] = (unsigned char)bp.cls[cj];
          m.jl[w][p] = (unsigned char)real[cj];
        }
        w_need = std::max(w_need, real[cj]);
      }
    w0 += waves[i];
  }
  return true;
}

// Planning cost of an instance in streamed-byte units: per in-plane row the
// bytes of its tensor row plus the row's reduction; per step a fixed cost
// for the state update and output.  A blocked instance streams its blocks
// and reduces once per block.
void unit_costs(const modal_instance& I, double& row_cost, double& fixed_cost,
                const BlockPlan* bp = nullptr) {
  const int ntp = round4(I.n_t);
  if (I.kind == MODAL_KIND_VK && bp && bp->ok) {
    row_cost = 4.0 * (double)bp->floats / std::max(1, I.n_in) + 4.0 * 2048.0;
    fixed_cost = 8192.0;
  } else if (I.kind == MODAL_KIND_VK) {
    row_cost = 4.0 * I.n_t * ntp + 4096.0;
    fixed_cost = 8192.0;
  } else {
    row_cost = 0.0;
    fixed_cost = 8192.0 + 64.0 * ntp;
  }
}

// Packs the batch into at most `n_bins` workgroups of capacity `cap`
// (streamed-byte units).  An instance costlier than `cap` is cut into the
// fewest slabs of in-plane rows that each fit; then every item goes, largest
// first, to the fullest workgroup it still fits in (best-fit decreasing).
// Returns the number of workgroups used, or n_bins + 1 if it does not fit.
int pack(const modal_desc* d, const std::vector<double>& row_cost,
         const std::vector<double>& fixed_cost, double cap, int n_bins, std::vector<Unit>& units,
         std::vector<int>& bin_of, std::vector<double>& load) {
  units.clear();
  for (int b = 0; b < d->batch; ++b) {
    const modal_instance& I = d->inst[b];
    const int rows = I.kind == MODAL_KIND_VK ? I.n_in : 1;
    int S = 1;
    const double whole = fixed_cost[b] + rows * row_cost[b];
    const bool may_split = (d->flags & MODAL_FLAG_SPLIT_ANY) || whole >= kMinSplitCost;
    if (I.kind == MODAL_KIND_VK && whole > cap && may_split) {
      const double sync = (d->flags & MODAL_FLAG_SPLIT_ANY) ? 0.0 : split_cost(d);
      const int per = (int)std::floor((cap - sync - fixed_cost[b]) / row_cost[b]);
      if (per < 1) return n_bins + 1;
      S = (rows + per - 1) / per;
    }
    if (S > n_bins) return n_bins + 1;
    for (int s = 0; s < S; ++s) {
      const int r0 = (int)((long long)rows * s / S), r1 = (int)((long long)rows * (s + 1) / S);
      const double sync = S > 1 && !(d->flags & MODAL_FLAG_SPLIT_ANY) ? split_cost(d) : 0.0;
      units.push_back({b, r0, r1, s, sync + fixed_cost[b] + (r1 - r0) * row_cost[b]});
    }
  }
  std::vector<int> order(units.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return units[a].cost > units[b].cost; });
  std::multimap<double, int> open;  // remaining capacity -> bin
  bin_of.assign(units.size(), -1);
  load.clear();
  for (int i : order) {
    const double c = units[i].cost;
    auto it = open.lower_bound(c);  // tightest bin that still fits
    int bin;
    if (it != open.end()) {
      bin = it->second;
      open.erase(it);
    } else {
      if ((int)load.size() == n_bins) return n_bins + 1;
      bin = (int)load.size();
      load.push_back(0.0);
    }
    load[bin] += c;
    bin_of[i] = bin;
    open.insert({cap - load[bin], bin});
  }
  return (int)load.size();
}

// Smallest capacity (binary search) at which the batch packs into n_bins
// workgroups, and that packing.  (Filling workgroups in turn with slabs of
// unequal sizes instead brings the planned heaviest workgroup within 3 % of
// the mean on the 256-plate batch, against 14 % here, but measured 10 %
// slower: more units per workgroup and more exchanges.)
bool plan_batch(const modal_desc* d, const std::vector<double>& row_cost,
                const std::vector<double>& fixed_cost, double total, int n_bins,
                std::vector<Unit>& units, std::vector<int>& bin_of, std::vector<double>& load) {
  double max_item = 0;
  for (int b = 0; b < d->batch; ++b) {
    const double whole = fixed_cost[b] + (d->inst[b].kind == MODAL_KIND_VK ? d->inst[b].n_in : 1) * row_cost[b];
    const double one_row = ((d->flags & MODAL_FLAG_SPLIT_ANY) ? 0.0 : split_cost(d)) + fixed_cost[b] +
                           (d->inst[b].kind == MODAL_KIND_VK ? row_cost[b] : 0.0);
    const bool may_split = (d->flags & MODAL_FLAG_SPLIT_ANY) || whole >= kMinSplitCost;
    max_item = std::max(max_item, may_split ? std::min(whole, one_row) : whole);
  }
  double lo = std::max(total / n_bins, max_item), hi = std::max(lo, total) * 1.0001 + 1.0;
  if (pack(d, row_cost, fixed_cost, hi, n_bins, units, bin_of, load) > n_bins) return false;
  for (int it = 0; it < 40 && hi - lo > 1e-4 * lo; ++it) {
    const double mid = 0.5 * (lo + hi);
    std::vector<Unit> u2;
    std::vector<int> b2;
    std::vector<double> l2;
    if (pack(d, row_cost, fixed_cost, mid, n_bins, u2, b2, l2) <= n_bins) hi = mid;
    else lo = mid;
  }
  pack(d, row_cost, fixed_cost, hi, n_bins, units, bin_of, load);
  return true;
}

// Copies every instance's Ht into the padded device layout (rows of ntp
// floats).  Device sources are copied directly; host sources are padded into
// two pinned staging buffers that alternate with the asynchronous copies.
int upload_tensors(modal_ctx* c, const modal_desc* d, const std::vector<InstDev>& inst,
                   const std::vector<BlockPlan>& plans, hipStream_t stream) {
  const size_t kStage = 64u << 20;
  float* stage[2] = {nullptr, nullptr};
  hipEvent_t done[2] = {nullptr, nullptr};
  int rc = MODAL_OK;
  auto cleanup = [&]() {
    for (int i = 0; i < 2; ++i) {
      if (done[i]) (void)hipEventDestroy(done[i]);
      if (stage[i]) (void)hipHostFree(stage[i]);
    }
  };
#define UP_TRY(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) {                                                            \
      rc = fail(MODAL_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));        \
      cleanup();                                                                       \
      return rc;                                                                       \
    }                                                                                  \
  } while (0)
  int slot = 0;
  bool used[2] = {false, false};
  for (int b = 0; b < d->batch; ++b) {
    const modal_instance& I = d->inst[b];
    if (I.kind != MODAL_KIND_VK) continue;
    const InstDev& D = inst[b];
    if (D.blk) {
      // blocks gathered on the host threads, whole in-plane rows staged in
      // order (each block as wide as its column class)
      if (!stage[0]) {
        for (int i = 0; i < 2; ++i) {
          UP_TRY(hipHostMalloc((void**)&stage[i], kStage, hipHostMallocDefault));
          UP_TRY(hipEventCreateWithFlags(&done[i], hipEventDisableTiming));
        }
      }
      const BlockPlan& bp = plans[b];
      const int nin = D.nin;
      std::vector<long long> rs((size_t)nin + 1, 0);  // first float of each in-plane row
      for (int n = 0; n < nin; ++n) {
        long long sz = 0;
        for (int i = 0; i < 4; ++i) {
          const int je = bp.jmap[(size_t)n * 4 + i];
          const int R = bp.cls[i + 1] - bp.cls[i];
          if (je >= 0 && R > 0) sz += (long long)R * (bp.cls[(je & 7) + 1] - bp.cls[je & 7]);
        }
        rs[n + 1] = rs[n] + sz;
      }
      const long long stage_floats = (long long)(kStage / sizeof(float));
      for (int n0 = 0; n0 < nin;) {
        int n1 = n0 + 1;
        while (n1 < nin && rs[n1 + 1] - rs[n0] <= stage_floats) ++n1;
        if (rs[n1] - rs[n0] > stage_floats) {
          cleanup();
          return fail(MODAL_ENOMEM, "an in-plane row's blocks exceed the staging buffer");
        }
        if (used[slot]) UP_TRY(hipEventSynchronize(done[slot]));
        float* dst = stage[slot];
        auto fill_rows = [&](int a, int z) {
          for (int n = a; n < z; ++n) {
            const float* Hn = I.H + (size_t)n * D.nt * D.nt;
            const double sc = I.h_row_scale ? I.h_row_scale[n] : 1.0;
            for (int i = 0; i < 4; ++i) {
              const int je = bp.jmap[(size_t)n * 4 + i];
              const int R = bp.cls[i + 1] - bp.cls[i];
              if (je < 0 || R == 0) continue;
              const int tj = je & 7;
              const int W = bp.cls[tj + 1] - bp.cls[tj];
              float* out = dst + (bp.boff[(size_t)n * 4 + i] - rs[n0]);
              for (int r = 0; r < R; ++r, out += W) {
                const int p = bp.slot_mode[bp.cls[i] + r];
                if (p < 0) {
                  std::memset(out, 0, sizeof(float) * W);
                  continue;
                }
                const float* row = Hn + (size_t)p * D.nt;
                for (int s2 = 0; s2 < W; ++s2) {
                  const int q = bp.slot_mode[bp.cls[tj] + s2];
                  out[s2] = q < 0 ? 0.f : (I.h_row_scale ? (float)(sc * (double)row[q]) : row[q]);
                }
              }
            }
          }
        };
        const int nr = n1 - n0;
        const unsigned nth = (unsigned)std::max(1, std::min({16, nr, (int)std::thread::hardware_concurrency()}));
        std::vector<std::thread> th;
        for (unsigned t = 1; t < nth; ++t) th.emplace_back(fill_rows, n0 + (int)(nr * t / nth), n0 + (int)(nr * (t + 1) / nth));
        fill_rows(n0, n0 + (int)(nr / nth));
        for (auto& t : th) t.join();
        UP_TRY(hipMemcpyAsync(c->dH + D.h_off + rs[n0], dst, sizeof(float) * (size_t)(rs[n1] - rs[n0]),
                              hipMemcpyHostToDevice, stream));
        UP_TRY(hipEventRecord(done[slot], stream));
        used[slot] = true;
        slot ^= 1;
        n0 = n1;
      }
      continue;
    }
    hipPointerAttribute_t attr;
    bool on_device = false;
    if (hipPointerGetAttributes(&attr, I.H) == hipSuccess)
      on_device = attr.type == hipMemoryTypeDevice;
    else
      (void)hipGetLastError();
    if (on_device && !I.h_row_scale) {
      UP_TRY(hipMemcpy2DAsync(c->dH + D.h_off, sizeof(float) * D.ntp, I.H, sizeof(float) * D.nt,
                              sizeof(float) * D.nt, (size_t)D.nin * D.nt, hipMemcpyDeviceToDevice,
                              stream));
      continue;
    }
    // host rows (a device tensor with row scales is read back first)
    std::vector<float> host_copy;
    const float* src = I.H;
    if (on_device) {
      host_copy.resize((size_t)D.nin * D.nt * D.nt);
      UP_TRY(hipMemcpy(host_copy.data(), I.H, sizeof(float) * host_copy.size(), hipMemcpyDeviceToHost));
      src = host_copy.data();
    }
    if (!stage[0]) {
      for (int i = 0; i < 2; ++i) {
        UP_TRY(hipHostMalloc((void**)&stage[i], kStage, hipHostMallocDefault));
        UP_TRY(hipEventCreateWithFlags(&done[i], hipEventDisableTiming));
      }
    }
    const size_t rows = (size_t)D.nin * D.nt;
    const size_t rows_per = std::max<size_t>(1, kStage / (sizeof(float) * D.ntp));
    for (size_t r0 = 0; r0 < rows; r0 += rows_per) {
      const size_t nr = std::min(rows_per, rows - r0);
      if (used[slot]) UP_TRY(hipEventSynchronize(done[slot]));
      float* dst = stage[slot];
      for (size_t r = 0; r < nr; ++r) {
        const float* row = src + (r0 + r) * D.nt;
        if (I.h_row_scale) {
          const double sc = I.h_row_scale[(r0 + r) / D.nt];
          for (int k = 0; k < D.nt; ++k) dst[r * D.ntp + k] = (float)(sc * (double)row[k]);
        } else {
          std::memcpy(dst + r * D.ntp, row, sizeof(float) * D.nt);
        }
        for (int k = D.nt; k < D.ntp; ++k) dst[r * D.ntp + k] = 0.f;
      }
      UP_TRY(hipMemcpyAsync(c->dH + D.h_off + r0 * D.ntp, dst, sizeof(float) * nr * D.ntp,
                            hipMemcpyHostToDevice, stream));
      UP_TRY(hipEventRecord(done[slot], stream));
      used[slot] = true;
      slot ^= 1;
    }
  }
  if (stage[0]) {
    UP_TRY(hipStreamSynchronize(stream));
  }
#undef UP_TRY
  cleanup();
  return MODAL_OK;
}

// ------------------------------------------------------------ linear batches
// Roots of z^2 - g z - p for every mode of an all-linear batch, the free
// response q^n = A z1^n + B z2^n from q^0, q^-1, and the impulse response
// h(j) = C (z1^j - z2^j) with C = r / (z1 - z2).  False (recursion path) when
// a mode has a double or nearly double root.
bool linear_modes(const modal_desc* d, modal_ctx* c) {
  using cd = std::complex<double>;
  const double T = 1.0 / d->fs;
  for (int b = 0; b < d->batch; ++b) {
    const modal_instance& I = d->inst[b];
    for (int k = 0; k < I.n_t; ++k) {
      const Coef q = coefficients(d->scheme, I.omega[k], I.gamma[k], T);
      const double g = q.m - q.p + 1.0, p = q.p;
      const cd disc = cd(g * g + 4.0 * p, 0.0);
      const cd sq = std::sqrt(disc);
      const cd z1 = 0.5 * (g + sq), z2 = 0.5 * (g - sq);
      // A and B lose about eps / |z1 - z2| relative accuracy by cancellation;
      // near-double roots (critically damped modes) keep the recursion
      if (std::abs(z1 - z2) <= 1e-6 * std::max(std::abs(z1), 1e-300)) return false;
      // a root at zero (a mode that stops after one step) has no logarithm
      if (std::min(std::abs(z1), std::abs(z2)) < 1e-150) return false;
      const cd A = (I.xm1[k] * z1 * z2 - I.x0[k] * z1) / (z2 - z1);
      c->lz1.push_back(z1);
      c->lz2.push_back(z2);
      c->lA.push_back(A);
      c->lB.push_back(I.x0[k] - A);
      c->lC.push_back(q.r / (z1 - z2));
      c->lc.push_back(I.c_out[k]);
      c->lb.push_back(I.b_ext ? I.b_ext[k] : 0.0);
      c->lconj.push_back(g * g + 4.0 * p < 0.0);
    }
    c->le.emplace_back(I.e_ext, I.e_ext + I.n_exc);
  }
  return true;
}

int init_linear(modal_ctx* c, const modal_desc* d, hipStream_t stream) {
  using cd = std::complex<double>;
  const int B = d->batch;
  const size_t M = c->lz1.size();
  std::vector<float> epool(1, 0.f);
  std::vector<long long> eoff(B);
  c->lin_moff.assign(B + 1, 0);
  std::vector<LinForced> forced;
  for (int b = 0; b < B; ++b) {
    c->lin_moff[b + 1] = c->lin_moff[b] + d->inst[b].n_t;
    eoff[b] = (long long)epool.size();
    const long long ne = (long long)c->le[b].size();
    epool.insert(epool.end(), c->le[b].begin(), c->le[b].end());
    if (ne > 0) forced.push_back({b, eoff[b], ne});
    c->lin_max_exc = std::max(c->lin_max_exc, ne);
  }
  // device order within an instance: complex-conjugate pairs first
  std::vector<int> src;
  src.reserve(M);
  c->lin_mc.assign(B, 0);
  for (int b = 0; b < B; ++b) {
    for (int k = c->lin_moff[b]; k < c->lin_moff[b + 1]; ++k)
      if (c->lconj[k]) src.push_back(k);
    c->lin_mc[b] = (int)src.size();
    for (int k = c->lin_moff[b]; k < c->lin_moff[b + 1]; ++k)
      if (!c->lconj[k]) src.push_back(k);
  }
  std::vector<LinMode> modes(M);
  std::vector<LinInit> init(M);
  for (int b = 0; b < B; ++b)
    for (int slot = c->lin_moff[b]; slot < c->lin_moff[b + 1]; ++slot) {
      const int k = src[slot];
      const cd z1 = c->lz1[k], z2 = c->lz2[k];
      const double lm1 = std::log(std::abs(z1)), lm2 = std::log(std::abs(z2));
      const cd s1 = std::polar(std::exp(64.0 * lm1), 64.0 * std::arg(z1));
      const cd s2 = std::polar(std::exp(64.0 * lm2), 64.0 * std::arg(z2));
      LinMode& m = modes[slot];
      m.z1 = ffc(z1);
      m.z2 = ffc(z2);
      m.s1 = ffc(s1);
      m.s2 = ffc(s2);
      split((s1 + s2).real(), m.ah, m.al);
      split((s1 * s2).real(), m.bh, m.bl);
      m.conj = c->lconj[k];
      m.pad[0] = m.pad[1] = m.pad[2] = 0;
      LinInit& I = init[slot];
      I.z1 = ffc(z1);
      I.z2 = ffc(z2);
      I.A = ffc(c->lA[k]);
      I.B = ffc(c->lB[k]);
      I.C = ffc(c->lC[k]);
      split(c->lc[k], I.ch, I.cl);
      split(c->lb[k], I.bh, I.bl);
      I.e_off = eoff[b];
      I.n_exc = (long long)c->le[b].size();
      I.conj = c->lconj[k];
      I.pad[0] = I.pad[1] = I.pad[2] = 0;
    }
  c->n_forced = (int)forced.size();
  c->lin_h_stride = std::max<long long>(1, c->lin_max_exc);
  std::vector<LinSeg> hseg;
  for (int f = 0; f < c->n_forced; ++f) {
    const int b = (int)forced[f].inst;
    hseg.push_back({c->lin_moff[b], c->lin_mc[b], c->lin_moff[b + 1], 0, 2 * (long long)M, 1,
                    f * c->lin_h_stride, forced[f].n_exc - 1});
  }
  int r = dalloc(&c->dLinModes, sizeof(LinMode) * std::max<size_t>(M, 1));
  if (!r) r = dalloc(&c->dLinInit, sizeof(LinInit) * std::max<size_t>(M, 1));
  if (!r) r = dalloc(&c->dLinAmp, sizeof(FFc) * 2 * 3 * std::max<size_t>(M, 1));
  if (!r) r = dalloc(&c->dLinTab, sizeof(FFc) * 64 * std::max<size_t>(M, 1));
  if (!r) r = dalloc(&c->dLinSeg, sizeof(LinSeg) * std::max<size_t>(2 * (size_t)B, hseg.size()));
  if (!r) r = dalloc(&c->dLinForced, sizeof(LinForced) * std::max<size_t>(forced.size(), 1));
  if (!r) r = dalloc(&c->dLinH, sizeof(float2) * std::max<size_t>(1, forced.size() * c->lin_h_stride));
  if (!r) r = dalloc(&c->dE, sizeof(float) * epool.size());
  if (!r) r = dalloc(&c->dFlags, sizeof(int) * 2);
  if (r) return r;
  HIP_TRY(hipMemcpyAsync(c->dLinModes, modes.data(), sizeof(LinMode) * M, hipMemcpyHostToDevice, stream));
  HIP_TRY(hipMemcpyAsync(c->dLinInit, init.data(), sizeof(LinInit) * M, hipMemcpyHostToDevice, stream));
  HIP_TRY(hipMemcpyAsync(c->dE, epool.data(), sizeof(float) * epool.size(), hipMemcpyHostToDevice, stream));
  if (!forced.empty())
    HIP_TRY(hipMemcpyAsync(c->dLinForced, forced.data(), sizeof(LinForced) * forced.size(),
                           hipMemcpyHostToDevice, stream));
  if (!hseg.empty())
    HIP_TRY(hipMemcpyAsync(c->dLinSeg, hseg.data(), sizeof(LinSeg) * hseg.size(), hipMemcpyHostToDevice,
                           stream));
  HIP_TRY(launch_lin_amp(c->dLinInit, c->dLinModes, (int)M, c->dE, c->dLinAmp, c->dLinTab, stream));
  HIP_TRY(launch_lin_sum_ff(c->dLinModes, c->dLinAmp, c->dLinTab, c->dLinSeg, (int)hseg.size(), c->lin_max_exc - 1,
                            c->dLinH, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  for (int b = 0; b < B; ++b) {
    c->kind.push_back(d->inst[b].kind);
    c->nt.push_back(d->inst[b].n_t);
  }
  c->linear = true;
  c->state_floats = 0;
  return MODAL_OK;
}

// Outputs of steps [base, base + n) of every instance.  An unforced instance
// is one free-response segment; a forced one is split at the end of its
// excitation: before it, the free response plus the excitation convolved with
// the impulse response, from it on, the response to the state the excitation
// left (the post amplitude set).
int run_linear(modal_ctx* c, int64_t n, float* y, int64_t y_stride, hipStream_t s) {
  if (n <= 0) return MODAL_OK;
  const int B = c->batch;
  const long long base = c->steps, end = base + n;
  const long long M = (long long)c->lz1.size();
  std::vector<LinSeg> seg;
  seg.reserve(2 * (size_t)B);
  for (int b = 0; b < B; ++b) {
    const int m0 = c->lin_moff[b], mc = c->lin_mc[b], m1 = c->lin_moff[b + 1];
    const long long row = (long long)b * y_stride;
    const long long ne = (long long)c->le[b].size();
    if (ne == 0) {
      seg.push_back({m0, mc, m1, 0, 0, base, row, n});
      continue;
    }
    const long long w_end = std::min(end, ne);
    if (w_end > base) seg.push_back({m0, mc, m1, 0, 0, base, row, w_end - base});
    const long long p0 = std::max(base, ne);
    if (end > p0) seg.push_back({m0, mc, m1, 0, M, p0 - ne, row + (p0 - base), end - p0});
  }
  HIP_TRY(hipMemcpyAsync(c->dLinSeg, seg.data(), sizeof(LinSeg) * seg.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(launch_lin_sum(c->dLinModes, c->dLinAmp, c->dLinTab, c->dLinSeg, (int)seg.size(), n, y, s));
  const long long window = std::min(end, c->lin_max_exc) - base;
  HIP_TRY(launch_lin_conv(c->dLinForced, c->n_forced, c->dLinH, c->lin_h_stride, c->dE, base, n, window, y,
                          y_stride, s));
  // the host segment list must outlive the asynchronous copy
  HIP_TRY(hipStreamSynchronize(s));
  return MODAL_OK;
}

// ------------------------------------------------------------ shared tensor
struct SharedGroup {
  const float* H;
  int nt, nin;
  std::vector<int> members;
};

// Instances grouped by (H pointer, n_t, n_in); empty unless the batch takes
// the shared-tensor path (every instance VK with n_t <= 16 kSharedMaxKT,
// n_in <= kSharedMaxNin, and at least 16 instances per distinct tensor on
// average).
std::vector<SharedGroup> shared_groups(const modal_desc* d) {
  std::vector<SharedGroup> g;
  if (d->flags & (MODAL_FLAG_GRAD | MODAL_FLAG_NO_SHARED)) return g;
  std::map<std::tuple<const float*, int, int>, int> index;
  for (int b = 0; b < d->batch; ++b) {
    const modal_instance& I = d->inst[b];
    if (I.kind != MODAL_KIND_VK || I.n_t > 16 * kSharedMaxKT || I.n_in > kSharedMaxNin) return {};
    auto key = std::make_tuple(I.H, I.n_t, I.n_in);
    auto it = index.find(key);
    if (it == index.end()) {
      it = index.emplace(key, (int)g.size()).first;
      g.push_back({I.H, I.n_t, I.n_in, {}});
    }
    g[it->second].members.push_back(b);
  }
  if ((long long)d->batch < 16LL * (long long)g.size()) return {};
  return g;
}

// Builds a context on the shared-tensor path: packs each group's tensor
// once in the MFMA operand order, lays every instance out as one column of
// its group's workgroups and uploads coefficients, scales and state.
int init_shared(modal_ctx* c, const modal_desc* d, std::vector<SharedGroup>& groups,
                hipStream_t stream) {
  const double T = 1.0 / d->fs;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, dev));
  int kt = 1, nin_max = 1;
  long long wg2 = 0;
  for (auto& g : groups) {
    kt = std::max(kt, (g.nt + 15) / 16);
    nin_max = std::max(nin_max, g.nin);
    wg2 += ((long long)g.members.size() + 127) / 128;
  }
  // K steps of the launch: the groups' common count, else the widest
  int kc = -1;
  for (auto& g : groups) {
    const int gkc = (g.nt + 3) / 4;
    kc = kc < 0 || kc == gkc ? gkc : 4 * kt;
  }
  if (kc < 4 * kt - 3) kc = 4 * kt;
  const int kc4 = (kc + 3) / 4;
  // two column tiles per wave once that still gives every CU a workgroup and
  // two such workgroups still fit a CU's LDS; otherwise one, and more
  // workgroups per CU hide each other's barriers and reductions (65 536
  // plates at 40/40: 90.8 TFLOP/s with one tile, 83.2 with two)
  const bool two_fit = 2 * shared_lds_bytes(kt, kc, 2, nin_max) <=
                       (size_t)prop.maxSharedMemoryPerMultiProcessor;
  const int jt = wg2 >= prop.multiProcessorCount && two_fit ? 2 : 1;
  const int cols = 64 * jt, ktot = 16 * kt;
  long long n_wg = 0;
  for (auto& g : groups) n_wg += ((long long)g.members.size() + cols - 1) / cols;
  if (n_wg > (1 << 30) / cols) return fail(MODAL_EINVAL, "batch too large");
  const long long ncol = n_wg * cols, ncolk = ncol * ktot;

  // packed tensors: A[n][t][c][l] = H[n][16 t + l%16][4 c + l/16]
  std::vector<SharedWg> wgs;
  std::vector<SharedSlot> slots(ncol, SharedSlot{-1, 0, 0, 0});
  std::vector<float> apool, s2((size_t)n_wg * nin_max * cols, 0.f);
  std::vector<float> coef(8 * (size_t)ncolk, 0.f);
  c->state0.assign(4 * (size_t)ncolk, 0.f);
  c->unit_state_of_inst.assign(d->batch, 0);
  std::vector<float> epool(1, 0.f);
  for (auto& g : groups) {
    const size_t hn = (size_t)g.nin * g.nt * g.nt;
    std::vector<float> H(hn);
    hipPointerAttribute_t attr;
    bool on_device = false;
    if (hipPointerGetAttributes(&attr, g.H) == hipSuccess)
      on_device = attr.type == hipMemoryTypeDevice;
    else
      (void)hipGetLastError();
    if (on_device) HIP_TRY(hipMemcpy(H.data(), g.H, sizeof(float) * hn, hipMemcpyDeviceToHost));
    else std::memcpy(H.data(), g.H, sizeof(float) * hn);
    float hmax = 0.f, dmax = 0.f;
    for (int n = 0; n < g.nin; ++n)
      for (int k = 0; k < g.nt; ++k)
        for (int j = 0; j < g.nt; ++j) {
          const float a = H[((size_t)n * g.nt + k) * g.nt + j], b = H[((size_t)n * g.nt + j) * g.nt + k];
          if (!std::isfinite(a)) return fail(MODAL_EINVAL, "non-finite H (instance " + std::to_string(g.members[0]) + ")");
          hmax = std::max(hmax, std::fabs(a));
          dmax = std::max(dmax, std::fabs(a - b));
        }
    if (dmax > 1e-6f * hmax)
      return fail(MODAL_EINVAL, "H not symmetric in its last two indices (instance " +
                                    std::to_string(g.members[0]) + ")");
    // A[n][t][c4][l][e] = H[n][16 t + l%16][4 (4 c4 + e) + l/16], zero past n_t
    const size_t row = (size_t)kt * kc4 * 64 * 4;
    const long long a_off = (long long)apool.size();
    apool.resize(apool.size() + (((size_t)g.nin * row + 63) & ~(size_t)63), 0.f);
    for (int n = 0; n < g.nin; ++n)
      for (int t = 0; t < kt; ++t)
        for (int c4 = 0; c4 < kc4; ++c4)
          for (int l = 0; l < 64; ++l)
            for (int e = 0; e < 4; ++e) {
              const int k = 16 * t + l % 16, q = 4 * (4 * c4 + e) + l / 16;
              apool[a_off + n * row + (((size_t)t * kc4 + c4) * 64 + l) * 4 + e] =
                  k < g.nt && q < g.nt ? H[((size_t)n * g.nt + k) * g.nt + q] : 0.f;
            }
    c->coupling_bytes += 4LL * g.nin * g.nt * g.nt * (long long)g.members.size();
    for (size_t i0 = 0; i0 < g.members.size(); i0 += cols) {
      const long long w = (long long)wgs.size();
      wgs.push_back(SharedWg{a_off, g.nin, g.nt, kt, kc});
      c->padded_bytes += 4LL * g.nin * (long long)row;
      for (size_t i = i0; i < std::min(g.members.size(), i0 + cols); ++i) {
        const int b = g.members[i];
        const modal_instance& I = d->inst[b];
        const long long col = w * cols + (long long)(i - i0);
        SharedSlot& sl = slots[col];
        sl.out_row = b;
        sl.n_exc = I.n_exc;
        sl.e_off = (long long)epool.size();
        if (I.n_exc > 0) epool.insert(epool.end(), I.e_ext, I.e_ext + I.n_exc);
        for (int n = 0; n < g.nin; ++n) {
          const double sc = I.h_row_scale ? I.h_row_scale[n] : 1.0;
          s2[((size_t)w * nin_max + n) * cols + (i - i0)] = (float)(sc * sc);
        }
        const size_t o = (size_t)col * ktot;
        c->unit_state_of_inst[b] = (int)o;
        for (int k = 0; k < I.n_t; ++k) {
          const Coef q = coefficients(d->scheme, I.omega[k], I.gamma[k], T);
          split(q.m, coef[o + k], coef[ncolk + o + k]);
          split(q.p, coef[2 * ncolk + o + k], coef[3 * ncolk + o + k]);
          split(q.r, coef[4 * ncolk + o + k], coef[5 * ncolk + o + k]);
          coef[6 * ncolk + o + k] = (float)I.c_out[k];
          coef[7 * ncolk + o + k] = I.b_ext ? (float)I.b_ext[k] : 0.f;
          split(I.x0[k], c->state0[o + k], c->state0[ncolk + o + k]);
          split(I.x0[k] - I.xm1[k], c->state0[2 * ncolk + o + k], c->state0[3 * ncolk + o + k]);
        }
        c->flops += 2LL * g.nin * g.nt * g.nt + 4LL * g.nin * g.nt;
      }
    }
  }
  for (int b = 0; b < d->batch; ++b) {
    c->kind.push_back(d->inst[b].kind);
    c->nt.push_back(d->inst[b].n_t);
  }
  c->shared = true;
  c->sh_kt = kt;
  c->sh_kc = kc;
  c->sh_jt = jt;
  c->n_wg = (int)n_wg;
  c->n_units = (int)ncol;
  c->occ = 0;
  c->state_floats = (int)ncolk;
  c->lds_bytes = shared_lds_bytes(kt, kc, jt, nin_max);

  const size_t meta_bytes = sizeof(SharedWg) * wgs.size() + sizeof(SharedSlot) * slots.size();
  int r = dalloc(&c->dShA, sizeof(float) * (apool.size() + 64));
  if (!r) r = dalloc(&c->dMeta, meta_bytes);
  if (!r) r = dalloc(&c->dShS2, sizeof(float) * s2.size());
  if (!r) r = dalloc(&c->dCoef, sizeof(float) * coef.size());
  if (!r) r = dalloc(&c->dState, sizeof(float) * c->state0.size());
  c->n_ctr = d->batch;
  if (!r) r = dalloc(&c->dCtr, sizeof(unsigned int) * d->batch);
  if (!r) r = dalloc(&c->dFlags, sizeof(int) * 2);
  if (!r) r = dalloc(&c->dStep, sizeof(long long));
  if (!r) r = dalloc(&c->dE, sizeof(float) * epool.size());
  if (r) return r;
  char* meta = (char*)c->dMeta;
  SharedWg* dWg = (SharedWg*)meta;
  SharedSlot* dSlot = (SharedSlot*)(meta + sizeof(SharedWg) * wgs.size());
  HIP_TRY(hipMemcpyAsync(c->dShA, apool.data(), sizeof(float) * apool.size(), hipMemcpyHostToDevice, stream));
  HIP_TRY(hipMemcpyAsync(dWg, wgs.data(), sizeof(SharedWg) * wgs.size(), hipMemcpyHostToDevice, stream));
  HIP_TRY(hipMemcpyAsync(dSlot, slots.data(), sizeof(SharedSlot) * slots.size(), hipMemcpyHostToDevice, stream));
  HIP_TRY(hipMemcpyAsync(c->dShS2, s2.data(), sizeof(float) * s2.size(), hipMemcpyHostToDevice, stream));
  HIP_TRY(hipMemcpyAsync(c->dCoef, coef.data(), sizeof(float) * coef.size(), hipMemcpyHostToDevice, stream));
  HIP_TRY(hipMemcpyAsync(c->dE, epool.data(), sizeof(float) * epool.size(), hipMemcpyHostToDevice, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  SharedParams& P = c->SP;
  P.wg = dWg;
  P.slot = dSlot;
  P.A = c->dShA;
  P.s2 = c->dShS2;
  P.nin_max = nin_max;
  P.cols = cols;
  P.ktot = ktot;
  P.x_hi = c->dState;
  P.x_lo = P.x_hi + ncolk;
  P.d_hi = P.x_lo + ncolk;
  P.d_lo = P.d_hi + ncolk;
  P.m_hi = c->dCoef;
  P.m_lo = P.m_hi + ncolk;
  P.p_hi = P.m_lo + ncolk;
  P.p_lo = P.p_hi + ncolk;
  P.r_hi = P.p_lo + ncolk;
  P.r_lo = P.r_hi + ncolk;
  P.c_out = P.r_lo + ncolk;
  P.b_ext = P.c_out + ncolk;
  P.e_ext = c->dE;
  P.step_base = c->dStep;
  P.flags = c->dFlags;
  return MODAL_OK;
}

}  // namespace

extern "C" {

const char* modal_last_error(void) { return g_err.c_str(); }

namespace {

// FNV-1a, 64 bits
struct Fnv {
  uint64_t h = 1469598103934665603ull;
  void add(const void* p, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) {
      h ^= b[i];
      h *= 1099511628211ull;
    }
  }
  void add_int(int32_t v) { add(&v, sizeof v); }
};

int tune_key(const modal_desc* d, std::string& key) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, dev));
  Fnv f;
  f.add(prop.name, strnlen(prop.name, sizeof(prop.name)));
  f.add_int(d->batch);
  f.add_int(d->scheme);
  f.add_int(d->flags & ~(MODAL_FLAG_ASYNC | MODAL_FLAG_GRAPH));
  for (int b = 0; b < d->batch; ++b) {
    const modal_instance& I = d->inst[b];
    f.add_int(I.kind);
    f.add_int(I.n_t);
    f.add_int(I.n_in);
    f.add_int(I.mode_class != nullptr);
    f.add_int(I.h_row_scale != nullptr);
  }
  char buf[17];
  snprintf(buf, sizeof buf, "%016llx", (unsigned long long)f.h);
  key = buf;
  return MODAL_OK;
}

// The integer after "name": in the JSON object text that follows `from`.
bool json_int(const std::string& text, size_t from, size_t to, const char* name, int& v) {
  const std::string pat = std::string("\"") + name + "\"";
  const size_t p = text.find(pat, from);
  if (p == std::string::npos || p >= to) return false;
  const size_t c = text.find(':', p + pat.size());
  if (c == std::string::npos || c >= to) return false;
  char* end = nullptr;
  const long x = std::strtol(text.c_str() + c + 1, &end, 10);
  if (end == text.c_str() + c + 1) return false;
  v = (int)x;
  return true;
}

// Launch shape for `d` from the autotuner's cache, if listed.
bool tuned_shape(const modal_desc* d, int& waves, int& max_wg, int& split_kb) {
  FILE* fp = std::fopen(d->tune_cache, "rb");
  if (!fp) return false;
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof buf, fp)) > 0) text.append(buf, n);
  std::fclose(fp);
  std::string key;
  if (tune_key(d, key)) return false;
  const size_t k = text.find("\"" + key + "\"");
  if (k == std::string::npos) return false;
  const size_t end = text.find('}', k);
  int w = 0, m = 0;
  if (!json_int(text, k, end, "waves", w) || !json_int(text, k, end, "max_workgroups", m)) return false;
  if ((w != 1 && w != 4 && w != 8) || m < 1) return false;
  waves = w;
  max_wg = m;
  int sk = 0;  // optional: the planner's per-slab exchange cost
  if (json_int(text, k, end, "split_cost_kb", sk) && sk > 0 && sk <= (1 << 20) && split_kb == 0) split_kb = sk;
  return true;
}

}  // namespace

int modal_tune_key(const modal_desc* d, char* out, int32_t len) {
  if (!out || len < 17) return fail(MODAL_EINVAL, "out NULL or len < 17");
  int rc = validate(d);
  if (rc) return rc;
  std::string key;
  rc = tune_key(d, key);
  if (rc) return rc;
  std::memcpy(out, key.c_str(), 17);
  return MODAL_OK;
}

int modal_init(modal_ctx** out, const modal_desc* d_in, void* stream_) {
  if (!out) return fail(MODAL_EINVAL, "out is NULL");
  *out = nullptr;
  g_err.clear();
  int rc = validate(d_in);
  if (rc) return rc;
  // the autotuner's launch shape for this batch, if cached
  modal_desc tuned = *d_in;
  if (d_in->tune_cache && d_in->waves == 0 && d_in->max_workgroups == 0)
    (void)tuned_shape(d_in, tuned.waves, tuned.max_workgroups, tuned.split_cost_kb);
  const modal_desc* d = &tuned;
  hipStream_t stream = (hipStream_t)stream_;
  const double T = 1.0 / d->fs;
  int device = 0;
  HIP_TRY(hipGetDevice(&device));
  {
    void* sp = nullptr;  // modal_run_noalloc's scratch, once per device
    HIP_TRY(resolve_scratch(device, &sp));
  }
  modal_ctx* c = new modal_ctx();
  c->device = device;
  c->batch = d->batch;
  c->scheme = d->scheme;
  c->flags = d->flags;
  c->fs = d->fs;
  c->chunk = d->chunk_steps;
  {
    bool all_linear = !(d->flags & (MODAL_FLAG_GRAD | MODAL_FLAG_RECURSE));
    for (int b = 0; b < d->batch && all_linear; ++b) all_linear = d->inst[b].kind == MODAL_KIND_LINEAR;
    if (all_linear && linear_modes(d, c)) {
      int r = init_linear(c, d, stream);
      if (r) {
        free_ctx(c);
        return r;
      }
      *out = c;
      return MODAL_OK;
    }
    c->lz1.clear(); c->lz2.clear(); c->lA.clear(); c->lB.clear(); c->lC.clear();
    c->lc.clear(); c->lb.clear(); c->le.clear();
  }
  {
    std::vector<SharedGroup> groups = shared_groups(d);
    if (!groups.empty()) {
      int r = init_shared(c, d, groups, stream);
      if (!r) r = modal_reset(c, stream_);
      if (!r && hipStreamSynchronize(stream) != hipSuccess) r = fail(MODAL_EHIP, "hipStreamSynchronize");
      if (r) {
        free_ctx(c);
        return r;
      }
      *out = c;
      return MODAL_OK;
    }
  }

  // ---------------- instance layout
  std::vector<InstDev> inst(d->batch);
  long long h_floats = 0, e_floats = 0;
  int mode_floats = 0;
  std::vector<double> row_cost(d->batch), fixed_cost(d->batch);
  int red_floats = 0;
  std::vector<int> qs_of(d->batch, 1), J_of(d->batch, 1);
  int dev0 = 0;
  HIP_TRY(hipGetDevice(&dev0));
  hipDeviceProp_t prop0;
  HIP_TRY(hipGetDeviceProperties(&prop0, dev0));
  bool latency = d->waves == 0 && d->max_workgroups == 0 && !(d->flags & MODAL_FLAG_SPLIT_ANY) &&
                 d->batch <= prop0.multiProcessorCount;
  if (latency) {
    double dense = 0.0;
    for (int b = 0; b < d->batch; ++b)
      if (d->inst[b].kind == MODAL_KIND_VK) dense += 4.0 * d->inst[b].n_in * (double)d->inst[b].n_t * d->inst[b].n_t;
    latency = dense <= kLatencyBytes;
  }
  // On-chip plan: a forward-only latency-bound batch whose instances each
  // fit one workgroup's registers (at most 64 modes; a von Karman tensor of
  // at most kChipWaves * rows in-plane rows) steps every instance in one
  // workgroup that holds its tensor for the launch, with no exchange
  // between workgroups.
  int chip_nt = 0, chip_rows = 0;
  std::vector<ChipMap> chip_maps;
  // A batch with no tensor at all (tension-modulated and linear instances,
  // each of at most kChipWaveModes modes) takes the one-wave variant.
  bool chip_wave = latency && !(d->flags & MODAL_FLAG_GRAD);
  for (int b = 0; b < d->batch && chip_wave; ++b)
    chip_wave = d->inst[b].kind != MODAL_KIND_VK && d->inst[b].n_t <= kChipWaveModes;
  if (latency && !(d->flags & MODAL_FLAG_GRAD) && !chip_wave) {
    int max_w = 0, max_rows = 0;
    bool ok = true;
    chip_maps.resize(d->batch);
    for (int b = 0; b < d->batch && ok; ++b) {
      int w = 0, r = 0;
      ok = chip_map(d->inst[b], chip_maps[b], w, r);
      max_w = std::max(max_w, w);
      max_rows = std::max(max_rows, r);
    }
    ok = ok && chip_shape(max_w, max_rows, chip_nt, chip_rows);
    if (!ok) {
      chip_nt = chip_rows = 0;
      chip_maps.clear();
    }
  }
  std::vector<BlockPlan> plans;
  if (!latency) plan_blocks(d, plans);
  else plans.assign(d->batch, BlockPlan{});
  std::vector<int> jmap_pool;
  c->mode_slot.assign(d->batch, {});
  for (int b = 0; b < d->batch; ++b) {
    const modal_instance& I = d->inst[b];
    InstDev& D = inst[b];
    D.kind = I.kind;
    D.nt = I.n_t;
    D.nin = I.kind == MODAL_KIND_VK ? I.n_in : 0;
    D.ntp = round4(I.n_t);
    if (plans[b].ok) {
      const BlockPlan& bp = plans[b];
      D.ntp = bp.cls[4];
      D.blk = 1;
      D.w = bp.w;
      for (int i = 0; i < 5; ++i) D.cls[i] = bp.cls[i];
      D.jmap_off = (long long)jmap_pool.size() / 4;
      for (int n = 0; n < D.nin; ++n) {
        for (int i = 0; i < 4; ++i) {  // with each stored block's rows per piece and pieces
        int je = bp.jmap[(size_t)n * 4 + i];
        const int R = bp.cls[i + 1] - bp.cls[i];
        if (je >= 0 && R > 0) {
          const int tlen = (bp.cls[(je & 7) + 1] - bp.cls[je & 7]) / 4;
          const int qs = std::min(R, (kSweepLoads * kWave) / tlen);
          je |= (qs << 4) | (((R + qs - 1) / qs) << 13);
        }
        jmap_pool.push_back(je);
      }
        jmap_pool.insert(jmap_pool.end(), bp.boff.begin() + 4 * n, bp.boff.begin() + 4 * n + 4);
      }
      c->mode_slot[b] = bp.mode_slot;
    }
    D.mode_off = mode_floats;
    mode_floats += D.ntp;
    D.kappa = (float)I.kappa;
    D.out_row = b;
    D.e_off = e_floats;
    D.n_exc = I.n_exc;
    e_floats += I.n_exc;
    D.h_off = 0;
    if (I.kind == MODAL_KIND_VK) {
      D.h_off = h_floats;
      D.row_off = c->rows_total;
      c->rows_total += D.nin;
      c->dense_bytes += 4LL * D.nin * D.nt * D.nt;
      c->flops += 2LL * D.nin * D.nt * D.nt + 4LL * D.nin * D.nt;
      if (D.blk) {
        const long long f = plans[b].floats;
        h_floats += (f + 63) & ~63LL;
        c->coupling_bytes += plans[b].stored_bytes;
        c->padded_bytes += 4 * f;
        c->n_blocked++;
        choose_sweep(plans[b].rmax, D.w / 4, qs_of[b], J_of[b]);
        // reduction buffer (one piece's slot layout), per-slot row dot
        // partials, row-dot vector
        red_floats = std::max(red_floats, 4 * kSweepLoads * kWave + kSweepLoads * kWave + D.ntp);
      } else {
        const long long f = (long long)D.nin * D.nt * D.ntp;
        h_floats += (f + 63) & ~63LL;  // 256-byte aligned instances
        c->coupling_bytes += 4LL * D.nin * D.nt * D.nt;
        c->padded_bytes += 4 * f;
        choose_sweep(D.nt, D.ntp / 4, qs_of[b], J_of[b]);
        // row double buffer; in latency-bound plans also two parked partial
        // rows (a row shared by several waves of a one-unit workgroup)
        red_floats = std::max(red_floats, 2 * qs_of[b] * D.ntp + (latency ? 2 * D.ntp : 0));
      }
    }
    unit_costs(I, row_cost[b], fixed_cost[b], &plans[b]);
  }
  c->mode_floats = mode_floats;
  for (int b = 0; b < d->batch; ++b) {
    const int g = (inst[b].ntp / 4 + kWave - 1) / kWave;
    c->gm = std::max(c->gm, g <= 1 ? 1 : (g <= 2 ? 2 : 4));
  }
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, dev));
  // Waves per workgroup.  A batch of small instances, at most one per CU, is
  // bound by the latency of each step rather than by bytes: eight waves share
  // a unit's rows when their reduction space fits the LDS (a single 40/40
  // plate steps in 10.4 us instead of 16.2 us).  Larger batches stream with
  // four waves and three workgroups per CU.
  c->nw = d->waves == 0 ? 4 : d->waves;
  if (d->waves == 0 && d->batch <= prop.multiProcessorCount) {
    bool small = true;
    if (!latency)
      for (int b = 0; b < d->batch && small; ++b)
        small = row_cost[b] * (inst[b].kind == KIND_VK ? inst[b].nin : 1) < kMinSplitCost;
    int o8 = 0;
    if (small) HIP_TRY(step_occupancy(&o8, c->gm, 8, step_lds_bytes(8, red_floats)));
    if (o8 >= 1) c->nw = 8;
  }
  c->lds_bytes = step_lds_bytes(c->nw, red_floats);

  // ---------------- partition over co-resident workgroups
  int occ = 0;
  HIP_TRY(step_occupancy(&occ, c->gm, c->nw, c->lds_bytes));
  c->red_floats = red_floats;
  if (d->flags & MODAL_FLAG_GRAD) {
    // the reverse kernel (with or without a tangent) must fit as many
    // co-resident workgroups as the plan uses; it shares the step kernel's
    // partition but may divide a unit's rows among fewer waves when its
    // reduction space does not fit the LDS with as many
    for (int tan = 0; tan < 2; ++tan) {
      int o = 0;
      c->nw_grad[tan] = c->nw;
      for (;;) {
        c->grad_lds_v[tan] = grad_lds_bytes(c->nw_grad[tan], (tan ? 3 : 2) * red_floats);
        HIP_TRY(grad_occupancy(&o, c->gm, tan == 1, c->nw_grad[tan], false, c->grad_lds_v[tan]));
        if (latency && o >= 1 && c->nw_grad[tan] > 1) {
          // the variant whose waves share a one-unit workgroup's row blocks
          int o2 = 0;
          HIP_TRY(grad_occupancy(&o2, c->gm, tan == 1, c->nw_grad[tan], true, c->grad_lds_v[tan]));
          o = std::min(o, o2);
        }
        if (o >= 1 || c->nw_grad[tan] == 1) break;
        c->nw_grad[tan] = c->nw_grad[tan] == 8 ? 4 : 1;
      }
      occ = std::min(occ, o);
    }
  }
  if (occ < 1) {
    free_ctx(c);
    return fail(MODAL_EHIP, "step kernel does not fit on a CU");
  }
  c->occ = occ;
  // Default budget per CU.  Measured on the 256-plate batch: with four
  // waves, 3 workgroups per CU (the occupancy limit) stream the parity-blocked
  // batch 17 % faster than 2, and the dense one at 6.1 TB/s (2: 6.4, 4: 5.6);
  // with one wave, 6 per CU reach 6.1 TB/s dense.  An explicit
  // max_workgroups (e.g. from the autotuner) overrides it.
  const int wg_per_cu = c->nw > 1 ? 3 : 6;
  int n_bins = occ * prop.multiProcessorCount;
  if (d->max_workgroups > 0) n_bins = std::min(n_bins, d->max_workgroups);
  else n_bins = std::min(n_bins, wg_per_cu * prop.multiProcessorCount);
  n_bins = std::max(1, std::min(n_bins, 1 << 20));
  double total = 0;
  for (int b = 0; b < d->batch; ++b)
    total += fixed_cost[b] + (inst[b].kind == KIND_VK ? inst[b].nin : 1) * row_cost[b];
  std::vector<Unit> units;
  std::vector<int> bin_of;
  std::vector<double> load;
  if (latency) {
    // one slab per workgroup, instances cut into slabs of about kLatencyRows
    // rows; only for a few instances: with many, the per-step exchanges of
    // all their slabs cost more than the rows they spread (64 plates at
    // 40/40 in 4 slabs each step in 16 us instead of 12)
    const int cap_slabs = d->batch > kLatencyMaxSplitBatch
                              ? 1
                              : std::max(1, prop.multiProcessorCount / d->batch);
    for (int b = 0; b < d->batch; ++b) {
      const int rows = inst[b].kind == KIND_VK ? inst[b].nin : 1;
      const double bytes = inst[b].kind == KIND_VK ? 4.0 * inst[b].nin * (double)inst[b].nt * inst[b].nt : 0.0;
      const int by_rows = (rows + kLatencyRows / 2) / kLatencyRows;
      const double slab_bytes = bytes > kLatencyBigTensor ? 0.5 * kLatencySlabBytes : kLatencySlabBytes;
      const int by_bytes = (int)std::ceil(bytes / slab_bytes);
      const int S = inst[b].kind == KIND_VK && !chip_nt
                        ? std::max(1, std::min({cap_slabs, rows, std::max(by_rows, by_bytes)}))
                        : 1;
      for (int sl = 0; sl < S; ++sl) {
        const int r0 = (int)((long long)rows * sl / S), r1 = (int)((long long)rows * (sl + 1) / S);
        const double cost = (S > 1 ? split_cost(d) : 0.0) + fixed_cost[b] + (r1 - r0) * row_cost[b];
        units.push_back({b, r0, r1, sl, cost});
        bin_of.push_back((int)load.size());
        load.push_back(cost);
      }
    }
    if ((int)load.size() > n_bins) {
      units.clear();
      bin_of.clear();
      load.clear();
      latency = false;
    }
  }
  if (!latency && !plan_batch(d, row_cost, fixed_cost, total, n_bins, units, bin_of, load)) {
    free_ctx(c);
    return fail(MODAL_EINVAL, "batch does not fit the workgroup budget");
  }
  c->makespan = *std::max_element(load.begin(), load.end());
  c->mean_load = total / n_bins;
  // workgroups actually used, renumbered densely; within a workgroup split
  // units come first so their partial forces are published early
  std::vector<int> used(n_bins, -1);
  int n_wg = 0;
  for (size_t i = 0; i < units.size(); ++i)
    if (used[bin_of[i]] < 0) used[bin_of[i]] = n_wg++;
  std::vector<int> nslab(d->batch, 0);
  for (auto& u : units) nslab[u.inst]++;
  std::vector<int> order(units.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const int wa = used[bin_of[a]], wb = used[bin_of[b]];
    if (wa != wb) return wa < wb;
    const bool sa = nslab[units[a].inst] > 1, sb = nslab[units[b].inst] > 1;
    if (sa != sb) return sa;
    return units[a].inst < units[b].inst;
  });
  std::vector<UnitDev> udev(units.size());
  std::vector<int> wg_begin(n_wg + 1, 0);
  int state_floats = 0;
  c->unit_state_of_inst.assign(d->batch, -1);
  for (size_t k = 0; k < order.size(); ++k) {
    const Unit& u = units[order[k]];
    UnitDev& U = udev[k];
    U.inst = u.inst;
    U.row0 = u.row0;
    U.row1 = u.row1;
    U.slab = u.slab;
    U.state_off = state_floats;
    if (c->unit_state_of_inst[u.inst] < 0) c->unit_state_of_inst[u.inst] = state_floats;
    state_floats += inst[u.inst].ntp;
    U.qs = qs_of[u.inst];
    U.J = J_of[u.inst];
    U.pad = 0;
    wg_begin[used[bin_of[order[k]]] + 1] = (int)k + 1;
  }
  for (int w = 1; w <= n_wg; ++w) wg_begin[w] = std::max(wg_begin[w], wg_begin[w - 1]);
  long long part_floats = 0;
  int n_ctr = 0;
  for (int b = 0; b < d->batch; ++b) {
    inst[b].nslab = nslab[b];
    inst[b].ctr_off = n_ctr;
    n_ctr += std::max(1, nslab[b]);
    inst[b].part_off = part_floats;
    if (nslab[b] > 1) {
      part_floats += 2LL * nslab[b] * inst[b].ntp;
      c->n_split++;
    }
  }
  c->n_wg = n_wg;
  c->n_units = (int)udev.size();
  c->n_ctr = n_ctr;
  // A latency-bound plan gives every workgroup one unit; its state and
  // coefficients then stay in LDS for the whole launch, which takes the
  // global round trips of the output and the update out of every step (a
  // lone 100/100 plate in 15 slabs steps in 12.0 us instead of 12.5, a
  // Berger plate in 2.4 us instead of 2.9).  Only
  // when the variant still fits every planned workgroup on the chip at once.
  c->res_stride = 0;
  if (latency && chip_nt && n_wg == d->batch) {
    c->chip_nt = chip_nt;
    c->chip_rows = chip_rows;
    c->nw = kChipWaves;
    c->lds_bytes = 0;
  } else if (latency && chip_wave && n_wg == d->batch) {
    int nt_max = 1;
    for (int b = 0; b < d->batch; ++b) nt_max = std::max(nt_max, d->inst[b].n_t);
    c->chip_wave = (nt_max + kWave - 1) / kWave;
    c->nw = 1;
    c->lds_bytes = 0;
  } else if (latency && n_wg == (int)udev.size() && (c->nw == 4 || c->nw == 8)) {
    int S = 0;
    for (int b = 0; b < d->batch; ++b) S = std::max(S, inst[b].ntp);
    const size_t lb = step_lds_bytes(c->nw, red_floats, S);
    int o = 0;
    HIP_TRY(step_occupancy(&o, c->gm, c->nw, lb, true));
    if (S > 0 && o >= 1 && (long long)o * prop.multiProcessorCount >= n_wg) {
      c->res_stride = S;
      c->lds_bytes = lb;
    }
  }
  c->state_floats = state_floats;
  c->units = udev;
  c->inst_host = inst;
  c->h_floats = h_floats;
  c->part_floats = part_floats;
  for (int b = 0; b < d->batch; ++b) {
    c->kind.push_back(d->inst[b].kind);
    for (int k = 0; k < d->inst[b].n_t; ++k) {
      c->omega.push_back(d->inst[b].omega[k]);
      c->gamma.push_back(d->inst[b].gamma[k]);
    }
  }

  // ---------------- coefficients, initial state
  std::vector<float> coef(9 * (size_t)mode_floats, 0.f);
  float *m_hi = &coef[0], *m_lo = m_hi + mode_floats, *p_hi = m_lo + mode_floats,
        *p_lo = p_hi + mode_floats, *r_hi = p_lo + mode_floats, *r_lo = r_hi + mode_floats,
        *cw = r_lo + mode_floats, *lam = cw + mode_floats, *bx = lam + mode_floats;
  c->nt.resize(d->batch);
  c->inst_mode_off.resize(d->batch);
  std::vector<float> xinit(4 * (size_t)mode_floats, 0.f);
  for (int b = 0; b < d->batch; ++b) {
    const modal_instance& I = d->inst[b];
    const int o = inst[b].mode_off;
    c->nt[b] = I.n_t;
    c->inst_mode_off[b] = o;
    const std::vector<int>& ms = c->mode_slot[b];
    for (int k = 0; k < I.n_t; ++k) {
      const int e = o + (ms.empty() ? k : ms[k]);  // internal slot of caller mode k
      const Coef q = coefficients(d->scheme, I.omega[k], I.gamma[k], T);
      split(q.m, m_hi[e], m_lo[e]);
      split(q.p, p_hi[e], p_lo[e]);
      split(q.r, r_hi[e], r_lo[e]);
      cw[e] = (float)I.c_out[k];
      lam[e] = I.lambda ? (float)I.lambda[k] : 0.f;
      bx[e] = I.b_ext ? (float)I.b_ext[k] : 0.f;
      split(I.x0[k], xinit[e], xinit[mode_floats + e]);
      split(I.x0[k] - I.xm1[k], xinit[2 * mode_floats + e], xinit[3 * mode_floats + e]);
    }
  }
  c->state0.assign(4 * (size_t)state_floats, 0.f);
  for (const UnitDev& U : udev) {
    const int o = inst[U.inst].mode_off, n = inst[U.inst].ntp;
    for (int a = 0; a < 4; ++a)
      std::memcpy(&c->state0[(size_t)a * state_floats + U.state_off], &xinit[(size_t)a * mode_floats + o],
                  sizeof(float) * n);
  }

  // ---------------- device memory
  const size_t meta_bytes = sizeof(InstDev) * d->batch + sizeof(UnitDev) * udev.size() +
                            sizeof(int) * (n_wg + 1);
#define ALLOC(p, bytes)                 \
  do {                                  \
    int r_ = dalloc(&(p), (bytes));     \
    if (r_) {                           \
      free_ctx(c);                      \
      return r_;                        \
    }                                   \
  } while (0)
  ALLOC(c->dH, sizeof(float) * (size_t)(h_floats + 64));
  ALLOC(c->dMeta, meta_bytes);
  ALLOC(c->dCoef, sizeof(float) * coef.size());
  ALLOC(c->dState, sizeof(float) * c->state0.size());
  ALLOC(c->dPart, sizeof(float) * (size_t)(part_floats + 64));
  ALLOC(c->dCtr, sizeof(unsigned int) * n_ctr);
  ALLOC(c->dFlags, sizeof(int) * (2 + 2 * d->batch));
  ALLOC(c->dStep, sizeof(long long));
  ALLOC(c->dE, sizeof(float) * (size_t)(e_floats + 1));
  ALLOC(c->dJmap, sizeof(int) * (jmap_pool.size() + 4));
  if (c->chip_nt) ALLOC(c->dChip, sizeof(ChipMap) * chip_maps.size());
#undef ALLOC
  auto bail = [&](int r) {
    free_ctx(c);
    return r;
  };
#define HIP_TRY_C(expr)                                                                   \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return bail(fail(MODAL_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)));   \
  } while (0)
  HIP_TRY_C(hipMemsetAsync(c->dH, 0, sizeof(float) * (size_t)(h_floats + 64), stream));
  {
    int r = upload_tensors(c, d, inst, plans, stream);
    if (r) return bail(r);
    if (!jmap_pool.empty())
      HIP_TRY_C(hipMemcpyAsync(c->dJmap, jmap_pool.data(), sizeof(int) * jmap_pool.size(),
                               hipMemcpyHostToDevice, stream));
    if (c->chip_nt)
      HIP_TRY_C(hipMemcpyAsync(c->dChip, chip_maps.data(), sizeof(ChipMap) * chip_maps.size(),
                               hipMemcpyHostToDevice, stream));
  }
  char* meta = (char*)c->dMeta;
  InstDev* dInst = (InstDev*)meta;
  UnitDev* dUnit = (UnitDev*)(meta + sizeof(InstDev) * d->batch);
  int* dWg = (int*)(meta + sizeof(InstDev) * d->batch + sizeof(UnitDev) * udev.size());
  HIP_TRY_C(hipMemcpyAsync(dInst, inst.data(), sizeof(InstDev) * d->batch, hipMemcpyHostToDevice, stream));
  HIP_TRY_C(hipMemcpyAsync(dUnit, udev.data(), sizeof(UnitDev) * udev.size(), hipMemcpyHostToDevice, stream));
  HIP_TRY_C(hipMemcpyAsync(dWg, wg_begin.data(), sizeof(int) * (n_wg + 1), hipMemcpyHostToDevice, stream));
  HIP_TRY_C(hipMemcpyAsync(c->dCoef, coef.data(), sizeof(float) * coef.size(), hipMemcpyHostToDevice, stream));
  {
    std::vector<float> epool((size_t)e_floats + 1, 0.f);
    for (int b = 0; b < d->batch; ++b)
      if (d->inst[b].n_exc > 0)
        std::memcpy(&epool[inst[b].e_off], d->inst[b].e_ext, sizeof(float) * d->inst[b].n_exc);
    HIP_TRY_C(hipMemcpyAsync(c->dE, epool.data(), sizeof(float) * epool.size(), hipMemcpyHostToDevice, stream));
    // symmetry / finiteness of the tensors
    HIP_TRY_C(hipMemsetAsync(c->dFlags, 0, sizeof(int) * (2 + 2 * d->batch), stream));
    HIP_TRY_C(launch_check(c->dH, dInst, d->batch, c->dFlags + 2, stream));
    std::vector<int> chk(2 * d->batch);
    HIP_TRY_C(hipMemcpyAsync(chk.data(), c->dFlags + 2, sizeof(int) * chk.size(), hipMemcpyDeviceToHost, stream));
    HIP_TRY_C(hipStreamSynchronize(stream));
    for (int b = 0; b < d->batch; ++b) {
      if (inst[b].kind != KIND_VK) continue;
      float dmax, hmax;
      std::memcpy(&dmax, &chk[2 * b], 4);
      std::memcpy(&hmax, &chk[2 * b + 1], 4);
      if (!std::isfinite(dmax) || !std::isfinite(hmax))
        return bail(fail(MODAL_EINVAL, "non-finite H (instance " + std::to_string(b) + ")"));
      if (dmax > 1e-6f * hmax)
        return bail(fail(MODAL_EINVAL, "H not symmetric in its last two indices (instance " +
                                           std::to_string(b) + ")"));
    }
  }
  StepParams& P = c->P;
  P.inst = dInst;
  P.jmap = c->dJmap;
  P.unit = dUnit;
  P.wg_begin = dWg;
  P.H = c->dH;
  P.m_hi = c->dCoef;
  P.m_lo = P.m_hi + mode_floats;
  P.p_hi = P.m_lo + mode_floats;
  P.p_lo = P.p_hi + mode_floats;
  P.r_hi = P.p_lo + mode_floats;
  P.r_lo = P.r_hi + mode_floats;
  P.c_out = P.r_lo + mode_floats;
  P.lam = P.c_out + mode_floats;
  P.b_ext = P.lam + mode_floats;
  P.e_ext = c->dE;
  P.x_hi = c->dState;
  P.x_lo = P.x_hi + state_floats;
  P.d_hi = P.x_lo + state_floats;
  P.d_lo = P.d_hi + state_floats;
  P.part = c->dPart;
  P.ctr = c->dCtr;
  P.flags = c->dFlags;
  P.timeout_ticks = d->barrier_us > 0 ? 100ull * (unsigned long long)d->barrier_us : kBarrierTicks;
  P.step_base = c->dStep;
  P.red_floats = red_floats;
  P.mode_floats = mode_floats;
  P.res_stride = c->res_stride;
  P.chip = c->dChip;
#undef HIP_TRY_C
  int r = modal_reset(c, stream_);
  if (r) return bail(r);
  HIP_TRY(hipStreamSynchronize(stream));
  *out = c;
  return MODAL_OK;
}

int modal_reset(modal_ctx* c, void* stream_) {
  if (!c) return fail(MODAL_EINVAL, "ctx is NULL");
  hipStream_t s = (hipStream_t)stream_;
  if (c->linear) {
    HIP_TRY(hipMemsetAsync(c->dFlags, 0, sizeof(int) * 2, s));
    c->steps = 0;
    return MODAL_OK;
  }
  HIP_TRY(hipMemcpyAsync(c->dState, c->state0.data(), sizeof(float) * c->state0.size(),
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemsetAsync(c->dCtr, 0, sizeof(unsigned int) * c->n_ctr, s));
  HIP_TRY(hipMemsetAsync(c->dFlags, 0, sizeof(int) * 2, s));
  HIP_TRY(hipMemsetAsync(c->dStep, 0, sizeof(long long), s));
  c->steps = 0;
  c->ckpt_broken = false;  // checkpoints of [0, ckpt_upto) stay valid
  c->ctr_stale = false;
  return MODAL_OK;
}

static int enqueue_run(modal_ctx* c, int64_t n_steps, float* y, int64_t y_stride, hipStream_t s) {
  const int64_t chunk = c->chunk > 0 ? c->chunk : n_steps;
  for (int64_t done = 0; done < n_steps; done += chunk) {
    const int64_t k = std::min<int64_t>(chunk, n_steps - done);
    if (c->shared) {
      SharedParams P = c->SP;
      P.y = y + done;
      P.y_stride = y_stride;
      P.n_steps = (int)k;
      HIP_TRY(launch_shared(P, c->sh_kt, c->sh_kc, c->sh_jt, c->n_wg, s));
    } else {
      StepParams P = c->P;
      P.y = y + done;
      P.y_stride = y_stride;
      P.n_steps = (int)k;
      if (c->run_ckpt) {
        P.ckpt = c->dCkpt;
        P.ckpt_every = kRunCkpt;
      }
      if (c->run_rec) {
        P.rec_x = c->dRecAll;
        P.rec_d = c->dRecAll + (size_t)c->recall_cap * c->mode_floats;
        P.rec_base = 0;
      }
      if (c->chip_wave)
        HIP_TRY(launch_chip_wave(P, c->chip_wave, c->n_wg, s));
      else if (c->chip_nt)
        HIP_TRY(launch_chip(P, c->chip_nt, c->chip_rows, c->n_wg, s));
      else
        HIP_TRY(launch_step(P, c->gm, c->nw, c->n_wg, c->lds_bytes, s));
    }
    HIP_TRY(launch_advance(c->dStep, (int)k, s));
  }
  return MODAL_OK;
}

int modal_check(modal_ctx* c, void* stream_) {
  if (!c) return fail(MODAL_EINVAL, "ctx is NULL");
  hipStream_t s = (hipStream_t)stream_;
  int fl[2] = {0, 0};
  HIP_TRY(hipMemcpyAsync(fl, c->dFlags, sizeof(fl), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (fl[0]) return fail(MODAL_EHANG, "a per-instance step barrier timed out");
  if (fl[1]) return fail(MODAL_ENONFINITE, "a modal state became non-finite");
  return MODAL_OK;
}

int modal_run(modal_ctx* c, int64_t n_steps, float* y, int64_t y_stride, void* stream_) {
  if (!c) return fail(MODAL_EINVAL, "ctx is NULL");
  if (n_steps < 0 || n_steps > (1LL << 31) - 1) return fail(MODAL_EINVAL, "n_steps out of range");
  if (n_steps == 0) return MODAL_OK;
  if (!y || y_stride < n_steps) return fail(MODAL_EINVAL, "y NULL or y_stride < n_steps");
  hipStream_t s = (hipStream_t)stream_;
  if (c->linear) {  // closed form at absolute steps: no persistent state, no graph
    int r = run_linear(c, n_steps, y, y_stride, s);
    if (r) return r;
    c->steps += n_steps;
    return MODAL_OK;
  }
  // gradient contexts record checkpoints while they run forward from step 0
  c->run_ckpt = false;
  if ((c->flags & MODAL_FLAG_GRAD) && !(c->flags & MODAL_FLAG_GRAPH) && !c->shared) {
    if (c->ckpt_broken || c->steps > c->ckpt_upto) {
      c->ckpt_broken = true;
    } else {
      const long long need = (c->steps + n_steps + kRunCkpt - 1) / kRunCkpt * 4LL * c->mode_floats;
      if (c->ckpt_floats < need && c->steps > 0) {
        c->ckpt_broken = true;  // growing would lose the slots already taken
      } else {
        if (c->ckpt_floats < need) {
          if (c->dCkpt) HIP_TRY(hipFree(c->dCkpt));
          c->dCkpt = nullptr;
          c->ckpt_floats = 0;
          c->ckpt_upto = 0;
          int r = dalloc(&c->dCkpt, sizeof(float) * (size_t)need);
          if (r) return r;
          c->ckpt_floats = need;
        }
        c->run_ckpt = true;
      }
    }
  }
  // and the whole trajectory, contiguous from step 0, while it fits
  c->run_rec = false;
  if (c->run_ckpt && c->steps <= c->rec_upto &&
      (double)(c->steps + n_steps) * 2.0 * c->mode_floats * sizeof(float) <= kRecAllBytes) {
    if (c->recall_cap >= c->steps + n_steps) {
      c->run_rec = true;
    } else if (c->steps == 0) {
      if (c->dRecAll) HIP_TRY(hipFree(c->dRecAll));
      c->dRecAll = nullptr;
      c->recall_cap = 0;
      c->rec_upto = 0;
      int r = dalloc(&c->dRecAll, sizeof(float) * 2 * (size_t)n_steps * c->mode_floats);
      if (r) return r;
      c->recall_cap = n_steps;
      c->run_rec = true;
    }
  }
  if (c->ctr_stale) {
    HIP_TRY(launch_ctr_fill(c->P.inst, c->batch, c->dStep, c->dCtr, s));
    c->ctr_stale = false;
  }
  if (c->flags & MODAL_FLAG_GRAPH) {
    hipGraphExec_t exec = nullptr;
    for (auto& g : c->graphs)
      if (g.n == n_steps && g.y == y && g.stride == y_stride) exec = g.exec;
    if (!exec) {
      // The caller's stream may be the legacy default stream, which cannot
      // be captured; record on a private stream and launch on the caller's.
      if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
      hipGraph_t graph;
      HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
      int r = enqueue_run(c, n_steps, y, y_stride, c->cap_stream);
      hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
      if (r) return r;
      if (e != hipSuccess) return fail(MODAL_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
      e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) return fail(MODAL_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
      c->graphs.push_back({n_steps, y_stride, y, exec});
    }
    HIP_TRY(hipGraphLaunch(exec, s));
  } else {
    const bool recorded = c->run_ckpt, recorded_all = c->run_rec;
    int r = enqueue_run(c, n_steps, y, y_stride, s);
    c->run_ckpt = false;
    c->run_rec = false;
    if (r) return r;
    if (recorded) c->ckpt_upto = std::max(c->ckpt_upto, c->steps + n_steps);
    if (recorded_all) c->rec_upto = std::max(c->rec_upto, c->steps + n_steps);
  }
  c->steps += n_steps;
  if (c->flags & MODAL_FLAG_ASYNC) return MODAL_OK;
  return modal_check(c, stream_);
}

int modal_run_noalloc(modal_ctx* c, int64_t n_steps, float* y, int64_t y_stride, void* stream_) {
  if (!c) return fail(MODAL_EINVAL, "ctx is NULL");
  if (n_steps < 0 || n_steps > (1LL << 31) - 1) return fail(MODAL_EINVAL, "n_steps out of range");
  if (n_steps == 0) return MODAL_OK;
  if (!y || y_stride < n_steps) return fail(MODAL_EINVAL, "y NULL or y_stride < n_steps");
  if (c->linear || c->shared)
    return fail(MODAL_ESTATE, "modal_run_noalloc steps the persistent recursion only; this context "
                              "runs the linear closed form or the shared-tensor path (use modal_run)");
  // scratch layout: arrival words [n_ctr] at 0, partial forces from the next
  // 256-byte boundary (the layout of the context's own buffers)
  const size_t ctr_bytes = (sizeof(unsigned int) * (size_t)c->n_ctr + 255) & ~(size_t)255;
  const size_t need = ctr_bytes + sizeof(float) * (size_t)(c->part_floats + 64);
  if (need > kScratchBytes)
    return fail(MODAL_EINVAL, "modal_run_noalloc: the batch's partial forces and arrival words need " +
                                  std::to_string(need) + " bytes; the scratch holds " +
                                  std::to_string(kScratchBytes) + " (use modal_run)");
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != c->device) return fail(MODAL_ESTATE, "the current device is not the context's");
  void* sp = nullptr;
  HIP_TRY(resolve_scratch(dev, &sp));  // resolved by modal_init: no allocation here
  unsigned char* base = static_cast<unsigned char*>(sp);
  unsigned int* ctr = reinterpret_cast<unsigned int*>(base);
  float* part = reinterpret_cast<float*>(base + ctr_bytes);
  hipStream_t s = (hipStream_t)stream_;
  // another call may have left other words behind: set them to where this
  // context's steps stand (a fill kernel, so a capturing caller records no
  // memset node)
  HIP_TRY(launch_ctr_fill(c->P.inst, c->batch, c->dStep, ctr, s));
  const int64_t chunk = c->chunk > 0 ? c->chunk : n_steps;
  for (int64_t done = 0; done < n_steps; done += chunk) {
    const int64_t k = std::min<int64_t>(chunk, n_steps - done);
    StepParams P = c->P;
    P.part = part;
    P.ctr = ctr;
    P.y = y + done;
    P.y_stride = y_stride;
    P.n_steps = (int)k;
    if (c->chip_wave)
      HIP_TRY(launch_chip_wave(P, c->chip_wave, c->n_wg, s));
    else if (c->chip_nt)
      HIP_TRY(launch_chip(P, c->chip_nt, c->chip_rows, c->n_wg, s));
    else
      HIP_TRY(launch_step(P, c->gm, c->nw, c->n_wg, c->lds_bytes, s));
    HIP_TRY(launch_advance(c->dStep, (int)k, s));
  }
  // no checkpoints were recorded: a gradient context's recorded checkpoints
  // stop at ckpt_upto, and a later modal_run past them marks them broken
  c->steps += n_steps;
  c->ctr_stale = true;
  if (c->flags & MODAL_FLAG_ASYNC) return MODAL_OK;
  return modal_check(c, stream_);
}

int modal_set_tangent(modal_ctx* c, int32_t b, const float* Hd, void* stream_) {
  if (!c || !Hd) return fail(MODAL_EINVAL, "NULL argument");
  if (c->shared) return fail(MODAL_ESTATE, "tangents need a context created with MODAL_FLAG_GRAD");
  if (b < 0 || b >= c->batch || c->kind[b] != MODAL_KIND_VK)
    return fail(MODAL_EINVAL, "tangent needs a VK instance index");
  hipStream_t s = (hipStream_t)stream_;
  if (!c->dHd) {
    int r = dalloc(&c->dHd, sizeof(float) * (size_t)(c->h_floats + 64));
    if (r) return r;
    HIP_TRY(hipMemsetAsync(c->dHd, 0, sizeof(float) * (size_t)(c->h_floats + 64), s));
  }
  const InstDev& D = c->inst_host[b];
  HIP_TRY(hipMemcpy2DAsync(c->dHd + D.h_off, sizeof(float) * D.ntp, Hd, sizeof(float) * D.nt,
                           sizeof(float) * D.nt, (size_t)D.nin * D.nt, hipMemcpyDefault, s));
  HIP_TRY(hipStreamSynchronize(s));
  c->tangent = true;
  return MODAL_OK;
}

namespace {

// Device copies of a transfer-function call's inputs as float-float pairs
// (split from the host's FP64 values) and room for its outputs; freed when
// the call returns.
struct TfCall {
  float2* coef = nullptr;
  int* off = nullptr;
  FFc* z = nullptr;
  FFc* out = nullptr;  // H, or dL/dH for the gradient
  float2* g = nullptr;
  ~TfCall() {
    for (void* p : {(void*)coef, (void*)off, (void*)z, (void*)out, (void*)g})
      if (p) (void)hipFree(p);
  }
};

int tf_check(const int32_t* mode_off, int32_t batch, int32_t n_freq, int& modes) {
  if (batch < 1 || batch > 65535 || n_freq < 1) return fail(MODAL_EINVAL, "batch or n_freq");
  for (int b = 0; b < batch; ++b)
    if (mode_off[b] < 0 || mode_off[b + 1] < mode_off[b]) return fail(MODAL_EINVAL, "mode_off not increasing");
  modes = mode_off[batch];
  return MODAL_OK;
}

int tf_upload(TfCall& t, const double* coef, const int32_t* mode_off, int32_t batch, const double* omega,
              int32_t n_freq, int modes, hipStream_t s) {
  std::vector<float2> cf(5 * (size_t)std::max(modes, 1));
  for (size_t i = 0; i < 5 * (size_t)modes; ++i) split(coef[i], cf[i].x, cf[i].y);
  std::vector<FFc> zf(n_freq);
  for (int k = 0; k < n_freq; ++k) zf[k] = ffc(std::polar(1.0, omega[k]));
  int r = dalloc(&t.coef, sizeof(float2) * cf.size());
  if (!r) r = dalloc(&t.off, sizeof(int) * (batch + 1));
  if (!r) r = dalloc(&t.z, sizeof(FFc) * n_freq);
  if (!r) r = dalloc(&t.out, sizeof(FFc) * (size_t)batch * n_freq);
  if (r) return r;
  HIP_TRY(hipMemcpyAsync(t.coef, cf.data(), sizeof(float2) * cf.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(t.off, mode_off, sizeof(int) * (batch + 1), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(t.z, zf.data(), sizeof(FFc) * n_freq, hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));  // the host vectors go out of scope
  return MODAL_OK;
}

}  // namespace

int modal_tf_response(const double* coef, const int32_t* mode_off, int32_t batch, const double* omega,
                      int32_t n_freq, double* H, void* stream_) {
  if (!coef || !mode_off || !omega || !H) return fail(MODAL_EINVAL, "NULL argument");
  int modes = 0;
  int r = tf_check(mode_off, batch, n_freq, modes);
  if (r) return r;
  hipStream_t s = (hipStream_t)stream_;
  TfCall t;
  r = tf_upload(t, coef, mode_off, batch, omega, n_freq, modes, s);
  if (r) return r;
  HIP_TRY(launch_tf_response(t.coef, t.off, batch, t.z, n_freq, t.out, s));
  std::vector<FFc> h((size_t)batch * n_freq);
  HIP_TRY(hipMemcpyAsync(h.data(), t.out, sizeof(FFc) * h.size(), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (size_t i = 0; i < h.size(); ++i) {
    H[2 * i] = (double)h[i].rh + (double)h[i].rl;
    H[2 * i + 1] = (double)h[i].ih + (double)h[i].il;
  }
  return MODAL_OK;
}

int modal_tf_grad(const double* coef, const int32_t* mode_off, int32_t batch, int32_t max_modes,
                  const double* omega, int32_t n_freq, const double* dL_dH, double* g_coef, void* stream_) {
  if (!coef || !mode_off || !omega || !dL_dH || !g_coef) return fail(MODAL_EINVAL, "NULL argument");
  int modes = 0;
  int r = tf_check(mode_off, batch, n_freq, modes);
  if (r) return r;
  if (max_modes < 0) return fail(MODAL_EINVAL, "max_modes");
  for (int b = 0; b < batch; ++b)
    if (mode_off[b + 1] - mode_off[b] > max_modes) return fail(MODAL_EINVAL, "an instance has more than max_modes modes");
  hipStream_t s = (hipStream_t)stream_;
  TfCall t;
  r = tf_upload(t, coef, mode_off, batch, omega, n_freq, modes, s);
  if (r) return r;
  std::vector<FFc> gh((size_t)batch * n_freq);
  for (size_t i = 0; i < gh.size(); ++i) {
    split(dL_dH[2 * i], gh[i].rh, gh[i].rl);
    split(dL_dH[2 * i + 1], gh[i].ih, gh[i].il);
  }
  r = dalloc(&t.g, sizeof(float2) * 5 * (size_t)std::max(modes, 1));
  if (r) return r;
  HIP_TRY(hipMemcpyAsync(t.out, gh.data(), sizeof(FFc) * gh.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(launch_tf_grad(t.coef, t.off, batch, max_modes, t.z, n_freq, t.out, t.g, s));
  std::vector<float2> g(5 * (size_t)std::max(modes, 1));
  HIP_TRY(hipMemcpyAsync(g.data(), t.g, sizeof(float2) * g.size(), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int b = 0; b < batch; ++b)
    for (int m = mode_off[b]; m < mode_off[b + 1]; ++m)
      for (int j = 0; j < 5; ++j) g_coef[5 * (size_t)m + j] = (double)g[5 * (size_t)m + j].x + (double)g[5 * (size_t)m + j].y;
  return MODAL_OK;
}

int modal_set_tensor(modal_ctx* c, int32_t b, const float* H, void* stream_) {
  if (!c || !H) return fail(MODAL_EINVAL, "NULL argument");
  if (c->shared || c->linear) return fail(MODAL_ESTATE, "the context keeps no per-instance tensor");
  if (b < 0 || b >= c->batch || c->kind[b] != MODAL_KIND_VK)
    return fail(MODAL_EINVAL, "set_tensor needs a VK instance index");
  const InstDev& D = c->inst_host[b];
  if (D.blk) return fail(MODAL_ESTATE, "the instance's tensor is stored parity-blocked");
  hipStream_t s = (hipStream_t)stream_;
  // the kernels use the symmetry of every row in its last two indices
  hipPointerAttribute_t attr;
  bool on_device = false;
  if (hipPointerGetAttributes(&attr, H) == hipSuccess)
    on_device = attr.type == hipMemoryTypeDevice;
  else
    (void)hipGetLastError();
  bool symmetric = true;
  if (on_device) {
    int bad = 0;
    // the first per-instance check slot (used only while modal_init runs)
    HIP_TRY(hipMemsetAsync(c->dFlags + 2, 0, sizeof(int), s));
    HIP_TRY(launch_sym_check(H, D.nin, D.nt, c->dFlags + 2, s));
    HIP_TRY(hipMemcpyAsync(&bad, c->dFlags + 2, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    symmetric = bad == 0;
  } else {
    const size_t per = (size_t)D.nt * D.nt;
    for (int n = 0; n < D.nin && symmetric; ++n)
      for (int i = 0; i < D.nt && symmetric; ++i)
        for (int j = i + 1; j < D.nt; ++j)
          if (H[n * per + (size_t)i * D.nt + j] != H[n * per + (size_t)j * D.nt + i]) {
            symmetric = false;
            break;
          }
  }
  if (!symmetric) return fail(MODAL_EINVAL, "tensor is not symmetric in its last two indices");
  HIP_TRY(hipMemcpy2DAsync(c->dH + D.h_off, sizeof(float) * D.ntp, H, sizeof(float) * D.nt,
                           sizeof(float) * D.nt, (size_t)D.nin * D.nt, hipMemcpyDefault, s));
  HIP_TRY(hipStreamSynchronize(s));
  c->ckpt_upto = 0;  // recorded checkpoints and trajectory belong to the old tensor
  c->rec_upto = 0;
  return MODAL_OK;
}

int modal_grad(modal_ctx* c, int64_t n_steps, const float* ybar, int64_t y_stride, int32_t ckpt_every,
               double* g_omega, double* g_gamma, double* g_c, double* g_x0, double* g_xm1,
               double* g_scale, double* g_theta, double* g_row, float* const* g_H, void* stream_) {
  if (!c) return fail(MODAL_EINVAL, "ctx is NULL");
  if (!(c->flags & MODAL_FLAG_GRAD)) return fail(MODAL_ESTATE, "context not created with MODAL_FLAG_GRAD");
  if (n_steps < 1 || n_steps > (1LL << 31) - 1 || !ybar || y_stride < n_steps)
    return fail(MODAL_EINVAL, "n_steps, dL_dy or y_stride");
  if (ckpt_every < 0) return fail(MODAL_EINVAL, "ckpt_every < 0");
  const int K = ckpt_every > 0 ? ckpt_every : 512;
  const long long nseg = (n_steps + K - 1) / K;
  hipStream_t s = (hipStream_t)stream_;
  const int mf = c->mode_floats, sf = c->state_floats;
  // checkpoints of the last forward runs, if they cover the steps with this
  // spacing, replace the forward pass
  const bool reuse = K == kRunCkpt && !c->ckpt_broken && c->ckpt_upto >= n_steps &&
                     !(c->flags & MODAL_FLAG_GRAPH) && c->ckpt_floats >= nseg * 4LL * mf;
  // buffers (grown on demand)
  if (c->ckpt_floats < nseg * 4LL * mf) {
    if (c->dCkpt) HIP_TRY(hipFree(c->dCkpt));
    c->dCkpt = nullptr;
    c->ckpt_floats = 0;
    c->ckpt_upto = 0;
    int r = dalloc(&c->dCkpt, sizeof(float) * (size_t)(nseg * 4LL * mf));
    if (r) return r;
    c->ckpt_floats = nseg * 4LL * mf;
  }
  if (c->rec_floats < 2LL * K * mf) {
    if (c->dRec) HIP_TRY(hipFree(c->dRec));
    c->dRec = nullptr;
    c->rec_floats = 0;
    int r = dalloc(&c->dRec, sizeof(float) * (size_t)(2LL * K * mf));
    if (r) return r;
    c->rec_floats = 2LL * K * mf;
  }
  if (g_row && c->rows_total > 0 && c->rrec_floats < (long long)K * c->rows_total) {
    if (c->dRrec) HIP_TRY(hipFree(c->dRrec));
    c->dRrec = nullptr;
    c->rrec_floats = 0;
    int r = dalloc(&c->dRrec, sizeof(float) * (size_t)K * c->rows_total);
    if (!r && !c->dRacc) r = dalloc(&c->dRacc, sizeof(float) * 2 * (size_t)c->rows_total);
    if (r) return r;
    c->rrec_floats = (long long)K * c->rows_total;
  }
  // full tensor gradient jobs (instances with an output buffer)
  std::vector<TGradJob> tjobs;
  int tj_nin = 0, tj_nt = 0;
  if (g_H) {
    for (int b = 0; b < c->batch; ++b) {
      if (!g_H[b]) continue;
      if (c->kind[b] != MODAL_KIND_VK) return fail(MODAL_EINVAL, "g_H given for an instance that is not VK");
      const InstDev& D = c->inst_host[b];
      tjobs.push_back({g_H[b], D.nt, D.nin, D.mode_off, D.row_off});
      tj_nin = std::max(tj_nin, D.nin);
      tj_nt = std::max(tj_nt, D.nt);
    }
  }
  const bool tens_on = !tjobs.empty();
  if (tens_on) {
    if (c->urec_floats < (long long)K * mf) {
      if (c->dUrec) HIP_TRY(hipFree(c->dUrec));
      c->dUrec = nullptr;
      c->urec_floats = 0;
      int r = dalloc(&c->dUrec, sizeof(float) * (size_t)K * mf);
      if (r) return r;
      c->urec_floats = (long long)K * mf;
    }
    if (c->trec_floats < 2LL * K * c->rows_total) {
      if (c->dTrec) HIP_TRY(hipFree(c->dTrec));
      c->dTrec = nullptr;
      c->trec_floats = 0;
      int r = dalloc(&c->dTrec, sizeof(float) * 2 * (size_t)K * c->rows_total);
      if (r) return r;
      c->trec_floats = 2LL * K * c->rows_total;
    }
    if (c->tjobs_cap < (int)tjobs.size()) {
      if (c->dTJobs) HIP_TRY(hipFree(c->dTJobs));
      c->dTJobs = nullptr;
      c->tjobs_cap = 0;
      int r = dalloc(&c->dTJobs, sizeof(TGradJob) * tjobs.size());
      if (r) return r;
      c->tjobs_cap = (int)tjobs.size();
    }
    HIP_TRY(hipMemcpyAsync(c->dTJobs, tjobs.data(), sizeof(TGradJob) * tjobs.size(), hipMemcpyHostToDevice, s));
    for (const TGradJob& j : tjobs)
      HIP_TRY(hipMemsetAsync(j.out, 0, sizeof(float) * (size_t)j.nin * j.nt * j.nt, s));
  }
  if (!c->dAdj) {
    int r = dalloc(&c->dAdj, sizeof(float) * 4 * (size_t)sf);
    if (!r) r = dalloc(&c->dAcc, sizeof(float) * 12 * (size_t)sf);
    if (!r) r = dalloc(&c->dGPart, sizeof(float) * (size_t)(2 * c->part_floats + 64));
    if (!r) r = dalloc(&c->dGCtr, sizeof(unsigned int) * c->n_ctr);
    if (r) return r;
  }
  // forward from the initial state with checkpoints (unless the last runs
  // recorded them)
  int r = modal_reset(c, stream_);
  if (r) return r;
  // the forward pass also records the whole trajectory while it fits, so
  // that the reverse sweep needs no segment recomputes
  bool rec_now = false;
  if (!reuse) {
    StepParams P = c->P;
    P.y = nullptr;
    P.ckpt = c->dCkpt;
    P.ckpt_every = K;
    P.n_steps = (int)n_steps;
    if ((double)n_steps * 2.0 * mf * sizeof(float) <= kRecAllBytes) {
      if (c->recall_cap < n_steps) {
        if (c->dRecAll) HIP_TRY(hipFree(c->dRecAll));
        c->dRecAll = nullptr;
        c->recall_cap = 0;
        c->rec_upto = 0;
        int r2 = dalloc(&c->dRecAll, sizeof(float) * 2 * (size_t)n_steps * mf);
        if (r2) return r2;
        c->recall_cap = n_steps;
      }
      P.rec_x = c->dRecAll;
      P.rec_d = c->dRecAll + (size_t)c->recall_cap * mf;
      P.rec_base = 0;
      rec_now = true;
    }
    HIP_TRY(launch_step(P, c->gm, c->nw, c->n_wg, c->lds_bytes, s));
    // slots now hold this spacing's checkpoints, and the record this run
    c->ckpt_upto = K == kRunCkpt ? std::max<long long>(c->ckpt_upto, n_steps) : 0;
    c->rec_upto = rec_now ? n_steps : 0;
  }
  HIP_TRY(hipMemsetAsync(c->dAdj, 0, sizeof(float) * 4 * (size_t)sf, s));
  HIP_TRY(hipMemsetAsync(c->dAcc, 0, sizeof(float) * 12 * (size_t)sf, s));
  HIP_TRY(hipMemsetAsync(c->dGCtr, 0, sizeof(unsigned int) * c->n_ctr, s));
  const bool rows_on = g_row && c->rows_total > 0;
  if (rows_on) HIP_TRY(hipMemsetAsync(c->dRacc, 0, sizeof(float) * 2 * (size_t)c->rows_total, s));
  GradParams G{};
  const StepParams& F = c->P;
  G.inst = F.inst;
  G.unit = F.unit;
  G.wg_begin = F.wg_begin;
  G.H = F.H;
  G.Hd = c->tangent ? c->dHd : nullptr;
  G.m_hi = F.m_hi; G.m_lo = F.m_lo; G.p_hi = F.p_hi; G.p_lo = F.p_lo;
  G.r_hi = F.r_hi; G.r_lo = F.r_lo;
  G.c_out = F.c_out; G.lam = F.lam; G.b_ext = F.b_ext; G.e_ext = F.e_ext;
  // the whole trajectory recorded by the last runs, if it covers the steps,
  // replaces the segment recomputes
  const bool reuse_rec = rec_now || (reuse && c->dRecAll && c->rec_upto >= n_steps);
  G.mode_floats = mf;
  G.ybar = ybar;
  G.ybar_stride = y_stride;
  G.qb_hi = c->dAdj; G.qb_lo = c->dAdj + sf; G.db_hi = c->dAdj + 2 * (size_t)sf; G.db_lo = c->dAdj + 3 * (size_t)sf;
  G.acc = c->dAcc;
  G.state_floats = sf;
  G.part = c->dGPart;
  G.ctr = c->dGCtr;
  G.flags = F.flags;
  G.timeout_ticks = F.timeout_ticks;
  G.red_floats = (c->tangent ? 3 : 2) * c->red_floats;
  G.rrec = rows_on ? c->dRrec : nullptr;
  G.rows_total = c->rows_total;
  G.urec = tens_on ? c->dUrec : nullptr;
  G.trec = tens_on ? c->dTrec : nullptr;
  for (long long seg = nseg - 1; seg >= 0; --seg) {
    const long long s0 = seg * K;
    const int len = (int)std::min<long long>(K, n_steps - s0);
    if (reuse_rec) {
      G.rec_x = c->dRecAll + (size_t)s0 * mf;
      G.rec_d = c->dRecAll + (size_t)(c->recall_cap + s0) * mf;
    } else {
      HIP_TRY(launch_restore(c->dCkpt, seg, mf, F.inst, F.unit, c->n_units, c->dState, sf, c->dStep, s0,
                             c->dCtr, s));
      StepParams P = c->P;
      P.y = nullptr;
      P.rec_x = c->dRec;
      P.rec_d = c->dRec + (size_t)K * mf;
      P.rec_base = s0;
      P.n_steps = len;
      HIP_TRY(launch_step(P, c->gm, c->nw, c->n_wg, c->lds_bytes, s));
      G.rec_x = c->dRec;
      G.rec_d = c->dRec + (size_t)K * mf;
    }
    G.seg_base = s0;
    G.seg_len = len;
    G.done_before = n_steps - s0 - len;
    HIP_TRY(launch_grad(G, c->gm, c->tangent, c->nw_grad[c->tangent], c->res_stride > 0 && c->nw_grad[c->tangent] > 1,
                        c->n_wg, c->grad_lds_v[c->tangent], s));
    if (rows_on) HIP_TRY(launch_row_sum(c->dRrec, len, c->rows_total, c->dRacc, s));
    if (tens_on)
      HIP_TRY(launch_tensor_grad(c->dTJobs, (int)tjobs.size(), tj_nin, tj_nt, G.rec_x, c->dUrec, c->dTrec, mf,
                                 c->rows_total, len, s));
  }
  r = modal_check(c, stream_);
  if (r) return r;
  if (g_row) {
    std::vector<float> ra(2 * (size_t)c->rows_total);
    if (rows_on)
      HIP_TRY(hipMemcpyAsync(ra.data(), c->dRacc, sizeof(float) * ra.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int i = 0; i < c->rows_total; ++i)
      g_row[i] = (double)ra[i] + (double)ra[(size_t)c->rows_total + i];
  }
  std::vector<float> acc(12 * (size_t)sf), adj(4 * (size_t)sf);
  HIP_TRY(hipMemcpyAsync(acc.data(), c->dAcc, sizeof(float) * acc.size(), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(adj.data(), c->dAdj, sizeof(float) * adj.size(), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  auto A = [&](int k, int i) { return (double)acc[(size_t)(2 * k) * sf + i] + (double)acc[(size_t)(2 * k + 1) * sf + i]; };
  // per instance: its slab-0 unit holds the accumulators; every unit its theta partial
  std::vector<int> slab0(c->batch, -1);
  std::vector<double> theta(c->batch, 0.0);
  for (const UnitDev& U : c->units) {
    if (U.slab == 0) slab0[U.inst] = U.state_off;
    theta[U.inst] += A(5, U.state_off);
  }
  const double T = 1.0 / c->fs;
  size_t o = 0;
  for (int b = 0; b < c->batch; ++b) {
    const int so = slab0[b];
    double gs = 0.0;
    for (int k = 0; k < c->nt[b]; ++k, ++o) {
      const double gm = A(0, so + k), gp = A(1, so + k), gr = A(2, so + k);
      double dw[3], dg[3];
      coefficient_derivs(c->scheme, c->omega[o], c->gamma[o], T, dw, dg);
      if (g_omega) g_omega[o] = gm * dw[0] + gp * dw[1] + gr * dw[2];
      if (g_gamma) g_gamma[o] = gm * dg[0] + gp * dg[1] + gr * dg[2];
      if (g_c) g_c[o] = A(3, so + k);
      gs += A(4, so + k);
      const Coef q = coefficients(c->scheme, c->omega[o], c->gamma[o], T);
      const double qb0 = (double)adj[so + k] + (double)adj[(size_t)sf + so + k];
      const double db1 = (double)adj[2 * (size_t)sf + so + k] + (double)adj[3 * (size_t)sf + so + k];
      const double d0b = -q.p * db1;  // d^0 = q^0 - q^-1 only feeds d^1
      if (g_x0) g_x0[o] = qb0 + d0b;
      if (g_xm1) g_xm1[o] = -d0b;
    }
    if (g_scale) g_scale[b] = gs;
    if (g_theta) g_theta[b] = theta[b];
  }
  return modal_reset(c, stream_);
}

int modal_get_state(modal_ctx* c, double* x, double* xm1, void* stream_) {
  if (!c || !x || !xm1) return fail(MODAL_EINVAL, "NULL argument");
  hipStream_t s = (hipStream_t)stream_;
  if (c->linear) {
    HIP_TRY(hipStreamSynchronize(s));
    const long long n = c->steps;
    size_t o = 0;
    for (int b = 0; b < c->batch; ++b)
      for (int k = 0; k < c->nt[b]; ++k, ++o) {
        for (int back = 0; back < 2; ++back) {
          const long long t = n - back;
          std::complex<double> v = c->lA[o] * std::pow(c->lz1[o], (double)t) +
                                   c->lB[o] * std::pow(c->lz2[o], (double)t);
          const std::vector<float>& e = c->le[b];
          for (long long m = 0; m < std::min<long long>((long long)e.size(), t); ++m) {
            const double lag = (double)(t - m);
            v += c->lb[o] * (double)e[m] * c->lC[o] *
                 (std::pow(c->lz1[o], lag) - std::pow(c->lz2[o], lag));
          }
          (back == 0 ? x : xm1)[o] = v.real();
        }
      }
    return MODAL_OK;
  }
  std::vector<float> st(c->state0.size());
  HIP_TRY(hipMemcpyAsync(st.data(), c->dState, sizeof(float) * st.size(), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const size_t S = c->state_floats;
  size_t o = 0;
  for (int b = 0; b < c->batch; ++b) {
    const int so0 = c->unit_state_of_inst[b];
    const std::vector<int>* ms = b < (int)c->mode_slot.size() && !c->mode_slot[b].empty() ? &c->mode_slot[b] : nullptr;
    for (int k = 0; k < c->nt[b]; ++k, ++o) {
      const int so = so0 + (ms ? (*ms)[k] - k : 0);
      const double xv = (double)st[so + k] + (double)st[S + so + k];
      const double dv = (double)st[2 * S + so + k] + (double)st[3 * S + so + k];
      x[o] = xv;
      xm1[o] = xv - dv;
    }
  }
  return MODAL_OK;
}

int modal_info(const modal_ctx* c, int64_t info[15]) {
  if (!c || !info) return fail(MODAL_EINVAL, "NULL argument");
  info[0] = c->n_wg;
  info[1] = c->n_units;
  info[2] = c->n_split;
  info[3] = c->coupling_bytes;
  info[4] = c->padded_bytes;
  info[5] = c->steps;
  info[6] = (int64_t)c->lds_bytes;
  info[7] = c->occ;
  info[8] = (int64_t)c->makespan;
  info[9] = (int64_t)c->mean_load;
  info[10] = c->shared ? 1 : (c->linear ? 2 : (c->chip_nt || c->chip_wave ? 3 : 0));
  info[11] = c->flops;
  info[12] = c->n_blocked;
  info[13] = c->shared ? c->coupling_bytes : c->dense_bytes;
  info[14] = c->res_stride;
  return MODAL_OK;
}

void modal_destroy(modal_ctx* c) { free_ctx(c); }

int modal_plan(const modal_desc* d, int32_t n_workgroups, int64_t out[4]) {
  g_err.clear();
  if (!out || n_workgroups < 1) return fail(MODAL_EINVAL, "out NULL or n_workgroups < 1");
  int rc = validate(d);
  if (rc) return rc;
  std::vector<double> row_cost(d->batch), fixed_cost(d->batch);
  double total = 0;
  for (int b = 0; b < d->batch; ++b) {
    unit_costs(d->inst[b], row_cost[b], fixed_cost[b]);
    total += fixed_cost[b] + (d->inst[b].kind == MODAL_KIND_VK ? d->inst[b].n_in : 1) * row_cost[b];
  }
  std::vector<Unit> units;
  std::vector<int> bin_of;
  std::vector<double> load;
  if (!plan_batch(d, row_cost, fixed_cost, total, n_workgroups, units, bin_of, load))
    return fail(MODAL_EINVAL, "batch does not fit the workgroup budget");
  out[0] = (int64_t)units.size();
  out[1] = (int64_t)load.size();
  out[2] = (int64_t)*std::max_element(load.begin(), load.end());
  out[3] = (int64_t)(total / n_workgroups);
  return MODAL_OK;
}

}  // extern "C"
