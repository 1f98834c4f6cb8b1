// Host side of the proposal network: layer bookkeeping, forward, backward
// and Adam around the kernels of mlp_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mlp.h"
#include "../../include/modal.h"

namespace modal {
hipError_t launch_gemm(const float* A, long long lda, int a_kc, const float* B, long long ldb, int b_kc, float* C,
                       long long ldc, int M, int N, int K, int epi, const float* bias, const float* mask,
                       float* part, hipStream_t s);
hipError_t launch_adam_dev(float* p, const float* g, float* m, float* v, long long n, const float* sched, int k,
                           float b1, float b2, float eps, hipStream_t s);
hipError_t launch_gather_rows(const float* src, const long long* idx, int B, int d, float* dst, hipStream_t s);
hipError_t launch_mse_grad(const float* y, const float* z, const long long* idx, int B, int d, float* g,
                           float* acc, hipStream_t s);
constexpr int kMaxSplit = 8;
hipError_t launch_colsum(const float* G, int M, int N, float* db, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, long long n, float lr, float b1,
                       float b2, float eps, int t, hipStream_t s);
}  // namespace modal

using namespace modal;

namespace {
thread_local std::string g_mlp_err;
int mfail(int code, const std::string& m) {
  g_mlp_err = m;
  return code;
}
#define MHIP(expr)                                                                     \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return mfail(MODAL_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)
enum { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_RELU = 2, EPI_MASK = 3 };
}  // namespace

struct mlp_ctx {
  int L = 0, max_batch = 0, max_d = 0, last_batch = 0;
  std::vector<int> dims;
  std::vector<long long> w_off, b_off, act_off;
  long long n_params = 0, act_floats = 0;
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr, *act = nullptr, *d0 = nullptr,
        *d1 = nullptr, *kpart = nullptr;  // kpart: split-K partial tiles
  // mlp_train_epoch: Adam's step count so far and the recorded epochs, each
  // with the device table its Adam steps read (learning rate, then the bias
  // corrections 1 - beta1^t, 1 - beta2^t of each step) and the host copy it
  // was last filled from
  int t = 0;
  hipStream_t cap = nullptr;
  struct Epoch {
    const float *X, *Z;
    const int64_t* order;
    int n_steps, B;
    float b1, b2, eps;
    float* loss;
    hipGraphExec_t exec;
    float* sched;
    std::vector<float> host;
    hipEvent_t copied;  // the last copy from `host` has been made
  };
  std::vector<Epoch> epochs;
};

extern "C" {

const char* mlp_last_error(void) { return g_mlp_err.c_str(); }

void mlp_destroy(mlp_ctx* c) {
  if (!c) return;
  for (float* q : {c->p, c->g, c->m, c->v, c->act, c->d0, c->d1, c->kpart})
    if (q) (void)hipFree(q);
  for (auto& e : c->epochs) {
    (void)hipGraphExecDestroy(e.exec);
    (void)hipFree(e.sched);
    if (e.copied) (void)hipEventDestroy(e.copied);
  }
  if (c->cap) (void)hipStreamDestroy(c->cap);
  delete c;
}

int mlp_init(mlp_ctx** out, int32_t n_layers, const int32_t* dims, int32_t max_batch, void* stream) {
  if (!out || n_layers < 1 || !dims || max_batch < 1) return mfail(MODAL_EINVAL, "bad arguments");
  *out = nullptr;
  for (int l = 0; l <= n_layers; ++l)
    if (dims[l] < 1 || dims[l] > (1 << 16)) return mfail(MODAL_EINVAL, "layer width out of range");
  mlp_ctx* c = new mlp_ctx();
  c->L = n_layers;
  c->max_batch = max_batch;
  c->dims.assign(dims, dims + n_layers + 1);
  for (int l = 0; l < n_layers; ++l) {
    c->w_off.push_back(c->n_params);
    c->n_params += (long long)dims[l] * dims[l + 1];
    c->b_off.push_back(c->n_params);
    c->n_params += dims[l + 1];
  }
  for (int l = 0; l <= n_layers; ++l) {
    c->act_off.push_back(c->act_floats);
    c->act_floats += (long long)max_batch * dims[l];
    c->max_d = std::max(c->max_d, dims[l]);
  }
  hipStream_t s = (hipStream_t)stream;
  const size_t pb = sizeof(float) * (size_t)c->n_params;
  float** bufs[] = {&c->p, &c->g, &c->m, &c->v};
  for (float** b : bufs) {
    if (hipMalloc((void**)b, pb) != hipSuccess) {
      mlp_destroy(c);
      return mfail(MODAL_ENOMEM, "hipMalloc params");
    }
    if (hipMemsetAsync(*b, 0, pb, s) != hipSuccess) {
      mlp_destroy(c);
      return mfail(MODAL_EHIP, "memset");
    }
  }
  if (hipMalloc((void**)&c->act, sizeof(float) * (size_t)c->act_floats) != hipSuccess ||
      hipMalloc((void**)&c->d0, sizeof(float) * (size_t)max_batch * c->max_d) != hipSuccess ||
      hipMalloc((void**)&c->d1, sizeof(float) * (size_t)max_batch * c->max_d) != hipSuccess ||
      hipMalloc((void**)&c->kpart, sizeof(float) * (size_t)kMaxSplit * std::max(max_batch, c->max_d) *
                                       c->max_d) != hipSuccess) {
    mlp_destroy(c);
    return mfail(MODAL_ENOMEM, "hipMalloc activations");
  }
  *out = c;
  return MODAL_OK;
}

int mlp_n_params(const mlp_ctx* c, int64_t* n) {
  if (!c || !n) return mfail(MODAL_EINVAL, "NULL");
  *n = c->n_params;
  return MODAL_OK;
}

int mlp_set_params(mlp_ctx* c, const float* host, void* stream) {
  if (!c || !host) return mfail(MODAL_EINVAL, "NULL");
  hipStream_t s = (hipStream_t)stream;
  MHIP(hipMemcpyAsync(c->p, host, sizeof(float) * (size_t)c->n_params, hipMemcpyHostToDevice, s));
  MHIP(hipMemsetAsync(c->m, 0, sizeof(float) * (size_t)c->n_params, s));
  MHIP(hipMemsetAsync(c->v, 0, sizeof(float) * (size_t)c->n_params, s));
  MHIP(hipStreamSynchronize(s));
  c->t = 0;
  return MODAL_OK;
}

int mlp_get(mlp_ctx* c, int32_t which, float* host, void* stream) {
  if (!c || !host || which < 0 || which > 1) return mfail(MODAL_EINVAL, "bad arguments");
  hipStream_t s = (hipStream_t)stream;
  MHIP(hipMemcpyAsync(host, which == 0 ? c->p : c->g, sizeof(float) * (size_t)c->n_params,
                      hipMemcpyDeviceToHost, s));
  MHIP(hipStreamSynchronize(s));
  return MODAL_OK;
}

}  // extern "C"

namespace {

// the layers on the input already in act (layer 0)
int forward_layers(mlp_ctx* c, int B, hipStream_t s) {
  for (int l = 0; l < c->L; ++l) {
    const int in = c->dims[l], out = c->dims[l + 1];
    const float* a = c->act + c->act_off[l];
    float* z = c->act + c->act_off[l + 1];
    // Z[b, o] = sum_i a[b, i] W[o, i]: A(b, i) = a[b in + i], B(i, o) = W[o in + i]
    MHIP(launch_gemm(a, in, 1, c->p + c->w_off[l], in, 1, z, out, B, out, in,
                     l + 1 < c->L ? EPI_BIAS_RELU : EPI_BIAS, c->p + c->b_off[l], nullptr, c->kpart, s));
  }
  c->last_batch = B;
  return MODAL_OK;
}

// the gradients for the output gradient already in d0
int backward_layers(mlp_ctx* c, hipStream_t s) {
  const int B = c->last_batch;
  float* gcur = c->d0;
  float* gnext = c->d1;
  for (int l = c->L - 1; l >= 0; --l) {
    const int in = c->dims[l], out = c->dims[l + 1];
    const float* a = c->act + c->act_off[l];
    // dW[o, i] = sum_b g[b, o] a[b, i]: A(o, b) = g[b out + o] (o contiguous),
    // B(b, i) = a[b in + i] (i contiguous)
    MHIP(launch_gemm(gcur, out, 0, a, in, 0, c->g + c->w_off[l], in, out, in, B, EPI_STORE, nullptr,
                     nullptr, c->kpart, s));
    MHIP(launch_colsum(gcur, B, out, c->g + c->b_off[l], s));
    if (l > 0) {
      // g_prev[b, i] = (sum_o g[b, o] W[o, i]) * [a[b, i] > 0]: A(b, o) =
      // g[b out + o] (o contiguous), B(o, i) = W[o in + i] (i contiguous)
      MHIP(launch_gemm(gcur, out, 1, c->p + c->w_off[l], in, 0, gnext, in, B, in, out, EPI_MASK,
                       nullptr, a, c->kpart, s));
      std::swap(gcur, gnext);
    }
  }
  return MODAL_OK;
}

}  // namespace

extern "C" {

int mlp_forward(mlp_ctx* c, const float* x, int32_t B, float* y, void* stream) {
  if (!c || !x || !y || B < 1 || B > c->max_batch) return mfail(MODAL_EINVAL, "bad arguments");
  hipStream_t s = (hipStream_t)stream;
  MHIP(hipMemcpyAsync(c->act, x, sizeof(float) * (size_t)B * c->dims[0], hipMemcpyDeviceToDevice, s));
  int r = forward_layers(c, B, s);
  if (r) return r;
  MHIP(hipMemcpyAsync(y, c->act + c->act_off[c->L], sizeof(float) * (size_t)B * c->dims[c->L],
                      hipMemcpyDeviceToDevice, s));
  return MODAL_OK;
}

int mlp_backward(mlp_ctx* c, const float* dy, void* stream) {
  if (!c || !dy || c->last_batch < 1) return mfail(MODAL_ESTATE, "backward needs a forward first");
  hipStream_t s = (hipStream_t)stream;
  MHIP(hipMemcpyAsync(c->d0, dy, sizeof(float) * (size_t)c->last_batch * c->dims[c->L],
                      hipMemcpyDeviceToDevice, s));
  return backward_layers(c, s);
}

int mlp_train_step(mlp_ctx* c, const float* X, const float* Z, const int64_t* idx, int32_t B, float lr,
                   float beta1, float beta2, float eps, int32_t t, float* loss_acc, void* stream) {
  if (!c || !X || !Z || !idx || B < 1 || B > c->max_batch || t < 1) return mfail(MODAL_EINVAL, "bad arguments");
  hipStream_t s = (hipStream_t)stream;
  const long long* ix = reinterpret_cast<const long long*>(idx);
  MHIP(launch_gather_rows(X, ix, B, c->dims[0], c->act, s));
  int r = forward_layers(c, B, s);
  if (r) return r;
  MHIP(launch_mse_grad(c->act + c->act_off[c->L], Z, ix, B, c->dims[c->L], c->d0, loss_acc, s));
  r = backward_layers(c, s);
  if (r) return r;
  MHIP(launch_adam(c->p, c->g, c->m, c->v, c->n_params, lr, beta1, beta2, eps, t, s));
  return MODAL_OK;
}

int mlp_train_epoch(mlp_ctx* c, const float* X, const float* Z, const int64_t* order, int32_t n_steps,
                    int32_t B, float lr, float beta1, float beta2, float eps, float* loss_acc, void* stream) {
  if (!c || !X || !Z || !order || n_steps < 1 || B < 1 || B > c->max_batch)
    return mfail(MODAL_EINVAL, "bad arguments");
  hipStream_t s = (hipStream_t)stream;
  mlp_ctx::Epoch* ep = nullptr;
  for (auto& e : c->epochs)
    if (e.X == X && e.Z == Z && e.order == order && e.n_steps == n_steps && e.B == B && e.b1 == beta1 &&
        e.b2 == beta2 && e.eps == eps && e.loss == loss_acc)
      ep = &e;
  if (!ep) {
    float* sched = nullptr;
    MHIP(hipMalloc((void**)&sched, sizeof(float) * (1 + 2 * (size_t)n_steps)));
    hipGraphExec_t exec = nullptr;
    // record the epoch once on a private stream (the caller's may be the
    // legacy default stream, which cannot be captured)
    if (!c->cap) MHIP(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
    hipGraph_t graph;
    MHIP(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    int r = MODAL_OK;
    for (int st = 0; st < n_steps && !r; ++st) {
      const long long* ix = reinterpret_cast<const long long*>(order) + (long long)st * B;
      hipError_t e = launch_gather_rows(X, ix, B, c->dims[0], c->act, c->cap);
      if (e == hipSuccess) r = forward_layers(c, B, c->cap);
      if (e == hipSuccess && !r)
        e = launch_mse_grad(c->act + c->act_off[c->L], Z, ix, B, c->dims[c->L], c->d0, loss_acc, c->cap);
      if (e == hipSuccess && !r) r = backward_layers(c, c->cap);
      if (e == hipSuccess && !r)
        e = launch_adam_dev(c->p, c->g, c->m, c->v, c->n_params, sched, st, beta1, beta2, eps, c->cap);
      if (e != hipSuccess) r = mfail(MODAL_EHIP, std::string("recording an epoch: ") + hipGetErrorString(e));
    }
    hipError_t e = hipStreamEndCapture(c->cap, &graph);
    if (!r && e != hipSuccess) r = mfail(MODAL_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    if (!r) {
      e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) r = mfail(MODAL_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    if (r) {
      (void)hipFree(sched);
      return r;
    }
    hipEvent_t ev = nullptr;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) {
      (void)hipGraphExecDestroy(exec);
      (void)hipFree(sched);
      return mfail(MODAL_EHIP, std::string("hipEventCreate: ") + hipGetErrorString(e));
    }
    c->epochs.push_back({X, Z, order, n_steps, B, beta1, beta2, eps, loss_acc, exec, sched, {}, ev});
    ep = &c->epochs.back();
  } else {
    MHIP(hipEventSynchronize(ep->copied));  // before its host table is rewritten
  }
  // this epoch's schedule, the corrections formed on the host as
  // mlp_adam_step forms them
  std::vector<float>& h = ep->host;
  h.assign(1 + 2 * (size_t)n_steps, 0.f);
  h[0] = lr;
  for (int k = 0; k < n_steps; ++k) {
    const float t = (float)(c->t + k + 1);
    h[1 + 2 * k] = 1.f - powf(beta1, t);
    h[2 + 2 * k] = 1.f - powf(beta2, t);
  }
  MHIP(hipMemcpyAsync(ep->sched, h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice, s));
  MHIP(hipEventRecord(ep->copied, s));
  MHIP(hipGraphLaunch(ep->exec, s));
  c->t += n_steps;
  c->last_batch = B;
  return MODAL_OK;
}

int mlp_adam_step(mlp_ctx* c, float lr, float b1, float b2, float eps, int32_t t, void* stream) {
  if (!c || t < 1) return mfail(MODAL_EINVAL, "bad arguments");
  MHIP(launch_adam(c->p, c->g, c->m, c->v, c->n_params, lr, b1, b2, eps, t, (hipStream_t)stream));
  return MODAL_OK;
}

}  // extern "C"
