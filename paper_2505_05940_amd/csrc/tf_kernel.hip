// Transfer-function response of linear modal systems and its gradient
// (gfx950, float-float arithmetic on FP32 pairs; the FP64 inputs are split
// into pairs on the host and the results recombined there).
//
// With impulse invariance each mode is the discrete system
// b1 z / (z^2 + a1 z + a2) (paper: Sec. 3.2, transfer function); the linear
// string fits of Sec. 4.3 add a second numerator coefficient b2 per mode and
// free output weights w, and compare the magnitude response on a Bark-scale
// frequency grid with the target's spectral envelope:
//   H_b(e^{i Omega_k}) = sum_{mu of b} w_mu (b1_mu z + b2_mu) / (z^2 + a1_mu z + a2_mu).
// Coefficients per mode are (a1, a2, b1, b2, w), each a float-float pair;
// z_k = e^{i Omega_k} comes from the host as a float-float complex number.
//
// tf_response: one thread per (instance, frequency), modes read as uniform
// loads.  tf_grad: one wave per mode, lanes over the frequencies, for
// L = sum_k Re(conj(g_k) H_k): with N = b1 z + b2, D = z^2 + a1 z + a2,
//   dH/dw = N/D, dH/db1 = w z/D, dH/db2 = w/D, dH/da1 = -w N z/D^2,
//   dH/da2 = -w N/D^2.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace modal {

namespace {

__device__ __forceinline__ ff fneg(ff a) { return {-a.hi, -a.lo}; }
__device__ __forceinline__ ff fsub(ff a, ff b) { return ff_add(a, fneg(b)); }

// a / b to about float-float precision: two correction steps on the FP32
// quotient of the high parts
__device__ __forceinline__ ff fdiv(ff a, ff b) {
  const float q1 = a.hi / b.hi;
  ff r = fsub(a, ff_mul_f(b, q1));
  const float q2 = r.hi / b.hi;
  r = fsub(r, ff_mul_f(b, q2));
  const float q3 = r.hi / b.hi;
  const ff q = fast_two_sum(q1, q2);
  return ff_add(q, {q3, 0.f});
}

struct cx {
  ff re, im;
};
__device__ __forceinline__ cx cmul(cx x, cx y) {
  return {fsub(ff_mul(x.re, y.re), ff_mul(x.im, y.im)), ff_add(ff_mul(x.re, y.im), ff_mul(x.im, y.re))};
}
__device__ __forceinline__ cx cadd(cx x, cx y) { return {ff_add(x.re, y.re), ff_add(x.im, y.im)}; }
__device__ __forceinline__ cx cscale(cx x, ff s) { return {ff_mul(x.re, s), ff_mul(x.im, s)}; }
// 1 / d = conj(d) / |d|^2
__device__ __forceinline__ cx cinv(cx d) {
  const ff n = ff_add(ff_mul(d.re, d.re), ff_mul(d.im, d.im));
  return {fdiv(d.re, n), fdiv(fneg(d.im), n)};
}
__device__ __forceinline__ cx ld(const FFc& v) { return {{v.rh, v.rl}, {v.ih, v.il}}; }
__device__ __forceinline__ ff ldf(const float2 v) { return {v.x, v.y}; }

// Re(conj(g) v)
__device__ __forceinline__ ff re_dot(cx g, cx v) { return ff_add(ff_mul(g.re, v.re), ff_mul(g.im, v.im)); }

__device__ __forceinline__ ff wave_sum_ff(ff v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = ff_add(v, {__shfl_xor(v.hi, o), __shfl_xor(v.lo, o)});
  return v;
}

}  // namespace

// coef [modes][5] float-float (a1, a2, b1, b2, w); z [n_freq]; H [batch][n_freq]
__global__ void __launch_bounds__(64) tf_response_kernel(const float2* __restrict__ coef,
                                                         const int* __restrict__ mode_off,
                                                         const FFc* __restrict__ z, int n_freq,
                                                         FFc* __restrict__ H) {
  const int b = blockIdx.y;
  const int k = blockIdx.x * 64 + threadIdx.x;
  if (k >= n_freq) return;
  const cx zk = ld(z[k]);
  const cx z2 = cmul(zk, zk);
  cx acc = {{0.f, 0.f}, {0.f, 0.f}};
  for (int m = mode_off[b]; m < mode_off[b + 1]; ++m) {
    const float2* p = coef + 5LL * m;
    const ff a1 = ldf(p[0]), a2 = ldf(p[1]), b1 = ldf(p[2]), b2 = ldf(p[3]), w = ldf(p[4]);
    const cx N = cadd(cscale(zk, b1), cx{b2, {0.f, 0.f}});
    const cx D = cadd(z2, cadd(cscale(zk, a1), cx{a2, {0.f, 0.f}}));
    acc = cadd(acc, cscale(cmul(N, cinv(D)), w));
  }
  H[(long long)b * n_freq + k] = FFc{acc.re.hi, acc.re.lo, acc.im.hi, acc.im.lo};
}

// grid: (ceil(max_modes / 4), batch); 4 waves per block, wave = mode
__global__ void __launch_bounds__(256) tf_grad_kernel(const float2* __restrict__ coef,
                                                      const int* __restrict__ mode_off,
                                                      const FFc* __restrict__ z, int n_freq,
                                                      const FFc* __restrict__ gH,
                                                      float2* __restrict__ g_coef) {
  const int b = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int m = mode_off[b] + blockIdx.x * 4 + (threadIdx.x >> 6);
  if (m >= mode_off[b + 1]) return;
  const float2* p = coef + 5LL * m;
  const ff a1 = ldf(p[0]), a2 = ldf(p[1]), b1 = ldf(p[2]), b2 = ldf(p[3]), w = ldf(p[4]);
  ff ga1 = {0.f, 0.f}, ga2 = ga1, gb1 = ga1, gb2 = ga1, gw = ga1;
  for (int k = lane; k < n_freq; k += 64) {
    const cx zk = ld(z[k]);
    const cx z2 = cmul(zk, zk);
    const cx N = cadd(cscale(zk, b1), cx{b2, {0.f, 0.f}});
    const cx D = cadd(z2, cadd(cscale(zk, a1), cx{a2, {0.f, 0.f}}));
    const cx iD = cinv(D);
    const cx ND = cmul(N, iD);    // N / D
    const cx ND2 = cmul(ND, iD);  // N / D^2
    const cx g = ld(gH[(long long)b * n_freq + k]);
    gw = ff_add(gw, re_dot(g, ND));
    gb1 = ff_add(gb1, ff_mul(w, re_dot(g, cmul(zk, iD))));
    gb2 = ff_add(gb2, ff_mul(w, re_dot(g, iD)));
    ga1 = fsub(ga1, ff_mul(w, re_dot(g, cmul(ND2, zk))));
    ga2 = fsub(ga2, ff_mul(w, re_dot(g, ND2)));
  }
  ga1 = wave_sum_ff(ga1);
  ga2 = wave_sum_ff(ga2);
  gb1 = wave_sum_ff(gb1);
  gb2 = wave_sum_ff(gb2);
  gw = wave_sum_ff(gw);
  if (lane == 0) {
    float2* o = g_coef + 5LL * m;
    o[0] = make_float2(ga1.hi, ga1.lo);
    o[1] = make_float2(ga2.hi, ga2.lo);
    o[2] = make_float2(gb1.hi, gb1.lo);
    o[3] = make_float2(gb2.hi, gb2.lo);
    o[4] = make_float2(gw.hi, gw.lo);
  }
}

hipError_t launch_tf_response(const float2* coef, const int* mode_off, int batch, const FFc* z, int n_freq,
                              FFc* H, hipStream_t s) {
  hipLaunchKernelGGL(tf_response_kernel, dim3((n_freq + 63) / 64, batch), dim3(64), 0, s, coef, mode_off, z,
                     n_freq, H);
  return hipGetLastError();
}

hipError_t launch_tf_grad(const float2* coef, const int* mode_off, int batch, int max_modes, const FFc* z,
                          int n_freq, const FFc* gH, float2* g_coef, hipStream_t s) {
  if (max_modes < 1) return hipSuccess;
  hipLaunchKernelGGL(tf_grad_kernel, dim3((max_modes + 3) / 4, batch), dim3(256), 0, s, coef, mode_off, z, n_freq,
                     gH, g_coef);
  return hipGetLastError();
}

}  // namespace modal
