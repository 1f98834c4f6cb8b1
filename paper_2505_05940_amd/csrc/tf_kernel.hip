// Transfer-function response of linear modal systems and its gradient
// (gfx950, FP64).
//
// With impulse invariance each mode is the discrete system
// b1 z / (z^2 + a1 z + a2) (paper: Sec. 3.2, transfer function); the linear
// string fits of Sec. 4.3 add a second numerator coefficient b2 per mode and
// free output weights w, and compare the magnitude response on a Bark-scale
// frequency grid with the target's spectral envelope:
//   H_b(e^{i Omega_k}) = sum_{mu of b} w_mu (b1_mu z + b2_mu) / (z^2 + a1_mu z + a2_mu).
// Coefficients per mode are (a1, a2, b1, b2, w), FP64.
//
// tf_response: one thread per (instance, frequency), modes read as uniform
// (scalar) loads.  tf_grad: one wave per mode, lanes over the frequencies,
// for L = sum_k Re(conj(g_k) H_k): with N = b1 z + b2, D = z^2 + a1 z + a2,
//   dH/dw = N/D, dH/db1 = w z/D, dH/db2 = w/D, dH/da1 = -w N z/D^2,
//   dH/da2 = -w N/D^2.
#include <hip/hip_runtime.h>

namespace modal {

namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  const double s = 1.0 / (b.x * b.x + b.y * b.y);
  return make_double2((a.x * b.x + a.y * b.y) * s, (a.y * b.x - a.x * b.y) * s);
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

}  // namespace

__global__ void __launch_bounds__(64) tf_response_kernel(const double* __restrict__ coef,
                                                         const int* __restrict__ mode_off,
                                                         const double* __restrict__ omega, int n_freq,
                                                         double2* __restrict__ H) {
  const int b = blockIdx.y;
  const int k = blockIdx.x * 64 + threadIdx.x;
  if (k >= n_freq) return;
  double s, c;
  sincos(omega[k], &s, &c);
  const double2 z = make_double2(c, s);
  const double2 z2 = cmul(z, z);
  double2 acc = make_double2(0.0, 0.0);
  for (int m = mode_off[b]; m < mode_off[b + 1]; ++m) {
    const double* p = coef + 5LL * m;
    const double a1 = p[0], a2 = p[1], b1 = p[2], b2 = p[3], w = p[4];
    const double2 N = make_double2(b1 * z.x + b2, b1 * z.y);
    const double2 D = make_double2(z2.x + a1 * z.x + a2, z2.y + a1 * z.y);
    const double2 q = cdiv(N, D);
    acc.x += w * q.x;
    acc.y += w * q.y;
  }
  H[(long long)b * n_freq + k] = acc;
}

// grid: (ceil(max_modes / 4), batch); 4 waves per block, wave = mode
__global__ void __launch_bounds__(256) tf_grad_kernel(const double* __restrict__ coef,
                                                      const int* __restrict__ mode_off,
                                                      const double* __restrict__ omega, int n_freq,
                                                      const double2* __restrict__ gH,
                                                      double* __restrict__ g_coef) {
  const int b = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int m = mode_off[b] + blockIdx.x * 4 + (threadIdx.x >> 6);
  if (m >= mode_off[b + 1]) return;
  const double* p = coef + 5LL * m;
  const double a1 = p[0], a2 = p[1], b1 = p[2], b2 = p[3], w = p[4];
  double ga1 = 0.0, ga2 = 0.0, gb1 = 0.0, gb2 = 0.0, gw = 0.0;
  for (int k = lane; k < n_freq; k += 64) {
    double s, c;
    sincos(omega[k], &s, &c);
    const double2 z = make_double2(c, s);
    const double2 z2 = cmul(z, z);
    const double2 N = make_double2(b1 * z.x + b2, b1 * z.y);
    const double2 D = make_double2(z2.x + a1 * z.x + a2, z2.y + a1 * z.y);
    const double2 iD = cdiv(make_double2(1.0, 0.0), D);
    const double2 ND = cmul(N, iD);       // N / D
    const double2 ND2 = cmul(ND, iD);     // N / D^2
    const double2 g = gH[(long long)b * n_freq + k];
    // Re(conj(g) v) = g.x v.x + g.y v.y
    auto re = [&](double2 v) { return g.x * v.x + g.y * v.y; };
    gw += re(ND);
    gb1 += w * re(cmul(z, iD));
    gb2 += w * re(iD);
    ga1 -= w * re(cmul(ND2, z));
    ga2 -= w * re(ND2);
  }
  ga1 = wave_sum_d(ga1);
  ga2 = wave_sum_d(ga2);
  gb1 = wave_sum_d(gb1);
  gb2 = wave_sum_d(gb2);
  gw = wave_sum_d(gw);
  if (lane == 0) {
    double* o = g_coef + 5LL * m;
    o[0] = ga1;
    o[1] = ga2;
    o[2] = gb1;
    o[3] = gb2;
    o[4] = gw;
  }
}

hipError_t launch_tf_response(const double* coef, const int* mode_off, int batch, const double* omega,
                              int n_freq, double* H, hipStream_t s) {
  hipLaunchKernelGGL(tf_response_kernel, dim3((n_freq + 63) / 64, batch), dim3(64), 0, s, coef, mode_off,
                     omega, n_freq, reinterpret_cast<double2*>(H));
  return hipGetLastError();
}

hipError_t launch_tf_grad(const double* coef, const int* mode_off, int batch, int max_modes, const double* omega,
                          int n_freq, const double* gH, double* g_coef, hipStream_t s) {
  if (max_modes < 1) return hipSuccess;
  hipLaunchKernelGGL(tf_grad_kernel, dim3((max_modes + 3) / 4, batch), dim3(256), 0, s, coef, mode_off, omega,
                     n_freq, reinterpret_cast<const double2*>(gH), g_coef);
  return hipGetLastError();
}

}  // namespace modal
