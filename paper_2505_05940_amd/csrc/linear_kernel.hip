// Time-parallel evaluation of linear modal systems (gfx950, FP64).
//
// Without a nonlinear force each mode of the recursion of the modal
// oscillator update (paper: Sec. 3.2), q^{n+1} = g q^n + p q^{n-1} + r f^n,
// is solved in closed form by the roots z1, z2 of z^2 - g z - p: the free
// response is A z1^n + B z2^n, and a unit force at step m adds
// h(n - m) = C (z1^(n-m) - z2^(n-m)), C = r / (z1 - z2), for n > m.  The paper
// evaluates such responses by repeated multiplication with the discrete
// eigenvalues in a prefix sum over time (Sec. 4.3, linear string fits).
//
// Here every output sample of every mode is a value Re(P1 z1^n + P2 z2^n)
// for one of three amplitude sets:
//   free   (P1, P2) = c (A, B),         exponent n, every step before the
//                                        excitation ends (and all steps of an
//                                        unforced instance);
//   post   (P1, P2) = c (V1, V2),       exponent n - n_exc, every step from
//                                        n_exc on, where Vk = A z_k^{n_exc} +
//                                        b C sum_{m < n_exc} e[m] z_k^{n_exc - m}
//                                        (the state the excitation leaves);
//   impulse(P1, P2) = c b C (1, -1),    exponent = lag, the output-space impulse
//                                        response used inside the excitation
//                                        window.
// Complex-conjugate root pairs keep one root with the amplitude doubled.
//
// Within an instance the complex-conjugate pairs come first.
//
// lin_sum: each lane owns the steps s0 + lane + 64 t (t < R) of a segment, so
// stores are coalesced.  Per mode it takes the first two values directly and
// the rest from the three-term recurrence y(n + 64) = a y(n) - b y(n - 64),
// a = z1^64 + z2^64, b = (z1 z2)^64, which both root terms satisfy: one
// multiply, one fused multiply-add and one add per mode and step.  The first
// power z1^(nb + lane) is z1^nb, which every lane computes for a different mode
// of a group of 64 (exp of nb log|z| and sincospi of nb arg/pi, whose
// reduction is exact) and reads back by lane, times z1^lane from a table built
// once.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace modal {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// z^n from log|z| and arg(z)/pi
__device__ __forceinline__ double2 cpow_polar(double lmag, double fpi, long long n) {
  const double mag = exp((double)n * lmag);
  double s, c;
  sincospi((double)n * fpi, &s, &c);
  return make_double2(mag * c, mag * s);
}

__device__ __forceinline__ double readlane_d(double v, int j) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), j),
                          __builtin_amdgcn_readlane(__double2loint(v), j));
}

// Adds Re(u z^(64 t)) for t < R to acc, given u and the recurrence of its mode.
template <int R>
__device__ __forceinline__ void add_mode(double (&acc)[R], double2 u, const LinMode& md) {
  double y0 = u.x, y1 = cmul(u, md.s1).x;
  acc[0] += y0;
  acc[1] += y1;
#pragma unroll
  for (int t = 2; t < R; ++t) {
    const double y2 = md.a * y1 - md.b * y0;
    acc[t] += y2;
    y0 = y1;
    y1 = y2;
  }
}

// The same for two modes at once (two independent recurrences).
template <int R>
__device__ __forceinline__ void add_mode_pair(double (&acc)[R], double2 u, const LinMode& md, double2 v,
                                              const LinMode& me) {
  double y0 = u.x, y1 = cmul(u, md.s1).x;
  double x0 = v.x, x1 = cmul(v, me.s1).x;
  acc[0] += y0 + x0;
  acc[1] += y1 + x1;
#pragma unroll
  for (int t = 2; t < R; ++t) {
    const double y2 = md.a * y1 - md.b * y0;
    const double x2 = me.a * x1 - me.b * x0;
    acc[t] += y2 + x2;
    y0 = y1;
    y1 = y2;
    x0 = x1;
    x1 = x2;
  }
}

template <int R, typename OutT>
__global__ __launch_bounds__(kLinWaves * 64) void lin_sum_kernel(const LinMode* __restrict__ modes,
                                                                 const double4* __restrict__ amp,
                                                                 const double2* __restrict__ ztab,
                                                                 const LinSeg* __restrict__ segs,
                                                                 OutT* __restrict__ out) {
  const LinSeg sg = segs[blockIdx.y];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long s0 = ((long long)blockIdx.x * kLinWaves + wave) * (64LL * R);
  if (s0 >= sg.len) return;
  const long long nb = sg.e0 + s0, n0 = nb + lane;
  const double4* Pa = amp + sg.amp_off;
  double acc[R];
#pragma unroll
  for (int t = 0; t < R; ++t) acc[t] = 0.0;
  // complex-conjugate root pairs [m0, mc), two modes at a time
  for (int kb = sg.m0; kb < sg.mc; kb += 64) {
    double2 zb = make_double2(0.0, 0.0);  // z1^nb of mode kb + lane
    if (kb + lane < sg.mc) zb = cpow_polar(modes[kb + lane].lm1, modes[kb + lane].f1, nb);
    const int kn = min(64, sg.mc - kb);
    int j = 0;
    for (; j + 1 < kn; j += 2) {
      const int k = kb + j;
      const LinMode md = modes[k], me = modes[k + 1];
      const double4 P = Pa[k], Q = Pa[k + 1];
      const double2 wu = cmul(make_double2(readlane_d(zb.x, j), readlane_d(zb.y, j)), ztab[(size_t)k * 64 + lane]);
      const double2 wv = cmul(make_double2(readlane_d(zb.x, j + 1), readlane_d(zb.y, j + 1)),
                              ztab[(size_t)(k + 1) * 64 + lane]);
      add_mode_pair<R>(acc, cmul(make_double2(P.x, P.y), wu), md, cmul(make_double2(Q.x, Q.y), wv), me);
    }
    if (j < kn) {
      const int k = kb + j;
      const LinMode md = modes[k];
      const double4 P = Pa[k];
      const double2 wu = cmul(make_double2(readlane_d(zb.x, j), readlane_d(zb.y, j)), ztab[(size_t)k * 64 + lane]);
      add_mode<R>(acc, cmul(make_double2(P.x, P.y), wu), md);
    }
  }
  // real root pairs [mc, m1): both roots, powers taken directly
  for (int k = sg.mc; k < sg.m1; ++k) {
    const LinMode md = modes[k];
    const double4 P = Pa[k];
    const double2 u1 = cmul(make_double2(P.x, P.y), cpow_polar(md.lm1, md.f1, n0));
    const double2 u2 = cmul(make_double2(P.z, P.w), cpow_polar(md.lm2, md.f2, n0));
    double y0 = u1.x + u2.x;
    double y1 = cmul(u1, md.s1).x + cmul(u2, md.s2).x;
    acc[0] += y0;
    acc[1] += y1;
#pragma unroll
    for (int t = 2; t < R; ++t) {
      const double y2 = md.a * y1 - md.b * y0;
      acc[t] += y2;
      y0 = y1;
      y1 = y2;
    }
  }
  OutT* o = out + sg.out_off;
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const long long i = s0 + lane + 64LL * t;
    if (i < sg.len) o[i] = (OutT)acc[t];
  }
}

// z1^l, l < 64, of every mode
__global__ void lin_tab_kernel(const LinMode* __restrict__ modes, int M, double2* __restrict__ ztab) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 64LL * M) return;
  const LinMode md = modes[i >> 6];
  ztab[i] = cpow_polar(md.lm1, md.f1, i & 63);
}

// Amplitude sets [free | post | impulse] of every mode; the post set runs the
// excitation through each root (V <- (V + b C e[m]) z), one thread per mode.
__global__ void lin_amp_kernel(const LinInit* __restrict__ init, int M, const float* __restrict__ e_ext,
                               double4* __restrict__ amp) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  const LinInit I = init[k];
  double2 v1 = I.A, v2 = I.B;
  const double2 bc = make_double2(I.b * I.C.x, I.b * I.C.y);
  const float* e = e_ext + I.e_off;
  for (long long m = 0; m < I.n_exc; ++m) {
    const double em = (double)e[m];
    v1 = cmul(make_double2(v1.x + bc.x * em, v1.y + bc.y * em), I.z1);
    v2 = cmul(make_double2(v2.x - bc.x * em, v2.y - bc.y * em), I.z2);
  }
  const double f = I.conj ? 2.0 * I.c : I.c;
  const double k2 = I.conj ? 0.0 : I.c;
  amp[k] = make_double4(f * I.A.x, f * I.A.y, k2 * I.B.x, k2 * I.B.y);
  amp[M + k] = make_double4(f * v1.x, f * v1.y, k2 * v2.x, k2 * v2.y);
  amp[2 * (size_t)M + k] = make_double4(f * bc.x, f * bc.y, -k2 * bc.x, -k2 * bc.y);
}

// Inside the excitation window: y[n - base] += sum_{m < n} e[m] h(n - m) for
// n in [base, min(base + n_steps, n_exc)); h row holds lags 1 .. n_exc - 1.
__global__ void lin_conv_kernel(const LinForced* __restrict__ forced, const double* __restrict__ h,
                                long long h_stride, const float* __restrict__ e_ext, long long base,
                                long long n_steps, float* __restrict__ y, long long y_stride) {
  const LinForced F = forced[blockIdx.y];
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long n = base + i;
  if (i >= n_steps || n >= F.n_exc) return;
  const float* e = e_ext + F.e_off;
  const double* hb = h + blockIdx.y * h_stride - 1;  // hb[lag], lag >= 1
  double v = 0.0;
  for (long long m = 0; m < n; ++m) v += (double)e[m] * hb[n - m];
  float* yo = y + F.inst * y_stride + i;
  *yo = (float)((double)*yo + v);
}

hipError_t launch_lin_sum(const LinMode* modes, const double4* amp, const double2* ztab, const LinSeg* segs,
                          int n_segs, long long max_len, float* out, hipStream_t s) {
  if (max_len < 1 || n_segs < 1) return hipSuccess;
  const long long per_block = 64LL * kLinWaves * kLinRun;
  dim3 grid((unsigned)((max_len + per_block - 1) / per_block), n_segs);
  hipLaunchKernelGGL((lin_sum_kernel<kLinRun, float>), grid, dim3(64 * kLinWaves), 0, s, modes, amp, ztab,
                     segs, out);
  return hipGetLastError();
}

hipError_t launch_lin_sum_f64(const LinMode* modes, const double4* amp, const double2* ztab,
                              const LinSeg* segs, int n_segs, long long max_len, double* out, hipStream_t s) {
  if (max_len < 1 || n_segs < 1) return hipSuccess;
  const long long per_block = 64LL * kLinWaves * kLinRun;
  dim3 grid((unsigned)((max_len + per_block - 1) / per_block), n_segs);
  hipLaunchKernelGGL((lin_sum_kernel<kLinRun, double>), grid, dim3(64 * kLinWaves), 0, s, modes, amp, ztab,
                     segs, out);
  return hipGetLastError();
}

hipError_t launch_lin_amp(const LinInit* init, const LinMode* modes, int M, const float* e_ext, double4* amp,
                          double2* ztab, hipStream_t s) {
  if (M < 1) return hipSuccess;
  hipLaunchKernelGGL(lin_tab_kernel, dim3((unsigned)((64LL * M + 255) / 256)), dim3(256), 0, s, modes, M, ztab);
  hipLaunchKernelGGL(lin_amp_kernel, dim3((M + 127) / 128), dim3(128), 0, s, init, M, e_ext, amp);
  return hipGetLastError();
}

hipError_t launch_lin_conv(const LinForced* forced, int n_forced, const double* h, long long h_stride,
                           const float* e_ext, long long base, long long n_steps, long long window,
                           float* y, long long y_stride, hipStream_t s) {
  if (n_forced < 1 || window < 1) return hipSuccess;
  dim3 grid((unsigned)((window + 255) / 256), n_forced);
  hipLaunchKernelGGL(lin_conv_kernel, grid, dim3(256), 0, s, forced, h, h_stride, e_ext, base, n_steps, y,
                     y_stride);
  return hipGetLastError();
}

}  // namespace modal
