// Time-parallel evaluation of linear modal systems (gfx950, float-float
// arithmetic on FP32 pairs; the FP64 work stays on the host).
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
// Within an instance the complex-conjugate pairs come first.
//
// The host computes the roots, amplitudes and 64th powers in FP64 and hands
// them over as float-float pairs (about 48 bits); every product and sum on
// the device is a float-float operation (Dekker/Knuth error-free
// transformations with explicit fmaf), so the result keeps the FP64
// closed form's accuracy well below the FP32 output's rounding.
//
// lin_sum: each lane owns the steps s0 + lane + 64 t (t < R) of a segment, so
// stores are coalesced.  Per mode it takes the first two values directly and
// the rest from the three-term recurrence y(n + 64) = a y(n) - b y(n - 64),
// which both root terms satisfy.  The first power z1^(nb + lane) is z1^nb,
// which every lane computes by binary exponentiation for a different mode of
// a group of 64 and reads back by lane, times z1^lane from a table built
// once the same way.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace modal {

namespace {

__device__ __forceinline__ ff ffneg(ff a) { return {-a.hi, -a.lo}; }

struct ffcx {
  ff re, im;
};

__device__ __forceinline__ ffcx load_ffc(const FFc& v) { return {{v.rh, v.rl}, {v.ih, v.il}}; }

__device__ __forceinline__ ffcx cmulx(ffcx x, ffcx y) {
  const ff a = ff_mul(x.re, y.re), b = ff_mul(x.im, y.im);
  const ff c = ff_mul(x.re, y.im), d = ff_mul(x.im, y.re);
  return {ff_add(a, ffneg(b)), ff_add(c, d)};
}

__device__ __forceinline__ ffcx caddx(ffcx x, ffcx y) { return {ff_add(x.re, y.re), ff_add(x.im, y.im)}; }

// x * s for a float s
__device__ __forceinline__ ffcx cscalef(ffcx x, float s) { return {ff_mul_f(x.re, s), ff_mul_f(x.im, s)}; }

// x * s for a float-float s
__device__ __forceinline__ ffcx cscale(ffcx x, ff s) { return {ff_mul(x.re, s), ff_mul(x.im, s)}; }

// z^n, n >= 0, by binary exponentiation (relative error about 2^k ulp of
// float-float after k squarings)
__device__ ffcx cpowx(ffcx z, long long n) {
  ffcx r = {{1.f, 0.f}, {0.f, 0.f}};
  ffcx b = z;
  while (n > 0) {
    if (n & 1) r = cmulx(r, b);
    n >>= 1;
    if (n > 0) b = cmulx(b, b);
  }
  return r;
}

__device__ __forceinline__ float rl(float v, int j) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
}
__device__ __forceinline__ ffcx readlane_c(ffcx v, int j) {
  return {{rl(v.re.hi, j), rl(v.re.lo, j)}, {rl(v.im.hi, j), rl(v.im.lo, j)}};
}

// Re(x y)
__device__ __forceinline__ ff re_mul(ffcx x, ffcx y) {
  return ff_add(ff_mul(x.re, y.re), ffneg(ff_mul(x.im, y.im)));
}

// y2 = a y1 - b y0
__device__ __forceinline__ ff rec_step(ff a, ff b, ff y1, ff y0) {
  return ff_add(ff_mul(a, y1), ffneg(ff_mul(b, y0)));
}

// Adds Re(u z^(64 t)) for t < R to acc, given u and the recurrence of its mode.
template <int R>
__device__ __forceinline__ void add_mode(ff (&acc)[R], ffcx u, const LinMode& md) {
  const ff a = {md.ah, md.al}, b = {md.bh, md.bl};
  ff y0 = u.re, y1 = re_mul(u, load_ffc(md.s1));
  acc[0] = ff_add(acc[0], y0);
  acc[1] = ff_add(acc[1], y1);
#pragma unroll
  for (int t = 2; t < R; ++t) {
    const ff y2 = rec_step(a, b, y1, y0);
    acc[t] = ff_add(acc[t], y2);
    y0 = y1;
    y1 = y2;
  }
}

// The same for two modes at once (two independent recurrences).
template <int R>
__device__ __forceinline__ void add_mode_pair(ff (&acc)[R], ffcx u, const LinMode& md, ffcx v,
                                              const LinMode& me) {
  const ff a = {md.ah, md.al}, b = {md.bh, md.bl};
  const ff a2 = {me.ah, me.al}, b2 = {me.bh, me.bl};
  ff y0 = u.re, y1 = re_mul(u, load_ffc(md.s1));
  ff x0 = v.re, x1 = re_mul(v, load_ffc(me.s1));
  acc[0] = ff_add(acc[0], ff_add(y0, x0));
  acc[1] = ff_add(acc[1], ff_add(y1, x1));
#pragma unroll
  for (int t = 2; t < R; ++t) {
    const ff y2 = rec_step(a, b, y1, y0);
    const ff x2 = rec_step(a2, b2, x1, x0);
    acc[t] = ff_add(acc[t], ff_add(y2, x2));
    y0 = y1;
    y1 = y2;
    x0 = x1;
    x1 = x2;
  }
}

__device__ __forceinline__ void put(float* o, long long i, ff v) { o[i] = v.hi + v.lo; }
__device__ __forceinline__ void put(float2* o, long long i, ff v) { o[i] = make_float2(v.hi, v.lo); }

}  // namespace

// amp: per amplitude set and mode, (P1, P2) as two FFc; OutT float (output
// samples) or float2 (float-float impulse responses).
template <int R, typename OutT>
__global__ __launch_bounds__(kLinWaves * 64) void lin_sum_kernel(const LinMode* __restrict__ modes,
                                                                 const FFc* __restrict__ amp,
                                                                 const FFc* __restrict__ ztab,
                                                                 const LinSeg* __restrict__ segs,
                                                                 OutT* __restrict__ out) {
  const LinSeg sg = segs[blockIdx.y];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long s0 = ((long long)blockIdx.x * kLinWaves + wave) * (64LL * R);
  if (s0 >= sg.len) return;
  const long long nb = sg.e0 + s0, n0 = nb + lane;
  const FFc* Pa = amp + 2 * sg.amp_off;
  ff acc[R];
#pragma unroll
  for (int t = 0; t < R; ++t) acc[t] = {0.f, 0.f};
  // complex-conjugate root pairs [m0, mc), two modes at a time
  for (int kb = sg.m0; kb < sg.mc; kb += 64) {
    ffcx zb = {{0.f, 0.f}, {0.f, 0.f}};  // z1^nb of mode kb + lane
    if (kb + lane < sg.mc) zb = cpowx(load_ffc(modes[kb + lane].z1), nb);
    const int kn = min(64, sg.mc - kb);
    int j = 0;
    for (; j + 1 < kn; j += 2) {
      const int k = kb + j;
      const LinMode md = modes[k], me = modes[k + 1];
      const ffcx wu = cmulx(readlane_c(zb, j), load_ffc(ztab[(size_t)k * 64 + lane]));
      const ffcx wv = cmulx(readlane_c(zb, j + 1), load_ffc(ztab[(size_t)(k + 1) * 64 + lane]));
      add_mode_pair<R>(acc, cmulx(load_ffc(Pa[2 * k]), wu), md, cmulx(load_ffc(Pa[2 * (k + 1)]), wv), me);
    }
    if (j < kn) {
      const int k = kb + j;
      const LinMode md = modes[k];
      const ffcx wu = cmulx(readlane_c(zb, j), load_ffc(ztab[(size_t)k * 64 + lane]));
      add_mode<R>(acc, cmulx(load_ffc(Pa[2 * k]), wu), md);
    }
  }
  // real root pairs [mc, m1): both roots, powers taken directly per lane
  for (int k = sg.mc; k < sg.m1; ++k) {
    const LinMode md = modes[k];
    const ffcx u1 = cmulx(load_ffc(Pa[2 * k]), cpowx(load_ffc(md.z1), n0));
    const ffcx u2 = cmulx(load_ffc(Pa[2 * k + 1]), cpowx(load_ffc(md.z2), n0));
    const ff a = {md.ah, md.al}, b = {md.bh, md.bl};
    ff y0 = ff_add(u1.re, u2.re);
    ff y1 = ff_add(re_mul(u1, load_ffc(md.s1)), re_mul(u2, load_ffc(md.s2)));
    acc[0] = ff_add(acc[0], y0);
    acc[1] = ff_add(acc[1], y1);
#pragma unroll
    for (int t = 2; t < R; ++t) {
      const ff y2 = rec_step(a, b, y1, y0);
      acc[t] = ff_add(acc[t], y2);
      y0 = y1;
      y1 = y2;
    }
  }
  OutT* o = out + sg.out_off;
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const long long i = s0 + lane + 64LL * t;
    if (i < sg.len) put(o, i, acc[t]);
  }
}

// z1^l, l < 64, of every mode
__global__ void lin_tab_kernel(const LinMode* __restrict__ modes, int M, FFc* __restrict__ ztab) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 64LL * M) return;
  const ffcx v = cpowx(load_ffc(modes[i >> 6].z1), i & 63);
  ztab[i] = FFc{v.re.hi, v.re.lo, v.im.hi, v.im.lo};
}

// Amplitude sets [free | post | impulse] of every mode; the post set runs the
// excitation through each root (V <- (V + b C e[m]) z), one thread per mode.
__global__ void lin_amp_kernel(const LinInit* __restrict__ init, int M, const float* __restrict__ e_ext,
                               FFc* __restrict__ amp) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  const LinInit I = init[k];
  const ffcx A = load_ffc(I.A), B = load_ffc(I.B), z1 = load_ffc(I.z1), z2 = load_ffc(I.z2);
  ffcx v1 = A, v2 = B;
  const ffcx bc = cscale(load_ffc(I.C), ff{I.bh, I.bl});
  const ffcx mbc = {ffneg(bc.re), ffneg(bc.im)};
  const float* e = e_ext + I.e_off;
  for (long long m = 0; m < I.n_exc; ++m) {
    const float em = e[m];
    v1 = cmulx(caddx(v1, cscalef(bc, em)), z1);
    v2 = cmulx(caddx(v2, cscalef(mbc, em)), z2);
  }
  const ff c = {I.ch, I.cl};
  const ff f = I.conj ? ff{2.f * I.ch, 2.f * I.cl} : c;
  const ff k2 = I.conj ? ff{0.f, 0.f} : c;
  auto st = [&](size_t slot, ffcx v) { amp[slot] = FFc{v.re.hi, v.re.lo, v.im.hi, v.im.lo}; };
  st(2 * (size_t)k, cscale(A, f));
  st(2 * (size_t)k + 1, cscale(B, k2));
  st(2 * ((size_t)M + k), cscale(v1, f));
  st(2 * ((size_t)M + k) + 1, cscale(v2, k2));
  st(2 * (2 * (size_t)M + k), cscale(bc, f));
  st(2 * (2 * (size_t)M + k) + 1, cscale(mbc, k2));
}

// Inside the excitation window: y[n - base] += sum_{m < n} e[m] h[n - m] for
// n in [base, min(base + n_steps, n_exc)); the h row (float-float) holds lags
// 1 .. n_exc - 1; the sum is float-float.
__global__ void lin_conv_kernel(const LinForced* __restrict__ forced, const float2* __restrict__ h,
                                long long h_stride, const float* __restrict__ e_ext, long long base,
                                long long n_steps, float* __restrict__ y, long long y_stride) {
  const LinForced F = forced[blockIdx.y];
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long n = base + i;
  if (i >= n_steps || n >= F.n_exc) return;
  const float* e = e_ext + F.e_off;
  const float2* hb = h + blockIdx.y * h_stride - 1;  // hb[lag], lag >= 1
  ff v = {0.f, 0.f};
  for (long long m = 0; m < n; ++m) {
    const float2 hl = hb[n - m];
    v = ff_add(v, ff_mul_f({hl.x, hl.y}, e[m]));
  }
  float* yo = y + F.inst * y_stride + i;
  const ff s = ff_add({*yo, 0.f}, v);
  *yo = s.hi + s.lo;
}

hipError_t launch_lin_sum(const LinMode* modes, const FFc* amp, const FFc* ztab, const LinSeg* segs,
                          int n_segs, long long max_len, float* out, hipStream_t s) {
  if (max_len < 1 || n_segs < 1) return hipSuccess;
  const long long per_block = 64LL * kLinWaves * kLinRun;
  dim3 grid((unsigned)((max_len + per_block - 1) / per_block), n_segs);
  hipLaunchKernelGGL((lin_sum_kernel<kLinRun, float>), grid, dim3(64 * kLinWaves), 0, s, modes, amp, ztab,
                     segs, out);
  return hipGetLastError();
}

hipError_t launch_lin_sum_ff(const LinMode* modes, const FFc* amp, const FFc* ztab, const LinSeg* segs,
                             int n_segs, long long max_len, float2* out, hipStream_t s) {
  if (max_len < 1 || n_segs < 1) return hipSuccess;
  const long long per_block = 64LL * kLinWaves * kLinRun;
  dim3 grid((unsigned)((max_len + per_block - 1) / per_block), n_segs);
  hipLaunchKernelGGL((lin_sum_kernel<kLinRun, float2>), grid, dim3(64 * kLinWaves), 0, s, modes, amp, ztab,
                     segs, out);
  return hipGetLastError();
}

hipError_t launch_lin_amp(const LinInit* init, const LinMode* modes, int M, const float* e_ext, FFc* amp,
                          FFc* ztab, hipStream_t s) {
  if (M < 1) return hipSuccess;
  hipLaunchKernelGGL(lin_tab_kernel, dim3((unsigned)((64LL * M + 255) / 256)), dim3(256), 0, s, modes, M, ztab);
  hipLaunchKernelGGL(lin_amp_kernel, dim3((M + 127) / 128), dim3(128), 0, s, init, M, e_ext, amp);
  return hipGetLastError();
}

hipError_t launch_lin_conv(const LinForced* forced, int n_forced, const float2* h, long long h_stride,
                           const float* e_ext, long long base, long long n_steps, long long window,
                           float* y, long long y_stride, hipStream_t s) {
  if (n_forced < 1 || window < 1) return hipSuccess;
  dim3 grid((unsigned)((window + 255) / 256), n_forced);
  hipLaunchKernelGGL(lin_conv_kernel, grid, dim3(256), 0, s, forced, h, h_stride, e_ext, base, n_steps, y,
                     y_stride);
  return hipGetLastError();
}

}  // namespace modal
