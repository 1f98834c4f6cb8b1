// On-chip time stepping of small modal systems (gfx950): one workgroup of
// kChipWaves waves per instance, with the instance's whole coupling tensor
// held in registers for the launch.
//
// The streaming step kernel re-reads Ht from the memory hierarchy every
// sample and, for a lone instance, spreads its rows over several workgroups
// that exchange partial forces through global memory each step; a small
// plate's step is then bound by the latency of those round trips, not by its
// arithmetic.  Here the tensor of an instance with at most 64 transverse
// modes is loaded once, laid out by the instance's ChipMap: lane p stands
// for mode perm[p], wave w keeps the in-plane rows row[w][r] (r < R), and
// for each of them lane p holds the W entries h[r][t] = Ht[n][perm[jb + t]][perm[p]]
// (t < jl, zero past it) of the one run of columns that can be nonzero
// against it: all modes for a tensor without classes; for a sine-family
// tensor, whose entries vanish unless the parity classes of the two columns
// and the row match (Sec. 5, sparsity), only the partner class, a quarter of
// them.  Per sample (paper: Sec. 3.1 modal forces, Sec. 3.2 modal update)
//   1. wave 0 publishes q^n (fp32 high part, lane order) to LDS and writes
//      the output y^n = sum_k c_k q_k^n;
//   2. every wave forms, for its rows, V[n, p] = sum_t h[r][t] q[jb + t]
//      (a wave's rows share jb, so each q read serves all of them),
//      eta_n = sum_p V[n, p] q_p (a DPP sum over the wave) and its partial
//      force F_p = sum_n eta_n V[n, p];
//   3. wave 0 adds the waves' partial forces (LDS) and advances its lane's
//      mode in float-float arithmetic, d+ = m X - p d + r (b e - F),
//      X+ = X + d+, exactly as the streaming kernel does.
// Tension-modulated instances need no tensor: wave 0 forms
// F_k = kappa lambda_k q_k sum_j lambda_j q_j^2 itself.  Linear instances
// have F = 0.  Two workgroup barriers per sample and no global memory
// besides the excitation sample and the output.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.h"
#include "kernels.h"

namespace modal {

namespace {

// R sums over the 64 lanes at once (the DPP steps of wave_sum interleaved so
// that their latencies overlap)
template <int R>
__device__ __forceinline__ void wave_sums(float (&v)[R]) {
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] += dpp_mov<0xB1>(v[r]);
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] += dpp_mov<0x4E>(v[r]);
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] += dpp_mov<0x141>(v[r]);
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] += dpp_mov<0x140>(v[r]);
#pragma unroll
  for (int r = 0; r < R; ++r)
    v[r] = (lane_value(v[r], 0) + lane_value(v[r], 16)) + (lane_value(v[r], 32) + lane_value(v[r], 48));
}

}  // namespace

// W: tensor columns held per row and lane (>= every jl, multiple of 4);
// R: rows per wave (>= every wave's row count).
template <int W, int R>
__global__ void __launch_bounds__(kWave * kChipWaves) chip_kernel(StepParams P) {
  // q^n (high parts) in lane order, zero past the last lane so that a run of
  // W columns from any jb reads zeros beyond the modes
  __shared__ float4 xc4[(kWave + 64) / 4];
  __shared__ float red[kChipWaves][kWave];  // per-wave partial forces
  float* Xc = reinterpret_cast<float*>(xc4);
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
  const UnitDev U = P.unit[P.wg_begin[blockIdx.x]];
  const InstDev I = P.inst[U.inst];
  const ChipMap& M = P.chip[U.inst];
  const int nt = I.nt;
  const bool vk = I.kind == KIND_VK;
  const int k = M.perm[lane];  // this lane's mode (-1: none)
  const int jb = M.jb[wave][lane];
  const int jl = M.jl[wave][lane];

  float h[R][W];
#pragma unroll
  for (int t = 0; t < W; ++t) {
    const int j = (vk && k >= 0 && t < jl) ? M.perm[jb + t] : -1;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int n = M.row[wave][r];
      h[r][t] = (j >= 0 && n >= 0) ? P.H[I.h_off + ((long long)n * nt + j) * I.ntp + k] : 0.f;
    }
  }
  for (int i = threadIdx.x; i < kWave + 64; i += kWave * kChipWaves) Xc[i] = 0.f;
  __syncthreads();

  // wave 0: its lane's mode, state and coefficients
  float xh = 0.f, xl = 0.f, dh = 0.f, dl = 0.f;
  float mh = 0.f, ml = 0.f, ph = 0.f, pl = 0.f, rh = 0.f, rl = 0.f, bx = 0.f, cw = 0.f, lam = 0.f;
  if (wave == 0) {
    if (k >= 0) {
      const int so = U.state_off + k, mo = I.mode_off + k;
      xh = P.x_hi[so];
      xl = P.x_lo[so];
      dh = P.d_hi[so];
      dl = P.d_lo[so];
      mh = P.m_hi[mo];
      ml = P.m_lo[mo];
      ph = P.p_hi[mo];
      pl = P.p_lo[mo];
      rh = P.r_hi[mo];
      rl = P.r_lo[mo];
      bx = P.b_ext[mo];
      cw = P.c_out[mo];
      lam = P.lam[mo];
    }
    Xc[lane] = xh;
  }
  const float4* xq = reinterpret_cast<const float4*>(Xc + jb);
  const long long base = *P.step_base;
  bool bad = false;
  for (int s = 0; s < P.n_steps; ++s) {
    const long long n = base + s;
    __syncthreads();  // q^n in LDS; the previous step's partial forces consumed
    float e = 0.f;
    if (wave == 0) {
      if (n < I.n_exc) e = P.e_ext[I.e_off + n];
      const float yv = wave_sum(cw * xh);
      if (lane == 0 && P.y) P.y[(long long)I.out_row * P.y_stride + s] = yv;
    }
    float F = 0.f;
    if (vk) {
      float V[R];
#pragma unroll
      for (int r = 0; r < R; ++r) V[r] = 0.f;
#pragma unroll
      for (int t4 = 0; t4 < W / 4; ++t4) {
        const float4 q = xq[t4];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          V[r] = fmaf(h[r][4 * t4], q.x, V[r]);
          V[r] = fmaf(h[r][4 * t4 + 1], q.y, V[r]);
          V[r] = fmaf(h[r][4 * t4 + 2], q.z, V[r]);
          V[r] = fmaf(h[r][4 * t4 + 3], q.w, V[r]);
        }
      }
      const float qk = Xc[lane];
      float eta[R];
#pragma unroll
      for (int r = 0; r < R; ++r) eta[r] = V[r] * qk;
      wave_sums<R>(eta);
#pragma unroll
      for (int r = 0; r < R; ++r) F = fmaf(eta[r], V[r], F);
      red[wave][lane] = F;
      __syncthreads();  // every wave's partial force
      if (wave == 0) {
        F = red[0][lane];
#pragma unroll
        for (int w = 1; w < kChipWaves; ++w) F += red[w][lane];
      }
    } else if (I.kind == KIND_TENSION && wave == 0) {
      const float S = wave_sum(lam * xh * xh) * I.kappa;
      F = lam * xh * S;
    }
    if (wave == 0) {
      ff_step(xh, xl, dh, dl, mh, ml, ph, pl, rh, rl, fmaf(bx, e, -F));
      bad |= !isfinite(xh);
      if (k >= 0) Xc[lane] = xh;
    }
  }
  if (wave == 0) {
    if (k >= 0) {
      const int so = U.state_off + k;
      P.x_hi[so] = xh;
      P.x_lo[so] = xl;
      P.d_hi[so] = dh;
      P.d_lo[so] = dl;
    }
    if (__any(bad) && lane == 0) atomicOr(&P.flags[1], 1);
  }
}

// Instances without a coupling tensor (tension-modulated and linear ones)
// of up to 64 M modes (M <= kChipWaveModes / 64), one wave each: lane p
// steps modes p, p + 64, ..., p + 64 (M - 1).  Per sample: the output and, for the tension
// force F_k = kappa lam_k q_k sum_j lam_j q_j^2, one more sum over the wave
// (DPP), then every mode's float-float update; no barrier and no memory
// traffic but the output and the excitation, read 64 samples ahead.
template <int M>
__global__ void __launch_bounds__(kWave) chip_wave_kernel(StepParams P) {
  const int lane = threadIdx.x;
  const UnitDev U = P.unit[P.wg_begin[blockIdx.x]];
  const InstDev I = P.inst[U.inst];
  const int nt = I.nt;
  const bool tension = I.kind == KIND_TENSION;
  float xh[M], xl[M], dh[M], dl[M], mh[M], ml[M], ph[M], pl[M], rh[M], rl[M], bx[M], cw[M], lam[M];
#pragma unroll
  for (int i = 0; i < M; ++i) {
    const int k = lane + kWave * i;
    const bool live = k < nt;
    const int so = U.state_off + k, mo = I.mode_off + k;
    xh[i] = live ? P.x_hi[so] : 0.f;
    xl[i] = live ? P.x_lo[so] : 0.f;
    dh[i] = live ? P.d_hi[so] : 0.f;
    dl[i] = live ? P.d_lo[so] : 0.f;
    mh[i] = live ? P.m_hi[mo] : 0.f;
    ml[i] = live ? P.m_lo[mo] : 0.f;
    ph[i] = live ? P.p_hi[mo] : 0.f;
    pl[i] = live ? P.p_lo[mo] : 0.f;
    rh[i] = live ? P.r_hi[mo] : 0.f;
    rl[i] = live ? P.r_lo[mo] : 0.f;
    bx[i] = live ? P.b_ext[mo] : 0.f;
    cw[i] = live ? P.c_out[mo] : 0.f;
    lam[i] = live ? P.lam[mo] : 0.f;
  }
  const long long base = *P.step_base;
  // excitation samples 64 at a time, lane j holding step 64 c + j of chunk
  // c; each chunk's loads are issued a chunk ahead, and the steps of a chunk
  // read no memory, so no step waits on the vector-memory counter
  auto chunk = [&](long long n0) {
    const long long m = n0 + lane;
    return m < I.n_exc ? P.e_ext[I.e_off + m] : 0.f;
  };
  float en = chunk(base);
  bool bad = false;
  for (int s0 = 0; s0 < P.n_steps; s0 += kWave) {
    const float ec = en;
    en = chunk(base + s0 + kWave);
    const int js = min(kWave, P.n_steps - s0);
    for (int j = 0; j < js; ++j) {
      const float e = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ec), j));
      float yp = 0.f, sp = 0.f;
#pragma unroll
      for (int i = 0; i < M; ++i) {
        yp = fmaf(cw[i], xh[i], yp);
        sp = fmaf(lam[i] * xh[i], xh[i], sp);
      }
      const float yv = wave_sum(yp);
      if (lane == 0 && P.y) P.y[(long long)I.out_row * P.y_stride + s0 + j] = yv;
      const float S = tension ? wave_sum(sp) * I.kappa : 0.f;
#pragma unroll
      for (int i = 0; i < M; ++i) {
        const float F = lam[i] * xh[i] * S;
        ff_step(xh[i], xl[i], dh[i], dl[i], mh[i], ml[i], ph[i], pl[i], rh[i], rl[i], fmaf(bx[i], e, -F));
        bad |= !isfinite(xh[i]);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < M; ++i) {
    const int k = lane + kWave * i;
    if (k < nt) {
      const int so = U.state_off + k;
      P.x_hi[so] = xh[i];
      P.x_lo[so] = xl[i];
      P.d_hi[so] = dh[i];
      P.d_lo[so] = dl[i];
    }
  }
  if (__any(bad) && lane == 0) atomicOr(&P.flags[1], 1);
}

// m: modes per lane, at least the batch's largest n_t / 64
hipError_t launch_chip_wave(const StepParams& P, int m, int n_wg, hipStream_t s) {
  if (P.ckpt || P.rec_x) return hipErrorInvalidValue;  // forward-only contexts
  static_assert(kChipWaveModes == 4 * kWave, "one kernel per modes-per-lane count");
  switch (m) {
    case 1: hipLaunchKernelGGL(chip_wave_kernel<1>, dim3(n_wg), dim3(kWave), 0, s, P); break;
    case 2: hipLaunchKernelGGL(chip_wave_kernel<2>, dim3(n_wg), dim3(kWave), 0, s, P); break;
    case 3: hipLaunchKernelGGL(chip_wave_kernel<3>, dim3(n_wg), dim3(kWave), 0, s, P); break;
    case 4: hipLaunchKernelGGL(chip_wave_kernel<4>, dim3(n_wg), dim3(kWave), 0, s, P); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Widths and rows per wave with a kernel: W R <= 200 tensor floats per lane
// (with the rest of the kernel's registers, at most two waves per SIMD).
bool chip_shape(int max_w, int max_rows, int& w_tile, int& rows) {
  static const int widths[] = {8, 16, 20, 24, 32, 40, 48, 64};
  static const int counts[] = {1, 2, 3, 4, 5, 6, 7, 8, 10, 12};
  int w = 0, r = 0;
  for (int x : widths)
    if (x >= max_w) {
      w = x;
      break;
    }
  for (int x : counts)
    if (x >= std::max(1, max_rows)) {
      r = x;
      break;
    }
  if (!w || !r || w * r > 200) return false;
  w_tile = w;
  rows = r;
  return true;
}

hipError_t launch_chip(const StepParams& P, int w_tile, int rows, int n_wg, hipStream_t s) {
  if (P.ckpt || P.rec_x || !P.chip) return hipErrorInvalidValue;  // forward-only contexts
#define CL(WW, RR)                                                                               \
  if (w_tile == WW && rows == RR) {                                                              \
    hipLaunchKernelGGL((chip_kernel<WW, RR>), dim3(n_wg), dim3(kWave * kChipWaves), 0, s, P);    \
    return hipGetLastError();                                                                    \
  }
  CL(8, 1) CL(8, 2) CL(8, 3) CL(8, 4) CL(8, 5) CL(8, 6) CL(8, 7) CL(8, 8) CL(8, 10) CL(8, 12)
  CL(16, 1) CL(16, 2) CL(16, 3) CL(16, 4) CL(16, 5) CL(16, 6) CL(16, 7) CL(16, 8) CL(16, 10) CL(16, 12)
  CL(20, 1) CL(20, 2) CL(20, 3) CL(20, 4) CL(20, 5) CL(20, 6) CL(20, 7) CL(20, 8) CL(20, 10)
  CL(24, 1) CL(24, 2) CL(24, 3) CL(24, 4) CL(24, 5) CL(24, 6) CL(24, 7) CL(24, 8)
  CL(32, 1) CL(32, 2) CL(32, 3) CL(32, 4) CL(32, 5) CL(32, 6)
  CL(40, 1) CL(40, 2) CL(40, 3) CL(40, 4) CL(40, 5)
  CL(48, 1) CL(48, 2) CL(48, 3) CL(48, 4)
  CL(64, 1) CL(64, 2) CL(64, 3)
#undef CL
  return hipErrorInvalidValue;
}

}  // namespace modal
