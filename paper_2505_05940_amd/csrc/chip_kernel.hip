// On-chip time stepping of small modal systems (gfx950): one workgroup of
// kChipWaves waves per instance, with the instance's whole coupling tensor
// held in registers for the launch.
//
// The streaming step kernel re-reads Ht from the memory hierarchy every
// sample and, for a lone instance, spreads its rows over several workgroups
// that exchange partial forces through global memory each step; a small
// plate's step is then bound by the latency of those round trips, not by its
// arithmetic.  Here the tensor of an instance with at most 64 transverse
// modes is loaded once: wave w keeps the in-plane rows n = w + kChipWaves r
// (r < R), lane k the column k of each, h[r][j] = Ht[n][j][k] (j < NT).  Per
// sample (paper: Sec. 3.1 modal forces, Sec. 3.2 modal update)
//   1. wave 0 publishes q^n (fp32 high part) to LDS and writes the output
//      y^n = sum_k c_k q_k^n;
//   2. every wave forms, for its rows, V[n, k] = sum_j Ht[n][j][k] q_j
//      (q broadcast from LDS), eta_n = sum_k V[n, k] q_k (a DPP sum over the
//      wave) and its partial force F_k = sum_n eta_n V[n, k];
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

// NT: tensor columns held per row (>= nt of every instance, multiple of 8);
// R: rows per wave (>= ceil(nin / kChipWaves)).
template <int NT, int R>
__global__ void __launch_bounds__(kWave * kChipWaves) chip_kernel(StepParams P) {
  __shared__ float4 xs4[kWave / 4];               // q^n (high parts), zero past nt
  __shared__ float red[kChipWaves][kWave];       // per-wave partial forces
  float* Xs = reinterpret_cast<float*>(xs4);
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const UnitDev U = P.unit[P.wg_begin[blockIdx.x]];
  const InstDev I = P.inst[U.inst];
  const int nt = I.nt;
  const bool vk = I.kind == KIND_VK;
  const bool mine = lane < nt;  // this lane's mode exists

  float h[R][NT];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int n = wave + kChipWaves * r;
    const float* row = P.H + I.h_off + (long long)n * nt * I.ntp + lane;
#pragma unroll
    for (int j = 0; j < NT; ++j) h[r][j] = (vk && mine && n < I.nin && j < nt) ? row[(long long)j * I.ntp] : 0.f;
  }

  // wave 0: its lane's mode, state and coefficients
  float xh = 0.f, xl = 0.f, dh = 0.f, dl = 0.f;
  float mh = 0.f, ml = 0.f, ph = 0.f, pl = 0.f, rh = 0.f, rl = 0.f, bx = 0.f, cw = 0.f, lam = 0.f;
  if (wave == 0) {
    if (mine) {
      const int so = U.state_off + lane, mo = I.mode_off + lane;
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
    Xs[lane] = xh;
  }
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
      for (int j4 = 0; j4 < NT / 4; ++j4) {
        const float4 q = xs4[j4];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          V[r] = fmaf(h[r][4 * j4], q.x, V[r]);
          V[r] = fmaf(h[r][4 * j4 + 1], q.y, V[r]);
          V[r] = fmaf(h[r][4 * j4 + 2], q.z, V[r]);
          V[r] = fmaf(h[r][4 * j4 + 3], q.w, V[r]);
        }
      }
      const float qk = Xs[lane];
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
      if (mine) Xs[lane] = xh;
    }
  }
  if (wave == 0) {
    if (mine) {
      const int so = U.state_off + lane;
      P.x_hi[so] = xh;
      P.x_lo[so] = xl;
      P.d_hi[so] = dh;
      P.d_lo[so] = dl;
    }
    if (__any(bad) && lane == 0) atomicOr(&P.flags[1], 1);
  }
}

// Column widths and rows per wave with a kernel: R NT <= 200 floats of
// tensor per lane (with the rest of the kernel's registers, at most two
// waves per SIMD).
bool chip_shape(int max_nt, int max_rows, int& nt_tile, int& rows) {
  static const int widths[] = {16, 32, 40, 48, 64};
  rows = std::max(1, max_rows);
  for (int w : widths)
    if (w >= max_nt) {
      nt_tile = w;
      return rows * w <= 200 && rows <= 8;
    }
  return false;
}

hipError_t launch_chip(const StepParams& P, int nt_tile, int rows, int n_wg, hipStream_t s) {
  if (P.ckpt || P.rec_x) return hipErrorInvalidValue;  // forward-only contexts
#define CL(W, RR)                                                                                \
  if (nt_tile == W && rows == RR) {                                                              \
    hipLaunchKernelGGL((chip_kernel<W, RR>), dim3(n_wg), dim3(kWave * kChipWaves), 0, s, P);     \
    return hipGetLastError();                                                                    \
  }
  CL(16, 1) CL(16, 2) CL(16, 3) CL(16, 4) CL(16, 5) CL(16, 6) CL(16, 7) CL(16, 8)
  CL(32, 1) CL(32, 2) CL(32, 3) CL(32, 4) CL(32, 5) CL(32, 6)
  CL(40, 1) CL(40, 2) CL(40, 3) CL(40, 4) CL(40, 5)
  CL(48, 1) CL(48, 2) CL(48, 3) CL(48, 4)
  CL(64, 1) CL(64, 2) CL(64, 3)
#undef CL
  return hipErrorInvalidValue;
}

}  // namespace modal
