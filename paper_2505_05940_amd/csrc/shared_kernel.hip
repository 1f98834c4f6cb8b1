// Time loop for batches that share one coupling tensor up to a per-row scale
// (gfx950, FP32 MFMA).
//
// With Ht_b[n][k][q] = s_b[n] H0[n][k][q] for every instance b of a group,
// the von Karman force of the nonlinear plate equation (paper: Sec. 2.1) is
//   V0[n][k][b] = sum_q H0[n][k][q] X[q][b]          (one product per n)
//   eta0[n][b]  = sum_k V0[n][k][b] X[k][b]
//   F[k][b]     = sum_n s_b[n]^2 eta0[n][b] V0[n][k][b]
// so a step is, per in-plane row n, a dense (n_t x n_t) by (n_t x columns)
// product followed by per-column reductions.  The product runs on
// v_mfma_f32_16x16x4f32: lane l supplies A[l%16][l/16] and B[l/16][l%16]
// and receives D[4 (l/16) + r][l%16] in accumulator r.  H0[n] is the A
// operand, pre-packed per (n, 16-row tile t, 4-wide K step c) in lane order
// so that a workgroup stages one row n with coalesced 16-byte loads into
// LDS (double-buffered, the next row in flight while the current one is
// multiplied); X (FP32 high part of the float-float state) is the B operand,
// held in registers for the whole step.  Every column keeps its own
// float-float state and coefficients and the update is the increment form of
// the forward kernel, so the only difference from it is the order of the
// FP32 sums inside the contraction.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace modal {

typedef float v4f __attribute__((ext_vector_type(4)));

template <int KT, int JT>
__global__ void __launch_bounds__(kWave * kSharedWaves) shared_kernel(SharedParams P) {
  constexpr int KC = 4 * KT;                      // K steps of 4 at most
  constexpr int CW = 16 * JT;                     // columns per wave
  constexpr int ABUF = KT * KC * 64;              // floats of one packed row n (max)
  constexpr int NA = (ABUF / 4 + kWave * kSharedWaves - 1) / (kWave * kSharedWaves);
  extern __shared__ float4 lds4[];
  float* Abuf = reinterpret_cast<float*>(lds4);   // [2][ABUF]
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
  const int col16 = lane & 15, quad = lane >> 4;
  float* xs = Abuf + 2 * ABUF + wave * (16 * KT) * CW;  // this wave's X: [16 KT][CW]
  const SharedWg W = P.wg[blockIdx.x];
  const int kt = W.kt, kc = W.kc;
  const int nA4 = kt * kc * 16;  // float4 per packed row n of this group
  const float4* Ag = reinterpret_cast<const float4*>(P.A + W.a_off);
  const int wcol = wave * CW;
  const long long col0 = (long long)blockIdx.x * P.cols + wcol;  // first global column of the wave

  // X^n of the wave's columns into LDS
  for (int i = lane; i < 16 * KT * CW; i += kWave) {
    const int k = i / CW, cc = i % CW;
    xs[i] = P.x_hi[(col0 + cc) * P.ktot + k];
  }
  SharedSlot sl[JT];
#pragma unroll
  for (int j = 0; j < JT; ++j) sl[j] = P.slot[col0 + 16 * j + col16];
  __builtin_amdgcn_wave_barrier();
  wave_lds_sync();
  const long long base = *P.step_base;

  for (int s = 0; s < P.n_steps; ++s) {
    const long long nabs = base + s;
    float Xb[JT][KC];
    v4f Xd[JT][KT], F[JT][KT];
#pragma unroll
    for (int j = 0; j < JT; ++j) {
#pragma unroll
      for (int c = 0; c < KC; ++c) Xb[j][c] = xs[(4 * c + quad) * CW + 16 * j + col16];
#pragma unroll
      for (int t = 0; t < KT; ++t) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          Xd[j][t][r] = xs[(16 * t + 4 * quad + r) * CW + 16 * j + col16];
          F[j][t][r] = 0.f;
        }
      }
    }
    // stage row n = 0
    float4 pre[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int idx = tid + kWave * kSharedWaves * i;
      pre[i] = idx < nA4 ? Ag[idx] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    __syncthreads();  // every wave is done with the previous step's buffers
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int idx = tid + kWave * kSharedWaves * i;
      if (idx < nA4) reinterpret_cast<float4*>(Abuf)[idx] = pre[i];
    }
    __syncthreads();
    for (int n = 0; n < W.nin; ++n) {
      const float* Ac = Abuf + (n & 1) * ABUF;
      const bool more = n + 1 < W.nin;
      if (more) {
        const float4* src = Ag + (long long)(n + 1) * nA4;
#pragma unroll
        for (int i = 0; i < NA; ++i) {
          const int idx = tid + kWave * kSharedWaves * i;
          if (idx < nA4) pre[i] = src[idx];
        }
      }
      float s2[JT];
#pragma unroll
      for (int j = 0; j < JT; ++j)
        s2[j] = P.s2[((long long)blockIdx.x * P.nin_max + n) * P.cols + wcol + 16 * j + col16];
      v4f acc[JT][KT];
#pragma unroll
      for (int j = 0; j < JT; ++j)
#pragma unroll
        for (int t = 0; t < KT; ++t) acc[j][t] = (v4f){0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int c = 0; c < KC; ++c) {
        if (c < kc) {
#pragma unroll
          for (int t = 0; t < KT; ++t) {
            if (t < kt) {
              const float a = Ac[(t * kc + c) * 64 + lane];
#pragma unroll
              for (int j = 0; j < JT; ++j)
                acc[j][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, Xb[j][c], acc[j][t], 0, 0, 0);
            }
          }
        }
      }
#pragma unroll
      for (int j = 0; j < JT; ++j) {
        float eta = 0.f;
#pragma unroll
        for (int t = 0; t < KT; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) eta = fmaf(acc[j][t][r], Xd[j][t][r], eta);
        eta += __shfl_xor(eta, 16, kWave);
        eta += __shfl_xor(eta, 32, kWave);
        const float e = s2[j] * eta;
#pragma unroll
        for (int t = 0; t < KT; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) F[j][t][r] = fmaf(e, acc[j][t][r], F[j][t][r]);
      }
      if (more) {
        float4* dst = reinterpret_cast<float4*>(Abuf + ((n + 1) & 1) * ABUF);
#pragma unroll
        for (int i = 0; i < NA; ++i) {
          const int idx = tid + kWave * kSharedWaves * i;
          if (idx < nA4) dst[idx] = pre[i];
        }
      }
      __syncthreads();
    }
    // output y^n = c . X^n and the float-float update of every (mode, column)
    bool bad = false;
#pragma unroll
    for (int j = 0; j < JT; ++j) {
      const long long col = col0 + 16 * j + col16;
      const float e = nabs < sl[j].n_exc ? P.e_ext[sl[j].e_off + nabs] : 0.f;
      float ypart = 0.f;
#pragma unroll
      for (int t = 0; t < KT; ++t) {
        const int k = 16 * t + 4 * quad;
        const long long o = col * P.ktot + k;
        float4 xh = ld4(P.x_hi + o), xl = ld4(P.x_lo + o);
        float4 dh = ld4(P.d_hi + o), dl = ld4(P.d_lo + o);
        const float4 mh = ld4(P.m_hi + o), ml = ld4(P.m_lo + o);
        const float4 ph = ld4(P.p_hi + o), pl = ld4(P.p_lo + o);
        const float4 rh = ld4(P.r_hi + o), rl = ld4(P.r_lo + o);
        const float4 b = ld4(P.b_ext + o), cw = ld4(P.c_out + o);
        ypart += dot4(cw, xh);
        ff_step(xh.x, xl.x, dh.x, dl.x, mh.x, ml.x, ph.x, pl.x, rh.x, rl.x, fmaf(b.x, e, -F[j][t][0]));
        ff_step(xh.y, xl.y, dh.y, dl.y, mh.y, ml.y, ph.y, pl.y, rh.y, rl.y, fmaf(b.y, e, -F[j][t][1]));
        ff_step(xh.z, xl.z, dh.z, dl.z, mh.z, ml.z, ph.z, pl.z, rh.z, rl.z, fmaf(b.z, e, -F[j][t][2]));
        ff_step(xh.w, xl.w, dh.w, dl.w, mh.w, ml.w, ph.w, pl.w, rh.w, rl.w, fmaf(b.w, e, -F[j][t][3]));
        bad |= !(isfinite(xh.x) && isfinite(xh.y) && isfinite(xh.z) && isfinite(xh.w));
        st4(P.x_hi + o, xh);
        st4(P.x_lo + o, xl);
        st4(P.d_hi + o, dh);
        st4(P.d_lo + o, dl);
        float* xr = xs + k * CW + 16 * j + col16;
        xr[0] = xh.x;
        xr[CW] = xh.y;
        xr[2 * CW] = xh.z;
        xr[3 * CW] = xh.w;
      }
      ypart += __shfl_xor(ypart, 16, kWave);
      ypart += __shfl_xor(ypart, 32, kWave);
      if (quad == 0 && sl[j].out_row >= 0 && P.y)
        P.y[(long long)sl[j].out_row * P.y_stride + s] = ypart;
    }
    if (__any(bad) && lane == 0) atomicOr(&P.flags[1], 1);
    wave_lds_sync();  // the new X is visible to every lane of the wave
  }
}

// kt: 16-row tiles of the widest group (1..kSharedMaxKT); jt: 16-column
// tiles per wave (1 or 2).
hipError_t launch_shared(const SharedParams& P, int kt, int jt, int n_wg, hipStream_t s) {
#define SH(K, J)                                                                              \
  hipLaunchKernelGGL((shared_kernel<K, J>), dim3(n_wg), dim3(kWave * kSharedWaves),           \
                     shared_lds_bytes(K, J), s, P)
  if (jt == 1) {
    if (kt <= 1) SH(1, 1); else if (kt == 2) SH(2, 1); else if (kt == 3) SH(3, 1); else SH(4, 1);
  } else {
    if (kt <= 1) SH(1, 2); else if (kt == 2) SH(2, 2); else if (kt == 3) SH(3, 2); else SH(4, 2);
  }
#undef SH
  return hipGetLastError();
}

}  // namespace modal
