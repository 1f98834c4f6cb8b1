// Time loop for batches that share one coupling tensor up to a per-row scale
// (gfx950, FP32 MFMA).
//
// With Ht_b[n][k][q] = s_b[n] H0[n][k][q] for every instance b of a group,
// the von Karman force of the nonlinear plate equation (paper: Sec. 3.1) is
//   V0[n][k][b] = sum_q H0[n][k][q] X[q][b]          (one product per n)
//   eta0[n][b]  = sum_k V0[n][k][b] X[k][b]
//   F[k][b]     = sum_n s_b[n]^2 eta0[n][b] V0[n][k][b]
// so a step is, per in-plane row n, a dense (n_t x n_t) by (n_t x columns)
// product followed by per-column reductions.  The product runs on
// v_mfma_f32_16x16x4f32: lane l supplies A[l%16][l/16] and B[l/16][l%16]
// and receives D[4 (l/16) + r][l%16] in accumulator r.  H0[n] is the A
// operand, pre-packed per (n, 16-row tile t, group of four 4-wide K steps)
// with each lane's four operands adjacent, so that a workgroup stages one
// row n with coalesced 16-byte loads into LDS (double-buffered; rows are
// loaded two ahead of the one multiplied) and a wave reads its operands
// with 16-byte LDS reads; X (FP32 high part of the float-float state) is the
// B operand, held in registers for the whole step, and also kept in LDS in
// accumulator order for the eta reductions; the squared row scales of the
// workgroup's columns sit in LDS for the whole launch.  Every column keeps its own
// float-float state and coefficients and the update is the increment form of
// the forward kernel, so the only difference from it is the order of the
// FP32 sums inside the contraction.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace modal {

typedef float v4f __attribute__((ext_vector_type(4)));

// Sum of v over the four lanes l, l^16, l^32, l^48 (gfx950 lane swaps).
__device__ __forceinline__ float quad_sum(float v) {
  auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  v = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  auto q = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(q[0]) + __uint_as_float(q[1]);
}

// KT: 16-row tiles; KC: 4-wide K steps (compile time, packed rows padded to
// a multiple of 4 steps); JT: 16-column tiles per wave.
template <int KT, int KC, int JT>
__global__ void __launch_bounds__(kWave * kSharedWaves, (KT == 4 && JT == 2) ? 1 : 2)
    shared_kernel(SharedParams P) {
  constexpr int CW = 16 * JT;                     // columns per wave
  constexpr int NT = kWave * kSharedWaves;        // threads per workgroup
  constexpr int KC4 = (KC + 3) / 4;               // 16-byte groups of K steps per lane
  constexpr int ROW4 = KT * KC4 * 64;             // 16-byte slots of one packed row n
  constexpr int NA = (ROW4 + NT - 1) / NT;        // 16-byte loads per thread per row
  constexpr int ABUF4 = NA * NT;                  // staged row, padded to whole rounds
  extern __shared__ float4 lds4[];
  v4f* Abuf4 = reinterpret_cast<v4f*>(lds4);      // [2][ABUF4]
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
  const int col16 = lane & 15, quad = lane >> 4;
  float* xs = reinterpret_cast<float*>(Abuf4 + 2 * ABUF4) + wave * (16 * KT) * CW;  // [16 KT][CW]
  v4f* xdl = reinterpret_cast<v4f*>(Abuf4 + 2 * ABUF4 + kSharedWaves * 4 * KT * CW) +
             wave * JT * KT * 64;  // X in accumulator order: [j][t][lane]
  float* S2 = reinterpret_cast<float*>(Abuf4 + 2 * ABUF4 + 2 * kSharedWaves * 4 * KT * CW);  // [nin][cols]
  const SharedWg W = P.wg[blockIdx.x];
  const v4f* Ag = reinterpret_cast<const v4f*>(P.A + W.a_off);
  const int wcol = wave * CW;
  const long long col0 = (long long)blockIdx.x * P.cols + wcol;  // first global column of the wave

  // the workgroup's squared row scales, and X^n of the wave's columns, into LDS
  for (int i = tid; i < W.nin * P.cols; i += NT)
    S2[i] = P.s2[(long long)blockIdx.x * P.nin_max * P.cols + i];
  for (int i = lane; i < 16 * KT * CW; i += kWave) {
    const int k = i / CW, cc = i % CW;
    xs[i] = P.x_hi[(col0 + cc) * P.ktot + k];
  }
#pragma unroll
  for (int j = 0; j < JT; ++j)
#pragma unroll
    for (int t = 0; t < KT; ++t) {
      const long long o = (col0 + 16 * j + col16) * P.ktot + 16 * t + 4 * quad;
      const float4 x = ld4(P.x_hi + o);
      xdl[(j * KT + t) * 64 + lane] = (v4f){x.x, x.y, x.z, x.w};
    }
  SharedSlot sl[JT];
#pragma unroll
  for (int j = 0; j < JT; ++j) sl[j] = P.slot[col0 + 16 * j + col16];
  __syncthreads();
  const long long base = *P.step_base;

  for (int s = 0; s < P.n_steps; ++s) {
    const long long nabs = base + s;
    v4f F[JT][KT];
    float bq[JT][KC];  // B operands: X[4 c + l/16][column], the whole step
#pragma unroll
    for (int j = 0; j < JT; ++j) {
#pragma unroll
      for (int t = 0; t < KT; ++t) F[j][t] = (v4f){0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int c = 0; c < KC; ++c) bq[j][c] = xs[(4 * c + quad) * CW + 16 * j + col16];
    }
    // rows n are staged two ahead: A(n+1) waits in registers while row n
    // is multiplied out of LDS and A(n+2) is in flight.  Loads are
    // unconditional (index clamped) so nothing waits for them early.
    v4f preA[NA], preB[NA];
#define SH_LOAD(N, DST)                                                     \
  {                                                                         \
    const v4f* src_ = Ag + (long long)(N) * ROW4;                           \
    _Pragma("unroll") for (int i = 0; i < NA; ++i)                          \
      DST[i] = src_[min(tid + NT * i, ROW4 - 1)];                           \
  }
#define SH_STORE(N, SRC)                                                    \
  {                                                                         \
    v4f* dst_ = Abuf4 + ((N) & 1) * ABUF4;                                  \
    _Pragma("unroll") for (int i = 0; i < NA; ++i) dst_[tid + NT * i] = SRC[i]; \
  }
// one in-plane row n: prefetch A(n+2) into AFTER, multiply row n out of LDS,
// fold it into F, then stage A(n+1) from NEXT for the following row
#define SH_ROW(N, NEXT, AFTER)                                                                  \
  {                                                                                             \
    const int n_ = (N);                                                                         \
    SH_LOAD(min(n_ + 2, W.nin - 1), AFTER)                                                     \
    const v4f* Ac = Abuf4 + (n_ & 1) * ABUF4 + lane;                                            \
    v4f a[KT][KC4];                                                                             \
    _Pragma("unroll") for (int t = 0; t < KT; ++t)                                              \
    _Pragma("unroll") for (int c4 = 0; c4 < KC4; ++c4) a[t][c4] = Ac[(t * KC4 + c4) * 64];      \
    v4f acc[JT][KT];                                                                            \
    _Pragma("unroll") for (int j = 0; j < JT; ++j)                                              \
    _Pragma("unroll") for (int t = 0; t < KT; ++t) acc[j][t] = (v4f){0.f, 0.f, 0.f, 0.f};       \
    _Pragma("unroll") for (int c = 0; c < KC; ++c)                                              \
    _Pragma("unroll") for (int t = 0; t < KT; ++t)                                              \
    _Pragma("unroll") for (int j = 0; j < JT; ++j)                                              \
      acc[j][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t][c / 4][c % 4], bq[j][c], acc[j][t], 0, 0, 0); \
    _Pragma("unroll") for (int j = 0; j < JT; ++j) {                                            \
      float eta = 0.f;                                                                          \
      _Pragma("unroll") for (int t = 0; t < KT; ++t) {                                          \
        const v4f xd = xdl[(j * KT + t) * 64 + lane];                                           \
        _Pragma("unroll") for (int r = 0; r < 4; ++r) eta = fmaf(acc[j][t][r], xd[r], eta);    \
      }                                                                                         \
      const float e = S2[n_ * P.cols + wcol + 16 * j + col16] * quad_sum(eta);                  \
      _Pragma("unroll") for (int t = 0; t < KT; ++t)                                            \
      _Pragma("unroll") for (int r = 0; r < 4; ++r) F[j][t][r] = fmaf(e, acc[j][t][r], F[j][t][r]); \
    }                                                                                           \
    SH_STORE(n_ + 1, NEXT)                                                                      \
    block_lds_sync();                                                                           \
  }
    // (past the last row the prefetch repeats it and the stage goes to the
    // buffer no row reads again before the next step restages row 0)
    SH_LOAD(0, preA);
    __syncthreads();  // every wave is done with the previous step's buffers
    SH_STORE(0, preA);
    SH_LOAD(min(1, W.nin - 1), preB);
    __syncthreads();
    int n = 0;
    for (; n + 1 < W.nin; n += 2) {
      SH_ROW(n, preB, preA)
      SH_ROW(n + 1, preA, preB)
    }
    if (n < W.nin) SH_ROW(n, preB, preA)
#undef SH_ROW
#undef SH_LOAD
#undef SH_STORE
    // output y^n = c . X^n and the float-float update of every (mode, column):
    // one 4-mode group per (column tile j, row tile t), its state and
    // coefficients loaded one group ahead of the arithmetic
    bool bad = false;
    float ypart[JT];
    float eo[JT];
#pragma unroll
    for (int j = 0; j < JT; ++j) {
      ypart[j] = 0.f;
      eo[j] = nabs < sl[j].n_exc ? P.e_ext[sl[j].e_off + nabs] : 0.f;
    }
    struct Grp {
      float4 xh, xl, dh, dl, mh, ml, ph, pl, rh, rl, b, cw;
    };
    auto grp_off = [&](int u) -> long long {
      const int j = u / KT, t = u % KT;
      return (col0 + 16 * j + col16) * P.ktot + 16 * t + 4 * quad;
    };
    auto grp_load = [&](long long o) -> Grp {
      Grp g;
      g.xh = ld4(P.x_hi + o); g.xl = ld4(P.x_lo + o); g.dh = ld4(P.d_hi + o); g.dl = ld4(P.d_lo + o);
      g.mh = ld4(P.m_hi + o); g.ml = ld4(P.m_lo + o); g.ph = ld4(P.p_hi + o); g.pl = ld4(P.p_lo + o);
      g.rh = ld4(P.r_hi + o); g.rl = ld4(P.r_lo + o); g.b = ld4(P.b_ext + o); g.cw = ld4(P.c_out + o);
      return g;
    };
    Grp cur = grp_load(grp_off(0));
#pragma unroll
    for (int u = 0; u < JT * KT; ++u) {
      const int j = u / KT, t = u % KT;
      Grp nxt;
      if (u + 1 < JT * KT) nxt = grp_load(grp_off(u + 1));
      const long long o = grp_off(u);
      const float e = eo[j];
      float4 xh = cur.xh, xl = cur.xl, dh = cur.dh, dl = cur.dl;
      ypart[j] += dot4(cur.cw, xh);
      ff_step(xh.x, xl.x, dh.x, dl.x, cur.mh.x, cur.ml.x, cur.ph.x, cur.pl.x, cur.rh.x, cur.rl.x,
              fmaf(cur.b.x, e, -F[j][t][0]));
      ff_step(xh.y, xl.y, dh.y, dl.y, cur.mh.y, cur.ml.y, cur.ph.y, cur.pl.y, cur.rh.y, cur.rl.y,
              fmaf(cur.b.y, e, -F[j][t][1]));
      ff_step(xh.z, xl.z, dh.z, dl.z, cur.mh.z, cur.ml.z, cur.ph.z, cur.pl.z, cur.rh.z, cur.rl.z,
              fmaf(cur.b.z, e, -F[j][t][2]));
      ff_step(xh.w, xl.w, dh.w, dl.w, cur.mh.w, cur.ml.w, cur.ph.w, cur.pl.w, cur.rh.w, cur.rl.w,
              fmaf(cur.b.w, e, -F[j][t][3]));
      bad |= !(isfinite(xh.x) && isfinite(xh.y) && isfinite(xh.z) && isfinite(xh.w));
      st4(P.x_hi + o, xh);
      st4(P.x_lo + o, xl);
      st4(P.d_hi + o, dh);
      st4(P.d_lo + o, dl);
      float* xr = xs + (16 * t + 4 * quad) * CW + 16 * j + col16;
      xr[0] = xh.x;
      xr[CW] = xh.y;
      xr[2 * CW] = xh.z;
      xr[3 * CW] = xh.w;
      xdl[(j * KT + t) * 64 + lane] = (v4f){xh.x, xh.y, xh.z, xh.w};
      if (u + 1 < JT * KT) cur = nxt;
    }
#pragma unroll
    for (int j = 0; j < JT; ++j) {
      const float yv = quad_sum(ypart[j]);
      if (quad == 0 && sl[j].out_row >= 0 && P.y) P.y[(long long)sl[j].out_row * P.y_stride + s] = yv;
    }
    if (__any(bad) && lane == 0) atomicOr(&P.flags[1], 1);
    wave_lds_sync();  // the new X is visible to every lane of the wave
  }
}

// kt: 16-row tiles of the widest group (1..kSharedMaxKT); kc: 4-wide K
// steps of every group (4 kt - 3 .. 4 kt); jt: 16-column tiles per wave (1, 2).
#define SH_KC(K, C)                                                                           \
  if (kc == C) {                                                                              \
    if (jt == 1)                                                                              \
      hipLaunchKernelGGL((shared_kernel<K, C, 1>), dim3(n_wg), dim3(kWave * kSharedWaves),    \
                         shared_lds_bytes(K, C, 1, P.nin_max), s, P);                         \
    else                                                                                      \
      hipLaunchKernelGGL((shared_kernel<K, C, 2>), dim3(n_wg), dim3(kWave * kSharedWaves),    \
                         shared_lds_bytes(K, C, 2, P.nin_max), s, P);                         \
    return hipGetLastError();                                                                 \
  }
#define SH_KT(K)                                                                              \
  if (kt == K) {                                                                              \
    SH_KC(K, 4 * K - 3) SH_KC(K, 4 * K - 2) SH_KC(K, 4 * K - 1) SH_KC(K, 4 * K)               \
  }
hipError_t launch_shared(const SharedParams& P, int kt, int kc, int jt, int n_wg, hipStream_t s) {
  SH_KT(1) SH_KT(2) SH_KT(3) SH_KT(4)
  return hipErrorInvalidValue;
}
#undef SH_KT
#undef SH_KC

}  // namespace modal
