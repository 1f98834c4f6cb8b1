// Persistent time-stepping kernel for batches of modal systems (gfx950).
//
// One workgroup is one 64-lane wave.  A workgroup owns a fixed list of work
// units for the whole launch; a unit is either a whole instance or a slab of
// in-plane rows of a von Karman instance whose coupling tensor is split over
// several workgroups.  Per audio sample (paper: Sec. 2.2, modal oscillator
// update) each unit
//   1. publishes q^n (fp32 high part) to LDS and writes the output sample
//      y^n = sum_k c_k q_k^n (modal-to-physical transform at one point),
//   2. evaluates its share of the nonlinear modal force (Sec. 2.1):
//        von Karman, one pass over its rows of Ht:  V[n,k] = sum_j Ht[n][j][k] q_j
//        (Ht symmetric in its last two indices), eta_n = sum_k V[n,k] q_k,
//        F_k += eta_n V[n,k];
//        tension-modulated: F_k = kappa lambda_k q_k sum_j lambda_j q_j^2,
//   3. advances the state in float-float arithmetic in increment form
//        d^{n+1} = m q^n - p d^n + r (f_ext^n - F^n),  q^{n+1} = q^n + d^{n+1}
//      (m = g + p - 1 = -r omega^2 for Stormer-Verlet), where instances split
//      over several workgroups first exchange their partial forces through
//      global memory and wait on a per-instance arrival counter.
// The coupling tensor is streamed from HBM once per step with 16-byte
// non-temporal loads; each element is used once, so it goes straight to
// registers.  LDS holds q^n and the cross-lane reduction of V.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace modal {

// ---------------------------------------------------------------- float-float
// Error-free transformations (Knuth's TwoSum, Dekker's Fast2Sum, and the
// FMA-based exact product).  This file is compiled with -ffp-contract=off so
// only the explicit fmaf calls fuse.
struct ff {
  float hi, lo;
};
__device__ __forceinline__ ff two_sum(float a, float b) {
  float s = a + b;
  float bb = s - a;
  float e = (a - (s - bb)) + (b - bb);
  return {s, e};
}
__device__ __forceinline__ ff fast_two_sum(float a, float b) {
  float s = a + b;
  float e = b - (s - a);
  return {s, e};
}
__device__ __forceinline__ ff ff_add(ff a, ff b) {
  ff s = two_sum(a.hi, b.hi);
  ff t = two_sum(a.lo, b.lo);
  float e = s.lo + t.hi;
  s = fast_two_sum(s.hi, e);
  e = s.lo + t.lo;
  return fast_two_sum(s.hi, e);
}
__device__ __forceinline__ ff ff_mul(ff a, ff b) {
  float p = a.hi * b.hi;
  float e = fmaf(a.hi, b.hi, -p);
  e = fmaf(a.hi, b.lo, e);
  e = fmaf(a.lo, b.hi, e);
  return fast_two_sum(p, e);
}
__device__ __forceinline__ ff ff_mul_f(ff a, float b) {
  float p = a.hi * b;
  float e = fmaf(a.hi, b, -p);
  e = fmaf(a.lo, b, e);
  return fast_two_sum(p, e);
}

// d+ = m X - p d + r fe ;  X+ = X + d+
__device__ __forceinline__ void ff_step(float& xh, float& xl, float& dh, float& dl,
                                        float mh, float ml, float ph, float pl,
                                        float rh, float rl, float fe) {
  ff X{xh, xl}, D{dh, dl};
  ff a = ff_mul({mh, ml}, X);
  ff b = ff_mul({ph, pl}, D);
  ff t = ff_add(a, {-b.hi, -b.lo});
  t = ff_add(t, ff_mul_f({rh, rl}, fe));
  X = ff_add(X, t);
  xh = X.hi;
  xl = X.lo;
  dh = t.hi;
  dl = t.lo;
}

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ float4 f4(float v) { return make_float4(v, v, v, v); }
__device__ __forceinline__ float4 fma4(float4 a, float b, float4 c) {
  return make_float4(fmaf(a.x, b, c.x), fmaf(a.y, b, c.y), fmaf(a.z, b, c.z), fmaf(a.w, b, c.w));
}
__device__ __forceinline__ float4 add4(float4 a, float4 b) {
  return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
}
__device__ __forceinline__ float dot4(float4 a, float4 b) {
  return fmaf(a.w, b.w, fmaf(a.z, b.z, fmaf(a.y, b.y, a.x * b.x)));
}
__device__ __forceinline__ float4 ld4(const float* p) { return *reinterpret_cast<const float4*>(p); }
typedef float v4f __attribute__((ext_vector_type(4)));
// streaming 16-byte load with the non-temporal hint (read once per step)
__device__ __forceinline__ float4 ldnt4(const float* p) {
  const v4f v = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st4(float* p, float4 v) { *reinterpret_cast<float4*>(p) = v; }

// Timeout of a per-instance barrier in ticks of the 100 MHz wall clock.
constexpr unsigned long long kBarrierTimeout = 400000000ull;  // 4 s

// Waits until the instance's arrival counter reaches `target` (wrap-safe).
// Returns false if the wait was abandoned (timeout here or elsewhere).
__device__ bool wait_counter(unsigned int* ctr, unsigned int target, int* flags) {
  const unsigned long long t0 = wall_clock64();
  while (true) {
    unsigned int v = __hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    if ((int)(v - target) >= 0) return true;
    if (__hip_atomic_load(&flags[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    if (wall_clock64() - t0 > kBarrierTimeout) {
      __hip_atomic_store(&flags[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

// -------------------------------------------------------- von Karman rows
// Rows [row0, row1) of one instance's Ht.  Row n is an nt x ntp matrix
// (nc = ntp/4 float4 per stored row), read as consecutive blocks of qs
// stored rows.  A block is contiguous, so lane slot v = lane + 64 j
// (j < kSweepLoads) simply reads float4 number v of the block: stored row
// q0 + v / nc, columns 4 (v % nc) .. +3.  Each sweep is one fully coalesced
// 4 KB read per wave.  Slot accumulators are reduced over the qs sub-rows
// through LDS (double buffered by row parity, one wave barrier per row),
// giving V[n, :] on the lanes that own each float4 column group
// (k4 = lane + 64 g); then eta_n and the force update follow.
template <int GM>
__device__ void vk_rows(const float* __restrict__ Hb, int nt, int ntp, int qs, int row0,
                        int row1, const float* Xs, float* red, float4 (&Fa)[GM], int G,
                        int lane) {
  constexpr int J = kSweepLoads;
  const int nc = ntp >> 2;
  const int qsnc = qs * nc;
  int xsub[J];  // sub-row of slot j within a block, -1 if the slot is idle
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int v = lane + kWave * j;
    xsub[j] = v < qsnc ? v / nc : -1;
  }
  const int nfull = nt / qs;
  const int tail = nt - nfull * qs;
  const long long blk_floats = (long long)qs * ntp;
  const long long row_floats = (long long)nt * ntp;
  const float* rowp = Hb + (long long)row0 * row_floats + 4 * lane;
  for (int n = row0; n < row1; ++n, rowp += row_floats) {
    float4 acc[J];
#pragma unroll
    for (int j = 0; j < J; ++j) acc[j] = f4(0.f);
    const float* p = rowp;
    int q0 = 0;
#pragma unroll 2
    for (int b = 0; b < nfull; ++b, p += blk_floats, q0 += qs) {
#pragma unroll
      for (int j = 0; j < J; ++j) {
        if (xsub[j] >= 0) {
          const float4 h = ldnt4(p + 4 * kWave * j);
          acc[j] = fma4(h, Xs[q0 + xsub[j]], acc[j]);
        }
      }
    }
    if (tail) {
#pragma unroll
      for (int j = 0; j < J; ++j) {
        if (xsub[j] >= 0 && xsub[j] < tail) {
          const float4 h = ldnt4(p + 4 * kWave * j);
          acc[j] = fma4(h, Xs[q0 + xsub[j]], acc[j]);
        }
      }
    }
    float* rb = red + (n & 1) * qs * ntp;
#pragma unroll
    for (int j = 0; j < J; ++j)
      if (xsub[j] >= 0) st4(rb + 4 * (lane + kWave * j), acc[j]);
    __syncthreads();
    float eta = 0.f;
    float4 V[GM];
#pragma unroll
    for (int g = 0; g < GM; ++g) {
      V[g] = f4(0.f);
      const int k4 = lane + kWave * g;
      if (g < G && k4 < nc) {
        float4 s = ld4(rb + 4 * k4);
        for (int t = 1; t < qs; ++t) s = add4(s, ld4(rb + t * ntp + 4 * k4));
        V[g] = s;
        eta += dot4(s, ld4(Xs + 4 * k4));
      }
    }
    eta = wave_sum(eta);
#pragma unroll
    for (int g = 0; g < GM; ++g) Fa[g] = fma4(V[g], eta, Fa[g]);
  }
}

// Per-mode state update of the float4 groups owned by this lane.
template <int GM>
__device__ __forceinline__ void update_groups(const StepParams& P, const InstDev& I, int soff,
                                              const float4 (&F)[GM], long long n,
                                              int G, int lane) {
  const int nc = I.ntp >> 2;
  float e = 0.f;
  if (n < I.n_exc) e = P.e_ext[I.e_off + n];
  bool bad = false;
#pragma unroll
  for (int g = 0; g < GM; ++g) {
    const int k4 = lane + kWave * g;
    if (g < G && k4 < nc) {
      const int so = soff + 4 * k4;
      const int mo = I.mode_off + 4 * k4;
      float4 xh = ld4(P.x_hi + so), xl = ld4(P.x_lo + so);
      float4 dh = ld4(P.d_hi + so), dl = ld4(P.d_lo + so);
      const float4 mh = ld4(P.m_hi + mo), ml = ld4(P.m_lo + mo);
      const float4 ph = ld4(P.p_hi + mo), pl = ld4(P.p_lo + mo);
      const float4 rh = ld4(P.r_hi + mo), rl = ld4(P.r_lo + mo);
      const float4 b = ld4(P.b_ext + mo);
      const float4 f = F[g];
      ff_step(xh.x, xl.x, dh.x, dl.x, mh.x, ml.x, ph.x, pl.x, rh.x, rl.x, fmaf(b.x, e, -f.x));
      ff_step(xh.y, xl.y, dh.y, dl.y, mh.y, ml.y, ph.y, pl.y, rh.y, rl.y, fmaf(b.y, e, -f.y));
      ff_step(xh.z, xl.z, dh.z, dl.z, mh.z, ml.z, ph.z, pl.z, rh.z, rl.z, fmaf(b.z, e, -f.z));
      ff_step(xh.w, xl.w, dh.w, dl.w, mh.w, ml.w, ph.w, pl.w, rh.w, rl.w, fmaf(b.w, e, -f.w));
      bad |= !(isfinite(xh.x) && isfinite(xh.y) && isfinite(xh.z) && isfinite(xh.w));
      st4(P.x_hi + so, xh);
      st4(P.x_lo + so, xl);
      st4(P.d_hi + so, dh);
      st4(P.d_lo + so, dl);
    }
  }
  if (__any(bad) && lane == 0) atomicOr(&P.flags[1], 1);
}

// GM: float4 column groups per lane the launch supports (modes <= 256 GM).
template <int GM>
__global__ void __launch_bounds__(kWave) step_kernel(StepParams P) {
  extern __shared__ float4 lds4[];
  float* Xs = reinterpret_cast<float*>(lds4);
  float* red = Xs + kMaxModes;
  const int lane = threadIdx.x;
  const int u0 = P.wg_begin[blockIdx.x];
  const int u1 = P.wg_begin[blockIdx.x + 1];
  const long long base = *P.step_base;

  for (int s = 0; s < P.n_steps; ++s) {
    const long long n = base + s;
    // ---------------- phase 1: output, force, and update of whole units
    for (int u = u0; u < u1; ++u) {
      const UnitDev U = P.unit[u];
      const InstDev I = P.inst[U.inst];
      const int nc = I.ntp >> 2;
      const int G = (nc + kWave - 1) / kWave;
      float ypart = 0.f, spart = 0.f;
#pragma unroll
      for (int g = 0; g < GM; ++g) {
        const int k4 = lane + kWave * g;
        if (g < G && k4 < nc) {
          const float4 xh = ld4(P.x_hi + U.state_off + 4 * k4);
          const float4 c = ld4(P.c_out + I.mode_off + 4 * k4);
          ypart += dot4(c, xh);
          if (I.kind == KIND_VK) {
            st4(Xs + 4 * k4, xh);
          } else if (I.kind == KIND_TENSION) {
            const float4 l = ld4(P.lam + I.mode_off + 4 * k4);
            const float4 lx = make_float4(l.x * xh.x, l.y * xh.y, l.z * xh.z, l.w * xh.w);
            spart += dot4(lx, xh);
          }
        }
      }
      if (U.slab == 0) {
        const float yv = wave_sum(ypart);
        if (lane == 0) P.y[(long long)I.out_row * P.y_stride + s] = yv;
      }
      float4 Fa[GM];
#pragma unroll
      for (int g = 0; g < GM; ++g) Fa[g] = f4(0.f);
      if (I.kind == KIND_VK) {
        __syncthreads();
        vk_rows<GM>(P.H + I.h_off, I.nt, I.ntp, U.qs, U.row0, U.row1, Xs, red, Fa, G, lane);
      } else if (I.kind == KIND_TENSION) {
        const float S = wave_sum(spart) * I.kappa;
#pragma unroll
        for (int g = 0; g < GM; ++g) {
          const int k4 = lane + kWave * g;
          if (g < G && k4 < nc) {
            const float4 xh = ld4(P.x_hi + U.state_off + 4 * k4);
            const float4 l = ld4(P.lam + I.mode_off + 4 * k4);
            Fa[g] = make_float4(l.x * xh.x * S, l.y * xh.y * S, l.z * xh.z * S, l.w * xh.w * S);
          }
        }
      }
      if (I.nslab == 1) {
        update_groups<GM>(P, I, U.state_off, Fa, n, G, lane);
      } else {
        float* dst = P.part + I.part_off + ((long long)(n & 1) * I.nslab + U.slab) * I.ntp;
#pragma unroll
        for (int g = 0; g < GM; ++g) {
          const int k4 = lane + kWave * g;
          if (g < G && k4 < nc) st4(dst + 4 * k4, Fa[g]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (lane == 0)
          __hip_atomic_fetch_add(&P.ctr[U.inst], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
      __syncthreads();
    }
    // ---------------- phase 2: split instances wait, sum partials, update
    for (int u = u0; u < u1; ++u) {
      const UnitDev U = P.unit[u];
      const InstDev I = P.inst[U.inst];
      if (I.nslab == 1) continue;
      const unsigned int target = (unsigned int)I.nslab * (unsigned int)(n + 1);
      if (!wait_counter(&P.ctr[U.inst], target, P.flags)) return;
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      const int nc = I.ntp >> 2;
      const int G = (nc + kWave - 1) / kWave;
      const float* src = P.part + I.part_off + (long long)(n & 1) * I.nslab * I.ntp;
      float4 F[GM];
#pragma unroll
      for (int g = 0; g < GM; ++g) {
        F[g] = f4(0.f);
        const int k4 = lane + kWave * g;
        if (g < G && k4 < nc)
          for (int t = 0; t < I.nslab; ++t) F[g] = add4(F[g], ld4(src + (long long)t * I.ntp + 4 * k4));
      }
      update_groups<GM>(P, I, U.state_off, F, n, G, lane);
    }
  }
}

__global__ void advance_kernel(long long* step_base, int n_steps) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *step_base += n_steps;
}

// Symmetry and finiteness of each instance's Ht: out[2b] = max |H - H^T|,
// out[2b+1] = max |H|, both as float bits (non-negative floats order like
// their bit patterns); a non-finite entry reports +inf in both.
__global__ void check_kernel(const float* H, const InstDev* inst, int* out) {
  const InstDev I = inst[blockIdx.y];
  if (I.kind != KIND_VK) return;
  const long long total = (long long)I.nin * I.nt * I.nt;
  float dmax = 0.f, hmax = 0.f;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(e % I.nt);
    const long long r = e / I.nt;
    const int k = (int)(r % I.nt);
    const long long n = r / I.nt;
    const float* Hn = H + I.h_off + n * (long long)I.nt * I.ntp;
    const float a = Hn[(long long)k * I.ntp + j];
    const float b = Hn[(long long)j * I.ntp + k];
    if (!isfinite(a)) {
      dmax = INFINITY;
      hmax = INFINITY;
    } else {
      dmax = fmaxf(dmax, fabsf(a - b));
      hmax = fmaxf(hmax, fabsf(a));
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    dmax = fmaxf(dmax, __shfl_xor(dmax, o, kWave));
    hmax = fmaxf(hmax, __shfl_xor(hmax, o, kWave));
  }
  if ((threadIdx.x & (kWave - 1)) == 0) {
    atomicMax(&out[2 * blockIdx.y], __float_as_int(dmax));
    atomicMax(&out[2 * blockIdx.y + 1], __float_as_int(hmax));
  }
}

}  // namespace modal

// Launch wrappers used by the host code (same translation unit keeps the
// kernels' symbols local to this file).
namespace modal {
// gm: float4 column groups per lane needed by the widest instance (1, 2 or 4)
hipError_t launch_step(const StepParams& P, int gm, int n_wg, size_t lds_bytes, hipStream_t s) {
  if (gm <= 1)
    hipLaunchKernelGGL(step_kernel<1>, dim3(n_wg), dim3(kWave), lds_bytes, s, P);
  else if (gm <= 2)
    hipLaunchKernelGGL(step_kernel<2>, dim3(n_wg), dim3(kWave), lds_bytes, s, P);
  else
    hipLaunchKernelGGL(step_kernel<4>, dim3(n_wg), dim3(kWave), lds_bytes, s, P);
  return hipGetLastError();
}
hipError_t launch_advance(long long* step_base, int n, hipStream_t s) {
  hipLaunchKernelGGL(advance_kernel, dim3(1), dim3(64), 0, s, step_base, n);
  return hipGetLastError();
}
hipError_t launch_check(const float* H, const InstDev* inst, int batch, int* out, hipStream_t s) {
  hipLaunchKernelGGL(check_kernel, dim3(64, batch), dim3(256), 0, s, H, inst, out);
  return hipGetLastError();
}
hipError_t step_occupancy(int* blocks_per_cu, int gm, size_t lds_bytes) {
  if (gm <= 1)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, step_kernel<1>, kWave, lds_bytes);
  if (gm <= 2)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, step_kernel<2>, kWave, lds_bytes);
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, step_kernel<4>, kWave, lds_bytes);
}
}  // namespace modal
