// Device helpers shared by the forward and reverse kernels (gfx950).
#pragma once
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
__device__ __forceinline__ ff two_prod(float a, float b) {
  const float p = a * b;
  return {p, fmaf(a, b, -p)};
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
// Data-parallel move between lanes of a 16-lane row (DPP control word C).
template <int C>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), C, 0xF, 0xF, true));
}
__device__ __forceinline__ float lane_value(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
// Sum over the 64 lanes of a wave (all lanes active), the same on every lane.
// Within each 16-lane row four DPP exchanges (partner lane ^1, ^2, the mirror
// within 8 lanes, the mirror within 16) leave the row's sum on all its lanes,
// identical bits on each since every pairing is symmetric; the four row sums
// are then read out and added.  No LDS crossbar round trips, unlike a
// shuffle-based butterfly.
__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_mov<0x141>(v);  // row_half_mirror
  v += dpp_mov<0x140>(v);  // row_mirror
  return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
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
// Raw buffer resource over `bytes` bytes at p (stride 0).  Loads at byte
// offsets >= bytes are out of range and return zeros without a memory
// access; the last word is the standard gfx9 raw-buffer format word.  The
// callers' values are wave-uniform; readfirstlane states it so that the
// resource lives in scalar registers.
typedef int v4i __attribute__((ext_vector_type(4)));
__device__ __forceinline__ v4i buf_rsrc(const float* p, int bytes) {
  const unsigned long long a = reinterpret_cast<unsigned long long>(p);
  v4i r;
  r.x = __builtin_amdgcn_readfirstlane((int)(unsigned)a);
  r.y = __builtin_amdgcn_readfirstlane((int)((a >> 32) & 0xffffu));
  r.z = __builtin_amdgcn_readfirstlane(bytes);
  r.w = 0x00020000;
  return r;
}
// The LLVM raw buffer load intrinsic, declared directly.
__device__ v4f llvm_raw_buffer_load_v4f32(v4i rsrc, int voffset, int soffset, int aux)
    __asm("llvm.amdgcn.raw.buffer.load.v4f32");
// The partial forces that the slabs of a split instance exchange in global
// memory are written and read with the sc1 cache policy, which gfx950 keeps
// coherent across the XCDs' separate L2 caches: the policy of an agent-scope
// relaxed atomic access, here on 16-byte buffer accesses instead of four
// separate 4-byte atomics.  Publishing a partial then needs only a wait for
// its stores to complete before the arrival word (an agent-scope atomic) is
// stored, and reading one needs no L2 invalidation: an agent-scope release or
// acquire fence would write back or invalidate the whole L2 of the XCD on
// every step.  The resource spans one instance's exchange region (offsets
// past it read zeros and drop stores); byte offsets per lane.
constexpr int kCoherentPolicy = 16;  // sc1 bit of the buffer instructions' cache-policy operand
__device__ void llvm_raw_buffer_store_v4f32(v4f v, v4i rsrc, int voffset, int soffset, int aux)
    __asm("llvm.amdgcn.raw.buffer.store.v4f32");
__device__ __forceinline__ void st4_coherent(v4i r, int byte_off, float4 v) {
  v4f w;
  w.x = v.x;
  w.y = v.y;
  w.z = v.z;
  w.w = v.w;
  llvm_raw_buffer_store_v4f32(w, r, byte_off, 0, kCoherentPolicy);
}
__device__ __forceinline__ float4 ld4_coherent(v4i r, int byte_off) {
  const v4f v = llvm_raw_buffer_load_v4f32(r, byte_off, 0, kCoherentPolicy);
  return make_float4(v.x, v.y, v.z, v.w);
}
// After a wave's partial-force stores (st4_coherent): waits until the memory
// system has acknowledged them, so that an arrival word stored afterwards
// cannot be seen before them.  A workgroup-scope release fence emits no such
// wait when a workgroup's waves share one CU, and an agent-scope one would
// also write back the XCD's whole L2; the wait on the vector-memory counter
// alone is what the exchange needs.  It is also a compiler barrier.
__device__ __forceinline__ void publish_fence() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
// Before reading partials (ld4_coherent) once the words have been seen:
// keeps the compiler from moving the reads above the words' loads (the
// hardware issues them after the polling loop, whose exit depends on the
// words' values).
__device__ __forceinline__ void consume_fence() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup"); }

// sum over t = t0, t0 + dt, ... (t < n) of the float4 at byte offset
// off + t * stride of resource r (partial forces of other workgroups, read
// coherently), eight reads issued before the first add (sixteen measured
// slower); a fixed order, so every caller gets the same bits
__device__ __forceinline__ float4 sum_slabs4_coherent(v4i r, int off, int t0, int dt, int n, int stride) {
  float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
  int t = t0;
  for (; t + 7 * dt < n; t += 8 * dt) {
    float4 a[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = ld4_coherent(r, off + (t + i * dt) * stride);
#pragma unroll
    for (int i = 0; i < 8; ++i) s = add4(s, a[i]);
  }
  for (; t < n; t += dt) s = add4(s, ld4_coherent(r, off + t * stride));
  return s;
}

// sum over t < n of the float4 at p + t * stride (LDS), with four partial
// sums so that four reads are in flight before the first add waits
__device__ __forceinline__ float4 sum_strided4(const float* p, int n, int stride) {
  float4 s0 = ld4(p), s1 = make_float4(0.f, 0.f, 0.f, 0.f), s2 = s1, s3 = s1;
  int t = 1;
  for (; t + 3 < n; t += 4) {
    s1 = add4(s1, ld4(p + t * stride));
    s2 = add4(s2, ld4(p + (t + 1) * stride));
    s3 = add4(s3, ld4(p + (t + 2) * stride));
    s0 = add4(s0, ld4(p + (t + 3) * stride));
  }
  for (; t < n; ++t) s1 = add4(s1, ld4(p + t * stride));
  return add4(add4(s0, s1), add4(s2, s3));
}

// Sum over t = t0, t0 + dt, ... (t < n) of the float4 at p + t * stride
// (global memory written by other workgroups), with eight loads issued
// before the first add so that their latencies overlap; a fixed order, so
// every caller gets the same bits.
__device__ __forceinline__ float4 sum_slabs4(const float* p, int t0, int dt, int n, long long stride) {
  float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
  int t = t0;
  for (; t + 7 * dt < n; t += 8 * dt) {
    float4 a[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = *reinterpret_cast<const float4*>(p + (long long)(t + i * dt) * stride);
#pragma unroll
    for (int i = 0; i < 8; ++i) s = add4(s, a[i]);
  }
  for (; t < n; t += dt) s = add4(s, *reinterpret_cast<const float4*>(p + (long long)t * stride));
  return s;
}

// sum of n consecutive floats (LDS), four partial sums
__device__ __forceinline__ float sum_run(const float* p, int n) {
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
  int c = 0;
  for (; c + 3 < n; c += 4) {
    s0 += p[c];
    s1 += p[c + 1];
    s2 += p[c + 2];
    s3 += p[c + 3];
  }
  for (; c < n; ++c) s0 += p[c];
  return (s0 + s1) + (s2 + s3);
}
// streaming 16-byte load with the non-temporal hint (read once per step)
__device__ __forceinline__ float4 ldnt4(const float* p) {
  const v4f v = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st4(float* p, float4 v) { *reinterpret_cast<float4*>(p) = v; }

// 16-byte load through a buffer resource with cache policy POL: kStream,
// the non-temporal hint, for tensors streamed from HBM once per step (the
// batch), or kKeep, the default policy, for a latency-bound instance whose
// tensor stays in the caches from step to step (measured on a lone 200/200
// plate: forward 14.0 -> 12.1 us and reverse 18.2 -> 16.8 us per step; the
// 256-plate batch 233 -> 247 ms per launch with kKeep).
constexpr int kStream = 2, kKeep = 0;
template <int POL = kStream>
__device__ __forceinline__ float4 buf_ld4(v4i r, int voff) {
  const v4f v = llvm_raw_buffer_load_v4f32(r, voff, 0, POL);
  return make_float4(v.x, v.y, v.z, v.w);
}

// Orders this wave's LDS writes before its later LDS reads by other lanes.
// Workgroups are single waves, so no s_barrier is needed, and vector-memory
// loads in flight are not waited for.
__device__ __forceinline__ void wave_lds_sync() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_wave_barrier();
}

// Workgroup barrier for LDS traffic only: this wave's LDS operations are
// complete and every wave has arrived.  Unlike __syncthreads it does not
// wait for outstanding global loads, so prefetches stay in flight across it.
__device__ __forceinline__ void block_lds_sync() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}


// Waits until every slab's arrival word f[t] (t < nslab) has reached
// `target` (wrap-safe); called by a whole wave, whose lanes poll the words
// together, so that no slab's arrival waits on another's (each slab stores
// its own word; nothing is read-modify-written).  Returns false if the wait
// was abandoned (after `timeout` ticks here, or elsewhere).
__device__ inline bool wait_slabs(const unsigned int* f, int nslab, unsigned int target, int* flags,
                                  unsigned long long timeout) {
  const int lane = threadIdx.x & (kWave - 1);
  const unsigned long long t0 = wall_clock64();
  while (true) {
    bool ok = true;
    for (int t = lane; t < nslab; t += kWave) {
      const unsigned int v = __hip_atomic_load(f + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      ok = ok && (int)(v - target) >= 0;
    }
    if (__all(ok)) return true;
    if (__hip_atomic_load(&flags[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    if (wall_clock64() - t0 > timeout) {
      __hip_atomic_store(&flags[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

}  // namespace modal
