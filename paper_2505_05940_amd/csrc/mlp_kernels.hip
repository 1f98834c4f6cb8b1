// Kernels of the proposal network (a multilayer perceptron): a BF16 MFMA
// GEMM with FP32 accumulation and fused epilogues, the bias-gradient column
// sum, and the Adam update on FP32 master weights (gfx950).
//
// GEMM: C[m, n] = sum_k A(m, k) B(k, n), FP32 in memory and rounded to BF16
// when staged in LDS.  Each operand is read along whichever of its two
// indices is contiguous in memory, with 16-byte loads: A(m, k) = A[m lda + k]
// (k contiguous) or A[k lda + m] (m contiguous), B(k, n) = B[n ldb + k] or
// B[k ldb + n]; so one kernel serves Y = X W^T, dX = dY W and dW = dY^T X.
// A 128-thread workgroup computes a 32 x 64 tile of C (two waves, one 32 x 32
// quadrant each) over K tiles of 64 with gfx950's v_mfma_f32_32x32x16_bf16;
// the next K tile's global loads are issued before the current tile's MFMAs
// and written to the second of two LDS buffers afterwards.  Operand layout of
// the instruction: lane l supplies A[l % 32][8 (l/32) + i] and
// B[8 (l/32) + i][l % 32], i < 8 (the same k for both); it receives
// D[8 (r/4) + 4 (l/32) + r % 4][l % 32] in accumulator r < 16.  The LDS
// tiles are [m][k] and [n][k] with k contiguous (rows padded by 8), so each
// fragment is one 16-byte LDS read.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.h"

namespace modal {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

enum : int { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_RELU = 2, EPI_MASK = 3 };

// round-to-nearest-even FP32 -> BF16 bits
__device__ __forceinline__ unsigned short to_bf16(float f) {
  unsigned int u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);  // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

constexpr int TM = 32, TN = 64, TK = 64, TKP = TK + 8;
constexpr int kGemmThreads = 128;

// Four consecutive elements of a row of a row-major matrix (ld elements per
// row) starting at column c, zero outside [0, rows) x [0, cols); a 16-byte
// load when the whole group is inside and aligned.
__device__ __forceinline__ float4 ld_group(const float* __restrict__ X, long long ld, int r, int c, int rows,
                                           int cols, bool vec) {
  if (r >= rows) return make_float4(0.f, 0.f, 0.f, 0.f);
  const float* p = X + (long long)r * ld + c;
  if (vec && c + 3 < cols) return *reinterpret_cast<const float4*>(p);
  float v[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = c + i < cols ? p[i] : 0.f;
  return make_float4(v[0], v[1], v[2], v[3]);
}

// 16-byte load through a buffer resource (cached); an offset past the
// resource's size reads zeros without touching memory.
__device__ __forceinline__ float4 ld4_rsrc(v4i r, int voff) {
  const v4f v = llvm_raw_buffer_load_v4f32(r, voff, 0, 0);
  return make_float4(v.x, v.y, v.z, v.w);
}
constexpr int kOutside = 0x7ffffff0;  // a byte offset past every operand resource

// Stages one operand tile of R rows (m or n) by TK k into registers: R * TK
// / 4 float4 groups over the 128 threads.  KC: the operand's k index is
// contiguous in memory (groups run along k), else its m / n index is.
// VEC: the contiguous extent and the row stride are multiples of 4 and the
// base 16-byte aligned, so every group is whole and is one 16-byte buffer
// load, with no branch (groups outside the matrix read zeros); otherwise
// element by element.
template <int R, bool KC, bool VEC>
struct Stage {
  static constexpr int G = R * TK / 4 / kGemmThreads;  // groups per thread
  float4 v[G];
  __device__ __forceinline__ void load(const float* __restrict__ X, v4i rs, long long ld, int r0, int k0,
                                       int rows, int K, int tid) {
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const int q = tid + kGemmThreads * j;
      // group q: along k, row q / (TK/4) and k = 4 (q % (TK/4)); along the
      // rows, k row q / (R/4) and rows 4 (q % (R/4)) .. +3
      const int a = KC ? r0 + q / (TK / 4) : k0 + q / (R / 4);      // memory row
      const int c = KC ? k0 + 4 * (q % (TK / 4)) : r0 + 4 * (q % (R / 4));  // first column
      const int na = KC ? rows : K, nc = KC ? K : rows;
      if (VEC) {
        const bool in = a < na && c < nc;
        v[j] = ld4_rsrc(rs, in ? (int)(((long long)a * ld + c) * 4) : kOutside);
      } else {
        v[j] = ld_group(X, ld, a, c, na, nc, false);
      }
    }
  }
  __device__ __forceinline__ void store(unsigned short (*T)[TKP], int tid) const {
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const int q = tid + kGemmThreads * j;
      const unsigned short b0 = to_bf16(v[j].x), b1 = to_bf16(v[j].y), b2 = to_bf16(v[j].z),
                           b3 = to_bf16(v[j].w);
      if (KC) {
        const int r = q / (TK / 4), k = 4 * (q % (TK / 4));
        uint2 w;
        w.x = (unsigned int)b0 | ((unsigned int)b1 << 16);
        w.y = (unsigned int)b2 | ((unsigned int)b3 << 16);
        *reinterpret_cast<uint2*>(&T[r][k]) = w;
      } else {
        const int k = q / (R / 4), r = 4 * (q % (R / 4));
        T[r][k] = b0;
        T[r + 1][k] = b1;
        T[r + 2][k] = b2;
        T[r + 3][k] = b3;
      }
    }
  }
};

// blockIdx.z selects a slice [k0, k0 + kc) of K (split K); with several
// slices (gridDim.z > 1) each writes its raw partial tile to
// part[z][M][N] and gemm_reduce adds the slices and applies the epilogue.
template <bool AKC, bool BKC, bool VEC>
__global__ void __launch_bounds__(kGemmThreads) gemm_bf16(const float* __restrict__ A, long long lda,
                                                          const float* __restrict__ B, long long ldb,
                                                          float* __restrict__ C, long long ldc, int M, int N,
                                                          int K, int kc, int epi, const float* __restrict__ bias,
                                                          const float* __restrict__ mask, float* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) unsigned short As[2][TM][TKP];
  __shared__ __attribute__((aligned(16))) unsigned short Bs[2][TN][TKP];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  // operand resources sized to the matrices (the host keeps them below 2 GB)
  const v4i ra = buf_rsrc(A, VEC ? (int)(4 * (AKC ? (long long)M : (long long)K) * lda) : 0);
  const v4i rb = buf_rsrc(B, VEC ? (int)(4 * (BKC ? (long long)N : (long long)K) * ldb) : 0);
  Stage<TM, AKC, VEC> sa;
  Stage<TN, BKC, VEC> sb;
  v16f acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.f;
  // this slice's K range, in whole tiles: [kb0, kb0 + kc) clipped to K
  const int kb0 = blockIdx.z * kc;
  const int kend = min(K, kb0 + kc);
  const int nk = (kend - kb0 + TK - 1) / TK;
  // operands are read as if K ended at kend (zeros past it)
  sa.load(A, ra, lda, m0, kb0, M, kend, tid);
  sb.load(B, rb, ldb, n0, kb0, N, kend, tid);
  sa.store(As[0], tid);
  sb.store(Bs[0], tid);
  __syncthreads();
  for (int t = 0; t < nk; ++t) {
    const int cur = t & 1;
    if (t + 1 < nk) {  // next tile's loads in flight during this tile's MFMAs
      sa.load(A, ra, lda, m0, kb0 + (t + 1) * TK, M, kend, tid);
      sb.load(B, rb, ldb, n0, kb0 + (t + 1) * TK, N, kend, tid);
    }
#pragma unroll
    for (int kk = 0; kk < TK; kk += 16) {
      const int kb = kk + 8 * (lane >> 5);
      const v8bf a = *reinterpret_cast<const v8bf*>(&As[cur][lane & 31][kb]);
      const v8bf b = *reinterpret_cast<const v8bf*>(&Bs[cur][32 * wave + (lane & 31)][kb]);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    if (t + 1 < nk) {
      sa.store(As[cur ^ 1], tid);
      sb.store(Bs[cur ^ 1], tid);
    }
    __syncthreads();
  }
  const int col = n0 + 32 * wave + (lane & 31);
  if (gridDim.z > 1) {
    float* P = part + (long long)blockIdx.z * M * N;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = m0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      if (row < M && col < N) P[(long long)row * N + col] = acc[r];
    }
    return;
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = m0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    if (row < M && col < N) {
      float v = acc[r];
      if (epi == EPI_BIAS || epi == EPI_BIAS_RELU) v += bias[col];
      if (epi == EPI_BIAS_RELU) v = fmaxf(v, 0.f);
      if (epi == EPI_MASK) v = mask[row * ldc + col] > 0.f ? v : 0.f;
      C[row * ldc + col] = v;
    }
  }
}

// C[m, n] = epilogue(sum over the S slices of part[z][m][n]), slices added in
// order (deterministic)
__global__ void gemm_reduce(const float* __restrict__ part, int S, float* __restrict__ C, long long ldc, int M,
                            int N, int epi, const float* __restrict__ bias, const float* __restrict__ mask) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)M * N) return;
  const int row = (int)(i / N), col = (int)(i % N);
  float v = 0.f;
  for (int z = 0; z < S; ++z) v += part[(long long)z * M * N + i];
  if (epi == EPI_BIAS || epi == EPI_BIAS_RELU) v += bias[col];
  if (epi == EPI_BIAS_RELU) v = fmaxf(v, 0.f);
  if (epi == EPI_MASK) v = mask[row * ldc + col] > 0.f ? v : 0.f;
  C[row * ldc + col] = v;
}

// db[n] = sum_m G[m, n]  (G row-major [M, N]) in one pass: a workgroup of
// 1024 threads owns 64 columns, its 16 row phases each sum every 16th row
// (loads unrolled so that several are in flight), and the phases are added
// through LDS in a fixed order (deterministic).
__global__ void __launch_bounds__(1024) colsum(const float* __restrict__ G, int M, int N, float* __restrict__ db) {
  __shared__ float red[16][64];
  const int c = threadIdx.x & 63, ph = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + c;
  float s = 0.f;
  if (n < N) {
#pragma unroll 8
    for (int m = ph; m < M; m += 16) s += G[(long long)m * N + n];
  }
  red[ph][c] = s;
  __syncthreads();
  if (ph == 0 && n < N) {
    float t = 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) t += red[i][c];
    db[n] = t;
  }
}

// dst[b][:] = src[idx[b]][:] (rows of d floats)
__global__ void gather_rows(const float* __restrict__ src, const long long* __restrict__ idx, int d,
                            float* __restrict__ dst) {
  const long long r = idx[blockIdx.x];
  const float* s = src + r * d;
  float* o = dst + (long long)blockIdx.x * d;
  if ((d & 3) == 0 && ((reinterpret_cast<unsigned long long>(src) & 15) == 0)) {
    for (int i = threadIdx.x; i < d / 4; i += blockDim.x)
      reinterpret_cast<float4*>(o)[i] = reinterpret_cast<const float4*>(s)[i];
  } else {
    for (int i = threadIdx.x; i < d; i += blockDim.x) o[i] = s[i];
  }
}

// Mean squared error of y [B][d] against z[idx[b]][:] and its gradient:
// g = 2 (y - z) / (B d); *acc += sum (y - z)^2 / (B d).  One workgroup, a
// fixed summation order (deterministic).
__global__ void __launch_bounds__(1024) mse_grad(const float* __restrict__ y, const float* __restrict__ z,
                                                const long long* __restrict__ idx, int B, int d,
                                                float* __restrict__ g, float* __restrict__ acc) {
  __shared__ float red[1024];
  const float inv = 1.f / ((float)B * (float)d);
  float s = 0.f;
#pragma unroll 4
  for (int i = threadIdx.x; i < B * d; i += 1024) {
    const int b = i / d, j = i - b * d;
    const float e = y[i] - z[idx[b] * d + j];
    g[i] = 2.f * e * inv;
    s = fmaf(e, e, s);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0 && acc) *acc += red[0] * inv;
}

hipError_t launch_gather_rows(const float* src, const long long* idx, int B, int d, float* dst, hipStream_t s) {
  hipLaunchKernelGGL(gather_rows, dim3(B), dim3(256), 0, s, src, idx, d, dst);
  return hipGetLastError();
}
hipError_t launch_mse_grad(const float* y, const float* z, const long long* idx, int B, int d, float* g,
                           float* acc, hipStream_t s) {
  hipLaunchKernelGGL(mse_grad, dim3(1), dim3(1024), 0, s, y, z, idx, B, d, g, acc);
  return hipGetLastError();
}

// Adam (Kingma & Ba): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
// p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
__global__ void adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                     float* __restrict__ v, long long n, float lr, float b1, float b2, float eps,
                     float c1, float c2) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// Split K so that a launch has at least about 1024 workgroups (K slices of
// whole 64-wide tiles, at most kMaxSplit); part: scratch of kMaxSplit * M * N
// floats for the slices' partial tiles.
constexpr int kMaxSplit = 8;
hipError_t launch_gemm(const float* A, long long lda, int a_kc, const float* B, long long ldb, int b_kc, float* C,
                       long long ldc, int M, int N, int K, int epi, const float* bias, const float* mask,
                       float* part, hipStream_t s) {
  const int tiles = ((N + TN - 1) / TN) * ((M + TM - 1) / TM);
  const int ktiles = (K + TK - 1) / TK;
  int S = std::max(1, std::min({kMaxSplit, ktiles, (1024 + tiles - 1) / tiles}));
  if (!part) S = 1;
  const int kc = ((ktiles + S - 1) / S) * TK;
  S = (K + kc - 1) / kc;
  dim3 grid((N + TN - 1) / TN, (M + TM - 1) / TM, S);
  // whole 16-byte groups along each operand's contiguous index, aligned,
  // and operands addressable by 32-bit byte offsets
  auto aligned = [](const float* p) { return (reinterpret_cast<unsigned long long>(p) & 15) == 0; };
  const long long a_bytes = 4 * (a_kc ? (long long)M : (long long)K) * lda;
  const long long b_bytes = 4 * (b_kc ? (long long)N : (long long)K) * ldb;
  const bool vec = (lda & 3) == 0 && (ldb & 3) == 0 && aligned(A) && aligned(B) &&
                   ((a_kc ? K : M) & 3) == 0 && ((b_kc ? K : N) & 3) == 0 && a_bytes < kOutside &&
                   b_bytes < kOutside;
#define GL(AK, BK, V)                                                                                      \
  hipLaunchKernelGGL((gemm_bf16<AK, BK, V>), grid, dim3(kGemmThreads), 0, s, A, lda, B, ldb, C, ldc, M, N, K, \
                     kc, epi, bias, mask, part)
  if (vec) {
    if (a_kc && b_kc) GL(true, true, true); else if (a_kc) GL(true, false, true);
    else if (b_kc) GL(false, true, true); else GL(false, false, true);
  } else {
    if (a_kc && b_kc) GL(true, true, false); else if (a_kc) GL(true, false, false);
    else if (b_kc) GL(false, true, false); else GL(false, false, false);
  }
#undef GL
  if (S > 1) {
    const long long n = (long long)M * N;
    hipLaunchKernelGGL(gemm_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, part, S, C, ldc, M, N, epi,
                       bias, mask);
  }
  return hipGetLastError();
}

hipError_t launch_colsum(const float* G, int M, int N, float* db, hipStream_t s) {
  hipLaunchKernelGGL(colsum, dim3((N + 63) / 64), dim3(1024), 0, s, G, M, N, db);
  return hipGetLastError();
}

// Adam with the learning rate and the bias corrections read from device
// memory: lr = sched[0], c1 = sched[2 k + 1], c2 = sched[2 k + 2] for the
// k-th step of a recorded epoch, so that the recorded graph can be replayed
// with a new schedule (the host writes the table before each replay).
__global__ void adam_dev(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                         float* __restrict__ v, long long n, const float* __restrict__ sched, int k, float b1,
                         float b2, float eps) {
  const float lr = sched[0], c1 = sched[2 * k + 1], c2 = sched[2 * k + 2];
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}
hipError_t launch_adam_dev(float* p, const float* g, float* m, float* v, long long n, const float* sched, int k,
                           float b1, float b2, float eps, hipStream_t s) {
  const int blocks = (int)std::min<long long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(adam_dev, dim3(blocks), dim3(256), 0, s, p, g, m, v, n, sched, k, b1, b2, eps);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, long long n, float lr, float b1,
                       float b2, float eps, int t, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  const int blocks = (int)std::min<long long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(adam, dim3(blocks), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace modal
