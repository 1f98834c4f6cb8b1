// Kernels of the proposal network (a multilayer perceptron): a BF16 MFMA
// GEMM with FP32 accumulation and fused epilogues, the bias-gradient column
// sum, and the Adam update on FP32 master weights (gfx950).
//
// GEMM: C[m, n] = sum_k A(m, k) B(k, n) with A(m, k) = A[m sam + k sak] and
// B(k, n) = B[k sbk + n sbn] (FP32 in memory, rounded to BF16 when staged in
// LDS), so one kernel serves Y = X W^T, dX = dY W and dW = dY^T X.
// A 256-thread workgroup computes a 64 x 64 tile; each of its four waves owns
// a 32 x 32 quadrant accumulated by v_mfma_f32_32x32x8 bf16 over K tiles of
// 32.  Operand layout of that instruction: lane l supplies A[l % 32][4 (l/32)
// + i] and B[4 (l/32) + i][l % 32], i < 4; it receives D[8 (r/4) + 4 (l/32)
// + r % 4][l % 32] in accumulator r < 16.
#include <hip/hip_runtime.h>

namespace modal {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));

enum : int { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_RELU = 2, EPI_MASK = 3 };

// round-to-nearest-even FP32 -> BF16 bits
__device__ __forceinline__ short to_bf16(float f) {
  unsigned int u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (short)(u >> 16);  // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

constexpr int TM = 64, TN = 64, TK = 32;

__global__ void __launch_bounds__(256) gemm_bf16(const float* __restrict__ A, long long sam,
                                                 long long sak, const float* __restrict__ B,
                                                 long long sbk, long long sbn, float* __restrict__ C,
                                                 long long scm, int M, int N, int K, int epi,
                                                 const float* __restrict__ bias,
                                                 const float* __restrict__ mask) {
  __shared__ short As[TM][TK + 4];  // [m][k]
  __shared__ short Bs[TN][TK + 4];  // [n][k]
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int qm = wave >> 1, qn = wave & 1;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  v16f acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.f;
  for (int k0 = 0; k0 < K; k0 += TK) {
    // stage A and B tiles (2048 elements each, 8 per thread), zero-padded
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int idx = tid + 256 * e;
      const int i = idx / TK, k = idx % TK;
      const int gm = m0 + i, gk = k0 + k;
      As[i][k] = to_bf16(gm < M && gk < K ? A[gm * sam + gk * sak] : 0.f);
      const int gn = n0 + i;
      Bs[i][k] = to_bf16(gn < N && gk < K ? B[gk * sbk + gn * sbn] : 0.f);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; kk += 8) {
      v4s a, b;
      const int kb = kk + 4 * (lane >> 5);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a[i] = As[qm * 32 + (lane & 31)][kb + i];
        b[i] = Bs[qn * 32 + (lane & 31)][kb + i];
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  const int col = n0 + qn * 32 + (lane & 31);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = m0 + qm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    if (row < M && col < N) {
      float v = acc[r];
      if (epi == EPI_BIAS || epi == EPI_BIAS_RELU) v += bias[col];
      if (epi == EPI_BIAS_RELU) v = fmaxf(v, 0.f);
      if (epi == EPI_MASK) v = mask[row * scm + col] > 0.f ? v : 0.f;
      C[row * scm + col] = v;
    }
  }
}

// db[n] = sum_m G[m, n]  (G row-major [M, N])
__global__ void colsum(const float* __restrict__ G, int M, int N, float* __restrict__ db) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int m = 0; m < M; ++m) s += G[(long long)m * N + n];
  db[n] = s;
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

hipError_t launch_gemm(const float* A, long long sam, long long sak, const float* B, long long sbk,
                       long long sbn, float* C, long long scm, int M, int N, int K, int epi,
                       const float* bias, const float* mask, hipStream_t s) {
  dim3 grid((N + TN - 1) / TN, (M + TM - 1) / TM);
  hipLaunchKernelGGL(gemm_bf16, grid, dim3(256), 0, s, A, sam, sak, B, sbk, sbn, C, scm, M, N, K,
                     epi, bias, mask);
  return hipGetLastError();
}

hipError_t launch_colsum(const float* G, int M, int N, float* db, hipStream_t s) {
  hipLaunchKernelGGL(colsum, dim3((N + 255) / 256), dim3(256), 0, s, G, M, N, db);
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
