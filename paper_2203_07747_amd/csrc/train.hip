// Residual-network training on the GPU (Sec. VII: Adam on a mean-squared error).
//
// Forward: the layer-chain kernel with the batch as input, also saving every
// hidden activation h_l.  Backward, layer by layer from the output:
//   dW_l = delta_l^T h_{l-1},  db_l = sum_b delta_l,
//   delta_{l-1} = (delta_l W_l) * act'(a_{l-1})          (act' from the stash)
// with delta_{L+1} = dL/dy = 2 (y - y*) / (6 B).  The products are small GEMMs
// (K = batch for dW) done by one LDS-tiled matrix-core kernel with strided
// operands; the reductions are deterministic (fixed order).
#include <hip/hip_runtime.h>

#include "common.h"
#include "mlp_chain.h"

namespace rtn {

constexpr int TBM = 64, TBN = 64, TBK = 32;

__device__ inline float from_bits(float v) { return v; }
__device__ inline float from_bits(uint16_t v) { return bf16_to_f32(v); }

// C[m][n] (+)= sum_k A(m,k) B(k,n), A(m,k) = A[m*sAm + k*sAk], B(k,n) = B[k*sBk + n*sBn].
// Optional gate: C[m][n] *= act'(row m, feature n) read from a stash [M][ldg] in
// stash order.  One 64x64 output tile per workgroup, 4 waves of 32x32.
template <int P, typename S>
__global__ void __launch_bounds__(256)
gemm_strided(int M, int N, int K, const float* __restrict__ A, long sAm, long sAk, const float* __restrict__ B,
             long sBk, long sBn, float* __restrict__ C, long sCm, int accumulate, const S* __restrict__ gate,
             int ldg) {
  __shared__ float As[TBK][TBM + 1];
  __shared__ float Bs[TBK][TBN + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * TBM, n0 = blockIdx.x * TBN;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f32x16 acc = {};
  for (int k0 = 0; k0 < K; k0 += TBK) {
    for (int e = tid; e < TBK * TBM; e += 256) {
      // consecutive threads walk the operand's contiguous dimension
      int kk, mm;
      if (sAk == 1) { kk = e % TBK; mm = e / TBK; } else { mm = e % TBM; kk = e / TBM; }
      const int m = m0 + mm, k = k0 + kk;
      As[kk][mm] = (m < M && k < K) ? A[(long)m * sAm + (long)k * sAk] : 0.f;
    }
    for (int e = tid; e < TBK * TBN; e += 256) {
      int kk, nn;
      if (sBn == 1) { nn = e % TBN; kk = e / TBN; } else { kk = e % TBK; nn = e / TBK; }
      const int n = n0 + nn, k = k0 + kk;
      Bs[kk][nn] = (n < N && k < K) ? B[(long)k * sBk + (long)n * sBn] : 0.f;
    }
    __syncthreads();
    if constexpr (P == P_BF16) {
#pragma unroll
      for (int ks = 0; ks < TBK; ks += 16) {
        bf16x8 a, b;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          a[j] = (__bf16)As[ks + (lane >> 5) * 8 + j][wm + (lane & 31)];
          b[j] = (__bf16)Bs[ks + (lane >> 5) * 8 + j][wn + (lane & 31)];
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int ks = 0; ks < TBK; ks += 2) {
        const float a = As[ks + (lane >> 5)][wm + (lane & 31)];
        const float b = Bs[ks + (lane >> 5)][wn + (lane & 31)];
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
      }
    }
    __syncthreads();
  }
  const int n = n0 + wn + (lane & 31);
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int m = m0 + wm + (i >> 2) * 8 + (lane >> 5) * 4 + (i & 3);
    if (m < M && n < N) {
      float v = acc[i];
      if (gate) v *= from_bits(gate[(long)m * ldg + stash_pos(n)]);
      float* c = C + (long)m * sCm + n;
      *c = accumulate ? *c + v : v;
    }
  }
}

// loss = mean over (batch, 6) of (y - t)^2 and dL/dy = 2 (y - t) / (6 B); one block,
// fixed summation order.
__global__ void __launch_bounds__(1024) mse_kernel(int nel, const float* __restrict__ y, const float* __restrict__ t,
                                                   float* __restrict__ dy, float* __restrict__ loss) {
  __shared__ float red[1024];
  float s = 0.f;
  const float sc = 2.f / (float)nel;
  for (int i = threadIdx.x; i < nel; i += 1024) {
    const float e = y[i] - t[i];
    dy[i] = sc * e;
    s += e * e;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) *loss = red[0] / (float)nel;
}

// db[o] (+)= sum_b delta[b][o], column sums in fixed order (one thread per column).
__global__ void colsum_kernel(int rows, int cols, const float* __restrict__ d, float* __restrict__ db) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= cols) return;
  float s = 0.f;
  for (int b = 0; b < rows; ++b) s += d[(long)b * cols + o];
  db[o] += s;
}

// Adam with bias correction (bc1 = 1 - beta1^t, bc2 = 1 - beta2^t), no weight decay.
__global__ void adam_kernel(long n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, float lr, float b1, float b2, float eps, float bc1, float bc2) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  }
}

hipError_t launch_gemm_strided(int prec, int M, int N, int K, const float* A, long sAm, long sAk, const float* B,
                               long sBk, long sBn, float* C, long sCm, int accumulate, const void* gate,
                               int gate_is_f32, int ldg, hipStream_t st) {
  dim3 grid((N + TBN - 1) / TBN, (M + TBM - 1) / TBM);
  if (grid.x == 0 || grid.y == 0) return hipSuccess;
  if (prec == P_FP32) {
    if (gate_is_f32 || !gate)
      gemm_strided<P_FP32, float><<<grid, 256, 0, st>>>(M, N, K, A, sAm, sAk, B, sBk, sBn, C, sCm, accumulate,
                                                        (const float*)gate, ldg);
    else
      gemm_strided<P_FP32, uint16_t><<<grid, 256, 0, st>>>(M, N, K, A, sAm, sAk, B, sBk, sBn, C, sCm, accumulate,
                                                           (const uint16_t*)gate, ldg);
  } else {
    if (gate_is_f32 || !gate)
      gemm_strided<P_BF16, float><<<grid, 256, 0, st>>>(M, N, K, A, sAm, sAk, B, sBk, sBn, C, sCm, accumulate,
                                                        (const float*)gate, ldg);
    else
      gemm_strided<P_BF16, uint16_t><<<grid, 256, 0, st>>>(M, N, K, A, sAm, sAk, B, sBk, sBn, C, sCm, accumulate,
                                                           (const uint16_t*)gate, ldg);
  }
  return hipGetLastError();
}

hipError_t launch_mse(int nel, const float* y, const float* t, float* dy, float* loss, hipStream_t st) {
  mse_kernel<<<1, 1024, 0, st>>>(nel, y, t, dy, loss);
  return hipGetLastError();
}

hipError_t launch_colsum(int rows, int cols, const float* d, float* db, hipStream_t st) {
  colsum_kernel<<<(cols + 255) / 256, 256, 0, st>>>(rows, cols, d, db);
  return hipGetLastError();
}

hipError_t launch_adam(long n, float* p, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                       float bc1, float bc2, hipStream_t st) {
  int blocks = (int)((n + 255) / 256);
  if (blocks > 2048) blocks = 2048;
  adam_kernel<<<blocks, 256, 0, st>>>(n, p, g, m, v, lr, b1, b2, eps, bc1, bc2);
  return hipGetLastError();
}

}  // namespace rtn
