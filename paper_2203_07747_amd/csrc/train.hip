// Residual-network training on the GPU (Sec. VII: Adam on a mean-squared error).
//
// Forward: the layer-chain kernel with the batch as input, also saving every
// hidden activation h_l.  Backward, layer by layer from the output:
//   dW_l = delta_l^T h_{l-1},  db_l = sum_b delta_l,
//   delta_{l-1} = (delta_l W_l) * act'(a_{l-1})          (act' from the stash)
// with delta_{L+1} = dL/dy = 2 (y - y*) / (6 B).  The products are GEMMs with
// strided operands on one LDS-tiled matrix-core kernel; dW and db come from one
// product (db is the product with an extra all-ones column of h), split over
// the batch into K ranges whose partial tiles are summed in fixed order, so the
// result is deterministic.
#include <hip/hip_runtime.h>

#include "common.h"
#include "mlp_chain.h"

namespace rtn {

constexpr int TBM = 64, TBN = 64;
// K per LDS tile: 128 for bf16 (eight MFMAs per wave between barriers), 32 for
// fp32 (its fp32 tiles would not fit the static LDS at 128)
template <int P> constexpr int gemm_tbk() { return P == P_BF16 ? 128 : 32; }
__device__ inline float from_bits(float v) { return v; }
__device__ inline float from_bits(uint16_t v) { return bf16_to_f32(v); }

// Operand element type staged in LDS: the MFMA input type.
template <int P> struct GemmT { using T = float; };
template <> struct GemmT<P_BF16> { using T = uint16_t; };
__device__ inline void stage(float* d, float v) { *d = v; }
__device__ inline void stage(uint16_t* d, float v) { *d = f32_to_bf16_rne(v); }

struct GemmArgs {
  int M, N, K;
  const float* A;  // A(m, k) = A[m * sAm + k * sAk]
  long sAm, sAk;
  const float* B;  // B(k, n) = B[k * sBk + n * sBn]; with ones_col, B(k, N) = 1
  long sBk, sBn;
  float* C;        // C[m * sCm + n], n < N
  long sCm;
  float* Cone;     // nullable: C(m, N) of the ones column (a column sum of A)
  int accumulate;  // C += result, else C = result
  const void* gate;  // nullable: result *= act'(row m, feature n), stash [M][ldg] in stash order
  int gate_f32, ldg;
  float* part;     // split-K partial tiles [splits][M][N + 1] (splits > 1)
  int kchunk;      // K range of one split
};

__device__ inline float gemm_epilogue(const GemmArgs& g, int m, int n, float v) {
  if (g.gate && n < g.N) {
    const long gi = (long)m * g.ldg + stash_pos(n);
    v *= g.gate_f32 ? static_cast<const float*>(g.gate)[gi] : bf16_to_f32(static_cast<const uint16_t*>(g.gate)[gi]);
  }
  return v;
}

__device__ inline void gemm_store(const GemmArgs& g, int m, int n, float v) {
  float* c = n < g.N ? g.C + (long)m * g.sCm + n : g.Cone + m;
  *c = g.accumulate ? *c + v : v;
}

// C = A B (+ the ones column), one 64 x 64 output tile per workgroup and one K
// range per grid z-slice; four waves of 32 x 32 (MFMA 32x32x16 bf16 or 32x32x2
// fp32).  Operands are staged in LDS in the MFMA input type, k-contiguous per row
// of the tile, loaded with 16-byte global reads along whichever dimension is
// contiguous.  The next K tile's global reads are issued before the current
// tile's products and held in registers, so their latency overlaps the matrix
// work.  With one K range the epilogue is applied here, otherwise the fp32
// partial tile is written for gemm_reduce.
template <int P>
__global__ void __launch_bounds__(256) gemm_mfma(GemmArgs g, int ones_col) {
  using T = typename GemmT<P>::T;
  constexpr int TBK = gemm_tbk<P>();
  constexpr int PAD = 16 / sizeof(T);  // 16-byte row padding against bank conflicts
  constexpr int NA = TBM * TBK / 4 / 256, NB = TBN * TBK / 4 / 256;  // float4 groups per thread
  __shared__ __attribute__((aligned(16))) T As[TBM][TBK + PAD];
  __shared__ __attribute__((aligned(16))) T Bs[TBN][TBK + PAD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // XCD-aware tile order: workgroups are dealt to the 8 XCDs in turn, so
  // workgroup id goes to XCD id % 8; giving each XCD a contiguous eighth of the
  // (x fastest, then y, then z) tile order keeps the operand rows and columns its
  // tiles share -- or its whole K split -- in that XCD's L2.
  const int GX = gridDim.x, GY = gridDim.y, NWG = GX * GY * gridDim.z;
  int L = blockIdx.x + GX * (blockIdx.y + GY * blockIdx.z);
  if (NWG % 8 == 0) L = (L % 8) * (NWG / 8) + L / 8;
  const int bx = L % GX, by = (L / GX) % GY, bz = L / (GX * GY);
  const int m0 = by * TBM, n0 = bx * TBN;
  const int NN = g.N + ones_col;
  const int kb = bz * g.kchunk, ke = min(g.K, kb + g.kchunk);
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const bool a_vec_k = g.sAk == 1 && (g.sAm & 3) == 0 && ((uintptr_t)g.A & 15) == 0;
  const bool a_vec_m = g.sAm == 1 && (g.sAk & 3) == 0 && ((uintptr_t)g.A & 15) == 0;
  const bool b_vec_k = g.sBk == 1 && (g.sBn & 3) == 0 && ((uintptr_t)g.B & 15) == 0;
  const bool b_vec_n = g.sBn == 1 && (g.sBk & 3) == 0 && ((uintptr_t)g.B & 15) == 0;
  auto a_at = [&](int m, int k) -> float { return (m < g.M && k < ke) ? g.A[(long)m * g.sAm + (long)k * g.sAk] : 0.f; };
  auto b_at = [&](int k, int n) -> float {
    if (k >= ke || n >= NN) return 0.f;
    return n < g.N ? g.B[(long)k * g.sBk + (long)n * g.sBn] : 1.f;
  };
  // group e of the A tile: 4 consecutive k of row mm (a_vec_k) or 4 consecutive m at k
  auto a_load = [&](int k0, int e) -> float4 {
    if (a_vec_k) {
      const int mm = e / (TBK / 4), kk = (e % (TBK / 4)) * 4;
      const int m = m0 + mm, k = k0 + kk;
      if (m < g.M && k + 3 < ke) return *reinterpret_cast<const float4*>(g.A + (long)m * g.sAm + k);
      return make_float4(a_at(m, k), a_at(m, k + 1), a_at(m, k + 2), a_at(m, k + 3));
    }
    const int kk = e / (TBM / 4), mm = (e % (TBM / 4)) * 4;
    const int m = m0 + mm, k = k0 + kk;
    if (a_vec_m && m + 3 < g.M && k < ke) return *reinterpret_cast<const float4*>(g.A + m + (long)k * g.sAk);
    return make_float4(a_at(m, k), a_at(m + 1, k), a_at(m + 2, k), a_at(m + 3, k));
  };
  auto a_stage = [&](int e, float4 v) {
    if (a_vec_k) {
      const int mm = e / (TBK / 4), kk = (e % (TBK / 4)) * 4;
      stage(&As[mm][kk], v.x); stage(&As[mm][kk + 1], v.y); stage(&As[mm][kk + 2], v.z); stage(&As[mm][kk + 3], v.w);
    } else {
      const int kk = e / (TBM / 4), mm = (e % (TBM / 4)) * 4;
      stage(&As[mm][kk], v.x); stage(&As[mm + 1][kk], v.y); stage(&As[mm + 2][kk], v.z); stage(&As[mm + 3][kk], v.w);
    }
  };
  auto b_load = [&](int k0, int e) -> float4 {
    if (b_vec_k) {
      const int nn = e / (TBK / 4), kk = (e % (TBK / 4)) * 4;
      const int n = n0 + nn, k = k0 + kk;
      if (n < g.N && k + 3 < ke) return *reinterpret_cast<const float4*>(g.B + k + (long)n * g.sBn);
      return make_float4(b_at(k, n), b_at(k + 1, n), b_at(k + 2, n), b_at(k + 3, n));
    }
    const int kk = e / (TBN / 4), nn = (e % (TBN / 4)) * 4;
    const int n = n0 + nn, k = k0 + kk;
    if (b_vec_n && n + 3 < g.N && k < ke) return *reinterpret_cast<const float4*>(g.B + (long)k * g.sBk + n);
    return make_float4(b_at(k, n), b_at(k, n + 1), b_at(k, n + 2), b_at(k, n + 3));
  };
  auto b_stage = [&](int e, float4 v) {
    if (b_vec_k) {
      const int nn = e / (TBK / 4), kk = (e % (TBK / 4)) * 4;
      stage(&Bs[nn][kk], v.x); stage(&Bs[nn][kk + 1], v.y); stage(&Bs[nn][kk + 2], v.z); stage(&Bs[nn][kk + 3], v.w);
    } else {
      const int kk = e / (TBN / 4), nn = (e % (TBN / 4)) * 4;
      stage(&Bs[nn][kk], v.x); stage(&Bs[nn + 1][kk], v.y); stage(&Bs[nn + 2][kk], v.z); stage(&Bs[nn + 3][kk], v.w);
    }
  };
  // bf16: each thread moves one 8 (k) x 4 (row) block of each operand tile, read as
  // eight float4 along whichever dimension is contiguous in memory and written to
  // LDS as four 16-byte runs of 8 consecutive k (the transpose happens in
  // registers); fp32: groups of 4 as read.
  auto blk_load = [&](bool vec_k, bool vec_x, int k0, int x0, int nx, auto at, auto ptr, float4 (&r)[8]) {
    // vec_k: four runs of 8 k per thread, run p = jj 256 + tid at row p / 16, k 8 (p % 16), so
    // that 16 neighbouring lanes read one row's 512 contiguous bytes; else one block of 4
    // rows (tid % 16) x 8 k (tid / 16)
    // a tile wholly inside the operand (uniform over the workgroup) is read without
    // per-lane bounds checks, so that all sixteen reads are issued back to back
    const bool inside = x0 + 64 <= nx && k0 + TBK <= ke;
    if (vec_k && inside) {
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int pr = jj * 256 + tid, x = x0 + (pr >> 4), k = k0 + (pr & 15) * 8;
        r[2 * jj] = *reinterpret_cast<const float4*>(ptr(x, k));
        r[2 * jj + 1] = *reinterpret_cast<const float4*>(ptr(x, k + 4));
      }
    } else if (vec_k) {
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int pr = jj * 256 + tid, x = x0 + (pr >> 4), k = k0 + (pr & 15) * 8;
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          const int kk = k + 4 * hh;
          r[2 * jj + hh] = (x < nx && kk + 3 < ke)
                               ? *reinterpret_cast<const float4*>(ptr(x, kk))
                               : make_float4(at(kk, x), at(kk + 1, x), at(kk + 2, x), at(kk + 3, x));
        }
      }
    } else if (vec_x && inside) {
      const int xb = (tid & 15) * 4, kb8 = (tid >> 4) * 8, x = x0 + xb;
#pragma unroll
      for (int j = 0; j < 8; ++j) r[j] = *reinterpret_cast<const float4*>(ptr(x, k0 + kb8 + j));
    } else {
      const int xb = (tid & 15) * 4, kb8 = (tid >> 4) * 8, x = x0 + xb;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = k0 + kb8 + j;
        r[j] = (vec_x && x + 3 < nx && k < ke) ? *reinterpret_cast<const float4*>(ptr(x, k))
                                              : make_float4(at(k, x), at(k, x + 1), at(k, x + 2), at(k, x + 3));
      }
    }
  };
  auto blk_stage = [&](bool vec_k, T (*dst)[TBK + PAD], const float4 (&r)[8]) {
    if (vec_k) {
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int pr = jj * 256 + tid;
        i32x4 w;
        w[0] = (int)pack_bf16x2(r[2 * jj].x, r[2 * jj].y);
        w[1] = (int)pack_bf16x2(r[2 * jj].z, r[2 * jj].w);
        w[2] = (int)pack_bf16x2(r[2 * jj + 1].x, r[2 * jj + 1].y);
        w[3] = (int)pack_bf16x2(r[2 * jj + 1].z, r[2 * jj + 1].w);
        *reinterpret_cast<i32x4*>(&dst[pr >> 4][(pr & 15) * 8]) = w;
      }
    } else {
      const int xb = (tid & 15) * 4, kb8 = (tid >> 4) * 8;
      auto col = [&](int q, int j) { return q == 0 ? r[j].x : q == 1 ? r[j].y : q == 2 ? r[j].z : r[j].w; };
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        i32x4 w;
#pragma unroll
        for (int t = 0; t < 4; ++t) w[t] = (int)pack_bf16x2(col(q, 2 * t), col(q, 2 * t + 1));
        *reinterpret_cast<i32x4*>(&dst[xb + q][kb8]) = w;
      }
    }
  };
  auto a_ptr = [&](int m, int k) { return g.A + (long)m * g.sAm + (long)k * g.sAk; };
  auto b_ptr = [&](int n, int k) { return g.B + (long)k * g.sBk + (long)n * g.sBn; };
  auto a_at2 = [&](int k, int m) { return a_at(m, k); };
  auto b_at2 = [&](int k, int n) { return b_at(k, n); };
  float4 ra[8], rb[8];
  auto load_tiles = [&](int k0) {
    if constexpr (P == P_BF16) {
      blk_load(a_vec_k, a_vec_m, k0, m0, g.M, a_at2, a_ptr, ra);
      blk_load(b_vec_k, b_vec_n, k0, n0, g.N, b_at2, b_ptr, rb);
    } else {
#pragma unroll
      for (int j = 0; j < NA; ++j) ra[j] = a_load(k0, tid + j * 256);
#pragma unroll
      for (int j = 0; j < NB; ++j) rb[j] = b_load(k0, tid + j * 256);
    }
  };
  load_tiles(kb);
  f32x16 acc = {};
  for (int k0 = kb; k0 < ke; k0 += TBK) {
    if constexpr (P == P_BF16) {
      blk_stage(a_vec_k, As, ra);
      blk_stage(b_vec_k, Bs, rb);
    } else {
#pragma unroll
      for (int j = 0; j < NA; ++j) a_stage(tid + j * 256, ra[j]);
#pragma unroll
      for (int j = 0; j < NB; ++j) b_stage(tid + j * 256, rb[j]);
    }
    __syncthreads();
    if (k0 + TBK < ke) load_tiles(k0 + TBK);  // the next tile's reads, in flight during the products
    const int r = lane & 31, h = lane >> 5;
    if constexpr (P == P_BF16) {
#pragma unroll
      for (int ks = 0; ks < TBK; ks += 16) {
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(&As[wm + r][ks + h * 8]);
        const bf16x8 b = *reinterpret_cast<const bf16x8*>(&Bs[wn + r][ks + h * 8]);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int ks = 0; ks < TBK; ks += 2)
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(As[wm + r][ks + h], Bs[wn + r][ks + h], acc, 0, 0, 0);
    }
    __syncthreads();
  }
  // accumulator register i of lane l: row (i/4)*8 + (l/32)*4 + i%4, column l%32
  const int n = n0 + wn + (lane & 31);
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int m = m0 + wm + (i >> 2) * 8 + (lane >> 5) * 4 + (i & 3);
    if (m >= g.M || n >= NN) continue;
    if (gridDim.z == 1) gemm_store(g, m, n, gemm_epilogue(g, m, n, acc[i]));
    else g.part[((long)bz * g.M + m) * (g.N + 1) + n] = acc[i];
  }
}

// Sum of the split-K partial tiles in split order, then the epilogue.
__global__ void gemm_reduce(GemmArgs g, int ones_col, int splits) {
  const int NN = g.N + ones_col;
  const long total = (long)g.M * NN;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
    const int m = (int)(i / NN), n = (int)(i % NN);
    float v = 0.f;
    for (int z = 0; z < splits; ++z) v += g.part[((long)z * g.M + m) * (g.N + 1) + n];
    gemm_store(g, m, n, gemm_epilogue(g, m, n, v));
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

// Split-K factor for an M x N (+1) output with reduction length K: enough
// workgroups to cover the chip, K ranges of at least 256.
int gemm_splits(int M, int N, int K) {
  const long tiles = (long)((M + TBM - 1) / TBM) * ((N + 1 + TBN - 1) / TBN);
  long s = (2L * num_cu() + tiles - 1) / tiles;
  const long smax = K / 256 > 0 ? K / 256 : 1;
  if (s > smax) s = smax;
  if (s > 64) s = 64;
  return s < 1 ? 1 : (int)s;
}

hipError_t launch_gemm(int prec, int M, int N, int K, const float* A, long sAm, long sAk, const float* B, long sBk,
                       long sBn, float* C, long sCm, float* Cone, int accumulate, const void* gate, int gate_is_f32,
                       int ldg, float* part, hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int ones = Cone ? 1 : 0;
  const int splits = (part && K > 0) ? gemm_splits(M, N, K) : 1;
  GemmArgs g{M, N, K, A, sAm, sAk, B, sBk, sBn, C, sCm, Cone, accumulate, gate, gate_is_f32, ldg, part, 0};
  const int tbk = prec == P_BF16 ? gemm_tbk<P_BF16>() : gemm_tbk<P_FP32>();
  g.kchunk = K > 0 ? (K + splits - 1) / splits : tbk;
  g.kchunk = (g.kchunk + tbk - 1) / tbk * tbk;
  const int splits_used = K > 0 ? (K + g.kchunk - 1) / g.kchunk : 1;
  dim3 grid((N + ones + TBN - 1) / TBN, (M + TBM - 1) / TBM, splits_used);
  if (prec == P_FP32) gemm_mfma<P_FP32><<<grid, 256, 0, st>>>(g, ones);
  else gemm_mfma<P_BF16><<<grid, 256, 0, st>>>(g, ones);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || splits_used == 1) return e;
  const long total = (long)M * (N + ones);
  int blocks = (int)((total + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  gemm_reduce<<<blocks, 256, 0, st>>>(g, ones, splits_used);
  return hipGetLastError();
}

hipError_t launch_mse(int nel, const float* y, const float* t, float* dy, float* loss, hipStream_t st) {
  mse_kernel<<<1, 1024, 0, st>>>(nel, y, t, dy, loss);
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
