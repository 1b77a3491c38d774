// Small-batch (latency) path of the network value and Jacobian, fp32.
//
// With a single MPC instance (tens of nodes) the layer-chain kernels run on a
// handful of compute units: one workgroup carries a block of rows through all
// layers.  Here every layer is its own launch instead and spreads its output
// features over many workgroups (32 x 32 output tiles, 16 x 16 when that grid
// would be small) and its reduction over up to 16 waves per workgroup, so a
// layer of 20 nodes x 512 features still occupies 64-256 compute units.  J_D,
// the output layer and the RK4 step follow in one launch (lat_tail_kernel).  Same mathematics as the chain kernels
// (Sec. IV-A: network value and reverse-mode Jacobian once per node):
//   forward : h_l = SiLU(W_l h_{l-1} + b_l), act'(a_l) kept; y = W_{L+1} h_L + b_{L+1}
//   reverse : G_L = W_{L+1} (.) act'(a_L) (6 rows per node, formed while loading);
//             G_{l-1} = (G_l W_l) (.) act'(a_{l-1});  J_D = G_1 W_1
// Weights are the fp32 master copy, row-major [fan_out][fan_in]; activations,
// derivatives and cotangents are row-major [rows][width] in model workspace.
// Width-64 networks of at most 4 hidden layers take one fused launch instead,
// with every operand in LDS (lat_fused_kernel).
#include <hip/hip_runtime.h>

#include <atomic>

#include "common.h"
#include "mlp_chain.h"
#include "rk4_node.h"

namespace rtn {

// A operand (rows x K): z_0 packed from x, u | a row-major buffer | a shared
// weight matrix gated per node, wsrc(r % rpn, k) * gate_a[r / rpn][k] (G_L =
// W_{L+1} (.) act'(a_L) with 6 rows per node; the first tangent layer with 14) |
// a row-major buffer gated per node, A[r][k] * gate_a[r / rpn][k] (tangents).
// B operand: W [N][K] read transposed (forward) or W [K][N] (reverse).
// Epilogue: SiLU with derivative (and second derivative) | bias | derivative
// gate (and the ungated value) | none.
enum LatA { LA_Z0 = 0, LA_ACT = 1, LA_GOUT = 2, LA_TGATE = 3 };
enum LatB { LB_NT = 0, LB_NN = 1 };
enum LatE { LE_SILU = 0, LE_BIAS = 1, LE_GATE = 2, LE_NONE = 3 };

struct LatArgs {
  int M, N, K;                 // rows, output columns, reduction length
  const float* x;              // LA_Z0: [n][13]
  const float* u;              // LA_Z0: [n][4]
  const float* A;              // LA_ACT, LA_TGATE: [M][K]
  const float* wsrc;           // LA_GOUT: element (j, k) at wsrc[j * wj + k * wk]
  long wj, wk;
  const float* gate_a;         // LA_GOUT, LA_TGATE: [M / rpn][K]
  int rpn;                     // LA_GOUT, LA_TGATE: operand rows per node
  const float* W;              // LB_NT: [N][K]; LB_NN: [K][N]
  const float* bias;           // LE_SILU, LE_BIAS: [N]
  const float* gate;           // LE_GATE: act'(a) [M/6][N]
  float* out;                  // [M][N]
  float* dout;                 // LE_SILU: act'(a) [M][N]; LE_GATE (nullable): the ungated value [M][N]
  float* ddout;                // LE_SILU (nullable): act''(a) [M][N]
  int act;                     // LE_SILU: 0 SiLU, 1 identity
  int input;                   // LA_Z0: network input variant (net_feature)
};

typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kLatWaves = 16;
constexpr int kLatNarrowBelow = 128;  // 32 x 32 tiles of a launch below which 16 x 16 tiles are used

__device__ inline float lat_a(const LatArgs& p, int akind, int r, int k) {
  if (r >= p.M || k >= p.K) return 0.f;
  if (akind == LA_Z0) return net_feature(p.x + (size_t)r * kNx, p.u + (size_t)r * kNu, k, p.input);
  if (akind == LA_ACT) return p.A[(size_t)r * p.K + k];
  const int node = r / p.rpn, j = r - p.rpn * node;
  const float g = p.gate_a[(size_t)node * p.K + k];
  if (akind == LA_TGATE) return p.A[(size_t)r * p.K + k] * g;
  return p.wsrc[(size_t)j * p.wj + (size_t)k * p.wk] * g;
}

__device__ inline float lat_b(const LatArgs& p, int bkind, int k, int c) {
  if (k >= p.K || c >= p.N) return 0.f;
  return bkind == LB_NT ? p.W[(size_t)c * p.K + k] : p.W[(size_t)k * p.N + c];
}

// Four consecutive k of one operand row (VEC path: 16-byte aligned, k % 4 == 0).
__device__ inline float4 lat_a4(const LatArgs& p, int akind, int r, int k) {
  if (r >= p.M) return make_float4(0.f, 0.f, 0.f, 0.f);
  if (akind == LA_ACT) return *reinterpret_cast<const float4*>(p.A + (size_t)r * p.K + k);
  const int node = r / p.rpn, j = r - p.rpn * node;
  const float4 g = *reinterpret_cast<const float4*>(p.gate_a + (size_t)node * p.K + k);
  const float4 a = akind == LA_TGATE ? *reinterpret_cast<const float4*>(p.A + (size_t)r * p.K + k)
                                     : *reinterpret_cast<const float4*>(p.wsrc + (size_t)j * p.wj + k);
  return make_float4(a.x * g.x, a.y * g.y, a.z * g.z, a.w * g.w);
}

__device__ inline float4 lat_b4(const LatArgs& p, int bkind, int k, int c) {
  if (c >= p.N) return make_float4(0.f, 0.f, 0.f, 0.f);
  if (bkind == LB_NT) return *reinterpret_cast<const float4*>(p.W + (size_t)c * p.K + k);
  const float* w = p.W + (size_t)k * p.N + c;
  return make_float4(w[0], w[p.N], w[2 * (size_t)p.N], w[3 * (size_t)p.N]);
}

// Epilogue of one output element (row, col) with the reduced product s.
template <int EP> __device__ inline void lat_store(const LatArgs& p, int row, int col, float s) {
  const size_t o = (size_t)row * p.N + col;
  if constexpr (EP == LE_SILU) {
    const float a = s + p.bias[col];
    if (p.act == 0) {
      const float sg = 1.f / (1.f + __expf(-a));
      p.out[o] = a * sg;
      p.dout[o] = sg * (1.f + a * (1.f - sg));
      if (p.ddout) p.ddout[o] = sg * (1.f - sg) * (2.f + a * (1.f - 2.f * sg));
    } else {
      p.out[o] = a;
      p.dout[o] = 1.f;
      if (p.ddout) p.ddout[o] = 0.f;
    }
  } else if constexpr (EP == LE_BIAS) {
    p.out[o] = s + p.bias[col];
  } else if constexpr (EP == LE_GATE) {
    p.out[o] = s * p.gate[(size_t)(row / 6) * p.N + col];
    if (p.dout) p.dout[o] = s;
  } else {
    p.out[o] = s;
  }
}

// One 32 x 32 output tile per workgroup, the K-steps split over its waves
// (32x32x2 fp32 MFMA); partial tiles are summed in LDS in fixed wave order.
// Scalar path: wave w takes steps w, w + nw, ..., step s covering k = 2 s, 2 s + 1.
// VEC path (K % 8 == 0, aligned operands, a multiple of 4 steps per wave): the
// two k slots of the product run over the two halves of K, and wave w takes a
// contiguous run of steps, so that every lane reads its operand rows as float4
// (the row-major operands are otherwise read one strided float per row).
template <int AK, int BK, int EP, bool VEC>
__global__ void __launch_bounds__(kLatWaves * kWave) lat_layer(LatArgs p) {
  __shared__ float part[kLatWaves][32 * 33];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const int ksteps = (p.K + 1) / 2;
  f32x16 acc = {};
  const int r = r0 + (lane & 31), c = c0 + (lane & 31), kh = lane >> 5;
  // all of this wave's operands are loaded before the first product (the loads
  // are L2 hits whose latency, not bandwidth, bounds a layer at this size)
  constexpr int MAXS = 32;  // K-steps per wave: K <= 2 * 16 * 32 = 1024
  float av[MAXS], bv[MAXS];
  if constexpr (VEC) {
    const int S = ksteps / nw, kb = kh * (p.K >> 1) + wave * S;
#pragma unroll
    for (int j = 0; j < MAXS / 4; ++j) {
      float4 a4 = make_float4(0.f, 0.f, 0.f, 0.f), b4 = a4;
      if (4 * j < S) {
        a4 = lat_a4(p, AK, r, kb + 4 * j);
        b4 = lat_b4(p, BK, kb + 4 * j, c);
      }
      av[4 * j] = a4.x, av[4 * j + 1] = a4.y, av[4 * j + 2] = a4.z, av[4 * j + 3] = a4.w;
      bv[4 * j] = b4.x, bv[4 * j + 1] = b4.y, bv[4 * j + 2] = b4.z, bv[4 * j + 3] = b4.w;
    }
#pragma unroll
    for (int i = 0; i < MAXS; ++i)
      if (i < S) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i], bv[i], acc, 0, 0, 0);
  } else {
#pragma unroll
    for (int i = 0; i < MAXS; ++i) {
      const int s = wave + i * nw;
      const int k = 2 * s + kh;
      const bool live = s < ksteps;
      av[i] = live ? lat_a(p, AK, r, k) : 0.f;
      bv[i] = live ? lat_b(p, BK, k, c) : 0.f;
    }
#pragma unroll
    for (int i = 0; i < MAXS; ++i)
      if (wave + i * nw < ksteps) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i], bv[i], acc, 0, 0, 0);
  }
  // accumulator register i of lane l: row (i/4)*8 + (l/32)*4 + i%4, column l%32
#pragma unroll
  for (int i = 0; i < 16; ++i) part[wave][((i >> 2) * 8 + kh * 4 + (i & 3)) * 33 + (lane & 31)] = acc[i];
  __syncthreads();
  for (int e = threadIdx.x; e < 32 * 32; e += blockDim.x) {
    const int rr = e >> 5, cc = e & 31, row = r0 + rr, col = c0 + cc;
    float s = 0.f;
    for (int w = 0; w < nw; ++w) s += part[w][rr * 33 + cc];
    if (row >= p.M || col >= p.N) continue;
    lat_store<EP>(p, row, col, s);
  }
}

// Narrow form for small grids: one 16 x 16 output tile per workgroup (MFMA
// 16x16x4 fp32).  A layer of a few tens of rows is bound by how fast each
// compute unit pulls its operands in (tens of GB/s per unit at these latencies),
// so a quarter of the tile area spreads the layer over four times as many units,
// each moving half the operand bytes of a 32 x 32 tile.  K is split over the
// waves; lane l supplies row / column l % 16 at k slot l / 16.  Scalar path: wave
// w takes 4-k steps w, w + nw, ...; VEC path (K a multiple of 16 nw, aligned
// operands): the four k slots run over four contiguous quarters of the wave's K
// range, so every lane reads its operand row as float4.
template <int AK, int BK, int EP, bool VEC>
__global__ void __launch_bounds__(kLatWaves * kWave) lat_layer16(LatArgs p) {
  __shared__ float part[kLatWaves][16 * 17];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int li = lane & 15, kq = lane >> 4;
  const int r = blockIdx.y * 16 + li, c = blockIdx.x * 16 + li;
  f32x4 acc = {};
  constexpr int MAXS = 16;  // MFMA steps per wave: K <= 4 * 16 * 16 = 1024
  float av[MAXS], bv[MAXS];
  if constexpr (VEC) {
    const int QW = p.K / nw / 4, kb = wave * (p.K / nw) + kq * QW;
#pragma unroll
    for (int j = 0; j < MAXS / 4; ++j) {
      float4 a4 = make_float4(0.f, 0.f, 0.f, 0.f), b4 = a4;
      if (4 * j < QW) {
        a4 = lat_a4(p, AK, r, kb + 4 * j);
        b4 = lat_b4(p, BK, kb + 4 * j, c);
      }
      av[4 * j] = a4.x, av[4 * j + 1] = a4.y, av[4 * j + 2] = a4.z, av[4 * j + 3] = a4.w;
      bv[4 * j] = b4.x, bv[4 * j + 1] = b4.y, bv[4 * j + 2] = b4.z, bv[4 * j + 3] = b4.w;
    }
#pragma unroll
    for (int i = 0; i < MAXS; ++i)
      if (i < QW) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[i], acc, 0, 0, 0);
  } else {
    const int ksteps = (p.K + 3) / 4;
#pragma unroll
    for (int i = 0; i < MAXS; ++i) {
      const int s = wave + i * nw;
      const int k = 4 * s + kq;
      const bool live = s < ksteps;
      av[i] = live ? lat_a(p, AK, r, k) : 0.f;
      bv[i] = live ? lat_b(p, BK, k, c) : 0.f;
    }
#pragma unroll
    for (int i = 0; i < MAXS; ++i)
      if (wave + i * nw < ksteps) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[i], acc, 0, 0, 0);
  }
  // accumulator v of lane l: row 4 (l / 16) + v, column l % 16
#pragma unroll
  for (int v = 0; v < 4; ++v) part[wave][(4 * kq + v) * 17 + li] = acc[v];
  __syncthreads();
  for (int e = threadIdx.x; e < 16 * 16; e += blockDim.x) {
    const int rr = e >> 4, cc = e & 15, row = blockIdx.y * 16 + rr, col = blockIdx.x * 16 + cc;
    float s = 0.f;
    for (int w = 0; w < nw; ++w) s += part[w][rr * 17 + cc];
    if (row >= p.M || col >= p.N) continue;
    lat_store<EP>(p, row, col, s);
  }
}

template <int AK, int BK, int EP> static hipError_t lat_launch(const LatArgs& p, hipStream_t st) {
  if (p.M <= 0 || p.N <= 0) return hipSuccess;
  if (p.K > 2 * kLatWaves * 32) return hipErrorInvalidValue;
  auto al16 = [](const void* q) { return q == nullptr || reinterpret_cast<uintptr_t>(q) % 16 == 0; };
  if (((p.N + 31) / 32) * ((p.M + 31) / 32) < kLatNarrowBelow && p.K <= 4 * kLatWaves * 16) {
    const dim3 grid((p.N + 15) / 16, (p.M + 15) / 16);
    int nw = (p.K / 4 + 15) / 16;  // about 16 MFMA steps per wave
    if (nw > kLatWaves) nw = kLatWaves;
    if (nw < 4) nw = 4;  // (the epilogue runs on the same waves)
    const bool vec = p.K % (16 * nw) == 0 && al16(p.A) && al16(p.gate_a) && al16(p.W) &&
                     (AK != LA_GOUT || (p.wk == 1 && p.wj % 4 == 0 && al16(p.wsrc)));
    if constexpr (AK != LA_Z0) {
      if (vec) {
        lat_layer16<AK, BK, EP, true><<<grid, nw * kWave, 0, st>>>(p);
        return hipGetLastError();
      }
    }
    lat_layer16<AK, BK, EP, false><<<grid, nw * kWave, 0, st>>>(p);
    return hipGetLastError();
  }
  const int ksteps = (p.K + 1) / 2;
  int nw = (ksteps + 15) / 16;  // about 16 K-steps per wave, at most 16 waves
  if (nw > kLatWaves) nw = kLatWaves;
  if (nw < 1) nw = 1;
  dim3 grid((p.N + 31) / 32, (p.M + 31) / 32);
  const bool vec = p.K % 8 == 0 && ksteps % nw == 0 && (ksteps / nw) % 4 == 0 && al16(p.A) && al16(p.gate_a) &&
                   al16(p.W) && (AK != LA_GOUT || (p.wk == 1 && p.wj % 4 == 0 && al16(p.wsrc)));
  if constexpr (AK != LA_Z0) {  // the input features are formed, not loaded
    if (vec) {
      lat_layer<AK, BK, EP, true><<<grid, nw * kWave, 0, st>>>(p);
      return hipGetLastError();
    }
  }
  lat_layer<AK, BK, EP, false><<<grid, nw * kWave, 0, st>>>(p);
  return hipGetLastError();
}

hipError_t launch_lat_forward(const LatNet& net, int n, const float* x, const float* u, float* act, float* sp, float* y,
                              hipStream_t st, float* spp) {
  const int H = net.H, L = net.L;
  hipError_t e;
  for (int l = 0; l < L; ++l) {
    LatArgs p{};
    p.M = n;
    p.N = H;
    p.K = l == 0 ? kDin : H;
    p.x = x;
    p.u = u;
    p.A = act + (size_t)((l + 1) & 1) * n * H;  // h_{l-1}
    p.W = net.W[l];
    p.bias = net.b[l];
    p.out = act + (size_t)(l & 1) * n * H;      // h_l
    p.dout = sp + (size_t)l * n * H;
    p.ddout = spp ? spp + (size_t)l * n * H : nullptr;
    p.act = net.act;
    p.input = net.input;
    e = l == 0 ? lat_launch<LA_Z0, LB_NT, LE_SILU>(p, st) : lat_launch<LA_ACT, LB_NT, LE_SILU>(p, st);
    if (e != hipSuccess) return e;
  }
  if (!y) return hipSuccess;  // (the tail kernel forms it)
  LatArgs p{};
  p.M = n;
  p.N = kDout;
  p.K = H;
  p.A = act + (size_t)((L - 1) & 1) * n * H;
  p.W = net.W[L];
  p.bias = net.b[L];
  p.out = y;
  return lat_launch<LA_ACT, LB_NT, LE_BIAS>(p, st);
}

hipError_t launch_lat_reverse(const LatNet& net, int n, const float* sp, float* g, float* J, hipStream_t st,
                              float* adj) {
  const int H = net.H, L = net.L;
  const int M = 6 * n;
  hipError_t e;
  // G_{l-1} = (G_l W_l) (.) act'(a_{l-1}) for l = L..2 (1-based), G_L formed on load
  for (int l = L - 1; l >= 1; --l) {  // 0-based layer index of W_{l+1}
    LatArgs p{};
    p.M = M;
    p.N = H;
    p.K = H;
    p.W = net.W[l];  // [H][H], reduction over its rows
    p.gate = sp + (size_t)(l - 1) * n * H;
    p.out = g + (size_t)(l & 1) * M * H;
    p.dout = adj ? adj + (size_t)(l - 1) * M * H : nullptr;  // dy/dh of layer l (1-based)
    if (l == L - 1) {
      p.gate_a = sp + (size_t)(L - 1) * n * H;
      p.wsrc = net.W[L];
      p.wj = H;
      p.wk = 1;
      p.rpn = 6;
      e = lat_launch<LA_GOUT, LB_NN, LE_GATE>(p, st);
    } else {
      p.A = g + (size_t)((l + 1) & 1) * M * H;
      e = lat_launch<LA_ACT, LB_NN, LE_GATE>(p, st);
    }
    if (e != hipSuccess) return e;
  }
  if (!J) return hipSuccess;  // (the tail kernel forms it from G_1 in g + M H)
  LatArgs p{};
  p.M = M;
  p.N = kDin;
  p.K = H;
  p.W = net.W[0];  // [H][14]
  p.out = J;
  if (L == 1) {
    p.gate_a = sp;
    p.wsrc = net.W[L];
    p.wj = H;
    p.wk = 1;
    p.rpn = 6;
    return lat_launch<LA_GOUT, LB_NN, LE_NONE>(p, st);
  }
  p.A = g + (size_t)(1 & 1) * M * H;
  return lat_launch<LA_ACT, LB_NN, LE_NONE>(p, st);
}

// ---------------------------------------------------------------------------
// Small networks (width 64, at most 4 hidden layers): the forward pass, the
// reverse sweep and J_D of up to 16 nodes in one workgroup -- one launch
// instead of 2L + 1.  Every weight is staged into LDS once (odd row strides, so
// that the column reads of the forward products are conflict free); products run
// on MFMA 16x16x4 fp32, where lane l supplies row / column l % 16 at
// k = 4 s + l / 16 and accumulator v of lane l is element (4 (l / 16) + v, l % 16).
// With rk4 given, the same workgroup then takes its nodes through the RK4 step
// (value, Jacobian and node data handed over in LDS).
constexpr int kFzNodes = 16, kFzH = 64, kFzMaxL = 4, kFzThreads = 512;
constexpr int kFzS = kFzH + 1, kFzW0S = kDin + 1, kFzRows = kFzNodes * kDout;  // 96 cotangent rows

static_assert(kFzNodes == kNodesPerBlock, "one RK4 block per workgroup");

static size_t fz_lds_bytes(int L) {
  const size_t f = (size_t)kFzH * kFzW0S + (size_t)(L - 1) * kFzH * kFzS + kDout * kFzH + L * kFzH + 8 +
                   2 * kFzNodes * kFzS + (size_t)L * kFzNodes * kFzS + 2 * kFzRows * kFzS +
                   kNodesPerBlock * kNodeStride + kNodesPerBlock;
  return f * sizeof(float);
}

__device__ inline float fz_act(float a, int act, float* d) {
  if (act == 0) {
    const float sg = 1.f / (1.f + __expf(-a));
    *d = sg * (1.f + a * (1.f - sg));
    return a * sg;
  }
  *d = 1.f;
  return a;
}

// acc[i] += A_i (16 x 64) B (64 x 16) on MFMA 16x16x4 fp32: lane (r, kq) supplies
// A_i[r][k] = ap[i][k - kq] and B[k][c] = bp[(k - kq) bk] for k = 4 st + kq; every
// operand is read from LDS before the first product.
template <int NT>
__device__ inline void fz_k64(const float* const* ap, const float* bp, int bk, f32x4* acc) {
  float a[NT][kFzH / 4], b[kFzH / 4];
#pragma unroll
  for (int st = 0; st < kFzH / 4; ++st) {
    b[st] = bp[4 * st * bk];
#pragma unroll
    for (int i = 0; i < NT; ++i) a[i][st] = ap[i][4 * st];
  }
#pragma unroll
  for (int st = 0; st < kFzH / 4; ++st)
#pragma unroll
    for (int i = 0; i < NT; ++i) acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][st], b[st], acc[i], 0, 0, 0);
}

__global__ void __launch_bounds__(kFzThreads) lat_fused_kernel(LatNet net, int n, const float* __restrict__ x,
                                                               const float* __restrict__ u, float* __restrict__ y,
                                                               float* __restrict__ J, FusedRk4 rk) {
  extern __shared__ float lds[];
  const int L = net.L;
  float* w0 = lds;                         // W_1 [64][14], row stride 15
  float* wh = w0 + kFzH * kFzW0S;          // W_2..W_L [64][64], row stride 65
  float* wo = wh + (L - 1) * kFzH * kFzS;  // W_{L+1} [6][64]
  float* bs = wo + kDout * kFzH;           // b_1..b_L [64] each, then b_{L+1} [6]
  float* zf = bs + L * kFzH + 8;           // 2 x [16][65] activations (node rows)
  float* spd = zf + 2 * kFzNodes * kFzS;   // L x [16][65] act'(a_l)
  float* gb = spd + L * kFzNodes * kFzS;   // 2 x [96][65] cotangents, row (node, output)
  float* rs = gb + 2 * kFzRows * kFzS;     // RK4 node data [16][kNodeStride], then 16 flags
  const bool with_rk4 = rk.xn != nullptr;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, r = lane & 15, kq = lane >> 4;
  const int node0 = blockIdx.x * kFzNodes, nn = min(kFzNodes, n - node0);

  // every parameter and the block's x, u: all loads issued first (clamped indices,
  // so that every address is valid and no load sits under a branch), then stored
  {
    constexpr int nW0 = kFzH * kDin, nWh = kFzH * kFzH, nHi = nWh / kFzThreads;
    static_assert(nWh % kFzThreads == 0 && 2 * kFzThreads >= nW0 && kFzThreads >= kDout * kFzH &&
                      kFzThreads >= kFzMaxL * kFzH + kDout && kFzThreads >= kFzNodes * kNx,
                  "staging covers every parameter in one pass");
    const float* W0 = net.W[0];
    float v0[2], vh[kFzMaxL - 1][nHi];
#pragma unroll
    for (int i = 0; i < 2; ++i) v0[i] = W0[min(t + i * kFzThreads, nW0 - 1)];
#pragma unroll
    for (int l = 0; l < kFzMaxL - 1; ++l) {
      const bool live = l + 1 < L;  // uniform
      const float* src = live ? net.W[l + 1] : W0;
#pragma unroll
      for (int i = 0; i < nHi; ++i) vh[l][i] = src[live ? t + i * kFzThreads : 0];
    }
    const float vo = net.W[L][min(t, kDout * kFzH - 1)];
    const int nb = L * kFzH + kDout, lb = t < nb ? t >> 6 : 0;
    const float* bsrc = lb == 0 ? net.b[0] : lb == 1 ? net.b[1] : lb == 2 ? net.b[2] : lb == 3 ? net.b[3] : net.b[4];
    const float vb = bsrc[t < nb ? t & 63 : 0];
    const float vx = x[(size_t)node0 * kNx + min(t, nn * kNx - 1)];
    const float vu = u[(size_t)node0 * kNu + min(t, nn * kNu - 1)];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int e = t + i * kFzThreads, row = e / kDin;
      if (e < nW0) w0[row * kFzW0S + (e - row * kDin)] = v0[i];
    }
#pragma unroll
    for (int l = 0; l < kFzMaxL - 1; ++l)
      if (l + 1 < L)
#pragma unroll
        for (int i = 0; i < nHi; ++i) {
          const int e = t + i * kFzThreads;
          wh[l * kFzH * kFzS + (e >> 6) * kFzS + (e & 63)] = vh[l][i];
        }
    if (t < kDout * kFzH) wo[t] = vo;
    if (t < nb) bs[t] = vb;
    if (t < nn * kNx) rs[(t / kNx) * kNodeStride + t % kNx] = vx;
    if (t < nn * kNu) rs[(t >> 2) * kNodeStride + 13 + (t & 3)] = vu;
  }
  __syncthreads();
  for (int e = t; e < kFzNodes * kDin; e += kFzThreads) {  // network input features from the staged x, u
    const int q = e / kDin, k = e - q * kDin;
    const float* sn = rs + q * kNodeStride;
    zf[q * kFzS + k] = q < nn ? net_feature(sn, sn + 13, k, net.input) : 0.f;
  }
  __syncthreads();

  // forward: a_l = h_{l-1} W_l^T + b_l, h_l = act(a_l); wave w < 4 owns columns 16 w .. 16 w + 15
  int cur = 0;
  for (int l = 0; l < L; ++l) {
    if (wave < 4) {
      const int c = wave * 16 + r;
      const float* zin = zf + cur * kFzNodes * kFzS;
      f32x4 acc = {};
      if (l == 0) {
        float a[4], b[4];
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          const int k = 4 * st + kq;
          a[st] = k < kDin ? zin[r * kFzS + k] : 0.f;
          b[st] = k < kDin ? w0[c * kFzW0S + k] : 0.f;
        }
#pragma unroll
        for (int st = 0; st < 4; ++st) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[st], b[st], acc, 0, 0, 0);
      } else {
        const float* ap[1] = {zin + r * kFzS + kq};
        fz_k64<1>(ap, wh + (l - 1) * kFzH * kFzS + c * kFzS + kq, 1, &acc);
      }
      float* zout = zf + (cur ^ 1) * kFzNodes * kFzS;
      float wl[kDout];  // last layer: W_{L+1}[j][c], for the cotangent rows formed below
#pragma unroll
      for (int j = 0; j < kDout; ++j) wl[j] = wo[j * kFzH + c];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int q = 4 * kq + v;
        float dd;
        zout[q * kFzS + c] = fz_act(acc[v] + bs[l * kFzH + c], net.act, &dd);
        spd[l * kFzNodes * kFzS + q * kFzS + c] = dd;
        if (l == L - 1)  // G_L[(q, j)][c] = W_{L+1}[j][c] act'(a_L)[q][c], into cotangent buffer 0
#pragma unroll
          for (int j = 0; j < kDout; ++j) gb[(q * kDout + j) * kFzS + c] = wl[j] * dd;
      }
    }
    __syncthreads();
    cur ^= 1;
  }

  // reverse: G_{l-1} = (G_l W_l) (.) act'(a_{l-1}), from G_L (formed in the last
  // forward epilogue); wave w owns column tile w % 4 and row tiles w / 4, w / 4 + 2,
  // w / 4 + 4 below nrt (W_l read once for all of them)
  const int rows = nn * kDout, nrt = (rows + 15) / 16;
  int gc = 0;
  for (int l = L - 1; l >= 1; --l) {
    const float* gin = gb + gc * kFzRows * kFzS;
    float* gout = gb + (gc ^ 1) * kFzRows * kFzS;
    const int ct = wave & 3, rt0 = wave >> 2, c = ct * 16 + r, ntl = (nrt - rt0 + 1) / 2;  // uniform per wave
    const float* ap[3] = {gin + (rt0 * 16 + r) * kFzS + kq, gin + ((rt0 + 2) * 16 + r) * kFzS + kq,
                          gin + ((rt0 + 4) * 16 + r) * kFzS + kq};
    const float* bp = wh + (l - 1) * kFzH * kFzS + kq * kFzS + c;
    f32x4 acc[3] = {};
    if (ntl >= 3)
      fz_k64<3>(ap, bp, kFzS, acc);
    else if (ntl == 2)
      fz_k64<2>(ap, bp, kFzS, acc);
    else if (ntl == 1)
      fz_k64<1>(ap, bp, kFzS, acc);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      if (i >= ntl) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int p = (rt0 + 2 * i) * 16 + 4 * kq + v, q = p / kDout;
        gout[p * kFzS + c] = p < rows ? acc[i][v] * spd[(l - 1) * kFzNodes * kFzS + q * kFzS + c] : 0.f;
      }
    }
    __syncthreads();
    gc ^= 1;
  }

  // J_D = G_1 W_1 ([rows][64] x [64][14]): wave w < nrt owns row tile w; wave 7
  // meanwhile forms y = W_{L+1} h_L + b_{L+1} (one 16 x 16 tile, 6 columns live)
  if (wave < nrt) {
    const float* ap[1] = {gb + gc * kFzRows * kFzS + (wave * 16 + r) * kFzS + kq};
    f32x4 acc = {};
    fz_k64<1>(ap, w0 + kq * kFzW0S + r, kFzW0S, &acc);  // columns r >= 14 are dropped
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int pv = wave * 16 + 4 * kq + v;
      if (pv < rows && r < kDin) {
        J[((size_t)node0 * kDout + pv) * kDin + r] = acc[v];
        rs[(pv / kDout) * kNodeStride + 23 + (pv % kDout) * kDin + r] = acc[v];
      }
    }
  } else if (wave == 7) {
    const float* ap[1] = {zf + cur * kFzNodes * kFzS + r * kFzS + kq};
    f32x4 acc = {};
    fz_k64<1>(ap, wo + r * kFzH + kq, 1, &acc);  // columns r >= 6 read other LDS data and are dropped
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int q = 4 * kq + v;
      if (q < nn && r < kDout) {
        const float yv = acc[v] + bs[L * kFzH + r];
        y[((size_t)node0 + q) * kDout + r] = yv;
        rs[q * kNodeStride + 17 + r] = yv;
      }
    }
  }
  if (with_rk4)  // uniform; the routine's first barrier publishes rs
    rk4_block_lanes(rs, reinterpret_cast<int*>(rs + kNodesPerBlock * kNodeStride), nn, node0, t, rk.P, rk.dt, true,
                    rk.xn, rk.A, rk.B, rk.status, net.input);
}

bool lat_fused_fits(const LatNet& net) { return net.H == kFzH && net.L >= 1 && net.L <= kFzMaxL; }

hipError_t launch_lat_fused(const LatNet& net, int n, const float* x, const float* u, float* y, float* J,
                            hipStream_t st, const FusedRk4* rk4) {
  if (n <= 0) return hipSuccess;
  if (!lat_fused_fits(net)) return hipErrorInvalidValue;
  static std::atomic<unsigned long long> lds_set{0};  // devices (id < 64) whose LDS limit is raised
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev >= 64 || !(lds_set.load() >> dev & 1)) {
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(lat_fused_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)fz_lds_bytes(kFzMaxL));
    if (e != hipSuccess) return e;
    if (dev < 64) lds_set.fetch_or(1ull << dev);
  }
  lat_fused_kernel<<<(n + kFzNodes - 1) / kFzNodes, kFzThreads, fz_lds_bytes(net.L), st>>>(net, n, x, u, y, J,
                                                                                     rk4 ? *rk4 : FusedRk4{});
  return hipGetLastError();
}

// Tail of the per-layer path (width 128..1024, L >= 2): J_D = G_1 W_1, the value
// y = W_{L+1} h_L + b_{L+1} and the RK4 step of kTlNodes nodes in one workgroup --
// one launch instead of three.  Each workgroup reads G_1's rows of its nodes
// (6 per node), their h_L rows and all of W_1 and W_{L+1}; at a few nodes per
// workgroup these reads, not the arithmetic, set the time, so the nodes are
// spread thin over the workgroups.  The 16-row tiles of J_D and the tile of y
// run on MFMA 16x16x4 fp32 with K split over the 8 waves; within a wave the
// four k slots of a product run over four contiguous quarters of the wave's K
// range, so that every lane reads its operand rows as float4.  Rows past the
// block's last node repeat its last row (valid addresses) and are dropped.
// Partial tiles are summed in LDS in fixed wave order, then handed to
// rk4_block_lanes with the node data.
constexpr int kTlThreads = 512, kTlNodes = 4;
constexpr int kTlJTiles = (kTlNodes * kDout + 15) / 16, kTlTiles = kTlJTiles + 1;
static_assert(kTlNodes <= kNodesPerBlock, "one RK4 block per workgroup");

template <int S>  // K-steps per lane: H = 32 S
__global__ void __launch_bounds__(kTlThreads)
    lat_tail_kernel(int n, const float* __restrict__ hL, const float* __restrict__ G1, const float* __restrict__ W1,
                    const float* __restrict__ Wo, const float* __restrict__ bo, const float* __restrict__ x,
                    const float* __restrict__ u, float* __restrict__ y, float* __restrict__ J, FusedRk4 rk,
                    int input) {
  constexpr int H = 32 * S, CH = S < 16 ? S : 16;
  __shared__ float part[kTlThreads / kWave][kTlTiles][256];
  __shared__ float rs[kTlNodes * kNodeStride + kTlNodes];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, r = lane & 15, kq = lane >> 4;
  const int node0 = blockIdx.x * kTlNodes, nn = min(kTlNodes, n - node0), rows = nn * kDout;
  if (t < nn * kNx) rs[(t / kNx) * kNodeStride + t % kNx] = x[(size_t)node0 * kNx + t];
  if (t < nn * kNu) rs[(t >> 2) * kNodeStride + 13 + (t & 3)] = u[(size_t)node0 * kNu + t];
  const int kl = wave * (H / 8) + kq * S;  // this lane's k run [kl, kl + S)
  const float* arow[kTlTiles];
#pragma unroll
  for (int rt = 0; rt < kTlJTiles; ++rt)
    arow[rt] = G1 + ((size_t)node0 * kDout + min(rt * 16 + r, rows - 1)) * H + kl;
  arow[kTlJTiles] = hL + ((size_t)node0 + min(r, nn - 1)) * H + kl;
  const float* wy = Wo + (size_t)min(r, kDout - 1) * H + kl;  // columns r >= 6 (and >= 14 of J_D) are dropped
  const float* wj = W1 + (size_t)kl * kDin + min(r, kDin - 1);
  f32x4 acc[kTlTiles] = {};
#pragma unroll
  for (int c0 = 0; c0 < S; c0 += CH) {
    float a[kTlTiles][CH], bj[CH], by[CH];
#pragma unroll
    for (int i = 0; i < CH; i += 4) {
#pragma unroll
      for (int rt = 0; rt < kTlTiles; ++rt) {
        const float4 v = *reinterpret_cast<const float4*>(arow[rt] + c0 + i);
        a[rt][i] = v.x, a[rt][i + 1] = v.y, a[rt][i + 2] = v.z, a[rt][i + 3] = v.w;
      }
      const float4 w = *reinterpret_cast<const float4*>(wy + c0 + i);
      by[i] = w.x, by[i + 1] = w.y, by[i + 2] = w.z, by[i + 3] = w.w;
    }
#pragma unroll
    for (int i = 0; i < CH; ++i) bj[i] = wj[(size_t)(c0 + i) * kDin];
#pragma unroll
    for (int i = 0; i < CH; ++i) {
#pragma unroll
      for (int rt = 0; rt < kTlJTiles; ++rt)
        acc[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rt][i], bj[i], acc[rt], 0, 0, 0);
      acc[kTlJTiles] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[kTlJTiles][i], by[i], acc[kTlJTiles], 0, 0, 0);
    }
  }
#pragma unroll
  for (int rt = 0; rt < kTlTiles; ++rt)
#pragma unroll
    for (int v = 0; v < 4; ++v) part[wave][rt][(4 * kq + v) * 16 + r] = acc[rt][v];
  __syncthreads();
  for (int e = t; e < kTlTiles * 256; e += kTlThreads) {
    const int rt = e >> 8, el = e & 255, row = el >> 4, col = el & 15;
    float sum = 0.f;
#pragma unroll
    for (int w = 0; w < kTlThreads / kWave; ++w) sum += part[w][rt][el];
    if (rt < kTlJTiles) {
      const int p = rt * 16 + row;
      if (p < rows && col < kDin) {
        J[((size_t)node0 * kDout + p) * kDin + col] = sum;
        rs[(p / kDout) * kNodeStride + 23 + (p % kDout) * kDin + col] = sum;
      }
    } else if (row < nn && col < kDout) {
      const float yv = sum + bo[col];
      y[((size_t)node0 + row) * kDout + col] = yv;
      rs[row * kNodeStride + 17 + col] = yv;
    }
  }
  rk4_block_lanes(rs, reinterpret_cast<int*>(rs + kTlNodes * kNodeStride), nn, node0, t, rk.P, rk.dt, true, rk.xn,
                  rk.A, rk.B, rk.status, input);
}

bool lat_tail_fits(const LatNet& net) {
  const int H = net.H;
  return net.L >= 2 && (H == 128 || H == 256 || H == 512 || H == 1024) &&
         reinterpret_cast<uintptr_t>(net.W[net.L]) % 16 == 0;
}

hipError_t launch_lat_tail(const LatNet& net, int n, const float* act, const float* g, const float* x, const float* u,
                           float* y, float* J, const FusedRk4& rk, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (!lat_tail_fits(net)) return hipErrorInvalidValue;
  const int L = net.L, H = net.H;
  const float* hL = act + (size_t)((L - 1) & 1) * n * H;  // the forward pass's last activations
  const float* G1 = g + (size_t)6 * n * H;                // the reverse sweep's G_1
  const dim3 grid((n + kTlNodes - 1) / kTlNodes);
#define RTN_TAIL(S_)                                                                                              \
  lat_tail_kernel<S_><<<grid, kTlThreads, 0, st>>>(n, hL, G1, net.W[0], net.W[L], net.b[L], x, u, y, J, rk, net.input)
  switch (H) {
    case 128: RTN_TAIL(4); break;
    case 256: RTN_TAIL(8); break;
    case 512: RTN_TAIL(16); break;
    default: RTN_TAIL(32); break;
  }
#undef RTN_TAIL
  return hipGetLastError();
}

// Tangents T_l = d a_l / d z_0 (14 rows per node, row (node, c) holds column c of
// T_l) for l = 2..L (1-based): T_2 = W_2 (act'(a_1) (.) W_1) with W_1 read as a
// gated shared matrix, T_l = W_l (act'(a_{l-1}) (.) T_{l-1}).  tan [2][14n][H]
// ping-pong: layer l (0-based, l >= 1) lands in tan + (l & 1) * 14 n H.
hipError_t launch_lat_tangent(const LatNet& net, int n, int l, const float* sp, float* tan, hipStream_t st) {
  const int H = net.H;
  LatArgs p{};
  p.M = 14 * n;
  p.N = H;
  p.K = H;
  p.W = net.W[l];
  p.gate_a = sp + (size_t)(l - 1) * n * H;
  p.rpn = 14;
  p.out = tan + (size_t)(l & 1) * 14 * n * H;
  if (l == 1) {
    p.wsrc = net.W[0];  // W_1 [H][14]: element (c, g) at g * 14 + c
    p.wj = 1;
    p.wk = kDin;
    return lat_launch<LA_GOUT, LB_NT, LE_NONE>(p, st);
  }
  p.A = tan + (size_t)((l - 1) & 1) * 14 * n * H;
  return lat_launch<LA_TGATE, LB_NT, LE_NONE>(p, st);
}

}  // namespace rtn
