// Small-batch (latency) path of the network value and Jacobian, fp32.
//
// With a single MPC instance (tens of nodes) the layer-chain kernels run on a
// handful of compute units: one workgroup carries a block of rows through all
// layers.  Here every layer is its own launch instead and spreads its output
// features over many workgroups (32 x 32 output tiles) and its reduction over up
// to 16 waves per workgroup, so a layer of 20 nodes x 512 features still
// occupies 16-64 compute units.  Same mathematics as the chain kernels
// (Sec. IV-A: network value and reverse-mode Jacobian once per node):
//   forward : h_l = SiLU(W_l h_{l-1} + b_l), act'(a_l) kept; y = W_{L+1} h_L + b_{L+1}
//   reverse : G_L = W_{L+1} (.) act'(a_L) (6 rows per node, formed while loading);
//             G_{l-1} = (G_l W_l) (.) act'(a_{l-1});  J_D = G_1 W_1
// Weights are the fp32 master copy, row-major [fan_out][fan_in]; activations,
// derivatives and cotangents are row-major [rows][width] in model workspace.
#include <hip/hip_runtime.h>

#include "common.h"
#include "mlp_chain.h"

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

constexpr int kLatWaves = 16;

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

// One 32 x 32 output tile per workgroup; wave w reduces K-steps w, w + nw, ...
// (32x32x2 fp32 MFMA); partial tiles are summed in LDS in fixed wave order.
template <int AK, int BK, int EP>
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
  // accumulator register i of lane l: row (i/4)*8 + (l/32)*4 + i%4, column l%32
#pragma unroll
  for (int i = 0; i < 16; ++i) part[wave][((i >> 2) * 8 + kh * 4 + (i & 3)) * 33 + (lane & 31)] = acc[i];
  __syncthreads();
  for (int e = threadIdx.x; e < 32 * 32; e += blockDim.x) {
    const int rr = e >> 5, cc = e & 31, row = r0 + rr, col = c0 + cc;
    float s = 0.f;
    for (int w = 0; w < nw; ++w) s += part[w][rr * 33 + cc];
    if (row >= p.M || col >= p.N) continue;
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
}

template <int AK, int BK, int EP> static hipError_t lat_launch(const LatArgs& p, hipStream_t st) {
  if (p.M <= 0 || p.N <= 0) return hipSuccess;
  if (p.K > 2 * kLatWaves * 32) return hipErrorInvalidValue;
  const int ksteps = (p.K + 1) / 2;
  int nw = (ksteps + 15) / 16;  // about 16 K-steps per wave, at most 16 waves
  if (nw > kLatWaves) nw = kLatWaves;
  if (nw < 1) nw = 1;
  dim3 grid((p.N + 31) / 32, (p.M + 31) / 32);
  lat_layer<AK, BK, EP><<<grid, nw * kWave, 0, st>>>(p);
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
