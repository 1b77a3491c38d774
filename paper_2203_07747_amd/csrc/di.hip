// Double-integrator runtime workload (Sec. V).
//
// Nominal model x = [p, pdot], f_F(x, u) = [pdot, u]; residual f_D: a network
// from the state (2 values) to 2 values with n_hidden layers of any width up
// to 8192.  The Jacobian J_D (2 x 2) is carried forward: each node owns three
// activation rows, the value h_l and its derivatives along p and pdot,
//   h_1 = act(W_1 x + b_1),   T_1 = act'(a_1) (.) W_1
//   h_l = act(W_l h_{l-1} + b_l),   T_l = act'(a_l) (.) (W_l T_{l-1})
//   y = W_{L+1} h_L + b_{L+1},   J_D = W_{L+1} T_L,
// so one sweep over each weight matrix gives value and Jacobian (reverse mode
// would read every matrix twice; with two inputs the tangent rows cost less
// than the second read).  For wide layers the sweep streams the weights from
// HBM once and is bound by that; the rows of all nodes share each weight load.
//
// Then the first-order local approximation (eq. (4)) is held fixed in one RK4
// step (Sec. III) to give x_{k+1}, A_k, B_k (eq. (2)), and one real-time
// iteration solves the LQ subproblem by the Riccati recursion and a rollout.
#include "common.h"
#include "di.h"

namespace rtn {

namespace {

constexpr int kNodesPerTile = 10;  // 30 of the 32 rows of an MFMA tile
constexpr int kTileRows = 3 * kNodesPerTile;
constexpr int kMaxWaves = 16;

__device__ inline float di_act(float a, int act, float* dact) {
  if (act == 0) {
    const float s = 1.f / (1.f + __expf(-a));
    *dact = s * (1.f + a * (1.f - s));
    return a * s;
  }
  *dact = 1.f;
  return a;
}

// Position of activation row w (0 value, 1 d/dp, 2 d/dv) of node i, feature k, in
// a [3n][H] array: row-major, or (packed) in MFMA operand order, node tiles of 10
// nodes (30 rows padded to 32), then K-groups of 8, then the 64 lanes' float4s:
//   ((tile * H/8 + k/8) * 64 + lane) * 4 + k%4,  lane = row-in-tile + 32 ((k%8)/4),
// so that each wave's operand load is one contiguous 1 KB run.
template <bool PK>
__device__ inline size_t zpos(int i, int w, int k, int H) {
  if constexpr (PK) {
    const int tile = i / kNodesPerTile, r = 3 * (i - tile * kNodesPerTile) + w;
    const int lane = r + 32 * ((k >> 2) & 1);
    return (((size_t)tile * (H >> 3) + (k >> 3)) * 64 + lane) * 4 + (k & 3);
  } else {
    return ((size_t)3 * i + w) * H + k;
  }
}

template <bool PK>
__global__ void __launch_bounds__(256) di_first_layer(int n, int H, const float* __restrict__ W,
                                                      const float* __restrict__ b, int act,
                                                      const float* __restrict__ x, float* __restrict__ Z) {
  const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= (long)n * H) return;
  const int i = (int)(idx / H), c = (int)(idx % H);
  const float w0 = W[2 * c], w1 = W[2 * c + 1];
  float d;
  const float h = di_act(fmaf(w0, x[2 * i], fmaf(w1, x[2 * i + 1], b[c])), act, &d);
  Z[zpos<PK>(i, 0, c, H)] = h;
  Z[zpos<PK>(i, 1, c, H)] = d * w0;
  Z[zpos<PK>(i, 2, c, H)] = d * w1;
}

// Zout = epilogue(Zin W^T) for W [N][K]; one workgroup per 32 output columns,
// 10 nodes and one of KS slices of K, its waves splitting the slice.  MFMA
// 32x32x2 fp32: lane l supplies row (or column) l % 32 and, for the 4 products
// of one group of 8 K-values, k = 8 j + 4 (l / 32) + t.  PK (K % 8 == 0): Zin,
// Zout and W are in operand order (zpos; W packed the same way by column tiles,
// zero padded), so every operand load is a contiguous float4 per lane with no
// bounds check; otherwise row-major with element loads (small odd widths).
// With KS > 1 every workgroup stores its slice's partial tile and
// di_hidden_fixup adds the slices in order and applies the epilogue.
template <bool PK>
__global__ void __launch_bounds__(kMaxWaves * kWave)
di_hidden_layer(int n, int K, int N, const float* __restrict__ Zin, const float* __restrict__ W,
                const float* __restrict__ b, int act, float* __restrict__ Zout, float* __restrict__ partial) {
  __shared__ float part[kMaxWaves][kTileRows * 33];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int c0 = blockIdx.x * 32, node0 = blockIdx.y * kNodesPerTile;
  const int KS = gridDim.z, slice = blockIdx.z;
  const int rows = 3 * min(kNodesPerTile, n - node0);
  const int r = lane & 31, h = lane >> 5;
  const int groups = (K + 7) / 8;
  const int per = (groups + KS - 1) / KS;
  const int g0 = slice * per, g1 = min(groups, g0 + per);
  f32x16 acc = {};
  if constexpr (PK) {
    const float4* ap = reinterpret_cast<const float4*>(Zin) + (size_t)blockIdx.y * groups * 64 + lane;
    const float4* bp = reinterpret_cast<const float4*>(W) + (size_t)blockIdx.x * groups * 64 + lane;
    constexpr int U = 4;  // groups in flight per wave
    int j = g0 + wave;
    for (; j + (U - 1) * nw < g1; j += U * nw) {
      float4 av[U], bv[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        av[q] = ap[(size_t)(j + q * nw) * 64];
        bv[q] = bp[(size_t)(j + q * nw) * 64];
      }
#pragma unroll
      for (int q = 0; q < U; ++q) {
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[q].x, bv[q].x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[q].y, bv[q].y, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[q].z, bv[q].z, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[q].w, bv[q].w, acc, 0, 0, 0);
      }
    }
    for (; j < g1; j += nw) {
      const float4 a4 = ap[(size_t)j * 64], b4 = bp[(size_t)j * 64];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.x, b4.x, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.y, b4.y, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.z, b4.z, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.w, b4.w, acc, 0, 0, 0);
    }
  } else {
    const bool rv = r < rows, cv = c0 + r < N;
    const float* za = Zin + ((size_t)node0 * 3 + (rv ? r : 0)) * K;
    const float* wb = W + (size_t)(cv ? c0 + r : 0) * K;
    for (int j = g0 + wave; j < g1; j += nw) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int k = 8 * j + 4 * h + t;
        const float a = (rv && k < K) ? za[k] : 0.f;
        const float bb = (cv && k < K) ? wb[k] : 0.f;
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bb, acc, 0, 0, 0);
      }
    }
  }
  // accumulator register i of lane l: row (i/4)*8 + (l/32)*4 + i%4, column l%32
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int row = (i >> 2) * 8 + h * 4 + (i & 3);
    if (row < kTileRows) part[wave][row * 33 + r] = acc[i];
  }
  __syncthreads();
  if (KS > 1) {  // this slice's tile, summed over the waves in wave order
    float* pt = partial + (((size_t)slice * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x) * kTileRows * 32;
    for (int e = threadIdx.x; e < kTileRows * 32; e += blockDim.x) {
      float v = 0.f;
      for (int w = 0; w < nw; ++w) v += part[w][(e >> 5) * 33 + (e & 31)];
      pt[e] = v;
    }
    return;
  }
  for (int e = threadIdx.x; e < kNodesPerTile * 32; e += blockDim.x) {
    const int q = e >> 5, cc = e & 31, node = node0 + q, col = c0 + cc;
    if (3 * q >= rows || col >= N) continue;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f;
    for (int w = 0; w < nw; ++w) {
      s0 += part[w][(3 * q) * 33 + cc];
      s1 += part[w][(3 * q + 1) * 33 + cc];
      s2 += part[w][(3 * q + 2) * 33 + cc];
    }
    float d;
    const float hv = di_act(s0 + b[col], act, &d);
    Zout[zpos<PK>(node, 0, col, N)] = hv;
    Zout[zpos<PK>(node, 1, col, N)] = d * s1;
    Zout[zpos<PK>(node, 2, col, N)] = d * s2;
  }
}

// Sum of the KS partial tiles (in slice order) and the layer epilogue.
template <bool PK>
__global__ void __launch_bounds__(320) di_hidden_fixup(int n, int N, int KS, const float* __restrict__ partial,
                                                       const float* __restrict__ b, int act, float* __restrict__ Zout) {
  const int q = threadIdx.x >> 5, cc = threadIdx.x & 31;
  const int node = blockIdx.y * kNodesPerTile + q, col = blockIdx.x * 32 + cc;
  if (node >= n || col >= N) return;
  const size_t stride = (size_t)gridDim.y * gridDim.x * kTileRows * 32;
  const float* pp = partial + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * kTileRows * 32 + cc;
  float s0 = 0.f, s1 = 0.f, s2 = 0.f;
  for (int sl = 0; sl < KS; ++sl) {
    s0 += pp[sl * stride + (3 * q) * 32];
    s1 += pp[sl * stride + (3 * q + 1) * 32];
    s2 += pp[sl * stride + (3 * q + 2) * 32];
  }
  float d;
  const float hv = di_act(s0 + b[col], act, &d);
  Zout[zpos<PK>(node, 0, col, N)] = hv;
  Zout[zpos<PK>(node, 1, col, N)] = d * s1;
  Zout[zpos<PK>(node, 2, col, N)] = d * s2;
}

// y[i][j] = W[j] . h + b[j], J[i][j][m] = W[j] . T_m: one workgroup per (node, output).
__global__ void __launch_bounds__(256) di_output_layer(int n, int K, const float* __restrict__ W,
                                                       const float* __restrict__ b, const float* __restrict__ Z,
                                                       float* __restrict__ y, float* __restrict__ J) {
  __shared__ float red[3][4];
  const int i = blockIdx.x >> 1, j = blockIdx.x & 1, t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const float* w = W + (size_t)j * K;
  float s0 = 0.f, s1 = 0.f, s2 = 0.f;
  for (int k = t; k < K; k += 256) {
    const float wk = w[k];
    s0 = fmaf(wk, Z[zpos<false>(i, 0, k, K)], s0);
    s1 = fmaf(wk, Z[zpos<false>(i, 1, k, K)], s1);
    s2 = fmaf(wk, Z[zpos<false>(i, 2, k, K)], s2);
  }
  for (int off = 32; off > 0; off >>= 1) {
    s0 += __shfl_xor(s0, off);
    s1 += __shfl_xor(s1, off);
    s2 += __shfl_xor(s2, off);
  }
  if (lane == 0) {
    red[0][wave] = s0;
    red[1][wave] = s1;
    red[2][wave] = s2;
  }
  __syncthreads();
  if (t == 0) {
    y[2 * i + j] = red[0][0] + red[0][1] + red[0][2] + red[0][3] + b[j];
    J[(2 * i + j) * 2 + 0] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    J[(2 * i + j) * 2 + 1] = red[2][0] + red[2][1] + red[2][2] + red[2][3];
  }
  (void)n;
}

// Packed path: one workgroup per node, each thread a set of K-groups of 8;
// the node's three rows of a group are six float4s of the operand order and
// the two output rows two float4s each.
constexpr int kOutThreads = 1024;  // one K-group per thread at width 8192: all loads in flight at once

__global__ void __launch_bounds__(kOutThreads) di_output_packed(int n, int K, const float* __restrict__ W,
                                                                const float* __restrict__ b,
                                                                const float* __restrict__ Z, float* __restrict__ y,
                                                                float* __restrict__ J) {
  constexpr int NWV = kOutThreads / kWave;
  __shared__ float red[6][NWV];
  const int i = blockIdx.x, t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int G = K >> 3, tile = i / kNodesPerTile, r0 = 3 * (i - tile * kNodesPerTile);
  const float4* z4 = reinterpret_cast<const float4*>(Z) + (size_t)tile * G * 64;
  const float4* w0 = reinterpret_cast<const float4*>(W);
  const float4* w1 = reinterpret_cast<const float4*>(W + K);
  float s[2][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
  for (int j = t; j < G; j += kOutThreads) {
    const float4 a0 = w0[2 * j], a1 = w0[2 * j + 1], c0 = w1[2 * j], c1 = w1[2 * j + 1];
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      const float4 lo = z4[(size_t)j * 64 + r0 + w], hi = z4[(size_t)j * 64 + r0 + w + 32];
      s[0][w] += a0.x * lo.x + a0.y * lo.y + a0.z * lo.z + a0.w * lo.w + a1.x * hi.x + a1.y * hi.y + a1.z * hi.z +
                 a1.w * hi.w;
      s[1][w] += c0.x * lo.x + c0.y * lo.y + c0.z * lo.z + c0.w * lo.w + c1.x * hi.x + c1.y * hi.y + c1.z * hi.z +
                 c1.w * hi.w;
    }
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    float v = s[q / 3][q % 3];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) red[q][wave] = v;
  }
  __syncthreads();
  if (t < 6) {
    float v = 0.f;
    for (int w = 0; w < NWV; ++w) v += red[t][w];
    const int jo = t / 3, w = t % 3;
    if (w == 0) y[2 * i + jo] = v + b[jo];
    else J[(2 * i + jo) * 2 + (w - 1)] = v;
  }
  (void)n;
}

// One RK4 step of F(xi) = [xi_1, u] + y + J (xi - x) with the tangent
// S = d xi / d [x, u] (2 x 3) carried through the stages.
__device__ inline void di_rk4(const float x[2], float u, const float y[2], const float J[4], float dt, float xn[2],
                              float A[4], float B[2]) {
  const float cst[4] = {0.f, 0.5f, 0.5f, 1.f};
  const float wst[4] = {1.f, 2.f, 2.f, 1.f};
  // M = df_F/dx + J
  const float M00 = J[0], M01 = 1.f + J[1], M10 = J[2], M11 = J[3];
  float k0 = 0.f, k1 = 0.f, xa0 = 0.f, xa1 = 0.f;
  float dk[2][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}}, Sa[2][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const float cdt = cst[s] * dt;
    const float d0 = cdt * k0, d1 = cdt * k1;  // x_s - x
    float S[2][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      S[0][c] = (c == 0 ? 1.f : 0.f) + cdt * dk[0][c];
      S[1][c] = (c == 1 ? 1.f : 0.f) + cdt * dk[1][c];
    }
    k0 = (x[1] + d1) + y[0] + J[0] * d0 + J[1] * d1;
    k1 = u + y[1] + J[2] * d0 + J[3] * d1;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      dk[0][c] = M00 * S[0][c] + M01 * S[1][c];
      dk[1][c] = M10 * S[0][c] + M11 * S[1][c] + (c == 2 ? 1.f : 0.f);
    }
    xa0 += wst[s] * k0;
    xa1 += wst[s] * k1;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Sa[0][c] += wst[s] * dk[0][c];
      Sa[1][c] += wst[s] * dk[1][c];
    }
  }
  const float dt6 = dt / 6.f;
  xn[0] = x[0] + dt6 * xa0;
  xn[1] = x[1] + dt6 * xa1;
  A[0] = 1.f + dt6 * Sa[0][0];
  A[1] = dt6 * Sa[0][1];
  A[2] = dt6 * Sa[1][0];
  A[3] = 1.f + dt6 * Sa[1][1];
  B[0] = dt6 * Sa[0][2];
  B[1] = dt6 * Sa[1][2];
}

__device__ inline void di_node(int node, float dt, const float* x, const float* u, const float* y, const float* J,
                               float xn[2], float A[4], float B[2]) {
  const float xk[2] = {x[2 * node], x[2 * node + 1]};
  const float yk[2] = {y ? y[2 * node] : 0.f, y ? y[2 * node + 1] : 0.f};
  float Jk[4] = {0.f, 0.f, 0.f, 0.f};
  if (J)
    for (int i = 0; i < 4; ++i) Jk[i] = J[4 * node + i];
  di_rk4(xk, u[node], yk, Jk, dt, xn, A, B);
}

__global__ void __launch_bounds__(256) di_linearize_kernel(int n, float dt, const float* __restrict__ x,
                                                           const float* __restrict__ u, const float* __restrict__ y,
                                                           const float* __restrict__ J, float* __restrict__ xn,
                                                           float* __restrict__ A, float* __restrict__ B) {
  const int node = blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= n) return;
  float xo[2], Ao[4], Bo[2];
  di_node(node, dt, x, u, y, J, xo, Ao, Bo);
  for (int i = 0; i < 2; ++i) xn[2 * node + i] = xo[i];
  for (int i = 0; i < 4; ++i) A[4 * node + i] = Ao[i];
  for (int i = 0; i < 2; ++i) B[2 * node + i] = Bo[i];
}

// Per node LQ data in LDS (fp64): A 4 | B 2 | c 2 | q 2 | r 1 | K 2 | kff 1.
constexpr int kLqStride = 14;

// Stage node k of an instance (global node `node`) for the LQ solve: its
// linearisation (A, B, gap c = x_next - x_{k+1}) and the cost gradients.
__device__ inline void di_stage_node(double* s, int k, int N, int node, int inst, const DiCost& cost, double xr0,
                                     double xr1, const float* x, const float* u, const float* xN, const float* xo,
                                     const float* Ao, const float* Bo) {
  const float* succ = k + 1 < N ? x + 2 * (node + 1) : xN + 2 * inst;
  for (int i = 0; i < 4; ++i) s[i] = Ao[i];
  s[4] = Bo[0];
  s[5] = Bo[1];
  s[6] = (double)xo[0] - (double)succ[0];
  s[7] = (double)xo[1] - (double)succ[1];
  const double e0 = (double)x[2 * node] - xr0, e1 = (double)x[2 * node + 1] - xr1;
  s[8] = cost.Q[0] * e0 + cost.Q[1] * e1;
  s[9] = cost.Q[2] * e0 + cost.Q[3] * e1;
  s[10] = cost.R * (double)u[node];
}

// The Riccati recursion and the rollout of one instance on one lane:
//   Quu = R + B^T P B,  Qux = B^T P A,  g = P c + p,  qx = q + A^T g,  qu = r + B^T g
//   K = -Qux / Quu,  kff = -qu / Quu,  P <- sym(Q + A^T P A + Qux^T K),  p <- qx + Qux^T kff
//   du_k = K dx_k + kff,  dx_{k+1} = A dx_k + B du_k + c_k,  dx_0 = x0 - x_0.
__device__ inline void di_lq_solve(double* sm, int N, int k0, int inst, const DiCost& cost, double xr0, double xr1,
                                   const float* x, const float* xN, const float* x0, double* du, double* dx,
                                   double* dxN) {
  const double* Q = cost.Q;
  double P00 = cost.QN[0], P01 = cost.QN[1], P10 = cost.QN[2], P11 = cost.QN[3];
  const double eN0 = (double)xN[2 * inst] - xr0, eN1 = (double)xN[2 * inst + 1] - xr1;
  double p0 = P00 * eN0 + P01 * eN1, p1 = P10 * eN0 + P11 * eN1;
  for (int k = N - 1; k >= 0; --k) {
    double* s = sm + k * kLqStride;
    const double A00 = s[0], A01 = s[1], A10 = s[2], A11 = s[3], B0 = s[4], B1 = s[5];
    const double PB0 = P00 * B0 + P01 * B1, PB1 = P10 * B0 + P11 * B1;  // P B
    const double Quu = cost.R + B0 * PB0 + B1 * PB1;
    // Qux = B^T P A = (P^T B)^T A; P is kept symmetric
    const double Qux0 = PB0 * A00 + PB1 * A10, Qux1 = PB0 * A01 + PB1 * A11;
    const double g0 = P00 * s[6] + P01 * s[7] + p0, g1 = P10 * s[6] + P11 * s[7] + p1;
    const double qx0 = s[8] + A00 * g0 + A10 * g1, qx1 = s[9] + A01 * g0 + A11 * g1;
    const double qu = s[10] + B0 * g0 + B1 * g1;
    const double K0 = -Qux0 / Quu, K1 = -Qux1 / Quu, kf = -qu / Quu;
    // A^T P A
    const double PA00 = P00 * A00 + P01 * A10, PA01 = P00 * A01 + P01 * A11;
    const double PA10 = P10 * A00 + P11 * A10, PA11 = P10 * A01 + P11 * A11;
    const double X00 = Q[0] + A00 * PA00 + A10 * PA10 + Qux0 * K0;
    const double X01 = Q[1] + A00 * PA01 + A10 * PA11 + Qux0 * K1;
    const double X10 = Q[2] + A01 * PA00 + A11 * PA10 + Qux1 * K0;
    const double X11 = Q[3] + A01 * PA01 + A11 * PA11 + Qux1 * K1;
    P00 = X00;
    P11 = X11;
    P01 = P10 = 0.5 * (X01 + X10);
    p0 = qx0 + Qux0 * kf;
    p1 = qx1 + Qux1 * kf;
    s[11] = K0;
    s[12] = K1;
    s[13] = kf;
  }
  double d0 = (double)x0[2 * inst] - (double)x[2 * k0], d1 = (double)x0[2 * inst + 1] - (double)x[2 * k0 + 1];
  for (int k = 0; k < N; ++k) {
    const double* s = sm + k * kLqStride;
    const double v = s[11] * d0 + s[12] * d1 + s[13];
    du[k0 + k] = v;
    dx[2 * (k0 + k)] = d0;
    dx[2 * (k0 + k) + 1] = d1;
    const double n0 = s[0] * d0 + s[1] * d1 + s[4] * v + s[6];
    const double n1 = s[2] * d0 + s[3] * d1 + s[5] * v + s[7];
    d0 = n0;
    d1 = n1;
  }
  dxN[2 * inst] = d0;
  dxN[2 * inst + 1] = d1;
}

__device__ inline void di_store_lin(int node, const float* xo, const float* Ao, const float* Bo, float* xnout,
                                    float* Aout, float* Bout) {
  if (xnout)
    for (int i = 0; i < 2; ++i) xnout[2 * node + i] = xo[i];
  if (Aout)
    for (int i = 0; i < 4; ++i) Aout[4 * node + i] = Ao[i];
  if (Bout)
    for (int i = 0; i < 2; ++i) Bout[2 * node + i] = Bo[i];
}

// One instance per workgroup: the RK4 linearisation of its nodes (parallel, with
// the network's value and Jacobian from the layer kernels), then the LQ solve.
__global__ void __launch_bounds__(64) di_rti_kernel(const int* __restrict__ offsets, float dt, DiCost cost,
                                                    const float* __restrict__ x, const float* __restrict__ u,
                                                    const float* __restrict__ xN, const float* __restrict__ x0,
                                                    const float* __restrict__ xref, const float* __restrict__ y,
                                                    const float* __restrict__ J, double* __restrict__ du,
                                                    double* __restrict__ dx, double* __restrict__ dxN,
                                                    float* __restrict__ Aout, float* __restrict__ Bout,
                                                    float* __restrict__ xnout) {
  __shared__ double sm[kDiMaxHorizon * kLqStride];
  const int inst = blockIdx.x, t = threadIdx.x;
  const int k0 = offsets[inst], N = offsets[inst + 1] - k0;
  const double xr0 = xref ? xref[2 * inst] : 0.0, xr1 = xref ? xref[2 * inst + 1] : 0.0;
  for (int k = t; k < N; k += 64) {
    const int node = k0 + k;
    float xo[2], Ao[4], Bo[2];
    di_node(node, dt, x, u, y, J, xo, Ao, Bo);
    di_store_lin(node, xo, Ao, Bo, xnout, Aout, Bout);
    di_stage_node(sm + k * kLqStride, k, N, node, inst, cost, xr0, xr1, x, u, xN, xo, Ao, Bo);
  }
  __syncthreads();
  if (t == 0) di_lq_solve(sm, N, k0, inst, cost, xr0, xr1, x, xN, x0, du, dx, dxN);
}

// Small networks (width <= 64, instances of <= 64 nodes): the whole iteration in
// one workgroup per instance -- every layer, value and tangent rows, with the
// activations in LDS and the hidden weights read transposed (Wt[k][c] = W[c][k],
// so a wave's weight loads are contiguous), then RK4 and the LQ solve -- one
// launch instead of L + 2.  Nodes are taken 10 at a time (30 activation rows).
constexpr int kFusedMaxWidth = 64;  // wider layers run faster as separate kernels
constexpr int kFusedMaxHorizon = 64;
constexpr int kFusedThreads = 256;

template <int MAXS>
__global__ void __launch_bounds__(kFusedThreads)
di_fused_small(const int* __restrict__ offsets, int L, int H, int act, const float* __restrict__ params,
               const long* __restrict__ woff, float dt, DiCost cost, const float* __restrict__ x,
               const float* __restrict__ u, const float* __restrict__ xN, const float* __restrict__ x0,
               const float* __restrict__ xref, double* __restrict__ du, double* __restrict__ dx,
               double* __restrict__ dxN, float* __restrict__ Aout, float* __restrict__ Bout,
               float* __restrict__ xnout) {
  // activation rows [30][ZS]: the odd stride puts the 32 rows an MFMA operand
  // read touches on 32 different banks
  constexpr int ZS = kFusedMaxWidth + 1;
  __shared__ float za[kTileRows * ZS], zb[kTileRows * ZS], sraw[kTileRows * ZS];
  __shared__ float yj[kNodesPerTile * 6];
  __shared__ double sm[kFusedMaxHorizon * kLqStride];
  const int inst = blockIdx.x, t = threadIdx.x, lane = t & 63, wave = t >> 6, r = lane & 31, hh = lane >> 5;
  const int k0 = offsets[inst], N = offsets[inst + 1] - k0;
  const double xr0 = xref ? xref[2 * inst] : 0.0, xr1 = xref ? xref[2 * inst + 1] : 0.0;
  // this wave's 32-column tile of every hidden layer (at most one per wave)
  const int c = wave * 32 + r;
  const bool cv = c < H, rv = r < kTileRows, has_tile = wave * 32 < H;
  const int steps = (H + 1) / 2;  // <= MAXS
  // the lane's weights of hidden layer l (k = 2 s + l / 32), requested one layer ahead
  float bv[MAXS];
  auto fetch = [&](int l) {
    const float* Wt = params + woff[2 * l];
#pragma unroll
    for (int st = 0; st < MAXS; ++st) {
      const int k = 2 * st + hh;
      bv[st] = (cv && k < H) ? Wt[k * H + c] : 0.f;
    }
  };
  // woff: W_1, b_1, W_2^T, b_2, ..., W_out, b_out offsets into params
  for (int n0 = 0; n0 < N; n0 += kNodesPerTile) {
    const int nn = min(kNodesPerTile, N - n0);
    if (L > 1) fetch(1);
    {  // layer 1: h_1 and its tangents, per (node, column)
      const float* W1 = params + woff[0];
      const float* b1 = params + woff[1];
      for (int e = t; e < nn * H; e += kFusedThreads) {
        const int q = e / H, cc = e - q * H, node = k0 + n0 + q;
        const float w0 = W1[2 * cc], w1 = W1[2 * cc + 1];
        float d;
        const float hv = di_act(fmaf(w0, x[2 * node], fmaf(w1, x[2 * node + 1], b1[cc])), act, &d);
        za[(3 * q) * ZS + cc] = hv;
        za[(3 * q + 1) * ZS + cc] = d * w0;
        za[(3 * q + 2) * ZS + cc] = d * w1;
      }
    }
    __syncthreads();
    float* zi = za;
    float* zo = zb;
    for (int l = 1; l < L; ++l) {
      // S = Z W_l^T on MFMA 32x32x2 fp32: lane l supplies activation row l % 32 and
      // weight column l % 32 at k = 2 s + l / 32
      if (has_tile) {
        f32x16 acc = {};
#pragma unroll
        for (int st = 0; st < MAXS; ++st) {
          if (st < steps) {
            const int k = 2 * st + hh;
            const float a = (rv && k < H) ? zi[r * ZS + k] : 0.f;
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bv[st], acc, 0, 0, 0);
          }
        }
        if (l + 1 < L) fetch(l + 1);  // the next layer's weights load during this epilogue
        // accumulator register i: row (i/4)*8 + (l/32)*4 + i%4, column l%32
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int row = (i >> 2) * 8 + hh * 4 + (i & 3);
          if (row < kTileRows && cv) sraw[row * ZS + c] = acc[i];
        }
      }
      __syncthreads();
      const float* bl = params + woff[2 * l + 1];
      for (int e = t; e < nn * H; e += kFusedThreads) {  // bias, act, act' gating of the tangent rows
        const int q = e / H, cc = e - q * H;
        float d;
        const float hv = di_act(sraw[(3 * q) * ZS + cc] + bl[cc], act, &d);
        zo[(3 * q) * ZS + cc] = hv;
        zo[(3 * q + 1) * ZS + cc] = d * sraw[(3 * q + 1) * ZS + cc];
        zo[(3 * q + 2) * ZS + cc] = d * sraw[(3 * q + 2) * ZS + cc];
      }
      __syncthreads();
      float* tmp = zi;
      zi = zo;
      zo = tmp;
    }
    {  // output layer: y = W_out h + b, J = W_out T (60 dot products of length H)
      const float* Wo = params + woff[2 * L];
      const float* bo = params + woff[2 * L + 1];
      if (t < nn * 6) {
        const int q = t / 6, rr = t - 6 * q, j = rr / 3, w = rr - 3 * j;
        float sacc = 0.f;
#pragma unroll 8
        for (int k = 0; k < H; ++k) sacc = fmaf(Wo[j * H + k], zi[(3 * q + w) * ZS + k], sacc);
        // yj[q][0..1] = y, yj[q][2..5] = J row-major
        if (w == 0) yj[6 * q + j] = sacc + bo[j];
        else yj[6 * q + 2 + 2 * j + (w - 1)] = sacc;
      }
    }
    __syncthreads();
    if (t < nn) {  // RK4 of each node with its own f_D-bar, J_D
      const int k = n0 + t, node = k0 + k;
      const float xk[2] = {x[2 * node], x[2 * node + 1]};
      float xo[2], Ao[4], Bo[2];
      di_rk4(xk, u[node], yj + 6 * t, yj + 6 * t + 2, dt, xo, Ao, Bo);
      di_store_lin(node, xo, Ao, Bo, xnout, Aout, Bout);
      di_stage_node(sm + k * kLqStride, k, N, node, inst, cost, xr0, xr1, x, u, xN, xo, Ao, Bo);
    }
    __syncthreads();
  }
  if (t == 0) di_lq_solve(sm, N, k0, inst, cost, xr0, xr1, x, xN, x0, du, dx, dxN);
}

}  // namespace

hipError_t launch_di_first_layer(int n, int H, const float* W, const float* b, int act, const float* x, float* Z,
                                 hipStream_t st) {
  const long total = (long)n * H;
  if (total <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((total + 255) / 256);
  if (di_packed(H))
    di_first_layer<true><<<blocks, 256, 0, st>>>(n, H, W, b, act, x, Z);
  else
    di_first_layer<false><<<blocks, 256, 0, st>>>(n, H, W, b, act, x, Z);
  return hipGetLastError();
}

int di_slices(int n, int H) {
  // wide layers: K split so that about two workgroups per compute unit stream
  // the weights (the partial tiles are small next to the weights they replace)
  (void)n;
  if (H < 2048 || H >= 8192) return 1;  // at 8192 one workgroup per CU already streams near the bound
  int ks = 512 / ((H + 31) / 32);
  if (ks > 8) ks = 8;
  return ks < 1 ? 1 : ks;
}

size_t di_partial_floats(int n, int H) {
  const size_t tiles = (size_t)(n + kNodesPerTile - 1) / kNodesPerTile, ct = (H + 31) / 32;
  const int ks = di_slices(n, H);
  return ks > 1 ? (size_t)ks * tiles * ct * kTileRows * 32 : 0;
}

hipError_t launch_di_hidden_layer(int n, int H, const float* Zin, const float* W, const float* b, int act,
                                  float* Zout, float* partial, hipStream_t st) {
  if (n <= 0 || H <= 0) return hipSuccess;
  const int groups = (H + 7) / 8, ks = di_slices(n, H);
  int nw = (groups / ks) / 8;  // about eight groups of eight K-values per wave
  if (nw > kMaxWaves) nw = kMaxWaves;
  if (nw < 1) nw = 1;
  dim3 grid((H + 31) / 32, (n + kNodesPerTile - 1) / kNodesPerTile, ks);
  const bool pk = di_packed(H);
  if (pk)
    di_hidden_layer<true><<<grid, nw * kWave, 0, st>>>(n, H, H, Zin, W, b, act, Zout, partial);
  else
    di_hidden_layer<false><<<grid, nw * kWave, 0, st>>>(n, H, H, Zin, W, b, act, Zout, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || ks == 1) return e;
  dim3 g2(grid.x, grid.y);
  if (pk)
    di_hidden_fixup<true><<<g2, kNodesPerTile * 32, 0, st>>>(n, H, ks, partial, b, act, Zout);
  else
    di_hidden_fixup<false><<<g2, kNodesPerTile * 32, 0, st>>>(n, H, ks, partial, b, act, Zout);
  return hipGetLastError();
}

hipError_t launch_di_output_layer(int n, int K, const float* W, const float* b, const float* Z, float* y, float* J,
                                  hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (di_packed(K))
    di_output_packed<<<n, kOutThreads, 0, st>>>(n, K, W, b, Z, y, J);
  else
    di_output_layer<<<2 * n, 256, 0, st>>>(n, K, W, b, Z, y, J);
  return hipGetLastError();
}

size_t di_z_floats(int n, int H) {
  const size_t tiles = (size_t)(n + kNodesPerTile - 1) / kNodesPerTile;
  return di_packed(H) ? tiles * 32 * H : (size_t)3 * n * H;
}

void di_pack_weight(const float* W, int H, float* out) {
  const int G = H / 8, CT = (H + 31) / 32;
  for (int ct = 0; ct < CT; ++ct)
    for (int j = 0; j < G; ++j)
      for (int lane = 0; lane < 64; ++lane)
        for (int t = 0; t < 4; ++t) {
          const int row = 32 * ct + (lane & 31), k = 8 * j + 4 * (lane >> 5) + t;
          out[(((size_t)ct * G + j) * 64 + lane) * 4 + t] = row < H ? W[(size_t)row * H + k] : 0.f;
        }
}

hipError_t launch_di_linearize(int n, float dt, const float* x, const float* u, const float* y, const float* J,
                               float* xn, float* A, float* B, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  di_linearize_kernel<<<(n + 255) / 256, 256, 0, st>>>(n, dt, x, u, y, J, xn, A, B);
  return hipGetLastError();
}

bool di_fused_fits(int H, int max_horizon) { return H <= kFusedMaxWidth && max_horizon <= kFusedMaxHorizon; }

hipError_t launch_di_fused(int n_inst, const int* offsets, int L, int H, int act, const float* fused,
                           const long* woff, float dt, const DiCost& cost, const float* x, const float* u,
                           const float* xN, const float* x0, const float* xref, double* du, double* dx, double* dxN,
                           float* A, float* B, float* xn, hipStream_t st) {
  if (n_inst <= 0) return hipSuccess;
  if (H > kFusedMaxWidth || H < 1) return hipErrorInvalidValue;
  if (H <= 32)
    di_fused_small<16><<<n_inst, kFusedThreads, 0, st>>>(offsets, L, H, act, fused, woff, dt, cost, x, u, xN, x0,
                                                         xref, du, dx, dxN, A, B, xn);
  else
    di_fused_small<32><<<n_inst, kFusedThreads, 0, st>>>(offsets, L, H, act, fused, woff, dt, cost, x, u, xN, x0,
                                                         xref, du, dx, dxN, A, B, xn);
  return hipGetLastError();
}

hipError_t launch_di_rti(int n_inst, const int* offsets, float dt, const DiCost& cost, const float* x, const float* u,
                         const float* xN, const float* x0, const float* xref, const float* y, const float* J,
                         double* du, double* dx, double* dxN, float* A, float* B, float* xn, hipStream_t st) {
  if (n_inst <= 0) return hipSuccess;
  di_rti_kernel<<<n_inst, 64, 0, st>>>(offsets, dt, cost, x, u, xN, x0, xref, y, J, du, dx, dxN, A, B, xn);
  return hipGetLastError();
}

}  // namespace rtn
