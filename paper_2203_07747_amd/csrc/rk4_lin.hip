// One RK4 step of the nominal quadrotor model plus the node's affine residual,
// with its exact sensitivities -- the continuity parameters of the QP
// (Sec. IV-A, eq. (2) and the definitions that follow it; local approximation
// eq. (4); quadrotor model eq. (6); RK4 as in Sec. III).
//
//   F(x) = f_F(x, u_k) + f_D-bar + J_x (x - x_k)        (u held constant)
//   k_s  = F(x_k + c_s dt k_{s-1}),  c = (0, 1/2, 1/2, 1)
//   x_{k+1} = x_k + dt/6 (k_1 + 2 k_2 + 2 k_3 + k_4)
//   [A | B] = d x_{k+1} / d [x_k, u_k], carried as 13-vector tangents through the
//   four stages:  dk_s = (df_F/dx + J_x) dx_s  (+ df_F/du_j + J_u e_j for input j).
//
// The per-node routine and its work split (one lane per node for the state,
// 16 per node for the tangents) are in rk4_node.h.
#include "common.h"
#include "mlp_chain.h"
#include "quad_model.h"
#include "rk4_node.h"

namespace rtn {

// 64 nodes per workgroup: phase (1) of rk4_block then fills one wave.
constexpr int kRk4Nodes = 64, kRk4Threads = 256;

// three waves per SIMD (<= 168 registers): the tangent passes are latency bound
__global__ void __launch_bounds__(kRk4Threads) __attribute__((amdgpu_waves_per_eu(3)))
rk4_linearize_kernel(int n, QuadConst P, float dt, const float* __restrict__ x, const float* __restrict__ u,
                     const float* __restrict__ fD, const float* __restrict__ JD, float* __restrict__ xn,
                     float* __restrict__ A, float* __restrict__ B, uint8_t* __restrict__ status, int input) {
  __shared__ float sm[kRk4Nodes * kNodeStride];
  __shared__ float tr[kRk4Nodes * kTrajStride];
  __shared__ __align__(16) float stg[rk4_stage_floats(kRk4Threads)];
  __shared__ int flags[kRk4Nodes];
  const int tid = threadIdx.x;
  const int node0 = blockIdx.x * kRk4Nodes;
  const int nn = min(kRk4Nodes, n - node0);
  if (nn <= 0) return;
  // cooperative, coalesced staging of the block's node data
  for (int i = tid; i < nn * kNx; i += kRk4Threads)
    sm[(i / kNx) * kNodeStride + (i % kNx)] = x[(size_t)node0 * kNx + i];
  for (int i = tid; i < nn * kNu; i += kRk4Threads)
    sm[(i / kNu) * kNodeStride + 13 + (i % kNu)] = u[(size_t)node0 * kNu + i];
  for (int i = tid; i < nn * kDout; i += kRk4Threads)
    sm[(i / kDout) * kNodeStride + 17 + (i % kDout)] = fD ? fD[(size_t)node0 * kDout + i] : 0.f;
  for (int i = tid; i < nn * kDout * kDin; i += kRk4Threads)
    sm[(i / (kDout * kDin)) * kNodeStride + 23 + (i % (kDout * kDin))] =
        JD ? JD[(size_t)node0 * kDout * kDin + i] : 0.f;
  rk4_block(sm, tr, stg, flags, nn, node0, tid, kRk4Threads, P, dt, JD != nullptr, xn, A, B, status, input);
}

hipError_t launch_rk4_linearize(int n, const QuadConst& q, float dt, const float* x, const float* u, const float* fD,
                                const float* JD, float* xn, float* A, float* B, uint8_t* status, hipStream_t st,
                                int input) {
  if (n <= 0) return hipSuccess;
  const int blocks = (n + kRk4Nodes - 1) / kRk4Nodes;
  rk4_linearize_kernel<<<blocks, kRk4Threads, 0, st>>>(n, q, dt, x, u, fD, JD, xn, A, B, status, input);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256)
rk4_lanes_kernel(int n, QuadConst P, float dt, const float* __restrict__ x, const float* __restrict__ u,
                 const float* __restrict__ fD, const float* __restrict__ JD, float* __restrict__ xn,
                 float* __restrict__ A, float* __restrict__ B, uint8_t* __restrict__ status, int input) {
  __shared__ float sm[kNodesPerBlock * kNodeStride];
  __shared__ int flags[kNodesPerBlock];
  const int tid = threadIdx.x;
  const int node0 = blockIdx.x * kNodesPerBlock;
  const int nn = min(kNodesPerBlock, n - node0);
  if (nn <= 0) return;
  for (int i = tid; i < nn * kNx; i += 256) sm[(i / kNx) * kNodeStride + (i % kNx)] = x[(size_t)node0 * kNx + i];
  for (int i = tid; i < nn * kNu; i += 256) sm[(i / kNu) * kNodeStride + 13 + (i % kNu)] = u[(size_t)node0 * kNu + i];
  for (int i = tid; i < nn * kDout; i += 256)
    sm[(i / kDout) * kNodeStride + 17 + (i % kDout)] = fD ? fD[(size_t)node0 * kDout + i] : 0.f;
  for (int i = tid; i < nn * kDout * kDin; i += 256)
    sm[(i / (kDout * kDin)) * kNodeStride + 23 + (i % (kDout * kDin))] =
        JD ? JD[(size_t)node0 * kDout * kDin + i] : 0.f;
  rk4_block_lanes(sm, flags, nn, node0, tid, P, dt, JD != nullptr, xn, A, B, status, input);
}

hipError_t launch_rk4_lanes(int n, const QuadConst& q, float dt, const float* x, const float* u, const float* fD,
                            const float* JD, float* xn, float* A, float* B, uint8_t* status, hipStream_t st,
                            int input) {
  if (n <= 0) return hipSuccess;
  const int blocks = (n + kNodesPerBlock - 1) / kNodesPerBlock;
  rk4_lanes_kernel<<<blocks, 256, 0, st>>>(n, q, dt, x, u, fD, JD, xn, A, B, status, input);
  return hipGetLastError();
}

}  // namespace rtn

namespace rtn {

// ---------------------------------------------------------------------------
// Exact ("naive") linearisation of Sec. IV-A: the network and its Jacobian are
// evaluated at every RK4 stage point x_s, not only at the node.  Stage s needs
// k_{s-1}, so the four stages are sequential launches; between them the chain
// kernels evaluate f_D(x_s, u_k) and J_D(x_s, u_k) for all nodes at once.
//
// Per node state in the workspace (fp32): xs [13] (stage point), kp [13]
// (previous stage derivative), kacc [13] (weighted sum), dkp [17][13] and
// dacc [17][13] (tangent columns of the previous stage / weighted sum).
// Column c < 13 is the state direction c, 13..16 the input direction c - 13.
struct ExactWork {
  float* xs;
  float* kp;
  float* kacc;
  float* dkp;
  float* dacc;
};

// One stage: lanes 0..16 of a 32-lane half-wave carry the 17 tangent columns of one
// node (2 nodes per wave); every lane also forms the node's stage derivative.
__global__ void __launch_bounds__(256)
rk4_exact_stage_kernel(int n, int stage, QuadConst P, float dt, const float* __restrict__ x,
                       const float* __restrict__ u, const float* __restrict__ fD, const float* __restrict__ JD,
                       ExactWork w, float* __restrict__ xn, float* __restrict__ A, float* __restrict__ B) {
  const float cst[4] = {0.f, 0.5f, 0.5f, 1.f};
  const float wst[4] = {1.f, 2.f, 2.f, 1.f};
  const int node = (blockIdx.x * blockDim.x + threadIdx.x) >> 5;
  const int c = threadIdx.x & 31;
  if (node >= n || c >= 17) return;
  float xk[13], xs[13], uk[4], J[84], yb[6];
#pragma unroll
  for (int i = 0; i < 13; ++i) xk[i] = x[(size_t)node * 13 + i];
#pragma unroll
  for (int i = 0; i < 4; ++i) uk[i] = u[(size_t)node * 4 + i];
#pragma unroll
  for (int i = 0; i < 6; ++i) yb[i] = fD ? fD[(size_t)node * 6 + i] : 0.f;
#pragma unroll
  for (int i = 0; i < 84; ++i) J[i] = JD ? JD[(size_t)node * 84 + i] : 0.f;
  const float cdt = cst[stage] * dt;
  // stage point and tangent of this column
  float ds[13];
#pragma unroll
  for (int i = 0; i < 13; ++i) {
    const float kprev = stage ? w.kp[(size_t)node * 13 + i] : 0.f;
    xs[i] = xk[i] + cdt * kprev;
    const float dprev = stage ? w.dkp[((size_t)node * 17 + c) * 13 + i] : 0.f;
    ds[i] = ((i == c) ? 1.f : 0.f) + cdt * dprev;
  }
  float ks[13], dk[13], r6[6];
  const QuadInv I = quad_inv(P);
  nominal_rhs(xs, uk, P, I, ks);
#pragma unroll
  for (int r = 0; r < 6; ++r) ks[7 + r] += yb[r];
  nominal_tangent(xs, uk, P, I, ds, dk);
  residual_tangent(J, ds, r6);
#pragma unroll
  for (int r = 0; r < 6; ++r) dk[7 + r] += r6[r];
  if (c >= 13) {
    const int j = c - 13;
    const float h = P.arm * 0.70710678118654752f;
    const float sx[4] = {-1.f, -1.f, 1.f, 1.f}, sy[4] = {-1.f, 1.f, 1.f, -1.f}, sz[4] = {-1.f, 1.f, -1.f, 1.f};
    const float qw = xs[3], qx = xs[4], qy = xs[5], qz = xs[6];
    dk[7] += 2.f * (qx * qz + qw * qy) * I.m;
    dk[8] += 2.f * (qy * qz - qw * qx) * I.m;
    dk[9] += (qw * qw - qx * qx - qy * qy + qz * qz) * I.m;
    dk[10] += h * sx[j] * I.Jx;
    dk[11] += h * sy[j] * I.Jy;
    dk[12] += P.c_tau * sz[j] * I.Jz;
#pragma unroll
    for (int r = 0; r < 6; ++r) dk[7 + r] += J[r * kDin + 10 + j];
  }
  // accumulate; stash this stage for the next; at the last stage write the outputs
  float* dacc = w.dacc + ((size_t)node * 17 + c) * 13;
  float* dkp = w.dkp + ((size_t)node * 17 + c) * 13;
  const float dt6 = dt / 6.f;
#pragma unroll
  for (int i = 0; i < 13; ++i) {
    const float a = (stage ? dacc[i] : 0.f) + wst[stage] * dk[i];
    if (stage < 3) {
      dacc[i] = a;
      dkp[i] = dk[i];
    } else if (c < 13) {
      A[(size_t)node * 169 + i * 13 + c] = ((i == c) ? 1.f : 0.f) + dt6 * a;
    } else {
      B[(size_t)node * 52 + i * 4 + (c - 13)] = dt6 * a;
    }
  }
  if (c == 0) {
    const float cn = stage < 3 ? cst[stage + 1] * dt : 0.f;
#pragma unroll
    for (int i = 0; i < 13; ++i) {
      const float a = (stage ? w.kacc[(size_t)node * 13 + i] : 0.f) + wst[stage] * ks[i];
      if (stage < 3) {
        w.kacc[(size_t)node * 13 + i] = a;
        w.kp[(size_t)node * 13 + i] = ks[i];
        w.xs[(size_t)node * 13 + i] = xk[i] + cn * ks[i];  // next stage point
      } else {
        xn[(size_t)node * 13 + i] = xk[i] + dt6 * a;
      }
    }
  }
}

hipError_t launch_rk4_exact_stage(int n, int stage, const QuadConst& q, float dt, const float* x, const float* u,
                                  const float* fD, const float* JD, float* xs, float* kp, float* kacc, float* dkp,
                                  float* dacc, float* xn, float* A, float* B, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  ExactWork w{xs, kp, kacc, dkp, dacc};
  const int blocks = (n * 32 + 255) / 256;
  rk4_exact_stage_kernel<<<blocks, 256, 0, st>>>(n, stage, q, dt, x, u, fD, JD, w, xn, A, B);
  return hipGetLastError();
}

}  // namespace rtn
