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
// Work split: 16 lanes per node (4 nodes per wave).  Lane c < 10 carries the
// tangent of state column 3 + c (nothing depends on the position, so columns
// 0..2 of A are the identity's and need no work); lanes 10..13 carry input
// columns 0..3; lane 14 writes x_{k+1}; lane 15 writes A's position columns.
// Every lane recomputes the node's state trajectory (cheap) so no lane waits
// on another.
#include "common.h"
#include "mlp_chain.h"
#include "quad_model.h"

namespace rtn {

constexpr int kNodesPerBlock = 16;
constexpr int kNodeStride = 108;  // x 13 | u 4 | y 6 | J 84 | pad 1


// Network Jacobian J (w.r.t. the input slots) -> the residual's state Jacobian
// in the slot layout of the full input [v, omega, q, u], at the node x_k, for the
// body-velocity inputs: slots 0..2 hold v_B = R(q)^T v, so the v columns become
// J dv_B/dv = J R^T, the q columns J dv_B/dq (homogeneous in q), omega's are
// zero; the u slots are unchanged.  One row of six floats per call.
__device__ inline void vb_row_to_state(const float* xk, float* Jr) {
  const float w = xk[3], a = xk[4], b = xk[5], c = xk[6];
  const float v0 = xk[7], v1 = xk[8], v2 = xk[9];
  const float j0 = Jr[0], j1 = Jr[1], j2 = Jr[2];
  // R(q) (rows) of the homogeneous rotation q (.) p (.) conj(q)
  const float R00 = w * w + a * a - b * b - c * c, R01 = 2.f * (a * b - w * c), R02 = 2.f * (a * c + w * b);
  const float R10 = 2.f * (a * b + w * c), R11 = w * w - a * a + b * b - c * c, R12 = 2.f * (b * c - w * a);
  const float R20 = 2.f * (a * c - w * b), R21 = 2.f * (b * c + w * a), R22 = w * w - a * a - b * b + c * c;
  // d v_B / d v_i = column i of R^T = row i of R
  Jr[0] = j0 * R00 + j1 * R01 + j2 * R02;
  Jr[1] = j0 * R10 + j1 * R11 + j2 * R12;
  Jr[2] = j0 * R20 + j1 * R21 + j2 * R22;
  Jr[3] = Jr[4] = Jr[5] = 0.f;
  // d v_B / d (w, a, b, c): derivative of sum_i R_ic(q) v_i
  const float d0w = 2.f * (w * v0 + c * v1 - b * v2), d0a = 2.f * (a * v0 + b * v1 + c * v2);
  const float d0b = 2.f * (-b * v0 + a * v1 - w * v2), d0c = 2.f * (-c * v0 + w * v1 + a * v2);
  const float d1w = 2.f * (-c * v0 + w * v1 + a * v2), d1a = 2.f * (b * v0 - a * v1 + w * v2);
  const float d1b = 2.f * (a * v0 + b * v1 + c * v2), d1c = 2.f * (-w * v0 - c * v1 + b * v2);
  const float d2w = 2.f * (b * v0 - a * v1 + w * v2), d2a = 2.f * (c * v0 - w * v1 - a * v2);
  const float d2b = 2.f * (w * v0 + c * v1 - b * v2), d2c = 2.f * (a * v0 + b * v1 + c * v2);
  Jr[6] = j0 * d0w + j1 * d1w + j2 * d2w;
  Jr[7] = j0 * d0a + j1 * d1a + j2 * d2a;
  Jr[8] = j0 * d0b + j1 * d1b + j2 * d2b;
  Jr[9] = j0 * d0c + j1 * d1c + j2 * d2c;
}

// J_x d restricted to rows 7..12 (network inputs are v, omega, q).
__device__ inline void residual_tangent(const float* J, const float* d, float* out6) {
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    const float* Jr = J + r * kDin;
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) s += Jr[c] * d[7 + c] + Jr[3 + c] * d[10 + c];
#pragma unroll
    for (int c = 0; c < 4; ++c) s += Jr[6 + c] * d[3 + c];
    out6[r] = s;
  }
}

__global__ void __launch_bounds__(256)
rk4_linearize_kernel(int n, QuadConst P, float dt, const float* __restrict__ x, const float* __restrict__ u,
                     const float* __restrict__ fD, const float* __restrict__ JD, float* __restrict__ xn,
                     float* __restrict__ A, float* __restrict__ B, uint8_t* __restrict__ status, int input) {
  __shared__ float sm[kNodesPerBlock * kNodeStride];
  __shared__ int flags[kNodesPerBlock];
  const int tid = threadIdx.x;
  const int node0 = blockIdx.x * kNodesPerBlock;
  const int nn = min(kNodesPerBlock, n - node0);
  if (nn <= 0) return;
  // cooperative, coalesced staging of the block's node data
  for (int i = tid; i < nn * kNx; i += 256) sm[(i / kNx) * kNodeStride + (i % kNx)] = x[(size_t)node0 * kNx + i];
  for (int i = tid; i < nn * kNu; i += 256) sm[(i / kNu) * kNodeStride + 13 + (i % kNu)] = u[(size_t)node0 * kNu + i];
  for (int i = tid; i < nn * kDout; i += 256)
    sm[(i / kDout) * kNodeStride + 17 + (i % kDout)] = fD ? fD[(size_t)node0 * kDout + i] : 0.f;
  for (int i = tid; i < nn * kDout * kDin; i += 256)
    sm[(i / (kDout * kDin)) * kNodeStride + 23 + (i % (kDout * kDin))] = JD ? JD[(size_t)node0 * kDout * kDin + i] : 0.f;
  if (tid < kNodesPerBlock) flags[tid] = 0;
  __syncthreads();
  if (input != 0 && JD) {  // uniform over the block
    if (tid < nn * kDout) {
      float* sn = sm + (tid / kDout) * kNodeStride;
      vb_row_to_state(sn, sn + 23 + (tid % kDout) * kDin);
    }
    __syncthreads();
  }

  const int ln = tid >> 4, c = tid & 15;
  const bool active = ln < nn;
  const int node = node0 + ln;
  const float* s = sm + (active ? ln : 0) * kNodeStride;
  const float* xk = s;
  const float* uk = s + 13;
  const float* yb = s + 17;
  const float* J = s + 23;

  // which tangent this lane carries
  const int xcol = c < 10 ? 3 + c : -1;
  const int ucol = (c >= 10 && c < 14) ? c - 10 : -1;
  const float h = P.arm * 0.70710678118654752f;
  const QuadInv I = quad_inv(P);
  float fu[13];  // df_F/du_j + J_u e_j (state-independent parts added per stage)
  if (ucol >= 0) {
    const float sx[4] = {-1.f, -1.f, 1.f, 1.f}, sy[4] = {-1.f, 1.f, 1.f, -1.f}, sz[4] = {-1.f, 1.f, -1.f, 1.f};
#pragma unroll
    for (int i = 0; i < 13; ++i) fu[i] = 0.f;
    fu[10] = h * sx[ucol] * I.Jx;
    fu[11] = h * sy[ucol] * I.Jy;
    fu[12] = P.c_tau * sz[ucol] * I.Jz;
#pragma unroll
    for (int r = 0; r < 6; ++r) fu[7 + r] += J[r * kDin + 10 + ucol];
  }

  float xs[13], kp[13], ks[13], dk[13], dkp[13], ds[13], accx[13], accd[13];
#pragma unroll
  for (int i = 0; i < 13; ++i) { accx[i] = 0.f; accd[i] = 0.f; kp[i] = 0.f; dkp[i] = 0.f; }
  const float cst[4] = {0.f, 0.5f, 0.5f, 1.f};
  const float wst[4] = {1.f, 2.f, 2.f, 1.f};
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const float cdt = cst[st] * dt;
#pragma unroll
    for (int i = 0; i < 13; ++i) {
      xs[i] = xk[i] + cdt * kp[i];
      ds[i] = ((i == xcol) ? 1.f : 0.f) + cdt * dkp[i];
    }
    // stage derivative of the state
    nominal_rhs(xs, uk, P, I, ks);
    float dx[13], r6[6];
#pragma unroll
    for (int i = 0; i < 13; ++i) dx[i] = xs[i] - xk[i];
    residual_tangent(J, dx, r6);
#pragma unroll
    for (int r = 0; r < 6; ++r) ks[7 + r] += yb[r] + r6[r];
    // stage derivative of the tangent
    nominal_tangent(xs, uk, P, I, ds, dk);
    residual_tangent(J, ds, r6);
#pragma unroll
    for (int r = 0; r < 6; ++r) dk[7 + r] += r6[r];
    if (ucol >= 0) {
      // thrust direction at the stage point (the homogeneous q (.) e_z)
      const float qw = xs[3], qx = xs[4], qy = xs[5], qz = xs[6];
      dk[7] += 2.f * (qx * qz + qw * qy) * I.m;
      dk[8] += 2.f * (qy * qz - qw * qx) * I.m;
      dk[9] += (qw * qw - qx * qx - qy * qy + qz * qz) * I.m;
#pragma unroll
      for (int i = 7; i < 13; ++i) dk[i] += fu[i];
    }
#pragma unroll
    for (int i = 0; i < 13; ++i) {
      accx[i] += wst[st] * ks[i];
      accd[i] += wst[st] * dk[i];
      kp[i] = ks[i];
      dkp[i] = dk[i];
    }
  }

  const float dt6 = dt / 6.f;
  int bad = 0;
  if (active && c < 14) {
    float col[13];
#pragma unroll
    for (int i = 0; i < 13; ++i) {
      col[i] = ((i == xcol) ? 1.f : 0.f) + dt6 * accd[i];
      bad |= !isfinite(col[i]);
    }
    if (xcol >= 0) {
      float* Ab = A + (size_t)node * kNx * kNx + xcol;
#pragma unroll
      for (int i = 0; i < 13; ++i) Ab[i * kNx] = col[i];
    } else {
      float* Bb = B + (size_t)node * kNx * kNu + ucol;
#pragma unroll
      for (int i = 0; i < 13; ++i) Bb[i * kNu] = col[i];
    }
  } else if (active && c == 14) {
#pragma unroll
    for (int i = 0; i < 13; ++i) {
      const float v = xk[i] + dt6 * accx[i];
      bad |= !isfinite(v);
      xn[(size_t)node * kNx + i] = v;
    }
  } else if (active) {
    float* Ab = A + (size_t)node * kNx * kNx;
#pragma unroll
    for (int i = 0; i < 13; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) Ab[i * kNx + j] = (i == j) ? 1.f : 0.f;
  }
  if (status) {  // uniform over the block
    int mlp_bad = 0;
    if (active && c == 15) {
      for (int i = 0; i < 6; ++i) mlp_bad |= !isfinite(yb[i]);
      for (int i = 0; i < 84; ++i) mlp_bad |= !isfinite(J[i]);
    }
    if (active && (bad || mlp_bad)) atomicOr(&flags[ln], (bad ? 2 : 0) | (mlp_bad ? 1 : 0));
    __syncthreads();
    if (active && c == 0) status[node] = (uint8_t)flags[ln];
  }
}

hipError_t launch_rk4_linearize(int n, const QuadConst& q, float dt, const float* x, const float* u, const float* fD,
                                const float* JD, float* xn, float* A, float* B, uint8_t* status, hipStream_t st,
                                int input) {
  if (n <= 0) return hipSuccess;
  const int blocks = (n + kNodesPerBlock - 1) / kNodesPerBlock;
  rk4_linearize_kernel<<<blocks, 256, 0, st>>>(n, q, dt, x, u, fD, JD, xn, A, B, status, input);
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
