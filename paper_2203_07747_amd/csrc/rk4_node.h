// The per-node RK4 step with sensitivities (Sec. IV-A, eq. (2) and the
// definitions that follow it; local approximation eq. (4); quadrotor model
// eq. (6)) as block-level device routines: rk4_block for the stand-alone RK4
// kernel (throughput), rk4_block_lanes for the fused small-network kernels
// (latency).
//
// Tangents: 16 lanes per node; lane c < 10 carries the tangent of state column
// 3 + c (nothing depends on the position, so columns 0..2 of A are the identity's
// and need no work), lanes 10..13 input columns 0..3, lane 15 writes A's position
// columns.  rk4_block first runs each node's state through the four stages of F
// with one lane per node and leaves in LDS what the tangents need at each stage
// point (q, omega and the thrust direction over the mass), so the trajectory is
// formed once per node instead of once per lane.
#pragma once

#include "common.h"
#include "quad_model.h"

namespace rtn {

constexpr int kNodesPerBlock = 16;  // nodes per rk4_block_lanes call of the fused network kernels
constexpr int kNodeStride = 108;    // x 13 | u 4 | y 6 | J 84 | pad 1
constexpr int kTrajStride = 40;     // per node, 4 stages of: q 4 | omega 3 | thrust direction / mass 3

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

// Phase (1) for the node staged at s (x 13 | u 4 | y 6 | J 84): the stage points
// x_s = x_k + c_s dt k_{s-1}, k_s = F(x_s), x_{k+1}; per stage tr receives q and
// omega at x_s and R(q) e_z / m (the thrust direction: d f_F / d u_j has it in
// rows 7..9 for every rotor).  Returns whether x_{k+1} is finite.
__device__ inline bool rk4_trajectory(const float* s, const QuadConst& P, const QuadInv& I, float dt, float* tr,
                                      float* __restrict__ xn) {
  const float* xk = s;
  const float* uk = s + 13;
  const float* yb = s + 17;
  const float* J = s + 23;
  float kp[13], acc[13];
#pragma unroll
  for (int i = 0; i < 13; ++i) { kp[i] = 0.f; acc[i] = 0.f; }
  const float cst[4] = {0.f, 0.5f, 0.5f, 1.f};
  const float wst[4] = {1.f, 2.f, 2.f, 1.f};
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    asm volatile("" ::: "memory");  // J is re-read from LDS per stage, not held in registers
    const float cdt = cst[st] * dt;
    float xs[13], dx[13], ks[13], r6[6];
#pragma unroll
    for (int i = 0; i < 13; ++i) {
      xs[i] = xk[i] + cdt * kp[i];
      dx[i] = xs[i] - xk[i];
    }
    nominal_rhs(xs, uk, P, I, ks);
    residual_tangent(J, dx, r6);
#pragma unroll
    for (int r = 0; r < 6; ++r) ks[7 + r] += yb[r] + r6[r];
    const float qw = xs[3], qx = xs[4], qy = xs[5], qz = xs[6];
    float* t = tr + st * 10;
    t[0] = qw;
    t[1] = qx;
    t[2] = qy;
    t[3] = qz;
    t[4] = xs[10];
    t[5] = xs[11];
    t[6] = xs[12];
    t[7] = 2.f * (qx * qz + qw * qy) * I.m;
    t[8] = 2.f * (qy * qz - qw * qx) * I.m;
    t[9] = (qw * qw - qx * qx - qy * qy + qz * qz) * I.m;
#pragma unroll
    for (int i = 0; i < 13; ++i) {
      acc[i] += wst[st] * ks[i];
      kp[i] = ks[i];
    }
  }
  const float dt6 = dt / 6.f;
  bool ok = true;
#pragma unroll
  for (int i = 0; i < 13; ++i) {
    const float v = xk[i] + dt6 * acc[i];
    ok &= isfinite(v);
    xn[i] = v;
  }
  return ok;
}

// LDS -> global copy of cnt floats by the nt threads of a block: whole 16-byte
// words where the destination is 16-byte aligned (src is), then the rest.
__device__ inline void copy_out(float* __restrict__ dst, const float* src, int cnt, int tid, int nt) {
  int done = 0;
  if ((reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
    const int n4 = cnt >> 2;
    for (int i = tid; i < n4; i += nt) reinterpret_cast<float4*>(dst)[i] = reinterpret_cast<const float4*>(src)[i];
    done = n4 << 2;
  }
  for (int i = done + tid; i < cnt; i += nt) dst[i] = src[i];
}

// Staging floats of one pass of rk4_block's phase (2): A and B of nt / 16 nodes.
constexpr int rk4_stage_floats(int nt) { return ((nt / 16) * kNx * kNx + 3) / 4 * 4 + (nt / 16) * kNx * kNu; }

// Throughput form: RK4 step of the nn nodes staged in sm (node i at sm + i kNodeStride:
// x 13 | u 4 | y 6 | J 84), nodes node0 .. node0 + nn - 1 of the batch, by a block
// of nt threads (nt a multiple of 16; phase (2) takes nt / 16 nodes at a time).
// Every thread of the block calls it (it holds barriers).  has_J: J holds the
// network Jacobian (w.r.t. its inputs); tr: nn kTrajStride floats of LDS;
// flags: nn ints of LDS; stg: rk4_stage_floats(nt) floats of 16-byte aligned LDS,
// where each pass assembles its nodes' A and B before they go out as contiguous runs.
__device__ inline void rk4_block(float* sm, float* tr, float* stg, int* flags, int nn, int node0, int tid, int nt,
                                 const QuadConst& P, float dt, bool has_J, float* __restrict__ xn,
                                 float* __restrict__ A, float* __restrict__ B, uint8_t* __restrict__ status,
                                 int input) {
  if (input != 0 && has_J) {  // uniform over the block
    __syncthreads();
    for (int i = tid; i < nn * kDout; i += nt) {
      float* sn = sm + (i / kDout) * kNodeStride;
      vb_row_to_state(sn, sn + 23 + (i % kDout) * kDin);
    }
  }
  __syncthreads();
  const QuadInv I = quad_inv(P);
  for (int ln = tid; ln < nn; ln += nt) {
    const float* sn = sm + ln * kNodeStride;
    int f = rk4_trajectory(sn, P, I, dt, tr + ln * kTrajStride, xn + (size_t)(node0 + ln) * kNx) ? 0 : 2;
    if (status) {  // the network's value and Jacobian (bit 1)
      bool ok = true;
#pragma unroll
      for (int i = 0; i < kDout + kDout * kDin; ++i) ok &= isfinite(sn[17 + i]);
      f |= ok ? 0 : 1;
    }
    flags[ln] = f;
  }
  __syncthreads();

  const int c = tid & 15;
  // which tangent this lane carries
  const int xcol = c < 10 ? 3 + c : -1;
  const int ucol = (c >= 10 && c < 14) ? c - 10 : -1;
  const float h = P.arm * 0.70710678118654752f;
  const float dt6 = dt / 6.f;
  const float cst[4] = {0.f, 0.5f, 0.5f, 1.f};
  const float wst[4] = {1.f, 2.f, 2.f, 1.f};
  const int per = nt >> 4, slot = tid >> 4;
  float* stA = stg;                                 // [per][13][13]
  float* stB = stg + (per * kNx * kNx + 3) / 4 * 4;  // [per][13][4]
  // A's position columns are the identity (no stage derivative depends on the
  // position) and the passes write only columns 3..12: fill them once
  for (int i = tid; i < per * kNx * 3; i += nt) {
    const int row = (i / 3) % kNx, col = i % 3;
    stA[(i / (3 * kNx)) * kNx * kNx + row * kNx + col] = row == col ? 1.f : 0.f;
  }
  for (int base = 0; base < nn; base += per) {  // uniform trip count: the passes hold barriers
    const int ln = base + slot;
    const float* s = sm + ln * kNodeStride;
    const float* uk = s + 13;
    const float* J = s + 23;
    const float* trn = tr + ln * kTrajStride;
    int bad = 0;
    if (ln < nn && c < 14) {
      // input lanes: the state-independent part of d F / d u_j (mixer torques and
      // the network's J_u e_j); the thrust direction is added per stage
      float fu[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      const float uon = ucol >= 0 ? 1.f : 0.f;
      if (ucol >= 0) {
        const float sx[4] = {-1.f, -1.f, 1.f, 1.f}, sy[4] = {-1.f, 1.f, 1.f, -1.f},
                    sz[4] = {-1.f, 1.f, -1.f, 1.f};
        fu[3] = h * sx[ucol] * I.Jx;
        fu[4] = h * sy[ucol] * I.Jy;
        fu[5] = P.c_tau * sz[ucol] * I.Jz;
#pragma unroll
        for (int r = 0; r < 6; ++r) fu[r] += J[r * kDin + 10 + ucol];
      }
      float dkp[13], accd[13];
#pragma unroll
      for (int i = 0; i < 13; ++i) { dkp[i] = 0.f; accd[i] = 0.f; }
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        // J and the stage values are re-read from LDS per stage rather than held in
        // registers: 168 instead of 197 VGPRs, three waves per SIMD instead of two
        asm volatile("" ::: "memory");
        const float cdt = cst[st] * dt;
        const float* t = trn + st * 10;
        float xs[13], ds[13], dk[13], r6[6];
#pragma unroll
        for (int i = 0; i < 13; ++i) {
          xs[i] = 0.f;  // only q and omega are read by the tangent
          ds[i] = ((i == xcol) ? 1.f : 0.f) + cdt * dkp[i];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) xs[3 + i] = t[i];
#pragma unroll
        for (int i = 0; i < 3; ++i) xs[10 + i] = t[4 + i];
        nominal_tangent(xs, uk, P, I, ds, dk);
        residual_tangent(J, ds, r6);
#pragma unroll
        for (int r = 0; r < 6; ++r) dk[7 + r] += r6[r] + fu[r];
#pragma unroll
        for (int i = 0; i < 3; ++i) dk[7 + i] += uon * t[7 + i];
#pragma unroll
        for (int i = 0; i < 13; ++i) {
          accd[i] += wst[st] * dk[i];
          dkp[i] = dk[i];
        }
      }
      float col[13];
#pragma unroll
      for (int i = 0; i < 13; ++i) {
        col[i] = ((i == xcol) ? 1.f : 0.f) + dt6 * accd[i];
        bad |= !isfinite(col[i]);
      }
      // column xcol of A or ucol of B (one store sequence for both kinds of lane)
      float* dst = xcol >= 0 ? stA + slot * kNx * kNx + xcol : stB + slot * kNx * kNu + ucol;
      const int ld = xcol >= 0 ? kNx : kNu;
#pragma unroll
      for (int i = 0; i < 13; ++i) dst[i * ld] = col[i];
      if (bad) atomicOr(&flags[ln], 2);
    }
    __syncthreads();
    // the pass's nodes are consecutive: their A and B are contiguous in global memory
    const int m = nn - base < per ? nn - base : per;
    copy_out(A + (size_t)(node0 + base) * kNx * kNx, stA, m * kNx * kNx, tid, nt);
    copy_out(B + (size_t)(node0 + base) * kNx * kNu, stB, m * kNx * kNu, tid, nt);
    __syncthreads();
  }
  if (status) {  // uniform over the block
    __syncthreads();
    for (int i = tid; i < nn; i += nt) status[node0 + i] = (uint8_t)flags[i];
  }
}

// Latency form: RK4 step of nn <= kNodesPerBlock nodes staged in sm (node i at
// sm + i kNodeStride: x 13 | u 4 | y 6 | J 84), nodes node0 .. node0 + nn - 1 of
// the batch, 16 lanes per node; every lane also runs the node's state through the
// stages itself, so no lane waits on another (for one small batch the longest
// dependency chain, not the instruction count, sets the time).  Every thread of
// the block calls it (it holds barriers); threads with tid >= 16 kNodesPerBlock
// only take part in those.  has_J: J holds the network
// Jacobian (w.r.t. its inputs); flags: kNodesPerBlock ints of LDS.
__device__ inline void rk4_block_lanes(float* sm, int* flags, int nn, int node0, int tid, const QuadConst& P,
                                       float dt, bool has_J, float* __restrict__ xn, float* __restrict__ A, float* __restrict__ B,
                                 uint8_t* __restrict__ status, int input) {
  if (tid < kNodesPerBlock) flags[tid] = 0;
  __syncthreads();
  if (input != 0 && has_J) {  // uniform over the block
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

}  // namespace rtn
