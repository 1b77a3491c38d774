// The nominal quadrotor model of eq. (6) and its directional derivative, shared
// by the RK4 sensitivity kernels (first- and second-order local approximation).
#pragma once

#include "common.h"
#include "mlp_chain.h"

namespace rtn {

// Reciprocals of the mass and the principal inertias, formed once per thread:
// the model divides by these constants many times per stage.
struct QuadInv {
  float m, Jx, Jy, Jz;
};
__device__ inline QuadInv quad_inv(const QuadConst& P) {
  return QuadInv{1.f / P.mass, 1.f / P.Jx, 1.f / P.Jy, 1.f / P.Jz};
}

// f_F(x, u) with T = sum u, tau from the X-frame mixer; closed form of eq. (6).
__device__ inline void nominal_rhs(const float* x, const float* u, const QuadConst& P, const QuadInv& I, float* f) {
  const float qw = x[3], qx = x[4], qy = x[5], qz = x[6];
  const float wx = x[10], wy = x[11], wz = x[12];
  const float T = u[0] + u[1] + u[2] + u[3];
  const float h = P.arm * 0.70710678118654752f;
  f[0] = x[7];
  f[1] = x[8];
  f[2] = x[9];
  f[3] = 0.5f * (-qx * wx - qy * wy - qz * wz);
  f[4] = 0.5f * (qw * wx + qy * wz - qz * wy);
  f[5] = 0.5f * (qw * wy - qx * wz + qz * wx);
  f[6] = 0.5f * (qw * wz + qx * wy - qy * wx);
  const float Tm = T * I.m;
  f[7] = Tm * 2.f * (qx * qz + qw * qy);
  f[8] = Tm * 2.f * (qy * qz - qw * qx);
  f[9] = Tm * (qw * qw - qx * qx - qy * qy + qz * qz) - P.g;
  const float tx = h * (-u[0] - u[1] + u[2] + u[3]);
  const float ty = h * (-u[0] + u[1] + u[2] - u[3]);
  const float tz = P.c_tau * (-u[0] + u[1] - u[2] + u[3]);
  f[10] = (tx - (P.Jz - P.Jy) * wy * wz) * I.Jx;
  f[11] = (ty - (P.Jx - P.Jz) * wz * wx) * I.Jy;
  f[12] = (tz - (P.Jy - P.Jx) * wx * wy) * I.Jz;
}

// (df_F/dx) d at x (directional derivative along the state tangent d).
__device__ inline void nominal_tangent(const float* x, const float* u, const QuadConst& P, const QuadInv& I,
                                       const float* d, float* df) {
  const float qw = x[3], qx = x[4], qy = x[5], qz = x[6];
  const float wx = x[10], wy = x[11], wz = x[12];
  const float dqw = d[3], dqx = d[4], dqy = d[5], dqz = d[6];
  const float dwx = d[10], dwy = d[11], dwz = d[12];
  const float T = u[0] + u[1] + u[2] + u[3];
  df[0] = d[7];
  df[1] = d[8];
  df[2] = d[9];
  // product rule on q (x) (0, w) / 2
  df[3] = 0.5f * (-dqx * wx - dqy * wy - dqz * wz - qx * dwx - qy * dwy - qz * dwz);
  df[4] = 0.5f * (dqw * wx + dqy * wz - dqz * wy + qw * dwx + qy * dwz - qz * dwy);
  df[5] = 0.5f * (dqw * wy - dqx * wz + dqz * wx + qw * dwy - qx * dwz + qz * dwx);
  df[6] = 0.5f * (dqw * wz + dqx * wy - dqy * wx + qw * dwz + qx * dwy - qy * dwx);
  const float Tm = T * I.m;
  df[7] = Tm * 2.f * (dqx * qz + qx * dqz + dqw * qy + qw * dqy);
  df[8] = Tm * 2.f * (dqy * qz + qy * dqz - dqw * qx - qw * dqx);
  df[9] = Tm * 2.f * (qw * dqw - qx * dqx - qy * dqy + qz * dqz);
  df[10] = -(P.Jz - P.Jy) * (dwy * wz + wy * dwz) * I.Jx;
  df[11] = -(P.Jx - P.Jz) * (dwz * wx + wz * dwx) * I.Jy;
  df[12] = -(P.Jy - P.Jx) * (dwx * wy + wx * dwy) * I.Jz;
}

}  // namespace rtn
