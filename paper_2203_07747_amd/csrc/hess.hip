// Second-order local approximation (eq. (4) with its Hessian term, Sec. IV-A):
// the network Hessian H_D per node and one RK4 step of f_F plus the quadratic
// residual f_D** = f_D-bar + J_D dz + 1/2 dz^T H_D dz (dz = z_0(x, u) - z_0(x_k, u_k),
// parameters held fixed), with the step's exact derivatives A_k, B_k.
//
// H_D by the chain rule of second order (fp32):
//   H_j = sum_l T_l^T diag((dy_j/dh_l) (.) act''(a_l)) T_l,   T_l = d a_l / d z_0,
// one layer at a time (the tangents T_l come from the per-layer kernels).
#include <hip/hip_runtime.h>

#include "common.h"
#include "mlp_chain.h"
#include "quad_model.h"

namespace rtn {

// One workgroup per node: T_l (14 x H) and the six weights w_j = dy_j/dh_l (.)
// act''(a_l) are staged in LDS (rows padded by one float against bank
// conflicts); each thread forms whole entries (j, c <= d) of the symmetric 14 x 14
// blocks in a fixed summation order.
__global__ void __launch_bounds__(256)
hess_accumulate_kernel(LatNet net, int n, int l, const float* __restrict__ tan, const float* __restrict__ adj,
                       const float* __restrict__ spp, float* __restrict__ Hd, int accumulate) {
  extern __shared__ float sm[];
  const int H = net.H, L = net.L, HP = H + 1;
  float* Ts = sm;              // [14][HP]
  float* ws = sm + kDin * HP;  // [6][HP]
  const int node = blockIdx.x, t = threadIdx.x;
  const float* T = tan + (size_t)(l & 1) * 14 * n * H + (size_t)node * 14 * H;
  for (int i = t; i < kDin * H; i += blockDim.x) {
    const int c = i / H, f = i - c * H;
    Ts[c * HP + f] = l == 0 ? net.W[0][(size_t)f * kDin + c] : T[(size_t)c * H + f];
  }
  const float* pp = spp + (size_t)l * n * H + (size_t)node * H;
  for (int i = t; i < kDout * H; i += blockDim.x) {
    const int j = i / H, f = i - j * H;
    const float u = l == L - 1 ? net.W[L][(size_t)j * H + f] : adj[(size_t)l * 6 * n * H + ((size_t)node * 6 + j) * H + f];
    ws[j * HP + f] = u * pp[f];
  }
  __syncthreads();
  float* out = Hd + (size_t)node * kDout * kDin * kDin;
  for (int idx = t; idx < kDout * 105; idx += blockDim.x) {
    const int j = idx / 105;
    int p = idx - j * 105, c = 0;
    while (p >= kDin - c) {  // (c, d) with c <= d, row by row
      p -= kDin - c;
      ++c;
    }
    const int d = c + p;
    const float* a = Ts + c * HP;
    const float* b = Ts + d * HP;
    const float* w = ws + j * HP;
    float s = 0.f;
    for (int f = 0; f < H; ++f) s += a[f] * b[f] * w[f];
    float* e1 = out + (j * kDin + c) * kDin + d;
    float* e2 = out + (j * kDin + d) * kDin + c;
    const float v = accumulate ? *e1 + s : s;
    *e1 = v;
    if (d != c) *e2 = v;
  }
}

hipError_t launch_hess_accumulate(const LatNet& net, int n, int l, const float* tan, const float* adj,
                                  const float* spp, float* Hd, int accumulate, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const size_t lds = (size_t)(kDin + kDout) * (net.H + 1) * sizeof(float);
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(hess_accumulate_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hess_accumulate_kernel<<<n, 256, lds, st>>>(net, n, l, tan, adj, spp, Hd, accumulate);
  return hipGetLastError();
}

// RK4 of f_F + f_D** with the stage sensitivities.  8 nodes per workgroup, 16
// lanes per node as in the first-order kernel: lane c < 10 carries state column
// 3 + c, lanes 10..13 input column c - 10, lane 14 writes x_{k+1}, lane 15 A's
// position columns.  Per stage: dz (the 10 state entries of z_0; u is held at
// u_k), the residual value f_D-bar + J dz + dz^T H dz / 2 and its effective
// Jacobian J + H dz, which multiplies the tangent.
constexpr int kQNodes = 8;
constexpr int kQStride = 13 + 4 + 6 + 84 + 1176 + 1;  // x | u | y | J | H | pad
__constant__ int kZToX[10] = {7, 8, 9, 10, 11, 12, 3, 4, 5, 6};

__global__ void __launch_bounds__(128)
rk4_quadratic_kernel(int n, QuadConst P, float dt, const float* __restrict__ x, const float* __restrict__ u,
                     const float* __restrict__ fD, const float* __restrict__ JD, const float* __restrict__ HD,
                     float* __restrict__ xn, float* __restrict__ A, float* __restrict__ B) {
  __shared__ float sm[kQNodes * kQStride];
  const int tid = threadIdx.x;
  const int node0 = blockIdx.x * kQNodes;
  const int nn = min(kQNodes, n - node0);
  if (nn <= 0) return;
  for (int i = tid; i < nn * kNx; i += 128) sm[(i / kNx) * kQStride + (i % kNx)] = x[(size_t)node0 * kNx + i];
  for (int i = tid; i < nn * kNu; i += 128) sm[(i / kNu) * kQStride + 13 + (i % kNu)] = u[(size_t)node0 * kNu + i];
  for (int i = tid; i < nn * kDout; i += 128) sm[(i / kDout) * kQStride + 17 + (i % kDout)] = fD[(size_t)node0 * kDout + i];
  for (int i = tid; i < nn * 84; i += 128) sm[(i / 84) * kQStride + 23 + (i % 84)] = JD[(size_t)node0 * 84 + i];
  for (int i = tid; i < nn * 1176; i += 128) sm[(i / 1176) * kQStride + 107 + (i % 1176)] = HD[(size_t)node0 * 1176 + i];
  __syncthreads();
  const int ln = tid >> 4, c = tid & 15;
  const bool active = ln < nn;
  const int node = node0 + ln;
  const float* s = sm + (active ? ln : 0) * kQStride;
  const float* xk = s;
  const float* uk = s + 13;
  const float* yb = s + 17;
  const float* J = s + 23;    // [6][14]
  const float* Hs = s + 107;  // [6][14][14]
  const int xcol = c < 10 ? 3 + c : -1;
  const int ucol = (c >= 10 && c < 14) ? c - 10 : -1;
  const float h = P.arm * 0.70710678118654752f;
  const QuadInv I = quad_inv(P);
  float xs[13], kp[13], ks[13], dk[13], dkp[13], ds[13], accx[13], accd[13];
#pragma unroll
  for (int i = 0; i < 13; ++i) { accx[i] = 0.f; accd[i] = 0.f; kp[i] = 0.f; dkp[i] = 0.f; }
  const float cst[4] = {0.f, 0.5f, 0.5f, 1.f};
  const float wst[4] = {1.f, 2.f, 2.f, 1.f};
  for (int st = 0; st < 4; ++st) {
    const float cdt = cst[st] * dt;
#pragma unroll
    for (int i = 0; i < 13; ++i) {
      xs[i] = xk[i] + cdt * kp[i];
      ds[i] = ((i == xcol) ? 1.f : 0.f) + cdt * dkp[i];
    }
    float dz[10];
#pragma unroll
    for (int i = 0; i < 10; ++i) dz[i] = xs[kZToX[i]] - xk[kZToX[i]];
    nominal_rhs(xs, uk, P, I, ks);
    nominal_tangent(xs, uk, P, I, ds, dk);
    for (int j = 0; j < 6; ++j) {
      const float* Jj = J + j * kDin;
      const float* Hj = Hs + j * kDin * kDin;
      float val = yb[j], tv = 0.f;
      for (int a = 0; a < 10; ++a) {
        float ja = Jj[a], hz = 0.f;  // effective Jacobian entry J + H dz, and (H dz)_a
        for (int b = 0; b < 10; ++b) hz += Hj[a * kDin + b] * dz[b];
        val += (Jj[a] + 0.5f * hz) * dz[a];
        tv += (ja + hz) * ds[kZToX[a]];
      }
      if (ucol >= 0) {
        float hz = 0.f;
        for (int b = 0; b < 10; ++b) hz += Hj[(10 + ucol) * kDin + b] * dz[b];
        tv += Jj[10 + ucol] + hz;
      }
      ks[7 + j] += val;
      dk[7 + j] += tv;
    }
    if (ucol >= 0) {
      const float sx[4] = {-1.f, -1.f, 1.f, 1.f}, sy[4] = {-1.f, 1.f, 1.f, -1.f}, sz[4] = {-1.f, 1.f, -1.f, 1.f};
      const float qw = xs[3], qx = xs[4], qy = xs[5], qz = xs[6];
      dk[7] += 2.f * (qx * qz + qw * qy) * I.m;
      dk[8] += 2.f * (qy * qz - qw * qx) * I.m;
      dk[9] += (qw * qw - qx * qx - qy * qy + qz * qz) * I.m;
      dk[10] += h * sx[ucol] * I.Jx;
      dk[11] += h * sy[ucol] * I.Jy;
      dk[12] += P.c_tau * sz[ucol] * I.Jz;
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
  if (active && c < 14) {
    if (xcol >= 0) {
      float* Ab = A + (size_t)node * kNx * kNx + xcol;
#pragma unroll
      for (int i = 0; i < 13; ++i) Ab[i * kNx] = ((i == xcol) ? 1.f : 0.f) + dt6 * accd[i];
    } else {
      float* Bb = B + (size_t)node * kNx * kNu + ucol;
#pragma unroll
      for (int i = 0; i < 13; ++i) Bb[i * kNu] = dt6 * accd[i];
    }
  } else if (active && c == 14) {
#pragma unroll
    for (int i = 0; i < 13; ++i) xn[(size_t)node * kNx + i] = xk[i] + dt6 * accx[i];
  } else if (active) {
    float* Ab = A + (size_t)node * kNx * kNx;
#pragma unroll
    for (int i = 0; i < 13; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) Ab[i * kNx + j] = (i == j) ? 1.f : 0.f;
  }
}

hipError_t launch_rk4_quadratic(int n, const QuadConst& q, float dt, const float* x, const float* u, const float* fD,
                                const float* JD, const float* HD, float* xn, float* A, float* B, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  rk4_quadratic_kernel<<<(n + kQNodes - 1) / kQNodes, 128, 0, st>>>(n, q, dt, x, u, fD, JD, HD, xn, A, B);
  return hipGetLastError();
}

}  // namespace rtn
