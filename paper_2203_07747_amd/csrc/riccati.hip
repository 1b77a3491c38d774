// Feedback phase: batched backward Riccati recursion in fp64 (Sec. IV-B; QP of
// Sec. IV-A with the continuity condition eq. (2) and the quadratic cost of
// Sec. VI).  For each instance, from P_N = Q_N, p_N = q_N and k = N-1 down to 0:
//
//   Qxx = Q + A^T P A,  Quu = R + B^T P B,  Qux = B^T P A,   g = P c + p
//   qx  = q + A^T g,    qu  = r + B^T g
//   K   = -Quu^{-1} Qux,  kff = -Quu^{-1} qu               (Cholesky of the 4x4 Quu)
//   P  <- sym(Qxx + Qux^T K),  p <- qx + Qux^T kff
//
// One 64-lane workgroup per instance; the 13x13 matrices live in LDS in fp64.
// The products (P A, P [B | c], A^T and B^T times those, Qux^T K) run on fp64
// MFMA 16x16x4 with the matrices padded to 16 x 16; the 4x4 Cholesky solve on
// the lanes.  The recursion is sequential in k, so instances (not nodes) are
// the parallel axis.
#include <hip/hip_runtime.h>

#include "common.h"
#include "mlp_chain.h"

namespace rtn {

constexpr int NX = 13, NU = 4;
typedef double f64x4 __attribute__((ext_vector_type(4)));

struct RiccatiArgs {
  const int* offsets;   // [n_inst + 1]
  const double* Q;      // 13x13
  const double* R;      // 4x4
  const double* QN;     // 13x13
  const float* A;       // [n][13][13]
  const float* B;       // [n][13][4]
  const double* c;      // nullable [n][13]
  const double* q;      // nullable [n][13]
  const double* r;      // nullable [n][4]
  const double* qN;     // nullable [n_inst][13]
  double* K;            // [n][4][13]
  double* kff;          // [n][4]
  double* P;            // nullable [n][13][13]
};

// The recursion runs on one wave per workgroup: lanes exchange data through LDS,
// whose operations a wave issues and completes in order, so a wait for those
// (with a compiler memory barrier) orders them; __syncthreads would also wait for
// the next node's global loads, which are meant to stay in flight.
__device__ inline void wave_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

__global__ void __launch_bounds__(64) riccati_kernel(RiccatiArgs a) {
  __shared__ double sQ[NX * NX], sR[NU * NU];
  __shared__ double sA[NX * NX], sB[NX * NU], sP[NX * NX], sPA[NX * NX], sPB[NX * NU];
  __shared__ double sQxx[NX * NX], sQux[NU * NX], sQuu[NU * NU], sK[NU * NX];
  __shared__ double sc[NX], sp[NX], sg[NX], sqx[NX], squ[NU], skff[NU], sq[NX], sr[NU];
  const int inst = blockIdx.x, t = threadIdx.x, r = t & 15, kq = t >> 4;
  const int rc13 = min(r, NX - 1), rc4 = min(r, NU - 1);  // clamped: LDS reads stay unconditional
  const int k0 = a.offsets[inst], k1 = a.offsets[inst + 1];
  for (int i = t; i < NX * NX; i += 64) {
    sQ[i] = a.Q[i];
    sP[i] = a.QN[i];
  }
  for (int i = t; i < NU * NU; i += 64) sR[i] = a.R[i];
  for (int i = t; i < NX; i += 64) sp[i] = a.qN ? a.qN[(size_t)inst * NX + i] : 0.0;
  // node data is loaded into registers one step ahead, so that its global
  // latency overlaps the previous node's arithmetic
  float ra[3] = {}, rb = 0.f;
  double rc = 0.0, rq = 0.0, rr = 0.0;
  // (clamped indices and substitute addresses: every load is issued unconditionally,
  // so that no wait is forced where divergent paths join)
  const bool has_c = a.c != nullptr, has_q = a.q != nullptr, has_r = a.r != nullptr;
  const double* cptr = has_c ? a.c : a.Q;
  const double* qptr = has_q ? a.q : a.Q;
  const double* rptr = has_r ? a.r : a.Q;
  auto load_node = [&](int k) {
#pragma unroll
    for (int j = 0; j < 3; ++j) ra[j] = a.A[(size_t)k * NX * NX + min(t + 64 * j, NX * NX - 1)];
    rb = a.B[(size_t)k * NX * NU + min(t, NX * NU - 1)];
    rc = cptr[(has_c ? (size_t)k * NX : 0) + min(t, NX - 1)];
    rq = qptr[(has_q ? (size_t)k * NX : 0) + min(t, NX - 1)];
    rr = rptr[(has_r ? (size_t)k * NU : 0) + min(t, NU - 1)];
  };
  if (k1 > k0) load_node(k1 - 1);
  __syncthreads();
  for (int k = k1 - 1; k >= k0; --k) {
    // stage the node's data (fp32 A, B promoted exactly); the last barrier of the
    // previous step ended every read of these buffers
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int i = t + 64 * j;
      if (i < NX * NX) sA[i] = (double)ra[j];
    }
    if (t < NX * NU) sB[t] = (double)rb;
    if (t < NX) {
      sc[t] = has_c ? rc : 0.0;
      sq[t] = has_q ? rq : 0.0;
    }
    if (t < NU) sr[t] = has_r ? rr : 0.0;
    if (k > k0) load_node(k - 1);
    wave_sync();
    // P A, P [B | c] on fp64 MFMA 16x16x4 (13 x 13 padded to 16 x 16): lane (r, kq)
    // supplies row / column r at k = 4 s + kq; accumulator v of the lane is element
    // (kq + 4 v, r) (the fp64 form interleaves rows, unlike the fp32 one).  Column 4
    // of the second product gives g = P c + p.
    {
      f64x4 dPA = {}, dPB = {};
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int k = 4 * s4 + kq, kc = min(k, NX - 1);
        const bool kin = k < NX, rin = r < NX;
        const double p0 = sP[rc13 * NX + kc], a0 = sA[kc * NX + rc13], b0 = sB[kc * NU + rc4], c0 = sc[kc];
        const double pk = (rin && kin) ? p0 : 0.0;
        const double ak = (rin && kin) ? a0 : 0.0;
        const double bk = kin ? (r < NU ? b0 : (r == NU ? c0 : 0.0)) : 0.0;
        dPA = __builtin_amdgcn_mfma_f64_16x16x4f64(pk, ak, dPA, 0, 0, 0);
        dPB = __builtin_amdgcn_mfma_f64_16x16x4f64(pk, bk, dPB, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = kq + 4 * v;
        const double spi = sp[min(i, NX - 1)];
        if (i < NX) {
          if (r < NX) sPA[i * NX + r] = dPA[v];
          if (r < NU) sPB[i * NU + r] = dPB[v];
          if (r == NU) sg[i] = dPB[v] + spi;
        }
      }
    }
    wave_sync();
    // A^T and B^T times P A and [P B | g]: Qxx, qx, Qux, Quu, qu
    {
      f64x4 dQxx = {}, dAg = {}, dQux = {}, dBg = {};
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int k = 4 * s4 + kq, kc = min(k, NX - 1);
        const bool kin = k < NX, rin = r < NX;
        const double a0 = sA[kc * NX + rc13], b0 = sB[kc * NU + rc4], p0 = sPA[kc * NX + rc13], q0 = sPB[kc * NU + rc4],
                     g0 = sg[kc];
        const double at = (rin && kin) ? a0 : 0.0;      // A^T[r][k]
        const double bt = (r < NU && kin) ? b0 : 0.0;   // B^T[r][k]
        const double pa = (rin && kin) ? p0 : 0.0;      // (P A)[k][r]
        const double pb = kin ? (r < NU ? q0 : (r == NU ? g0 : 0.0)) : 0.0;
        dQxx = __builtin_amdgcn_mfma_f64_16x16x4f64(at, pa, dQxx, 0, 0, 0);
        dAg = __builtin_amdgcn_mfma_f64_16x16x4f64(at, pb, dAg, 0, 0, 0);
        dQux = __builtin_amdgcn_mfma_f64_16x16x4f64(bt, pa, dQux, 0, 0, 0);
        dBg = __builtin_amdgcn_mfma_f64_16x16x4f64(bt, pb, dBg, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = kq + 4 * v, ic = min(i, NX - 1), i4 = min(i, NU - 1);
        const double q0 = sQ[ic * NX + rc13], qv = sq[ic], r0 = sR[i4 * NU + rc4], rv = sr[i4];
        if (i < NX && r < NX) sQxx[i * NX + r] = q0 + dQxx[v];
        if (i < NX && r == NU) sqx[i] = qv + dAg[v];
        if (i < NU && r < NX) sQux[i * NX + r] = dQux[v];
        if (i < NU && r < NU) sQuu[i * NU + r] = r0 + dBg[v];
        if (i < NU && r == NU) squ[i] = rv + dBg[v];
      }
    }
    wave_sync();
    // K = -Quu^-1 Qux (columns 0..12), kff = -Quu^-1 qu (column 13): each lane
    // factors Quu = L L^T itself and solves its own right-hand side.
    if (t <= NX) {
      double Lc[NU][NU] = {}, il[NU];  // il: reciprocals of the diagonal (one division each)
      bool ok = true;
#pragma unroll
      for (int j = 0; j < NU; ++j) {
        double d = sQuu[j * NU + j];
#pragma unroll
        for (int m = 0; m < j; ++m) d -= Lc[j][m] * Lc[j][m];
        ok = ok && d > 0.0;
        const double ljj = sqrt(d);
        Lc[j][j] = ljj;
        il[j] = 1.0 / ljj;
#pragma unroll
        for (int i = j + 1; i < NU; ++i) {
          double s = 0.5 * (sQuu[i * NU + j] + sQuu[j * NU + i]);
#pragma unroll
          for (int m = 0; m < j; ++m) s -= Lc[i][m] * Lc[j][m];
          Lc[i][j] = s * il[j];
        }
      }
      double y[NU], x[NU];
#pragma unroll
      for (int i = 0; i < NU; ++i) {
        double s = t < NX ? sQux[i * NX + t] : squ[i];
#pragma unroll
        for (int m = 0; m < i; ++m) s -= Lc[i][m] * y[m];
        y[i] = s * il[i];
      }
#pragma unroll
      for (int i = NU - 1; i >= 0; --i) {
        double s = y[i];
#pragma unroll
        for (int m = i + 1; m < NU; ++m) s -= Lc[m][i] * x[m];
        x[i] = s * il[i];
      }
      const double nan = __builtin_nan("");
      for (int i = 0; i < NU; ++i) {
        const double v = ok ? -x[i] : nan;
        if (t < NX) sK[i * NX + t] = v;
        else skff[i] = v;
      }
    }
    wave_sync();
    // outputs of node k and the value function before it
    for (int e = t; e < NU * NX; e += 64) a.K[(size_t)k * NU * NX + e] = sK[e];
    if (t < NU) a.kff[(size_t)k * NU + t] = skff[t];
    {  // P = sym(Qxx + Qux^T K): both Qux^T K and its transpose K^T Qux in one K-step each
      const double q0 = sQux[kq * NX + rc13], k0v = sK[kq * NX + rc13];
      const double qk = r < NX ? q0 : 0.0, kk = r < NX ? k0v : 0.0;
      const f64x4 zero = {};
      const f64x4 dM = __builtin_amdgcn_mfma_f64_16x16x4f64(qk, kk, zero, 0, 0, 0);
      const f64x4 dMT = __builtin_amdgcn_mfma_f64_16x16x4f64(kk, qk, zero, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = kq + 4 * v, j = r, ic = min(i, NX - 1);
        const double xij = sQxx[ic * NX + rc13], xji = sQxx[rc13 * NX + ic];
        if (i < NX && j < NX) {
          const double pv = 0.5 * ((xij + dM[v]) + (xji + dMT[v]));
          sP[i * NX + j] = pv;
          if (a.P) a.P[(size_t)k * NX * NX + i * NX + j] = pv;
        }
      }
    }
    if (t < NX) {
      double s = sqx[t];
      for (int u = 0; u < NU; ++u) s += sQux[u * NX + t] * skff[u];
      sp[t] = s;
    }
    wave_sync();
  }
}

// Forward pass of the LQ solution (the primal step of the same QP): from the
// instance's initial deviation dx_0,
//   du_k = K_k dx_k + kff_k,   dx_{k+1} = A_k dx_k + B_k du_k + c_k.
// One 64-lane workgroup per instance; lane i < 13 owns state row i, lane i < 4
// input row i; the deviation vector lives in LDS between the two half-steps.
__global__ void __launch_bounds__(64)
lq_rollout_kernel(const int* __restrict__ offsets, const float* __restrict__ A, const float* __restrict__ B,
                  const double* __restrict__ c, const double* __restrict__ K, const double* __restrict__ kff,
                  const double* __restrict__ dx0, double* __restrict__ dx, double* __restrict__ du,
                  double* __restrict__ dxN) {
  __shared__ double sx[NX], su[NU];
  const int inst = blockIdx.x, t = threadIdx.x;
  const int k0 = offsets[inst], k1 = offsets[inst + 1];
  if (t < NX) sx[t] = dx0[(size_t)inst * NX + t];
  __syncthreads();
  for (int k = k0; k < k1; ++k) {
    if (t < NX && dx) dx[(size_t)k * NX + t] = sx[t];
    if (t < NU) {
      const double* Kr = K + ((size_t)k * NU + t) * NX;
      double s = kff[(size_t)k * NU + t];
      for (int j = 0; j < NX; ++j) s += Kr[j] * sx[j];
      su[t] = s;
      du[(size_t)k * NU + t] = s;
    }
    __syncthreads();
    double nx = 0.0;
    if (t < NX) {
      const float* Ar = A + ((size_t)k * NX + t) * NX;
      const float* Br = B + ((size_t)k * NX + t) * NU;
      nx = c ? c[(size_t)k * NX + t] : 0.0;
      for (int j = 0; j < NX; ++j) nx += (double)Ar[j] * sx[j];
      for (int j = 0; j < NU; ++j) nx += (double)Br[j] * su[j];
    }
    __syncthreads();
    if (t < NX) sx[t] = nx;
    __syncthreads();
  }
  if (t < NX && dxN) dxN[(size_t)inst * NX + t] = sx[t];
}

hipError_t launch_lq_rollout(int n_inst, const int* offsets, const float* A, const float* B, const double* c,
                             const double* K, const double* kff, const double* dx0, double* dx, double* du,
                             double* dxN, hipStream_t st) {
  if (n_inst <= 0) return hipSuccess;
  lq_rollout_kernel<<<n_inst, 64, 0, st>>>(offsets, A, B, c, K, kff, dx0, dx, du, dxN);
  return hipGetLastError();
}

// Lane `lane`'s value of v, in every lane (lane is a constant, v any double).
__device__ inline double wave_bcast(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane), hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// ---------------------------------------------------------------------------
// Input box lo_k <= du_k <= hi_k (the input rows of eq. (3)) by ADMM on the split
// du = z, z in the box (scaled dual y):
//   du-step: the LQ above with R + rho I and r_k - rho (z_k - y_k) -- the matrix
//            recursion (K_k, P_k) does not change between iterations, so it is
//            computed once (riccati_kernel) and each iteration is one backward pass
//            of the vectors and one rollout;
//   z-step : z_k = clip(a du_k + (1 - a) z_k + y_k, lo_k, hi_k);
//   y-step : y_k += a du_k + (1 - a) z_k_prev - z_k,
// with the over-relaxation a = 1.6 of Boyd et al. (Distributed optimization and
// statistical learning via ADMM, Sec. 3.4.3), which fixes the same minimiser and
// takes fewer iterations than a = 1.  Stops when max |du - z| and
// rho max |z - z_prev| are both below tol.  The returned inputs are z (inside the
// box) and the states rolled out with them; resid reports both measures of the
// last iteration.
struct BoxArgs {
  const int* offsets;
  const float* A;
  const float* B;
  const double* c;   // nullable
  const double* QN;  // 13x13
  const double* Rt;  // 4x4, R + rho I
  const double* q;   // nullable [n][13]
  const double* r;   // nullable [n][4]
  const double* qN;  // nullable [n_inst][13]
  const double* K;   // [n][4][13] of R + rho I
  const double* P;   // [n][13][13] of R + rho I
  const double* dx0; // [n_inst][13]
  const double* lo;  // [n][4]
  const double* hi;  // [n][4]
  double rho, tol;
  int max_iter;
  double* ws;        // [n][44]: Quu^-1 (16), z (4), y (4), kff (4), P_{k+1} c_k (13), pad
  double* du;        // [n][4]
  double* dx;        // nullable [n][13]
  double* dxN;       // nullable [n_inst][13]
  int* iters;        // nullable [n_inst]
  double* resid;     // nullable [n_inst][2]: primal, dual residual of the last iteration
};

constexpr double kBoxRelax = 1.6;

constexpr int kBoxWs = kBoxWsDoubles;

__global__ void __launch_bounds__(64) box_admm_kernel(BoxArgs a) {
  __shared__ double sPB[NX * NU], sQuu[NU * NU], sx[NX];
  const int inst = blockIdx.x, t = threadIdx.x;
  const int k0 = a.offsets[inst], k1 = a.offsets[inst + 1];
  auto Pnext = [&](int k) { return k + 1 < k1 ? a.P + (size_t)(k + 1) * NX * NX : a.QN; };
  // set-up: Quu_k^-1 = (R + rho I + B^T P_{k+1} B)^-1, z_k = clip(0), y_k = 0
  for (int k = k0; k < k1; ++k) {
    const float* Bk = a.B + (size_t)k * NX * NU;
    const double* Pn = Pnext(k);
    if (t < NX * NU) {
      const int m = t / NU, j = t % NU;
      double s = 0.0;
      for (int l = 0; l < NX; ++l) s += Pn[m * NX + l] * (double)Bk[l * NU + j];
      sPB[t] = s;
    }
    __syncthreads();
    if (t < NU * NU) {
      const int i = t / NU, j = t % NU;
      double s = a.Rt[t];
      for (int m = 0; m < NX; ++m) s += (double)Bk[m * NU + i] * sPB[m * NU + j];
      sQuu[t] = s;
    }
    __syncthreads();
    if (t < NU) {  // column t of the inverse: Cholesky solve of Quu x = e_t (symmetrised)
      double L[NU][NU] = {};
      for (int j = 0; j < NU; ++j) {
        double d = sQuu[j * NU + j];
        for (int m = 0; m < j; ++m) d -= L[j][m] * L[j][m];
        L[j][j] = sqrt(d);
        for (int i = j + 1; i < NU; ++i) {
          double s = 0.5 * (sQuu[i * NU + j] + sQuu[j * NU + i]);
          for (int m = 0; m < j; ++m) s -= L[i][m] * L[j][m];
          L[i][j] = s / L[j][j];
        }
      }
      double y[NU], x[NU];
      for (int i = 0; i < NU; ++i) {
        double s = i == t ? 1.0 : 0.0;
        for (int m = 0; m < i; ++m) s -= L[i][m] * y[m];
        y[i] = s / L[i][i];
      }
      for (int i = NU - 1; i >= 0; --i) {
        double s = y[i];
        for (int m = i + 1; m < NU; ++m) s -= L[m][i] * x[m];
        x[i] = s / L[i][i];
      }
      double* w = a.ws + (size_t)k * kBoxWs;
      for (int i = 0; i < NU; ++i) w[i * NU + t] = x[i];
      const double lo = a.lo[(size_t)k * NU + t], hi = a.hi[(size_t)k * NU + t];
      w[16 + t] = fmin(fmax(0.0, lo), hi);
      w[20 + t] = 0.0;
    }
    if (t < NX) {  // P_{k+1} c_k, fixed over the iterations
      double s = 0.0;
      if (a.c)
        for (int l = 0; l < NX; ++l) s += Pn[t * NX + l] * a.c[(size_t)k * NX + l];
      a.ws[(size_t)k * kBoxWs + 28 + t] = s;
    }
    __syncthreads();
  }
  // Iterations: one wave and no barriers.  Lanes 0..12 carry the state-sized
  // vectors (p_k in the backward pass, x_k in the rollout), lanes 16..19 the
  // input-sized ones (the affine term, z, y); the other lanes compute values that
  // are never read.  A value one lane computed reaches the others by readlane, and
  // each lane loads its operands for a node with addresses of its own, all before
  // the node's first product, so a step waits on no barrier and on one memory
  // round trip.  Every sum runs in the order of its definition.
  const bool sl = t < NX, il = t >= 16 && t < 16 + NU;
  const int ti = il ? t - 16 : 0, ts = sl ? t : 0;
  const bool hq = a.q != nullptr, hr = a.r != nullptr, hc = a.c != nullptr;
  const double rho = a.rho;
  int it = 0;
  for (; it < a.max_iter; ++it) {
    // backward pass of the linear terms: g = p_{k+1} + P_{k+1} c_k,
    // (q~, r~) = (q_k + A_k^T g, r_k - rho (z_k - y_k) + B_k^T g),
    // p_k = q~ + K_k^T r~ (state lanes), d_k = -Quu_k^-1 r~ (input lanes)
    double p = sl && a.qN ? a.qN[(size_t)inst * NX + ts] : 0.0;
    for (int k = k1 - 1; k >= k0; --k) {
      const double* w = a.ws + (size_t)k * kBoxWs;
      // column t of A_k or column i of B_k; column t of K_k or row i of Quu_k^-1
      const float* c13p = sl ? a.A + (size_t)k * NX * NX + ts : a.B + (size_t)k * NX * NU + ti;
      const int c13s = sl ? NX : NU;
      const double* c4p = sl ? a.K + (size_t)k * NU * NX + ts : w + ti * NU;
      const int c4s = sl ? NX : 1;
      float c13[NX];
      double c4[NU];
#pragma unroll
      for (int m = 0; m < NX; ++m) c13[m] = c13p[m * c13s];
#pragma unroll
      for (int j = 0; j < NU; ++j) c4[j] = c4p[j * c4s];
      const double qv = hq ? a.q[(size_t)k * NX + ts] : 0.0;
      const double rv = hr ? a.r[(size_t)k * NU + ti] : 0.0;
      const double pc = w[28 + ts], zv = w[16 + ti], yv = w[20 + ti];
      const double g = p + pc;
      double s1 = sl ? qv : rv - rho * (zv - yv);
#pragma unroll
      for (int m = 0; m < NX; ++m) s1 += (double)c13[m] * wave_bcast(g, m);
      double s2 = sl ? s1 : 0.0;
      if (sl) {
#pragma unroll
        for (int j = 0; j < NU; ++j) s2 += c4[j] * wave_bcast(s1, 16 + j);
      } else {
#pragma unroll
        for (int j = 0; j < NU; ++j) s2 -= c4[j] * wave_bcast(s1, 16 + j);
      }
      if (il) a.ws[(size_t)k * kBoxWs + 24 + ti] = s2;
      p = s2;
    }
    // rollout with du_k = d_k + K_k x_k, then the z- and y-steps of node k
    double x = sl ? a.dx0[(size_t)inst * NX + ts] : 0.0;
    double rp = 0.0, rd = 0.0;
    for (int k = k0; k < k1; ++k) {
      double* w = a.ws + (size_t)k * kBoxWs;
      const float* Ar = a.A + (size_t)k * NX * NX + ts * NX;   // row t of A_k
      const float* Br = a.B + (size_t)k * NX * NU + ts * NU;   // row t of B_k
      const double* Kr = a.K + (size_t)k * NU * NX + ti * NX;  // row i of K_k
      double c13[NX];
      float b4[NU];
      if (sl) {
#pragma unroll
        for (int j = 0; j < NX; ++j) c13[j] = (double)Ar[j];
      } else {
#pragma unroll
        for (int j = 0; j < NX; ++j) c13[j] = Kr[j];
      }
#pragma unroll
      for (int j = 0; j < NU; ++j) b4[j] = Br[j];
      const double cv = hc ? a.c[(size_t)k * NX + ts] : 0.0;
      const double dv = w[24 + ti], zv = w[16 + ti], yv = w[20 + ti];
      const double lo = a.lo[(size_t)k * NU + ti], hi = a.hi[(size_t)k * NU + ti];
      double s3 = sl ? cv : dv;
#pragma unroll
      for (int j = 0; j < NX; ++j) s3 += c13[j] * wave_bcast(x, j);
      if (il) {
        const double d = s3;
        const double dr = kBoxRelax * d + (1.0 - kBoxRelax) * zv;  // over-relaxed du
        const double zn = fmin(fmax(dr + yv, lo), hi);
        rp = fmax(rp, fabs(d - zn));
        rd = fmax(rd, rho * fabs(zn - zv));
        w[20 + ti] = yv + (dr - zn);
        w[16 + ti] = zn;
      }
      double s4 = s3;
#pragma unroll
      for (int j = 0; j < NU; ++j) s4 += (double)b4[j] * wave_bcast(s3, 16 + j);
      x = s4;
    }
    double mp = 0.0, md = 0.0;
#pragma unroll
    for (int j = 0; j < NU; ++j) {
      mp = fmax(mp, wave_bcast(rp, 16 + j));
      md = fmax(md, wave_bcast(rd, 16 + j));
    }
    if (t == 0 && a.resid) {
      a.resid[(size_t)inst * 2] = mp;
      a.resid[(size_t)inst * 2 + 1] = md;
    }
    if (mp < a.tol && md < a.tol) {
      ++it;
      break;
    }
  }
  // z was written by the input lanes; the rollout below reads it in the state lanes
  __syncthreads();
  // outputs: the box-feasible inputs z and the states they produce
  if (t < NX) sx[t] = a.dx0[(size_t)inst * NX + t];
  __syncthreads();
  for (int k = k0; k < k1; ++k) {
    const float* Ak = a.A + (size_t)k * NX * NX;
    const float* Bk = a.B + (size_t)k * NX * NU;
    const double* w = a.ws + (size_t)k * kBoxWs;
    if (t < NX && a.dx) a.dx[(size_t)k * NX + t] = sx[t];
    if (t >= 16 && t < 16 + NU) a.du[(size_t)k * NU + (t - 16)] = w[16 + (t - 16)];
    double nx = 0.0;
    if (t < NX) {
      nx = a.c ? a.c[(size_t)k * NX + t] : 0.0;
      for (int j = 0; j < NX; ++j) nx += (double)Ak[t * NX + j] * sx[j];
      for (int j = 0; j < NU; ++j) nx += (double)Bk[t * NU + j] * w[16 + j];
    }
    __syncthreads();
    if (t < NX) sx[t] = nx;
    __syncthreads();
  }
  if (t < NX && a.dxN) a.dxN[(size_t)inst * NX + t] = sx[t];
  if (t == 0 && a.iters) a.iters[inst] = it;
}

hipError_t launch_box_admm(int n_inst, const int* offsets, const float* A, const float* B, const double* c,
                           const double* QN, const double* Rt, const double* q, const double* r, const double* qN,
                           const double* K, const double* P, const double* dx0, const double* lo, const double* hi,
                           double rho, double tol, int max_iter, double* ws, double* du, double* dx, double* dxN,
                           int* iters, double* resid, hipStream_t st) {
  if (n_inst <= 0) return hipSuccess;
  BoxArgs a{offsets, A, B, c, QN, Rt, q, r, qN, K, P, dx0, lo, hi, rho, tol, max_iter, ws, du, dx, dxN, iters, resid};
  box_admm_kernel<<<n_inst, 64, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_riccati(int n_inst, const int* offsets, const double* Q, const double* R, const double* QN,
                          const float* A, const float* B, const double* c, const double* q, const double* r,
                          const double* qN, double* K, double* kff, double* P, hipStream_t st) {
  if (n_inst <= 0) return hipSuccess;
  RiccatiArgs a{offsets, Q, R, QN, A, B, c, q, r, qN, K, kff, P};
  riccati_kernel<<<n_inst, 64, 0, st>>>(a);
  return hipGetLastError();
}

}  // namespace rtn
