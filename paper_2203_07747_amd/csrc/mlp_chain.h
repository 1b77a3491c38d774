// Host-visible interface of the network kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace rtn {

// Device view of a network, passed by value to the kernels.  Layer index i is
// 0-based: fw[i] packs W_{i+1} (M = fan_out, K = fan_in), rw[i] packs W_{i+1}^T
// (M = fan_in, K = fan_out) for the hidden layers i < L.
struct NetView {
  int L;      // hidden layers
  int act;    // 0 SiLU, 1 identity
  int input;  // network input: 0 [v, w, q, u]; 1 v_B; 2 [v_B, u] (v_B in slots 0..2, u in 10..13)
  const void* fw[17];
  const void* rw[16];
  const float* bias[17];
  const float* w_out;   // fp32 W_{L+1} [6][H]
  const float* w_out_s; // the same, each row in stash order (element stash_pos(k) holds column k)
  const float* wscale;  // fp8: dequantisation scale of W_1..W_{L+1} (L+1)
  const float* ascale;  // fp8: scale of the forward operands z_0, h_1..h_L (L+1)
  const float* gscale;  // fp8: scale of the reverse operands G_1..G_L (L)
};

template <int P> struct StashT { using type = uint16_t; };
template <> struct StashT<0> { using type = float; };

int pack_geometry(int prec, int M, int K, int* MT, int* KS);
// Pack matrices of one precision into MFMA fragment order, in one launch (at
// most 34): each W fp32 row-major [M or K rows][cols], trans selects W^T.
struct PackSpec {
  const float* W;
  int cols, M, K, trans;
  const float* scale;
  void* out;
};
hipError_t launch_pack_layers(int prec, int n, const PackSpec* specs, hipStream_t st);
hipError_t launch_amax(const float* a, long n, float* out, hipStream_t st);
hipError_t launch_amax_to_scale(float* s, int n, hipStream_t st);
// Launch configuration of a layer-chain kernel: tile variant (0 = default
// shape, 1..4 = alternative shapes, widths 512 and 1024 only) and workgroup
// count (0 = two per compute unit; never more than there are row blocks).
struct ChainCfg {
  int variant = 0;
  int grid = 0;
};
constexpr int kChainVariants = 5;
// Tile shape of a (precision, width, direction, variant): whether it exists,
// waves per workgroup, rows per workgroup, and (when `occupancy` is set; this
// asks the device) workgroups resident per compute unit, else 0.
struct ChainGeom {
  int valid, waves, rows, resident_per_cu;
};
hipError_t chain_geometry(int prec, int H, int rev, int variant, int occupancy, ChainGeom* g);
hipError_t launch_mlp_forward(int prec, int H, const NetView& net, int n, const float* x, const float* u,
                              const float* zin, void* stash, float* y, float* amax, hipStream_t st,
                              float* hsave = nullptr, const ChainCfg& cfg = ChainCfg());
hipError_t launch_mlp_reverse(int prec, int H, const NetView& net, int n, const void* stash, float* J, float* amax,
                              hipStream_t st, const ChainCfg& cfg = ChainCfg());
// per-precision instantiations (chain_fp32.hip, chain_bf16.hip, chain_fp8.hip)
template <int P>
hipError_t chain_forward(int H, const ChainCfg& cfg, const NetView& net, int n, const float* x, const float* u,
                         const float* zin, void* stash, float* y, float* amax, float* hsave, hipStream_t st);
template <int P>
hipError_t chain_reverse(int H, const ChainCfg& cfg, const NetView& net, int n, const void* stash, float* J,
                         float* amax, hipStream_t st);
template <int P> hipError_t chain_geom(int H, int rev, int V, int occupancy, ChainGeom* g);
int stash_elem_bytes(int prec);
int num_cu();  // compute units of the current device (cached after the first call)
hipError_t launch_reorder_out(const float* W, int H, float* out, hipStream_t st);

// Small-batch per-layer path (layer_lat.hip), fp32 master weights: W[l] is
// W_{l+1} row-major [fan_out][fan_in], W[L] the output layer.
struct QuadConst {
  float mass, Jx, Jy, Jz, arm, c_tau, g;
};

struct LatNet {
  int L, H, act, input;
  const float* W[17];
  const float* b[17];
};
// act: [2][n][H] ping-pong activations; sp: [L][n][H] activation derivatives;
// g: [2][6n][H] ping-pong cotangents; y [n][6]; J [n][6][14] (y, J nullptr: the
// output layer / the J_D layer is left to launch_lat_tail).
// spp (nullable): act''(a) [L][n][H]; adj (nullable): dy/dh_l [L-1][6n][H] for the
// hidden layers below the last (dy/dh_L is W_{L+1}).
hipError_t launch_lat_forward(const LatNet& net, int n, const float* x, const float* u, float* act, float* sp, float* y,
                              hipStream_t st, float* spp = nullptr);
hipError_t launch_lat_reverse(const LatNet& net, int n, const float* sp, float* g, float* J, hipStream_t st,
                              float* adj = nullptr);
hipError_t launch_lat_tangent(const LatNet& net, int n, int l, const float* sp, float* tan, hipStream_t st);
// Width 64 and <= 4 hidden layers: value y [n][6] and Jacobian J [n][6][14] in one
// launch (16 nodes per workgroup, every operand in LDS); with rk4 given, the RK4
// step of launch_rk4_linearize follows in the same launch.
struct FusedRk4 {
  QuadConst P;
  float dt;
  float* xn;  // nullptr: network only
  float* A;
  float* B;
  uint8_t* status;  // nullable
};
bool lat_fused_fits(const LatNet& net);
// Width 128..1024 with L >= 2: J_D (from G_1 = g + 6 n H, left there by
// launch_lat_reverse with J = nullptr), y (from the last activations in act, left
// by launch_lat_forward with y = nullptr) and the RK4 step, one launch.
bool lat_tail_fits(const LatNet& net);
hipError_t launch_lat_tail(const LatNet& net, int n, const float* act, const float* g, const float* x, const float* u,
                           float* y, float* J, const FusedRk4& rk, hipStream_t st);
hipError_t launch_lat_fused(const LatNet& net, int n, const float* x, const float* u, float* y, float* J,
                            hipStream_t st, const FusedRk4* rk4 = nullptr);
// H_D [n][6][14][14] (+)= T_l^T diag(dy/dh_l (.) act''(a_l)) T_l for layer l (0-based);
// T_0 = W_1, dy/dh_{L-1} = W_{L+1}; accumulate = 0 for the first layer visited.
hipError_t launch_hess_accumulate(const LatNet& net, int n, int l, const float* tan, const float* adj,
                                  const float* spp, float* Hd, int accumulate, hipStream_t st);

hipError_t launch_rk4_quadratic(int n, const QuadConst& q, float dt, const float* x, const float* u, const float* fD,
                                const float* JD, const float* HD, float* xn, float* A, float* B, hipStream_t st);
// input: network input variant of JD's columns (0 full; 1, 2 body velocity)
hipError_t launch_rk4_linearize(int n, const QuadConst& q, float dt, const float* x, const float* u, const float* fD,
                                const float* JD, float* xn, float* A, float* B, uint8_t* status, hipStream_t st,
                                int input = 0);
// The same step for small batches, 16 nodes per workgroup (the latency form of
// the per-node routine: shortest dependency chain instead of fewest instructions).
hipError_t launch_rk4_lanes(int n, const QuadConst& q, float dt, const float* x, const float* u, const float* fD,
                            const float* JD, float* xn, float* A, float* B, uint8_t* status, hipStream_t st,
                            int input = 0);

hipError_t launch_rk4_exact_stage(int n, int stage, const QuadConst& q, float dt, const float* x, const float* u,
                                  const float* fD, const float* JD, float* xs, float* kp, float* kacc, float* dkp,
                                  float* dacc, float* xn, float* A, float* B, hipStream_t st);
hipError_t launch_lq_rollout(int n_inst, const int* offsets, const float* A, const float* B, const double* c,
                             const double* K, const double* kff, const double* dx0, double* dx, double* du,
                             double* dxN, hipStream_t st);
constexpr int kBoxWsDoubles = 44;  // per node ADMM state of launch_box_admm
hipError_t launch_box_admm(int n_inst, const int* offsets, const float* A, const float* B, const double* c,
                           const double* QN, const double* Rt, const double* q, const double* r, const double* qN,
                           const double* K, const double* P, const double* dx0, const double* lo, const double* hi,
                           double rho, double tol, int max_iter, double* ws, double* du, double* dx, double* dxN,
                           int* iters, double* resid, hipStream_t st);
hipError_t launch_riccati(int n_inst, const int* offsets, const double* Q, const double* R, const double* QN,
                          const float* A, const float* B, const double* c, const double* q, const double* r,
                          const double* qN, double* K, double* kff, double* P, hipStream_t st);

// C (+)= A B for A(m,k) = A[m*sAm + k*sAk], B(k,n) = B[k*sBk + n*sBn], C row stride
// sCm; Cone (nullable) (+)= the product with an all-ones column of B (column sums
// of A); gate (nullable): result *= act'(m, n) from a stash [M][ldg] in stash
// order; part (nullable): split-K scratch of gemm_part_floats(M, N, K) floats.
hipError_t launch_gemm(int prec, int M, int N, int K, const float* A, long sAm, long sAk, const float* B, long sBk,
                       long sBn, float* C, long sCm, float* Cone, int accumulate, const void* gate, int gate_is_f32,
                       int ldg, float* part, hipStream_t st);
int gemm_splits(int M, int N, int K);
inline long gemm_part_floats(int M, int N, int K) { return (long)gemm_splits(M, N, K) * M * (N + 1); }
hipError_t launch_mse(int nel, const float* y, const float* t, float* dy, float* loss, hipStream_t st);
hipError_t launch_adam(long n, float* p, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                       float bc1, float bc2, hipStream_t st);

}  // namespace rtn
