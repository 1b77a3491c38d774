// Kernels of the double-integrator runtime workload (Sec. V): a 2-input,
// 2-output residual network of any width, evaluated with its Jacobian by
// forward-mode tangents in the same weight sweep, and one real-time iteration
// (RK4 linearisation, Riccati recursion, rollout) per instance.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtn {

constexpr int kDiMaxHidden = 64;
constexpr int kDiMaxWidth = 8192;
constexpr int kDiMaxHorizon = 512;  // nodes per instance in one real-time iteration

// Activations of a node batch: three rows per node, [value h_l; dh_l/dp; dh_l/dv],
// for widths that are a multiple of 8 in MFMA operand order (node tiles of 10
// nodes padded to 32 rows), else row-major [3n][width]; di_z_floats is the size.
inline bool di_packed(int H) { return H % 8 == 0; }
size_t di_z_floats(int n, int H);
// Hidden weights W [H][H] (row-major) -> the operand order of the packed path,
// (H+31)/32 * 32 * H floats, zero padded (host).
void di_pack_weight(const float* W, int H, float* out);
inline size_t di_packed_weight_floats(int H) { return (size_t)(H + 31) / 32 * 32 * H; }
hipError_t launch_di_first_layer(int n, int H, const float* W, const float* b, int act, const float* x, float* Z,
                                 hipStream_t st);
// Wide layers split K into di_slices(n, H) slices (one workgroup each) to fill
// the device; a second kernel adds their partial tiles (di_partial_floats of
// scratch) in slice order.
int di_slices(int n, int H);
size_t di_partial_floats(int n, int H);
hipError_t launch_di_hidden_layer(int n, int H, const float* Zin, const float* W, const float* b, int act,
                                  float* Zout, float* partial, hipStream_t st);
hipError_t launch_di_output_layer(int n, int K, const float* W, const float* b, const float* Z, float* y, float* J,
                                  hipStream_t st);
// Per node RK4 step of the nominal model plus the affine residual (y, J nullable = 0).
hipError_t launch_di_linearize(int n, float dt, const float* x, const float* u, const float* y, const float* J,
                               float* xn, float* A, float* B, hipStream_t st);

struct DiCost {
  double Q[4], R, QN[4];
};
// One real-time iteration per instance (one workgroup each); A, B, xn nullable.
hipError_t launch_di_rti(int n_inst, const int* offsets, float dt, const DiCost& cost, const float* x, const float* u,
                         const float* xN, const float* x0, const float* xref, const float* y, const float* J,
                         double* du, double* dx, double* dxN, float* A, float* B, float* xn, hipStream_t st);

// The whole iteration in one workgroup per instance for small networks
// (di_fused_fits: width <= 64, <= 64 nodes per instance).  `fused` holds
// W_1, b_1, then W_l^T (k-major), b_l for the hidden layers, then W_out, b_out;
// woff [2L + 2] (device) their offsets.
bool di_fused_fits(int H, int max_horizon);
hipError_t launch_di_fused(int n_inst, const int* offsets, int L, int H, int act, const float* fused,
                           const long* woff, float dt, const DiCost& cost, const float* x, const float* u,
                           const float* xN, const float* x0, const float* xref, double* du, double* dx, double* dxN,
                           float* A, float* B, float* xn, hipStream_t st);

}  // namespace rtn
