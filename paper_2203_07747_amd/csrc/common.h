// Shared device/host definitions of the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtn {

constexpr int kWave = 64;
constexpr int kMaxHidden = 16;
constexpr int kDin = 14;
constexpr int kDout = 6;
constexpr int kNx = 13;
constexpr int kNu = 4;

enum Prec : int { P_FP32 = 0, P_BF16 = 1, P_FP8 = 2 };

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Operand slot order.
//
// Every MFMA used here is a 32x32 tile: lane l of a wave supplies row (A) or
// column (B) l % 32 and a group g = l / 32 of consecutive "slots" along the
// reduction dimension.  A dot product does not care in which order the
// reduction index is visited, so A and B only have to agree on which feature
// sits in which (group, slot).  We choose the order in which a 32x32 fp32
// accumulator holds its rows: accumulator register i of lane l holds row
// (i/4)*8 + g*4 + i%4.  With K-slots numbered the same way, the accumulator of
// one layer is, register for register, the operand of the next layer and can be
// written to LDS without a transpose.
//
// slot_feature(q, g): feature index of per-lane slot q (counted along K across
// all K-steps) in lane group g.
__host__ __device__ inline int slot_feature(int q, int g) {
  return 32 * (q >> 4) + ((q & 15) >> 2) * 8 + g * 4 + (q & 3);
}

// Network input feature k (0..13) of one node, xr = x row (13), ur = u row (4).
// input 0: z = [v, omega, q, u].  Inputs 1 and 2 are the simplified residual
// models of Sec. VI, fed the body-frame velocity v_B = conj(q) (.) v = R(q)^T v
// (homogeneous in q, like every q (.) v product of eq. (6)) in slots 0..2 and,
// for input 2, u in slots 10..13; every other slot is zero.
__device__ inline float net_feature(const float* __restrict__ xr, const float* __restrict__ ur, int k, int input) {
  if (input == 0) {
    if (k < 6) return xr[7 + k];
    if (k < 10) return xr[3 + (k - 6)];
    return ur[k - 10];
  }
  if (k < 3) {
    const float w = xr[3], a = xr[4], b = xr[5], c = xr[6];
    const float v0 = xr[7], v1 = xr[8], v2 = xr[9];
    if (k == 0) return (w * w + a * a - b * b - c * c) * v0 + 2.f * (a * b + w * c) * v1 + 2.f * (a * c - w * b) * v2;
    if (k == 1) return 2.f * (a * b - w * c) * v0 + (w * w - a * a + b * b - c * c) * v1 + 2.f * (b * c + w * a) * v2;
    return 2.f * (a * c + w * b) * v0 + 2.f * (b * c - w * a) * v1 + (w * w - a * a - b * b + c * c) * v2;
  }
  if (input == 2 && k >= 10) return ur[k - 10];
  return 0.f;
}

// Inverse for one 32-feature tile: position of feature k in "stash order"
// (tile, group, register), used for per-feature side arrays (the activation
// derivative stash) that are read by the same lane mapping.
__host__ __device__ inline int stash_pos(int k) {
  int t = k >> 5, r = k & 31;
  int g = (r >> 2) & 1;
  int i = (r >> 3) * 4 + (r & 3);
  return t * 32 + g * 16 + i;
}

// MFMA traits per precision.  E = K-slots per lane per instruction, KSTEP = K
// per instruction, KALIGN = padding granule of a reduction dimension.
template <int P> struct Mfma;

template <> struct Mfma<P_FP32> {
  using elem = float;
  using frag = float;
  static constexpr int E = 1, KSTEP = 2, KALIGN = 16;
  __device__ static inline f32x16 mma(frag a, frag b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
};

template <> struct Mfma<P_BF16> {
  using elem = uint16_t;
  using frag = bf16x8;
  static constexpr int E = 8, KSTEP = 16, KALIGN = 16;
  __device__ static inline f32x16 mma(frag a, frag b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};

template <> struct Mfma<P_FP8> {
  using elem = uint8_t;
  using frag = i32x8;
  static constexpr int E = 32, KSTEP = 64, KALIGN = 64;
  __device__ static inline f32x16 mma(frag a, frag b, f32x16 c) {
    // format 0 = FP8 E4M3 for both operands; block scales 127 = 2^0 (unscaled)
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 127, 0, 127);
  }
};

__host__ __device__ inline int round_up(int a, int b) { return (a + b - 1) / b * b; }

// Conversions used when writing operands --------------------------------------
// Round to nearest even (gfx950 converts in hardware: v_cvt_pk_bf16_f32).
__device__ inline uint16_t f32_to_bf16_rne(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ inline uint32_t pack_bf16x2(float lo, float hi) {
  typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
  bf16x2_t v = {(__bf16)lo, (__bf16)hi};
  return __builtin_bit_cast(uint32_t, v);
}
__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// Two floats -> two OCP E4M3 bytes (finite values saturated to +-448, round to
// nearest even; a NaN stays NaN, so a poisoned operand still reaches the status check).
__device__ inline float sat448(float a) { return a != a ? a : fminf(fmaxf(a, -448.f), 448.f); }
__device__ inline uint32_t f32x2_to_e4m3(float a, float b) {
  a = sat448(a);
  b = sat448(b);
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false) & 0xffffu;
}

template <int P> __device__ inline typename Mfma<P>::elem to_elem(float v, float inv_scale);
template <> __device__ inline float to_elem<P_FP32>(float v, float) { return v; }
template <> __device__ inline uint16_t to_elem<P_BF16>(float v, float) { return f32_to_bf16_rne(v); }

// max(|v|) into *p (calibration); non-negative floats order like their bit patterns
__device__ inline void atomic_amax(float* p, float v) {
  atomicMax(reinterpret_cast<unsigned int*>(p), __float_as_uint(fabsf(v)));
}

}  // namespace rtn
