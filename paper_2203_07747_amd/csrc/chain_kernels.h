// Residual network value and Jacobian on matrix cores (gfx950).
//
// Sec. IV-A evaluates the learned dynamics and its Jacobian for all shooting
// nodes as one batch.  Here the batch is a matrix of rows (one row per node for
// the forward pass, six rows per node -- one per network output -- for the
// reverse/adjoint sweep) and every layer is a product with the same weight
// matrix, so the whole batch is a chain of GEMMs.
//
// Layer-chain kernels.  One workgroup owns a block of R rows and carries it
// through every layer: the block's activations (forward) or cotangents
// (reverse) live in LDS as the B operand, each wave streams its slice of the
// weight matrix (the A operand) from L2, and the fp32 accumulators of a layer
// are written straight back to LDS as the next layer's operand.  We compute the
// transposed product C^T = W . H^T so that an accumulator register already is
// an operand slot (see slot_feature in common.h) and the write-back needs no
// transpose.  Weights are stored pre-packed in exact fragment order, so every
// weight load is one contiguous 64-lane vector load.
//
//   forward  : a_l = W_l h_{l-1} + b_l, h_l = act(a_l); stash act'(a_l); y = W_{L+1} h_L + b_{L+1}
//   reverse  : G_L = W_{L+1} * act'(a_L) (per node, 6 rows); G_{l-1} = (G_l W_l) * act'(a_{l-1});
//              J_D = G_1 W_1            (chain rule: J_D = W_{L+1} D_L W_L ... D_1 W_1)
//
// The activation-derivative stash goes through HBM between the two kernels
// (L * H values per node).
#pragma once

#include <type_traits>

#include "common.h"
#include "mlp_chain.h"

namespace rtn {

// Rows per workgroup and waves per workgroup for a (precision, width) pair.
// Limits: the B operand of R rows x H features (plus the staged activation
// derivatives of the reverse sweep) must fit in the 160 KB of LDS, and each
// wave's accumulators (H/32/NW M-tiles x R/32 row tiles x 16 floats) must fit its
// registers: <= 128 with two waves per SIMD (8 waves), <= 192 with one wave per
// SIMD (4 waves), where the accumulators live in AGPRs.
template <int P, int H, bool REV> struct ChainShapeDefault {
  // the reverse sweep keeps one wave per SIMD (big accumulator tile, staged act'
  // rows); the forward pass, whose epilogue (SiLU) is transcendental-heavy, keeps
  // two waves per SIMD so one wave's epilogue overlaps the other's matrix work
  static constexpr bool ONE_PER_SIMD = REV && P == P_BF16 && H == 512;
  static constexpr int NW = ONE_PER_SIMD ? 4 : (H >= 256 ? 8 : H / 32);
  static constexpr int R = P == P_FP32 ? (H <= 256 ? 128 : (H == 512 ? 64 : 32))
                         : P == P_BF16 ? (H <= 256 ? 128 : (H == 512 ? (REV ? 96 : 64) : 64))
                                       : (H <= 256 ? 128 : 64);
};

// Variant V = 0 is the default shape above; V = 1 and 2 are alternatives the
// autotuner may pick instead (widths 512 and 1024 only):
//   V = 1: default with one wave per SIMD       -> two waves per SIMD, 64 rows;
//          bf16/fp8 width 512, two waves per SIMD -> one wave per SIMD, 96 rows;
//          otherwise                             -> the same waves, half the rows
//   V = 2: one wave per SIMD with half the register file and at most 80 KB of
//          LDS (64 rows, else 32), so that two workgroups share a compute unit
//          and one's epilogue overlaps the other's matrix work.
//   V = 3: reverse, bf16/fp8 width 512: one wave per SIMD, 128 rows, all 256
//          accumulator registers in use -- a quarter less weight traffic from
//          L2 per matrix product than 96 rows.
//   V = 4: bf16/fp8 width 512: 128 rows over 8 waves (two per SIMD, each 2
//          M-tiles x 4 row tiles), one workgroup per CU: half the weight
//          traffic of two 64-row workgroups, and a 4-step weight ring.
//   V = 5, 6: bf16/fp8 width 512: variant 4 with 64 or 96 rows (2 or 3 row tiles
//          per wave).  Not choices of their own: variant 4 runs its last, partly
//          filled round of blocks in one of these shapes on all workgroups.
// OCC is the number of waves per SIMD the register budget is sized for.
template <int P, int H, bool REV = true, int V = 0> struct ChainShape {
  using D = ChainShapeDefault<P, H, REV>;
  static constexpr bool ALT_ONE = !D::ONE_PER_SIMD && H == 512 && P != P_FP32;
  static constexpr int ESZ = P == P_FP32 ? 4 : (P == P_BF16 ? 2 : 1);
  static constexpr int SPE = P == P_FP32 ? 4 : 2;
  // operand rows + (reverse) staged derivatives of a 64-row block within 80 KB
  static constexpr bool FITS64 = 64 * H * ESZ + (REV ? 12 * (H + 16 / SPE) * SPE : 0) <= 80 * 1024 &&
                                 (H / 32 / 4) * 2 * 16 <= 128;
  static constexpr int R2 = FITS64 ? 64 : 32;
  static constexpr int NW =
      V == 0 ? D::NW : V == 1 ? (D::ONE_PER_SIMD ? 8 : (ALT_ONE ? 4 : D::NW)) : V >= 4 ? 8 : 4;
  static constexpr int R = V == 0   ? D::R
                           : V == 1 ? (D::ONE_PER_SIMD ? 64 : (ALT_ONE ? 96 : D::R / 2))
                           : V == 2 ? R2
                           : V == 5 ? 64
                           : V == 6 ? 96
                                    : 128;
  static constexpr int OCC = V == 2 ? 2 : (NW <= 4 ? 1 : 2);
  static constexpr bool VALID =
      V == 0 || (V == 1 && H >= 512 && R >= 32) ||
      (V == 2 && H >= 512 && R * H * ESZ + (REV ? 7 * (H + 16 / SPE) * SPE : 0) <= 80 * 1024 &&
       (H / 32 / 4) * (R / 32) * 16 <= 128) ||
      (V == 3 && REV && H == 512 && P != P_FP32) || (V == 4 && H == 512 && P != P_FP32) ||
      ((V == 5 || V == 6) && H == 512 && P != P_FP32);
};

// OCC: waves per SIMD the kernel is built for (1: the whole register file and,
// with 4 waves, the whole LDS; 2: half of each when the workgroup has 4 waves).
template <int P, int H, int R, int NW, int OCC = (NW <= 4 ? 1 : 2)> struct Chain {
  static constexpr int kOcc = OCC;
  using M = Mfma<P>;
  using elem = typename M::elem;
  using frag = typename M::frag;
  static constexpr int E = M::E, KSTEP = M::KSTEP;
  static constexpr int RT = R / 32;
  static constexpr int MT = H / 32;
  static constexpr int MTW = MT / NW;
  static constexpr int KS_H = H / KSTEP;
  static constexpr int K1 = (kDin + M::KALIGN - 1) / M::KALIGN * M::KALIGN;
  static constexpr int KS_1 = K1 / KSTEP;
  static constexpr int B_BYTES = R * H * (int)sizeof(elem);
  static constexpr int PART_BYTES = NW * R * 16 * 4;
  static constexpr int LDS_BYTES = B_BYTES > PART_BYTES ? B_BYTES : PART_BYTES;
  // reverse sweep: the activation derivatives of the nodes a row block touches;
  // a block may start at any row (the tail launches), so R rows from offset 5
  // within a node reach floor((R + 4) / 6) + 1 nodes
  static constexpr int SP_NODES = (R + 4) / 6 + 1;
  static constexpr int SP_ELEM = P == P_FP32 ? 4 : 2;
  static constexpr int SPS = H + 16 / SP_ELEM;  // LDS row stride (elements): 16-byte pad against bank conflicts
  static constexpr int SP_BYTES = SP_NODES * SPS * SP_ELEM;
  static constexpr int SP_ROW_CHUNKS = H * SP_ELEM / 16;
  static constexpr int SP_CHUNKS_PER_THREAD = (SP_NODES * SP_ROW_CHUNKS + NW * kWave - 1) / (NW * kWave);
  // output weights stay resident in LDS for the whole kernel when they fit
  static constexpr int WOS = H + 4;  // LDS row stride (floats): 16-byte pad against bank conflicts
  static constexpr int LDS_CAP = 160 * 1024 * NW / (4 * OCC);
  static constexpr bool WO_IN_LDS = LDS_BYTES + SP_BYTES + kDout * WOS * 4 <= LDS_CAP;
  static constexpr int WO_BYTES = WO_IN_LDS ? kDout * WOS * 4 : 0;
  static constexpr int REV_LDS_BYTES = LDS_BYTES + SP_BYTES + WO_BYTES;
  static_assert(MT % NW == 0, "width must split evenly over the waves");
  static_assert(MTW * RT * 16 <= (OCC == 1 ? 256 : 128), "accumulator budget");
  static_assert(REV_LDS_BYTES <= LDS_CAP || LDS_BYTES <= LDS_CAP, "LDS budget");

  // LDS element index of (row tile, K-step, lane, slot-in-step) for an operand with KS K-steps.
  __device__ static inline int lidx(int rt, int s, int lane, int KS) { return ((rt * KS + s) * kWave + lane) * E; }

  // fp8: the 32 bytes of a lane's fragment are two 16-byte halves kept in separate
  // planes of the K-step's block, so every 16-byte LDS access of a wave has a
  // 16-byte lane stride (a 32-byte stride puts two lanes on each bank group)
  __device__ static inline int hidx(int rt, int s, int half, int lane, int KS) {
    return (((rt * KS + s) * 2 + half) * kWave + lane) * 16;
  }

  __device__ static inline frag lds_frag(const elem* lds, int rt, int s, int lane, int KS) {
    if constexpr (P == P_FP8) {
      const i32x4 lo = *reinterpret_cast<const i32x4*>(lds + hidx(rt, s, 0, lane, KS));
      const i32x4 hi = *reinterpret_cast<const i32x4*>(lds + hidx(rt, s, 1, lane, KS));
      return frag{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    } else {
      return *reinterpret_cast<const frag*>(lds + lidx(rt, s, lane, KS));
    }
  }

  // acc[i][r] = sum over NSTEPS K-steps from s0 of A(mt0+i, s) * B(r, s), NMT M-tiles.
  // Weight fragments stream through a PD-deep register ring (loads are issued PD steps
  // ahead of their use, hiding L2 latency); LDS operand fragments are double-buffered.
  // B operand read from the LDS operand region
  struct LdsB {
    static constexpr bool kPrefetch = true;  // read the next step's fragments one step ahead
    const elem* lds;
    int KS;
    __device__ inline frag operator()(int r, int s, int lane) const { return lds_frag(lds, r, s, lane, KS); }
  };

  template <int NMT, int NSTEPS, int RING = 0>
  __device__ static inline void gemm(f32x16 (&acc)[NMT][RT], const frag* __restrict__ Wp, int MTALL, int KS,
                                     int mt0, int s0, int rot, const elem* lds, int lane) {
    gemm_src<NMT, NSTEPS, RING>(acc, Wp, MTALL, mt0, s0, rot, LdsB{lds, KS}, lane);
  }

  // RING: bytes of weight fragments per lane in flight (0 = default for the wave count)
  template <int NMT, int NSTEPS, int RING, class BSrc>
  __device__ static inline void gemm_src(f32x16 (&acc)[NMT][RT], const frag* __restrict__ Wp, int MTALL,
                                         int mt0, int s0, int rot, const BSrc& bsrc, int lane) {
    // ring depth: up to 4 steps, at most 128 (two waves per SIMD) or 256 (one wave
    // per SIMD) bytes of weight fragments per lane
    constexpr int PD0 = (RING ? RING : (OCC == 1 ? 256 : 128)) / (NMT * (int)sizeof(frag));
    constexpr int PD1 = PD0 < 1 ? 1 : (PD0 > 4 ? 4 : PD0);
    constexpr int PD = NSTEPS < PD1 ? NSTEPS : PD1;
    static_assert(NSTEPS % PD == 0, "K-steps must be a multiple of the prefetch depth");
    static_assert((NSTEPS & (NSTEPS - 1)) == 0, "K-steps must be a power of two");
    // K-step visited at position s: the loop starts at a per-block rotation so that
    // workgroups running in lock-step read different parts of the weight matrix
    auto kstep = [&](int s) { return s0 + ((s + rot) & (NSTEPS - 1)); };
    auto wfrag = [&](int s, int i) { return Wp[((size_t)kstep(s) * MTALL + mt0 + i) * kWave + lane]; };
#pragma unroll
    for (int i = 0; i < NMT; ++i)
#pragma unroll
      for (int r = 0; r < RT; ++r) acc[i][r] = f32x16{};
    frag a[PD][NMT];
#pragma unroll
    for (int d = 0; d < PD; ++d)
#pragma unroll
      for (int i = 0; i < NMT; ++i) a[d][i] = wfrag(d, i);
    frag b[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) b[r] = bsrc(r, kstep(0), lane);
    // steady state: every step prefetches the weights PD steps ahead
    auto group = [&](int g) __attribute__((always_inline)) {
#pragma unroll
      for (int d = 0; d < PD; ++d) {
        const int s = g + d;
        frag bn[RT];
        if constexpr (BSrc::kPrefetch) {
#pragma unroll
          for (int r = 0; r < RT; ++r) bn[r] = bsrc(r, kstep(s + 1), lane);
        } else if (s > 0) {
#pragma unroll
          for (int r = 0; r < RT; ++r) b[r] = bsrc(r, kstep(s), lane);
        }
#pragma unroll
        for (int i = 0; i < NMT; ++i)
#pragma unroll
          for (int r = 0; r < RT; ++r) acc[i][r] = M::mma(a[d][i], b[r], acc[i][r]);
#pragma unroll
        for (int i = 0; i < NMT; ++i) a[d][i] = wfrag(s + PD, i);
        if constexpr (BSrc::kPrefetch) {
#pragma unroll
          for (int r = 0; r < RT; ++r) b[r] = bn[r];
          // next step's B reads first, then this step's MFMAs, then the weight loads
          __builtin_amdgcn_sched_group_barrier(0x100, RT, 0);
          __builtin_amdgcn_sched_group_barrier(0x008, NMT * RT, 0);
          __builtin_amdgcn_sched_group_barrier(0x020, NMT, 0);
        }
        // keep each step's loads where they are issued: PD steps ahead of their use
        __builtin_amdgcn_sched_barrier(0);
      }
    };
    if constexpr (sizeof(frag) >= 32) {
      // 32-byte (fp8) fragments: the loop over step groups stays rolled; unrolled,
      // the scheduler's early loads exceed the register file
#pragma unroll 1
      for (int g = 0; g < NSTEPS - PD; g += PD) group(g);
    } else {
      for (int g = 0; g < NSTEPS - PD; g += PD) group(g);
    }
    // drain: the last PD steps
#pragma unroll
    for (int d = 0; d < PD; ++d) {
      const int s = NSTEPS - PD + d;
      frag bn[RT];
      if constexpr (BSrc::kPrefetch) {
        if (d + 1 < PD) {
#pragma unroll
          for (int r = 0; r < RT; ++r) bn[r] = bsrc(r, kstep(s + 1), lane);
        }
      } else if (s > 0) {
#pragma unroll
        for (int r = 0; r < RT; ++r) b[r] = bsrc(r, kstep(s), lane);
      }
#pragma unroll
      for (int i = 0; i < NMT; ++i)
#pragma unroll
        for (int r = 0; r < RT; ++r) acc[i][r] = M::mma(a[d][i], b[r], acc[i][r]);
      if constexpr (BSrc::kPrefetch) {
        if (d + 1 < PD) {
#pragma unroll
          for (int r = 0; r < RT; ++r) b[r] = bn[r];
        }
      }
    }
  }

  // K-steps per wave when a narrow (one M-tile) layer splits its K over the waves.
  static constexpr int SPLIT = (KS_H + NW - 1) / NW;

  // Store 16 accumulator-ordered values of (row tile rt, M-tile mt) as operand slots
  // q = 16*mt .. 16*mt+15 of the next layer (K-steps over width H).
  __device__ static inline void put_operand(elem* lds, int rt, int mt, int lane, const float (&v)[16], float inv_scale) {
    if constexpr (P == P_FP32) {
#pragma unroll
      for (int i = 0; i < 16; ++i) lds[lidx(rt, 16 * mt + i, lane, KS_H)] = v[i];
    } else if constexpr (P == P_BF16) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        i32x4 w;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          w[j] = (int)pack_bf16x2(v[8 * h + 2 * j], v[8 * h + 2 * j + 1]);
        *reinterpret_cast<i32x4*>(lds + lidx(rt, 2 * mt + h, lane, KS_H)) = w;
      }
    } else {
      i32x4 w;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        w[j] = (int)(f32x2_to_e4m3(v[4 * j] * inv_scale, v[4 * j + 1] * inv_scale) |
                     (f32x2_to_e4m3(v[4 * j + 2] * inv_scale, v[4 * j + 3] * inv_scale) << 16));
      *reinterpret_cast<i32x4*>(lds + hidx(rt, mt >> 1, mt & 1, lane, KS_H)) = w;
    }
  }

  // E float slot values -> one operand fragment
  __device__ static inline frag to_frag(const float* v, float inv_scale) {
    if constexpr (P == P_FP32) {
      return v[0];
    } else if constexpr (P == P_BF16) {
      i32x4 w;
#pragma unroll
      for (int j = 0; j < 4; ++j) w[j] = (int)pack_bf16x2(v[2 * j], v[2 * j + 1]);
      return __builtin_bit_cast(frag, w);
    } else {
      i32x8 w;
#pragma unroll
      for (int j = 0; j < 8; ++j)
        w[j] = (int)(f32x2_to_e4m3(v[4 * j] * inv_scale, v[4 * j + 1] * inv_scale) |
                     (f32x2_to_e4m3(v[4 * j + 2] * inv_scale, v[4 * j + 3] * inv_scale) << 16));
      return w;
    }
  }

  // Write one operand element block (E slots of lane `lane`, K-step s) from float values.
  __device__ static inline void put_slots(elem* lds, int rt, int s, int lane, int KS, const float* v, float inv_scale) {
    elem* dst = lds + lidx(rt, s, lane, KS);
    if constexpr (P == P_FP32) {
      dst[0] = v[0];
    } else if constexpr (P == P_BF16) {
      i32x4 w;
#pragma unroll
      for (int j = 0; j < 4; ++j) w[j] = (int)pack_bf16x2(v[2 * j], v[2 * j + 1]);
      *reinterpret_cast<i32x4*>(dst) = w;
    } else {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        i32x4 w;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          w[j] = (int)(f32x2_to_e4m3(v[16 * h + 4 * j] * inv_scale, v[16 * h + 4 * j + 1] * inv_scale) |
                       (f32x2_to_e4m3(v[16 * h + 4 * j + 2] * inv_scale, v[16 * h + 4 * j + 3] * inv_scale) << 16));
        *reinterpret_cast<i32x4*>(lds + hidx(rt, s, h, lane, KS)) = w;
      }
    }
  }
};


// 16 consecutive stash values <-> floats, as 16-byte vector accesses.
template <typename S> __device__ inline void store16(S* dst, const float (&v)[16]);
template <> __device__ inline void store16<float>(float* dst, const float (&v)[16]) {
#pragma unroll
  for (int c = 0; c < 4; ++c) reinterpret_cast<float4*>(dst)[c] = make_float4(v[4 * c], v[4 * c + 1], v[4 * c + 2], v[4 * c + 3]);
}
template <> __device__ inline void store16<uint16_t>(uint16_t* dst, const float (&v)[16]) {
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    i32x4 w;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      w[j] = (int)pack_bf16x2(v[8 * c + 2 * j], v[8 * c + 2 * j + 1]);
    reinterpret_cast<i32x4*>(dst)[c] = w;
  }
}
// RL consecutive stash values (RL = 1, 8 or 16) -> floats
template <int RL> __device__ inline void load_run(const float* src, float* v) {
  if constexpr (RL == 1) {
    v[0] = src[0];
  } else {
#pragma unroll
    for (int c = 0; c < RL / 4; ++c) {
      const float4 t = reinterpret_cast<const float4*>(src)[c];
      v[4 * c] = t.x; v[4 * c + 1] = t.y; v[4 * c + 2] = t.z; v[4 * c + 3] = t.w;
    }
  }
}
template <int RL> __device__ inline void load_run(const uint16_t* src, float* v) {
  if constexpr (RL == 1) {
    v[0] = __uint_as_float(((uint32_t)src[0]) << 16);
  } else {
#pragma unroll
    for (int c = 0; c < RL / 8; ++c) {
      const i32x4 t = reinterpret_cast<const i32x4*>(src)[c];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        v[8 * c + 2 * j] = __uint_as_float(((uint32_t)t[j]) << 16);
        v[8 * c + 2 * j + 1] = __uint_as_float(((uint32_t)t[j]) & 0xffff0000u);
      }
    }
  }
}

template <typename S> __device__ inline S to_stash(float v);
template <> __device__ inline float to_stash<float>(float v) { return v; }
template <> __device__ inline uint16_t to_stash<uint16_t>(float v) { return f32_to_bf16_rne(v); }
__device__ inline float from_stash(float v) { return v; }
__device__ inline float from_stash(uint16_t v) { return bf16_to_f32(v); }

// ---------------------------------------------------------------------------
// Forward chain: z_0 -> h_1..h_L (stash act'), y.
template <int P, int H, int V>
__global__ void __attribute__((amdgpu_flat_work_group_size(1, ChainShape<P, H, false, V>::NW * kWave),
                               amdgpu_waves_per_eu(ChainShape<P, H, false, V>::OCC)))
mlp_forward_chain(NetView net, int n, const float* __restrict__ x, const float* __restrict__ u,
                  const float* __restrict__ zin, typename StashT<P>::type* __restrict__ stash,
                  float* __restrict__ y, float* __restrict__ amax, float* __restrict__ hsave, int row_begin,
                  int row_end) {
  constexpr int NW = ChainShape<P, H, false, V>::NW, R = ChainShape<P, H, false, V>::R;
  using C = Chain<P, H, R, NW, ChainShape<P, H, false, V>::OCC>;
  using elem = typename C::elem;
  using frag = typename C::frag;
  using S = typename StashT<P>::type;
  __shared__ __attribute__((aligned(16))) unsigned char smem[C::LDS_BYTES];
  elem* lds = reinterpret_cast<elem*>(smem);
  float* part = reinterpret_cast<float*>(smem);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 5;
  // rows (nodes) [row_begin, row_end) of the n, in blocks of R from row_begin
  const int nblocks = (row_end - row_begin + R - 1) / R;
  const float* dq = net.wscale;  // fp8 only
  for (int blk = blockIdx.x; blk < nblocks; blk += gridDim.x) {
    const int row0 = row_begin + blk * R;
    // z_0 (the network input features) into operand slots of K1 features
    for (int it = tid; it < C::RT * C::KS_1 * kWave; it += NW * kWave) {
      const int l = it % kWave, s = (it / kWave) % C::KS_1, rt = it / (kWave * C::KS_1);
      const int row = row0 + rt * 32 + (l & 31), gg = l >> 5;
      float v[C::E];
#pragma unroll
      for (int j = 0; j < C::E; ++j) {
        const int k = slot_feature(s * C::E + j, gg);
        float z = 0.f;
        if (row < row_end && k < kDin)
          z = zin ? zin[(size_t)row * kDin + k] : net_feature(x + (size_t)row * kNx, u + (size_t)row * kNu, k, net.input);
        v[j] = z;
      }
      if (amax) {  // calibration only: max |z_0| (padding slots hold zeros)
        float m = 0.f;
#pragma unroll
        for (int j = 0; j < C::E; ++j) m = fmaxf(m, fabsf(v[j]));
        atomic_amax(&amax[0], m);
      }
      C::put_slots(lds, rt, s, l, C::KS_1, v, P == P_FP8 ? 1.f / net.ascale[0] : 1.f);
    }
    __syncthreads();

    for (int layer = 0; layer < net.L; ++layer) {
      const int KS = layer == 0 ? C::KS_1 : C::KS_H;
      f32x16 acc[C::MTW][C::RT];
      if (layer == 0)
        C::template gemm<C::MTW, C::KS_1>(acc, reinterpret_cast<const frag*>(net.fw[0]), C::MT, C::KS_1, wave * C::MTW,
                                          0, blk, lds, lane);
      else
        C::template gemm<C::MTW, C::KS_H, (C::kOcc > 1 ? 64 : 0)>(acc, reinterpret_cast<const frag*>(net.fw[layer]), C::MT,
                                                              C::KS_H, wave * C::MTW, 0, blk, lds, lane);
      __syncthreads();
      const float scale = P == P_FP8 ? dq[layer] * net.ascale[layer] : 1.f;
      const float inv_next = P == P_FP8 ? 1.f / net.ascale[layer + 1] : 1.f;
      const float* bias = net.bias[layer];
      S* st = stash + (size_t)layer * n * H;
      float lmax = 0.f;  // calibration: this lane's max |h|
      // The activation is chosen once per layer, not per value: a branch inside the
      // 16-value loop would serialise each value's exp -> rcp -> product chain.
      // Row tiles outer, M-tiles inner: a wave's M-tiles of one row are adjacent in
      // the stash (MTW x 64 bytes), so their stores follow each other and reach
      // memory as whole lines.
      auto tiles = [&](auto silu) __attribute__((always_inline)) {
        float bm[C::MTW][16];
#pragma unroll
        for (int i = 0; i < C::MTW; ++i)
#pragma unroll
          for (int vi = 0; vi < 16; ++vi) bm[i][vi] = bias[(wave * C::MTW + i) * 32 + (vi >> 2) * 8 + g * 4 + (vi & 3)];
#pragma unroll
        for (int r = 0; r < C::RT; ++r) {
#pragma unroll
          for (int i = 0; i < C::MTW; ++i) {
            const int mt = wave * C::MTW + i;
            const int row = row0 + r * 32 + (lane & 31);
            float h[16], sp[16];
#pragma unroll
            for (int vi = 0; vi < 16; ++vi) {
              const float a = acc[i][r][vi] * scale + bm[i][vi];
              if constexpr (decltype(silu)::value) {
                // SiLU h = a s(a), s = logistic; act' = s (1 + a (1 - s)) = s + h (1 - s)
                const float sg = __builtin_amdgcn_rcpf(1.f + __expf(-a));
                h[vi] = a * sg;
                sp[vi] = __builtin_fmaf(h[vi], 1.f - sg, sg);
              } else {
                h[vi] = a;
                sp[vi] = 1.f;
              }
            }
            if (amax && row < row_end) {
#pragma unroll
              for (int vi = 0; vi < 16; ++vi) lmax = fmaxf(lmax, fabsf(h[vi]));
            }
            if (row < row_end) store16<S>(st + (size_t)row * H + mt * 32 + g * 16, sp);
            if (hsave && row < row_end) {  // training: h_l in natural feature order
              float* hd = hsave + ((size_t)layer * n + row) * H + mt * 32 + g * 4;
#pragma unroll
              for (int q4 = 0; q4 < 4; ++q4)
                reinterpret_cast<float4*>(hd + q4 * 8)[0] =
                    make_float4(h[4 * q4], h[4 * q4 + 1], h[4 * q4 + 2], h[4 * q4 + 3]);
            }
            C::put_operand(lds, r, mt, lane, h, inv_next);
          }
        }
      };
      if (net.act == 0)
        tiles(std::true_type{});
      else
        tiles(std::false_type{});
      if (amax) atomic_amax(&amax[layer + 1], lmax);
      __syncthreads();
    }

    // output layer y = W_{L+1} h_L + b: one 32-row M-tile (6 used), K split over the waves
    {
      f32x16 acc[1][C::RT];
      const int s0 = wave * C::SPLIT;
      if (s0 < C::KS_H)
        C::template gemm<1, C::SPLIT>(acc, reinterpret_cast<const frag*>(net.fw[net.L]), 1, C::KS_H, 0, s0, 0, lds, lane);
      else
        for (int r = 0; r < C::RT; ++r) acc[0][r] = f32x16{};
      __syncthreads();
#pragma unroll
      for (int r = 0; r < C::RT; ++r)
#pragma unroll
        for (int vi = 0; vi < 4; ++vi) part[(wave * R + r * 32 + (lane & 31)) * 8 + g * 4 + vi] = acc[0][r][vi];
      __syncthreads();
      const float scale = P == P_FP8 ? dq[net.L] * net.ascale[net.L] : 1.f;
      for (int t = tid; t < R * kDout; t += NW * kWave) {
        const int rr = t / kDout, j = t % kDout, row = row0 + rr;
        float s = 0.f;
        for (int w = 0; w < NW; ++w) s += part[(w * R + rr) * 8 + j];
        if (row < row_end) y[(size_t)row * kDout + j] = s * scale + net.bias[net.L][j];
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// Reverse (adjoint) chain: 6 rows per node; J_D[node][j][c] for the 14 inputs.
//
// The activation derivatives a row block needs in a layer's epilogue are the rows
// of its (at most R/6 + 2) nodes, contiguous in the stash.  They are fetched with
// 16-byte loads issued before the layer's K-loop (so their latency hides behind
// the matrix work) and parked in LDS when the loop ends; the next block's
// first-layer rows are fetched during the current block's last K-loop.
template <int P, int H, int V>
__global__ void __attribute__((amdgpu_flat_work_group_size(1, ChainShape<P, H, true, V>::NW * kWave),
                               amdgpu_waves_per_eu(ChainShape<P, H, true, V>::OCC)))
mlp_reverse_chain(NetView net, int n, const typename StashT<P>::type* __restrict__ stash,
                  float* __restrict__ J, float* __restrict__ amax, int row_begin, int row_end) {
  constexpr int NW = ChainShape<P, H, true, V>::NW, R = ChainShape<P, H, true, V>::R;
  using C = Chain<P, H, R, NW, ChainShape<P, H, true, V>::OCC>;
  using elem = typename C::elem;
  using frag = typename C::frag;
  using S = typename StashT<P>::type;
  constexpr int NT = NW * kWave;
  constexpr int CH = C::SP_CHUNKS_PER_THREAD;
  __shared__ __attribute__((aligned(16))) unsigned char smem[C::REV_LDS_BYTES];
  elem* lds = reinterpret_cast<elem*>(smem);
  float* part = reinterpret_cast<float*>(smem);
  S* sp_lds = reinterpret_cast<S*>(smem + C::LDS_BYTES);
  i32x4* sp_lds4 = reinterpret_cast<i32x4*>(smem + C::LDS_BYTES);
  float* wo_lds = reinterpret_cast<float*>(smem + C::LDS_BYTES + C::SP_BYTES);
  const float* wo = C::WO_IN_LDS ? wo_lds : net.w_out_s;
  const int wo_stride = C::WO_IN_LDS ? C::WOS : H;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 5;
  // rows [row_begin, row_end) of the 6 n, in blocks of R from row_begin
  const int nrows = row_end;
  const int nblocks = (row_end - row_begin + R - 1) / R;
  const int L = net.L;
  const size_t layer_stride = (size_t)n * H;

  i32x4 sp_reg[CH];
  // issue the loads of stash layer `layer` for the nodes of the block starting at row r0
  auto sp_fetch = [&](int layer, int r0) {
    const int node0 = r0 / 6;
    const int node1 = min(n, (min(r0 + R, nrows) + 5) / 6);
    const int nchunks = (node1 - node0) * H * (int)sizeof(S) / 16;
    const i32x4* src = reinterpret_cast<const i32x4*>(stash + (size_t)layer * layer_stride + (size_t)node0 * H);
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int idx = tid + c * NT;
      if (idx < nchunks) sp_reg[c] = __builtin_nontemporal_load(src + idx);
    }
  };
  auto sp_park = [&]() {
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int idx = tid + c * NT;
      const int nd = idx / C::SP_ROW_CHUNKS, w = idx - nd * C::SP_ROW_CHUNKS;
      if (nd < C::SP_NODES) sp_lds4[nd * (C::SPS * C::SP_ELEM / 16) + w] = sp_reg[c];
    }
  };

  if constexpr (C::WO_IN_LDS) {
    for (int i = tid; i < kDout * H / 4; i += NT) {
      const int j = i / (H / 4), c = i - j * (H / 4);
      reinterpret_cast<float4*>(wo_lds + j * C::WOS)[c] = reinterpret_cast<const float4*>(net.w_out_s)[i];
    }
  }
  if (blockIdx.x < nblocks) sp_fetch(L - 1, row_begin + blockIdx.x * R);
  for (int blk = blockIdx.x; blk < nblocks; blk += gridDim.x) {
    const int row0 = row_begin + blk * R;
    const int node0 = row0 / 6;
    sp_park();
    __syncthreads();
    // G_L[row][k] = W_{L+1}[row % 6][k] * act'(a_L)[row / 6][k]; the E slots of one
    // (row tile, K-step, lane) item are runs of consecutive stash positions
    constexpr int RL = C::E < 16 ? C::E : 16;
    {
      const float inv = P == P_FP8 ? 1.f / net.gscale[L - 1] : 1.f;
      float lmax = 0.f;
      // Work unit = (K-step, lane group, output j, quarter of the rows): the unit
      // loads the E weights W_{L+1}[j][slots] once and applies them to its rows
      // with row % 6 == j (every 24th row of the block), so each weight value is
      // read from L2 once per unit rather than once per row -- the L2 round trips
      // of these reads otherwise dominate this phase.  Rows past the end are
      // written as zeros.
      constexpr int NU = C::KS_H * 2 * kDout * 4;
      constexpr int UPT = (NU + NT - 1) / NT;  // units per thread
      const int jr = row0 % 6;
      // every unit's weights are requested before the first unit's rows are built
      float wv[UPT][C::E];
#pragma unroll
      for (int k = 0; k < UPT; ++k) {
        const int u = tid + k * NT;
        const int j = (u >> 2) % kDout, gg = (u / (4 * kDout)) & 1, sk = min(u, NU - 1) / (8 * kDout);
#pragma unroll
        for (int run = 0; run < C::E / RL; ++run) {
          const int q0 = sk * C::E + run * RL;
          const int pos = 32 * (q0 >> 4) + gg * 16 + (q0 & 15);  // stash order of slot q0
          load_run<RL>(wo + j * wo_stride + pos, wv[k] + run * RL);
        }
      }
#pragma unroll
      for (int k = 0; k < UPT; ++k) {
        const int u = tid + k * NT;
        if (u >= NU) break;
        const int qr = u & 3, j = (u >> 2) % kDout, gg = (u / (4 * kDout)) & 1, sk = u / (8 * kDout);
        // block rows i with (row0 + i) % 6 == j, this quarter: i = i0 + 6 qr + 24 m;
        // all of the unit's rows are read before the first is written (the
        // operand stores would otherwise hold back every following read)
        const int i0 = (j - jr + 6) % 6 + 6 * qr;
        constexpr int NI = (R + 23) / 24;
        float v[NI][C::E];
#pragma unroll
        for (int m = 0; m < NI; ++m) {
          const int row = row0 + i0 + 24 * m;
          const int node = (i0 + 24 * m < R && row < nrows) ? row / 6 : node0;
#pragma unroll
          for (int run = 0; run < C::E / RL; ++run) {
            const int q0 = sk * C::E + run * RL;
            const int pos = 32 * (q0 >> 4) + gg * 16 + (q0 & 15);
            load_run<RL>(sp_lds + (node - node0) * C::SPS + pos, v[m] + run * RL);
          }
        }
#pragma unroll
        for (int m = 0; m < NI; ++m) {
          const int i = i0 + 24 * m;
          if (i >= R) break;
          const bool live = row0 + i < nrows;
#pragma unroll
          for (int t = 0; t < C::E; ++t) v[m][t] = live ? wv[k][t] * v[m][t] : 0.f;
          if (amax) {
#pragma unroll
            for (int t = 0; t < C::E; ++t) lmax = fmaxf(lmax, fabsf(v[m][t]));
          }
          C::put_slots(lds, i >> 5, sk, gg * 32 + (i & 31), C::KS_H, v[m], inv);
        }
      }
      if (amax) atomic_amax(&amax[L - 1], lmax);
    }
    __syncthreads();

    for (int layer = L - 1; layer >= 1; --layer) {  // weights W_{layer+1}^T, stash of h_layer
      f32x16 acc[C::MTW][C::RT];
      sp_fetch(layer - 1, row0);
      C::template gemm<C::MTW, C::KS_H, (C::kOcc > 1 ? 64 : 0)>(acc, reinterpret_cast<const frag*>(net.rw[layer]),
                                                               C::MT, C::KS_H, wave * C::MTW, 0, blk, lds, lane);
      sp_park();
      __syncthreads();
      const float scale = P == P_FP8 ? net.wscale[layer] * net.gscale[layer] : 1.f;
      const float inv_next = P == P_FP8 ? 1.f / net.gscale[layer - 1] : 1.f;
      float lmax = 0.f;
      // with one wave per SIMD there are registers to read all of this wave's
      // activation-derivative runs (16 stash values = 32 or 64 bytes each, kept
      // packed) before their first use
      constexpr bool PRE = C::kOcc == 1 && C::MTW * C::RT <= 12;
      constexpr int PI = PRE ? C::MTW : 1, PR = PRE ? C::RT : 2;
      constexpr int RUN_CH = 16 * (int)sizeof(S) / 16;  // 16-byte chunks per run
      i32x4 spraw[PI][PR][RUN_CH];
      auto raw_load = [&](int i, int r, int mt, int row) {
        const int node = row < nrows ? row / 6 : node0;
        const i32x4* src = reinterpret_cast<const i32x4*>(sp_lds + (node - node0) * C::SPS + mt * 32 + g * 16);
#pragma unroll
        for (int c = 0; c < RUN_CH; ++c) spraw[i][r][c] = src[c];
      };
      if constexpr (PRE) {
#pragma unroll
        for (int i = 0; i < C::MTW; ++i)
#pragma unroll
          for (int r = 0; r < C::RT; ++r) raw_load(i, r, wave * C::MTW + i, row0 + r * 32 + (lane & 31));
      } else {
        // otherwise each run is read one tile ahead, before the previous tile's
        // operand stores (which the compiler cannot move loads across)
        raw_load(0, 0, wave * C::MTW, row0 + (lane & 31));
      }
#pragma unroll
      for (int i = 0; i < C::MTW; ++i) {
        const int mt = wave * C::MTW + i;
#pragma unroll
        for (int r = 0; r < C::RT; ++r) {
          const int row = row0 + r * 32 + (lane & 31);
          const int t = i * C::RT + r;
          const int pi = PRE ? i : 0, pr = PRE ? r : (t & 1);
          if constexpr (!PRE) {
            if (t + 1 < C::MTW * C::RT) {
              const int i1 = (t + 1) / C::RT, r1 = (t + 1) % C::RT;
              raw_load(0, (t + 1) & 1, wave * C::MTW + i1, row0 + r1 * 32 + (lane & 31));
            }
          }
          float sv[16];
          load_run<16>(reinterpret_cast<const S*>(spraw[pi][pr]), sv);
          float v[16];
#pragma unroll
          for (int vi = 0; vi < 16; ++vi) v[vi] = acc[i][r][vi] * scale * sv[vi];
          if (amax && row < nrows) {
#pragma unroll
            for (int vi = 0; vi < 16; ++vi) lmax = fmaxf(lmax, fabsf(v[vi]));
          }
          C::put_operand(lds, r, mt, lane, v, inv_next);
        }
      }
      if (amax) atomic_amax(&amax[layer - 1], lmax);
      __syncthreads();
    }

    // J_D = G_1 W_1: one M-tile (14 used), K split over the waves
    {
      f32x16 acc[1][C::RT];
      const int s0 = wave * C::SPLIT;
      if (s0 < C::KS_H)
        C::template gemm<1, C::SPLIT>(acc, reinterpret_cast<const frag*>(net.rw[0]), 1, C::KS_H, 0, s0, 0, lds, lane);
      else
        for (int r = 0; r < C::RT; ++r) acc[0][r] = f32x16{};
      // the next block's first rows: requested after the J_D product's weight loads,
      // which would otherwise return only after these (loads complete in order)
      if (blk + (int)gridDim.x < nblocks) sp_fetch(L - 1, row_begin + (blk + gridDim.x) * R);
      __syncthreads();
#pragma unroll
      for (int r = 0; r < C::RT; ++r)
#pragma unroll
        for (int vi = 0; vi < 8; ++vi)
          part[(wave * R + r * 32 + (lane & 31)) * 16 + (vi >> 2) * 8 + g * 4 + (vi & 3)] = acc[0][r][vi];
      __syncthreads();
      const float scale = P == P_FP8 ? net.wscale[0] * net.gscale[0] : 1.f;
      for (int t = tid; t < R * kDin; t += NT) {
        const int rr = t / kDin, c = t % kDin, row = row0 + rr;
        float s = 0.f;
        for (int w = 0; w < NW; ++w) s += part[(w * R + rr) * 16 + c];
        if (row < nrows) J[(size_t)row * kDin + c] = s * scale;
      }
      __syncthreads();
    }
  }
}


// ---------------------------------------------------------------------------
// Launchers (explicitly instantiated per precision in chain_fp32/bf16/fp8.hip)

// Workgroups for `blocks` row blocks: the configured count, else two per compute
// unit; never more than there are blocks.
inline int chain_grid(int blocks, const ChainCfg& cfg) {
  const int want = cfg.grid > 0 ? cfg.grid : 2 * num_cu();
  return blocks < want ? blocks : want;
}

// Variant 4 (128-row blocks, one workgroup per CU) with a last round of blocks that
// would keep at most three quarters of the resident workgroups busy: that round's
// rows go to a second launch of 64-row (up to half busy) or 96-row blocks, which
// spreads them over all CUs.  rows: rows of the launch; grid: workgroups kept.
struct TailPlan {
  int split;      // rows of the 128-row launch; rows [split, rows) go to the tail
  int tail_rows;  // 64 or 96 rows per tail block (0: no tail)
  int grid_main;  // workgroups of the 128-row launch
};
inline TailPlan tail_plan(int rows, int grid, const ChainCfg& cfg) {
  const int nblk = (rows + 127) / 128;
  const int slots = grid < num_cu() ? grid : num_cu();
  const int rem = slots > 0 ? nblk % slots : 0;
  if (nblk <= slots || rem == 0 || 4 * rem > 3 * slots) return {rows, 0, grid};
  return {(nblk - rem) * 128, 2 * rem <= slots ? 64 : 96, chain_grid(nblk - rem, cfg)};
}

template <int P, int H, int V>
hipError_t chain_forward_v(const ChainCfg& cfg, const NetView& net, int n, const float* x, const float* u,
                           const float* zin, void* stash, float* y, float* amax, float* hsave, hipStream_t st) {
  using Sh = ChainShape<P, H, false, V>;
  if constexpr (!Sh::VALID) {
    return hipErrorInvalidValue;
  } else {
    using S = typename StashT<P>::type;
    const int grid = chain_grid((n + Sh::R - 1) / Sh::R, cfg);
    if (grid <= 0) return hipSuccess;
    TailPlan tp{n, 0, grid};
    if constexpr (V == 4 && ChainShape<P, H, false, 5>::VALID) tp = tail_plan(n, grid, cfg);
    mlp_forward_chain<P, H, V><<<tp.grid_main, Sh::NW * kWave, 0, st>>>(net, n, x, u, zin, (S*)stash, y, amax,
                                                                        hsave, 0, tp.split);
    hipError_t e = hipGetLastError();
    if constexpr (V == 4 && ChainShape<P, H, false, 5>::VALID) {
      if (e == hipSuccess && tp.tail_rows == 64) {
        mlp_forward_chain<P, H, 5><<<(n - tp.split + 63) / 64, ChainShape<P, H, false, 5>::NW * kWave, 0, st>>>(
            net, n, x, u, zin, (S*)stash, y, amax, hsave, tp.split, n);
        e = hipGetLastError();
      } else if (e == hipSuccess && tp.tail_rows == 96) {
        mlp_forward_chain<P, H, 6><<<(n - tp.split + 95) / 96, ChainShape<P, H, false, 6>::NW * kWave, 0, st>>>(
            net, n, x, u, zin, (S*)stash, y, amax, hsave, tp.split, n);
        e = hipGetLastError();
      }
    }
    return e;
  }
}

template <int P, int H, int V>
hipError_t chain_reverse_v(const ChainCfg& cfg, const NetView& net, int n, const void* stash, float* J, float* amax,
                           hipStream_t st) {
  using Sh = ChainShape<P, H, true, V>;
  if constexpr (!Sh::VALID) {
    return hipErrorInvalidValue;
  } else {
    using S = typename StashT<P>::type;
    const int nrows = 6 * n;
    const int grid = chain_grid((nrows + Sh::R - 1) / Sh::R, cfg);
    if (grid <= 0) return hipSuccess;
    TailPlan tp{nrows, 0, grid};
    if constexpr (V == 4 && ChainShape<P, H, true, 5>::VALID) tp = tail_plan(nrows, grid, cfg);
    mlp_reverse_chain<P, H, V><<<tp.grid_main, Sh::NW * kWave, 0, st>>>(net, n, (const S*)stash, J, amax, 0,
                                                                        tp.split);
    hipError_t e = hipGetLastError();
    if constexpr (V == 4 && ChainShape<P, H, true, 5>::VALID) {
      if (e == hipSuccess && tp.tail_rows == 64) {
        mlp_reverse_chain<P, H, 5><<<(nrows - tp.split + 63) / 64, ChainShape<P, H, true, 5>::NW * kWave, 0, st>>>(
            net, n, (const S*)stash, J, amax, tp.split, nrows);
        e = hipGetLastError();
      } else if (e == hipSuccess && tp.tail_rows == 96) {
        mlp_reverse_chain<P, H, 6><<<(nrows - tp.split + 95) / 96, ChainShape<P, H, true, 6>::NW * kWave, 0, st>>>(
            net, n, (const S*)stash, J, amax, tp.split, nrows);
        e = hipGetLastError();
      }
    }
    return e;
  }
}

template <int P, int H, int V> hipError_t chain_geom_v(int rev, int occupancy, ChainGeom* g) {
  constexpr bool VF = ChainShape<P, H, false, V>::VALID, VR = ChainShape<P, H, true, V>::VALID;
  g->valid = rev ? VR : VF;
  g->waves = rev ? ChainShape<P, H, true, V>::NW : ChainShape<P, H, false, V>::NW;
  g->rows = rev ? ChainShape<P, H, true, V>::R : ChainShape<P, H, false, V>::R;
  g->resident_per_cu = 0;
  if (!g->valid || !occupancy) return hipSuccess;
  int nb = 0;
  hipError_t e = hipSuccess;
  if (rev) {
    if constexpr (VR)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, mlp_reverse_chain<P, H, V>, g->waves * kWave, 0);
  } else {
    if constexpr (VF)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, mlp_forward_chain<P, H, V>, g->waves * kWave, 0);
  }
  g->resident_per_cu = nb;
  return e;
}

#define RTN_CHAIN_SWITCH(FN, ...)                              \
  switch (H * 8 + V) {                                         \
    case 64 * 8: return FN<P, 64, 0>(__VA_ARGS__);             \
    case 128 * 8: return FN<P, 128, 0>(__VA_ARGS__);           \
    case 256 * 8: return FN<P, 256, 0>(__VA_ARGS__);           \
    case 512 * 8: return FN<P, 512, 0>(__VA_ARGS__);           \
    case 512 * 8 + 1: return FN<P, 512, 1>(__VA_ARGS__);       \
    case 512 * 8 + 2: return FN<P, 512, 2>(__VA_ARGS__);       \
    case 512 * 8 + 3: return FN<P, 512, 3>(__VA_ARGS__);       \
    case 512 * 8 + 4: return FN<P, 512, 4>(__VA_ARGS__);       \
    case 1024 * 8: return FN<P, 1024, 0>(__VA_ARGS__);         \
    case 1024 * 8 + 1: return FN<P, 1024, 1>(__VA_ARGS__);     \
    case 1024 * 8 + 2: return FN<P, 1024, 2>(__VA_ARGS__);     \
    default: return hipErrorInvalidValue;                      \
  }

template <int P>
hipError_t chain_forward(int H, const ChainCfg& cfg, const NetView& net, int n, const float* x, const float* u,
                         const float* zin, void* stash, float* y, float* amax, float* hsave, hipStream_t st) {
  const int V = cfg.variant;
  RTN_CHAIN_SWITCH(chain_forward_v, cfg, net, n, x, u, zin, stash, y, amax, hsave, st)
}

template <int P>
hipError_t chain_reverse(int H, const ChainCfg& cfg, const NetView& net, int n, const void* stash, float* J,
                         float* amax, hipStream_t st) {
  const int V = cfg.variant;
  RTN_CHAIN_SWITCH(chain_reverse_v, cfg, net, n, stash, J, amax, st)
}

template <int P> hipError_t chain_geom(int H, int rev, int V, int occupancy, ChainGeom* g) {
  RTN_CHAIN_SWITCH(chain_geom_v, rev, occupancy, g)
}

#undef RTN_CHAIN_SWITCH

}  // namespace rtn
