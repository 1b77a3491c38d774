// Weight packing, amax/scale kernels and the precision dispatch of the
// layer-chain kernels (whose templates are in chain_kernels.h and are compiled
// in one translation unit per precision).
#include "common.h"
#include "mlp_chain.h"

namespace rtn {

// W_{L+1} (6 x H) reordered so that element j*H + stash_pos(k) holds W[j][k].
__global__ void reorder_out_weights(const float* __restrict__ W, int H, float* __restrict__ out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < 6 * H; i += gridDim.x * blockDim.x) {
    const int j = i / H, k = i % H;
    out[j * H + stash_pos(k)] = W[i];
  }
}

hipError_t launch_reorder_out(const float* W, int H, float* out, hipStream_t st) {
  reorder_out_weights<<<(6 * H + 255) / 256, 256, 0, st>>>(W, H, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Operand packing: fp32 matrix -> fragment-ordered compute-type copy, K-step major
// (all M-tiles of one K-step are contiguous, so the weights that lock-stepped
// waves read at the same time are spread over the L2 channels):
//   out[((s*MT + mt)*64 + lane)*E + j] = A[m][k],  m = 32 mt + lane % 32,
//   k = slot_feature(s*E + j, lane / 32);  A = W (trans = 0) or W^T (trans = 1),
//   W fp32 row-major [rows][cols].  Zero outside M x K.
// One operand matrix of a batched pack (see launch_pack_layers).
struct PackJob {
  const float* W;
  int cols, M, K, trans;
  const float* scale;
  void* out;
  int MT, KS;
  long begin;  // first element of this job in the launch's element range
};
constexpr int kMaxPackJobs = 34;
struct PackJobs {
  int n;
  PackJob j[kMaxPackJobs];
};

template <int P>
__device__ inline void pack_element(const PackJob& q, long idx) {
  constexpr int E = Mfma<P>::E;
  const int j = idx % E;
  const int lane = (idx / E) % kWave;
  const int mt = (idx / ((long)E * kWave)) % q.MT;
  const int s = idx / ((long)E * kWave * q.MT);
  const int m = mt * 32 + (lane & 31);
  const int k = slot_feature(s * E + j, lane >> 5);
  float v = 0.f;
  if (m < q.M && k < q.K) v = q.trans ? q.W[(size_t)k * q.cols + m] : q.W[(size_t)m * q.cols + k];
  auto* out = static_cast<typename Mfma<P>::elem*>(q.out);
  if constexpr (P == P_FP32) out[idx] = v;
  else if constexpr (P == P_BF16) out[idx] = f32_to_bf16_rne(v);
  else out[idx] = (uint8_t)(f32x2_to_e4m3(v * (q.scale ? 1.f / q.scale[0] : 1.f), 0.f) & 0xffu);
}

// Every matrix of a model's precision in one launch (one launch per layer costs
// a few microseconds each after every optimiser step).
template <int P>
__global__ void pack_operands(PackJobs jobs, long total) {
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
    int q = 0;
    while (q + 1 < jobs.n && idx >= jobs.j[q + 1].begin) ++q;
    pack_element<P>(jobs.j[q], idx - jobs.j[q].begin);
  }
}

__global__ void amax_kernel(const float* __restrict__ a, long n, float* __restrict__ out) {
  float m = 0.f;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) m = fmaxf(m, fabsf(a[i]));
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0) atomic_amax(out, m);
}

// amax -> e4m3 scale (amax / 448, 1 when the tensor is all zero)
__global__ void amax_to_scale(float* s, int n) {
  int i = threadIdx.x;
  if (i < n) s[i] = s[i] > 0.f ? s[i] / 448.f : 1.f;
}

// ---------------------------------------------------------------------------
// Host launchers

int pack_geometry(int prec, int M, int K, int* MT, int* KS) {
  int E, KSTEP, KALIGN;
  if (prec == P_FP32) { E = 1; KSTEP = 2; KALIGN = 16; }
  else if (prec == P_BF16) { E = 8; KSTEP = 16; KALIGN = 16; }
  else { E = 32; KSTEP = 64; KALIGN = 64; }
  (void)E;
  *MT = (M + 31) / 32;
  *KS = round_up(K, KALIGN) / KSTEP;
  return *MT * *KS * kWave * E;  // elements
}

hipError_t launch_pack_layers(int prec, int n, const PackSpec* specs, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (n > kMaxPackJobs) return hipErrorInvalidValue;
  PackJobs jobs{};
  jobs.n = n;
  long total = 0;
  for (int i = 0; i < n; ++i) {
    const PackSpec& p = specs[i];
    PackJob& q = jobs.j[i];
    q.W = p.W;
    q.cols = p.cols;
    q.M = p.M;
    q.K = p.K;
    q.trans = p.trans;
    q.scale = p.scale;
    q.out = p.out;
    q.begin = total;
    total += pack_geometry(prec, p.M, p.K, &q.MT, &q.KS);
  }
  int blocks = (int)((total + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  if (prec == P_FP32)
    pack_operands<P_FP32><<<blocks, 256, 0, st>>>(jobs, total);
  else if (prec == P_BF16)
    pack_operands<P_BF16><<<blocks, 256, 0, st>>>(jobs, total);
  else
    pack_operands<P_FP8><<<blocks, 256, 0, st>>>(jobs, total);
  return hipGetLastError();
}

hipError_t launch_amax(const float* a, long n, float* out, hipStream_t st) {
  amax_kernel<<<64, 256, 0, st>>>(a, n, out);
  return hipGetLastError();
}

hipError_t launch_amax_to_scale(float* s, int n, hipStream_t st) {
  amax_to_scale<<<1, 64, 0, st>>>(s, n);
  return hipGetLastError();
}

static int g_num_cu = 0;
int num_cu() {
  if (!g_num_cu) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) == hipSuccess) g_num_cu = p.multiProcessorCount;
    if (g_num_cu <= 0) g_num_cu = 256;
  }
  return g_num_cu;
}

hipError_t launch_mlp_forward(int prec, int H, const NetView& net, int n, const float* x, const float* u,
                              const float* zin, void* stash, float* y, float* amax, hipStream_t st, float* hsave,
                              const ChainCfg& cfg) {
  if (prec == P_FP32) return chain_forward<P_FP32>(H, cfg, net, n, x, u, zin, stash, y, amax, hsave, st);
  if (prec == P_BF16) return chain_forward<P_BF16>(H, cfg, net, n, x, u, zin, stash, y, amax, hsave, st);
  return chain_forward<P_FP8>(H, cfg, net, n, x, u, zin, stash, y, amax, hsave, st);
}

hipError_t launch_mlp_reverse(int prec, int H, const NetView& net, int n, const void* stash, float* J, float* amax,
                              hipStream_t st, const ChainCfg& cfg) {
  if (prec == P_FP32) return chain_reverse<P_FP32>(H, cfg, net, n, stash, J, amax, st);
  if (prec == P_BF16) return chain_reverse<P_BF16>(H, cfg, net, n, stash, J, amax, st);
  return chain_reverse<P_FP8>(H, cfg, net, n, stash, J, amax, st);
}

hipError_t chain_geometry(int prec, int H, int rev, int variant, int occupancy, ChainGeom* g) {
  if (prec == P_FP32) return chain_geom<P_FP32>(H, rev, variant, occupancy, g);
  if (prec == P_BF16) return chain_geom<P_BF16>(H, rev, variant, occupancy, g);
  return chain_geom<P_FP8>(H, rev, variant, occupancy, g);
}

int stash_elem_bytes(int prec) { return prec == P_FP32 ? 4 : 2; }

}  // namespace rtn
