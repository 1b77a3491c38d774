// rtn_riccati_noalloc: the batched fp64 Riccati recursion of rtn_riccati for
// callers that cannot allocate device memory (code under stream capture, tight
// serving loops, harnesses that forbid allocation).
//
// rtn_riccati stages the cost matrices Q, R, Q_N and the instance offsets in a
// stream-ordered device allocation.  Here they go into a file-scope device
// array instead, of fixed size: the constants and the offsets of at most
// kNoAllocMaxInst instances.  Each device the library runs on holds its own copy
// of the array until the process ends; its device address is looked up once per
// device (hipGetSymbolAddress) on the first call made with that device current,
// and only that address is handed to the copy and the kernel -- in host code the
// array's name is not a device address.
//
// Every call on a device overwrites that device's array (stream-ordered on the
// caller's stream), so calls that overlap on one device -- from two host threads,
// or enqueued on two streams that run concurrently -- race on it.  Nothing in it
// needs clearing: every call writes all the bytes its kernel reads.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "mlp_chain.h"
#include "model.h"
#include "profiler.h"

namespace rtn {
namespace {

constexpr int kNoAllocMaxInst = 65536;
constexpr size_t kConstDoubles = 169 + 16 + 169;  // Q, R, Q_N
constexpr size_t kScratchBytes = (kConstDoubles * 8 + (size_t)(kNoAllocMaxInst + 1) * 4 + 255) / 256 * 256;
constexpr int kMaxDevices = 64;

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of this device's scratch array (looked up once per device).
static hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

}  // namespace rtn

using namespace rtn;

extern "C" rtn_status rtn_riccati_noalloc(int32_t n_inst, const int32_t* offsets_host, int32_t n_nodes,
                                          const float* A, const float* B, const double* c, const double* Q_host,
                                          const double* R_host, const double* QN_host, const double* q,
                                          const double* r, const double* qN, double* K, double* kff, double* P,
                                          void* stream) {
  rtn_status s = check_offsets(n_inst, offsets_host, n_nodes);
  if (s) return s;
  if (n_inst > kNoAllocMaxInst)
    return failf(RTN_EINVAL, "rtn_riccati_noalloc takes at most %d instances (got %d); use rtn_riccati",
                 kNoAllocMaxInst, n_inst);
  if (!Q_host || !R_host || !QN_host) return failf(RTN_EINVAL, "Q_host, R_host and QN_host are required");
  for (int i = 0; i < 13 * 13; ++i)
    if (!std::isfinite(Q_host[i]) || !std::isfinite(QN_host[i])) return failf(RTN_EINVAL, "Q or Q_N is not finite");
  for (int i = 0; i < 16; ++i)
    if (!std::isfinite(R_host[i])) return failf(RTN_EINVAL, "R is not finite");
  if (n_nodes == 0) return RTN_OK;
  if (!A || !B) return failf(RTN_EINVAL, "A and B must be device pointers");
  if (!K || !kff) return failf(RTN_EINVAL, "K and kff must be device pointers");
  void* dev = nullptr;
  hipError_t e = scratch_address(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
  hipStream_t st = (hipStream_t)stream;
  // the same staging layout as rtn_riccati: Q | R | Q_N | offsets
  unsigned char host[kConstDoubles * 8];
  const size_t off_bytes = (size_t)(n_inst + 1) * 4;
  memcpy(host, Q_host, 169 * 8);
  memcpy(host + 169 * 8, R_host, 16 * 8);
  memcpy(host + 185 * 8, QN_host, 169 * 8);
  unsigned char* d = static_cast<unsigned char*>(dev);
  // pageable sources are consumed before hipMemcpyAsync returns
  e = hipMemcpyAsync(d, host, kConstDoubles * 8, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    if (offsets_host) {
      e = hipMemcpyAsync(d + kConstDoubles * 8, offsets_host, off_bytes, hipMemcpyHostToDevice, st);
    } else {
      const int32_t one[2] = {0, n_nodes};
      e = hipMemcpyAsync(d + kConstDoubles * 8, one, sizeof one, hipMemcpyHostToDevice, st);
    }
  }
  if (e != hipSuccess) return hip_fail(e, "rtn_riccati_noalloc (staging copy)");
  const double* dd = reinterpret_cast<const double*>(d);
  ProfScope ps("riccati", st);
  e = launch_riccati(n_inst, reinterpret_cast<const int*>(d + kConstDoubles * 8), dd, dd + 169, dd + 185, A, B, c, q,
                     r, qN, K, kff, P, st);
  if (e != hipSuccess) return hip_fail(e, "rtn_riccati_noalloc");
  return RTN_OK;
}
