// C ABI of the double-integrator runtime workload (Sec. V): model ownership,
// argument validation and dispatch of the kernels in di.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/rtn.h"
#include "di.h"
#include "model.h"
#include "profiler.h"

using namespace rtn;

#define DI_TRY(expr)                                  \
  do {                                                \
    hipError_t _e = (expr);                           \
    if (_e != hipSuccess) return hip_fail(_e, #expr); \
  } while (0)

struct rtn_di_model {
  int L = 0, H = 0, act = 0;
  int64_t n_params = 0;
  std::vector<int64_t> w_off, b_off;  // into `params`, every tensor 64-float aligned
  float* params = nullptr;
  // workspace: activations [2][3n][H], f_D [n][2], J_D [n][2][2]; instance offsets
  float* Z = nullptr;
  float* yJ = nullptr;
  float* partial = nullptr;  // split-K partial tiles of the hidden layers
  float* fused = nullptr;    // small widths: the single-workgroup path's weights (hidden ones transposed)
  long* fused_off = nullptr;
  int64_t cap = 0;
  int* d_off = nullptr;
  std::vector<int32_t> off_host;
  struct Graph {
    uint64_t key[24];
    hipGraphExec_t exec;
    uint64_t last_use;
  };
  std::vector<Graph> graphs;
  uint64_t clock = 0;
  hipStream_t cap_stream = nullptr;

  ~rtn_di_model() {
    drop_graphs();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (void* p : {(void*)params, (void*)Z, (void*)yJ, (void*)partial, (void*)d_off, (void*)fused, (void*)fused_off})
      if (p) (void)hipFree(p);
  }
  void drop_graphs() {
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
    graphs.clear();
  }
  int fan_in(int l) const { return l == 0 ? 2 : H; }
  int fan_out(int l) const { return l == L ? 2 : H; }
};

namespace {

bool di_shape_ok(int32_t n_hidden, int32_t width) {
  return n_hidden >= 1 && n_hidden <= kDiMaxHidden && width >= 1 && width <= kDiMaxWidth;
}

int64_t di_count(int L, int H) { return 2LL * H + H + (int64_t)(L - 1) * ((int64_t)H * H + H) + 2LL * H + 2; }

rtn_status check_dt(float dt) {
  if (!(dt > 0.f) || !std::isfinite(dt)) return failf(RTN_EINVAL, "dt must be positive and finite");
  return RTN_OK;
}

rtn_status ensure_ws(rtn_di_model* m, int64_t n, hipStream_t st) {
  if (n <= m->cap) return RTN_OK;
  m->drop_graphs();
  DI_TRY(hipStreamSynchronize(st));
  for (void** p : {(void**)&m->Z, (void**)&m->yJ, (void**)&m->partial}) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
  }
  m->cap = 0;
  const int H = m->H;
  hipError_t e = hipMalloc((void**)&m->Z, 2 * di_z_floats((int)n, H) * 4);
  if (e == hipSuccess) e = hipMalloc((void**)&m->yJ, (size_t)n * 6 * 4);
  if (e == hipSuccess) e = hipMalloc((void**)&m->partial, di_partial_floats((int)n, H) * 4 + 16);
  if (e != hipSuccess) return failf(RTN_ENOMEM, "workspace for %lld nodes: %s", (long long)n, hipGetErrorString(e));
  m->cap = n;
  return RTN_OK;
}

// Network value and Jacobian of n nodes into y [n][2], J [n][2][2].
hipError_t enqueue_network(const rtn_di_model* m, int n, const float* x, float* y, float* J, hipStream_t st) {
  const size_t zs = di_z_floats(n, m->H);
  float* Za = m->Z;
  float* Zb = m->Z + zs;
  hipError_t e;
  {
    ProfScope ps("di_first_layer", st);
    if ((e = launch_di_first_layer(n, m->H, m->params + m->w_off[0], m->params + m->b_off[0], m->act, x, Za, st)))
      return e;
  }
  for (int l = 1; l < m->L; ++l) {
    ProfScope ps("di_hidden_layer", st);
    if ((e = launch_di_hidden_layer(n, m->H, Za, m->params + m->w_off[l], m->params + m->b_off[l], m->act, Zb,
                                    m->partial, st)))
      return e;
    std::swap(Za, Zb);
  }
  ProfScope ps("di_output_layer", st);
  return launch_di_output_layer(n, m->H, m->params + m->w_off[m->L], m->params + m->b_off[m->L], Za, y, J, st);
}

}  // namespace

extern "C" {

rtn_status rtn_di_param_count(int32_t n_hidden, int32_t width, int64_t* count) {
  if (!di_shape_ok(n_hidden, width))
    return failf(RTN_EINVAL, "n_hidden must be in [1, %d] and width in [1, %d] (got %d, %d)", kDiMaxHidden,
                 kDiMaxWidth, n_hidden, width);
  if (!count) return failf(RTN_EINVAL, "count is NULL");
  *count = di_count(n_hidden, width);
  return RTN_OK;
}

rtn_status rtn_di_model_create(int32_t n_hidden, int32_t width, int32_t activation, const float* params_host,
                               rtn_di_model** out) {
  if (!out) return failf(RTN_EINVAL, "out is NULL");
  *out = nullptr;
  int64_t count;
  rtn_status s = rtn_di_param_count(n_hidden, width, &count);
  if (s) return s;
  if (activation != RTN_ACT_SILU && activation != RTN_ACT_IDENTITY)
    return failf(RTN_EINVAL, "unknown activation %d", activation);
  if (!params_host) return failf(RTN_EINVAL, "params_host is NULL");
  rtn_di_model* m = new (std::nothrow) rtn_di_model();
  if (!m) return failf(RTN_ENOMEM, "host allocation");
  m->L = n_hidden;
  m->H = width;
  m->act = activation == RTN_ACT_SILU ? 0 : 1;
  m->n_params = count;
  // device layout: the user's tensors in order, each starting on a 256-byte
  // boundary; hidden-to-hidden weights in the operand order of the packed path
  // when the width allows it
  const bool pk = di_packed(m->H);
  std::vector<int64_t> user_off;
  int64_t off = 0, uoff = 0;
  auto align = [](int64_t v) { return (v + 63) / 64 * 64; };
  for (int l = 0; l <= m->L; ++l) {
    const int64_t nw = (int64_t)m->fan_out(l) * m->fan_in(l), nb = m->fan_out(l);
    const bool hid = l > 0 && l < m->L;
    m->w_off.push_back(off);
    user_off.push_back(uoff);
    off = align(off + (hid && pk ? (int64_t)di_packed_weight_floats(m->H) : nw));
    uoff += nw;
    m->b_off.push_back(off);
    user_off.push_back(uoff);
    off = align(off + nb);
    uoff += nb;
  }
  hipError_t e = hipMalloc((void**)&m->params, (size_t)off * 4);
  if (e != hipSuccess) {
    delete m;
    return failf(RTN_ENOMEM, "hipMalloc(%lld bytes): %s", (long long)off * 4, hipGetErrorString(e));
  }
  std::vector<float> packed(pk && m->L > 1 ? di_packed_weight_floats(m->H) : 0);
  for (int l = 0; l <= m->L && e == hipSuccess; ++l) {
    const int64_t nw = (int64_t)m->fan_out(l) * m->fan_in(l), nb = m->fan_out(l);
    if (pk && l > 0 && l < m->L) {
      di_pack_weight(params_host + user_off[2 * l], m->H, packed.data());
      e = hipMemcpy(m->params + m->w_off[l], packed.data(), packed.size() * 4, hipMemcpyHostToDevice);
    } else {
      e = hipMemcpy(m->params + m->w_off[l], params_host + user_off[2 * l], nw * 4, hipMemcpyHostToDevice);
    }
    if (e == hipSuccess)
      e = hipMemcpy(m->params + m->b_off[l], params_host + user_off[2 * l + 1], nb * 4, hipMemcpyHostToDevice);
  }
  if (e == hipSuccess && di_fused_fits(m->H, 1)) {
    // the single-workgroup path for small widths: W_1, b_1, W_l^T, b_l, ..., W_out, b_out
    std::vector<float> f;
    std::vector<long> fo;
    for (int l = 0; l <= m->L; ++l) {
      const int fo_ = m->fan_out(l), fi = m->fan_in(l);
      const float* W = params_host + user_off[2 * l];
      fo.push_back((long)f.size());
      if (l > 0 && l < m->L) {
        for (int k = 0; k < fi; ++k)
          for (int c = 0; c < fo_; ++c) f.push_back(W[(size_t)c * fi + k]);
      } else {
        f.insert(f.end(), W, W + (size_t)fo_ * fi);
      }
      fo.push_back((long)f.size());
      f.insert(f.end(), params_host + user_off[2 * l + 1], params_host + user_off[2 * l + 1] + fo_);
    }
    e = hipMalloc((void**)&m->fused, f.size() * 4);
    if (e == hipSuccess) e = hipMalloc((void**)&m->fused_off, fo.size() * sizeof(long));
    if (e == hipSuccess) e = hipMemcpy(m->fused, f.data(), f.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->fused_off, fo.data(), fo.size() * sizeof(long), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    delete m;
    return hip_fail(e, "copying parameters");
  }
  *out = m;
  return RTN_OK;
}

rtn_status rtn_di_model_destroy(rtn_di_model* model) {
  delete model;
  return RTN_OK;
}

rtn_status rtn_di_linearize(const rtn_di_model* model, float dt, int32_t n_nodes, const float* x, const float* u,
                            float* x_next, float* A, float* B, float* f_D, float* J_D, void* stream) {
  rtn_status s = check_dt(dt);
  if (s) return s;
  if (n_nodes < 0) return failf(RTN_EINVAL, "n_nodes must be >= 0 (got %d)", n_nodes);
  if (n_nodes == 0) return RTN_OK;
  if (!x || !u || !x_next || !A || !B) return failf(RTN_EINVAL, "x, u, x_next, A and B must be device pointers");
  hipStream_t st = (hipStream_t)stream;
  rtn_di_model* m = const_cast<rtn_di_model*>(model);
  float* y = nullptr;
  float* J = nullptr;
  if (m) {
    if ((s = ensure_ws(m, n_nodes, st))) return s;
    y = f_D ? f_D : m->yJ;
    J = J_D ? J_D : m->yJ + (size_t)2 * n_nodes;
    DI_TRY(enqueue_network(m, n_nodes, x, y, J, st));
  } else {
    if (f_D) DI_TRY(hipMemsetAsync(f_D, 0, (size_t)n_nodes * 2 * 4, st));
    if (J_D) DI_TRY(hipMemsetAsync(J_D, 0, (size_t)n_nodes * 4 * 4, st));
  }
  ProfScope ps("di_linearize", st);
  DI_TRY(launch_di_linearize(n_nodes, dt, x, u, y, J, x_next, A, B, st));
  return RTN_OK;
}

rtn_status rtn_di_rti(const rtn_di_model* model, float dt, int32_t n_inst, const int32_t* offsets_host,
                      int32_t n_nodes, const double* Q_host, const double* R_host, const double* QN_host,
                      const float* x, const float* u, const float* xN, const float* x0, const float* x_ref,
                      double* du, double* dx, double* dxN, float* A, float* B, float* x_next, void* stream) {
  rtn_status s = check_dt(dt);
  if (s) return s;
  if ((s = check_offsets(n_inst, offsets_host, n_nodes))) return s;
  if (!Q_host || !R_host || !QN_host) return failf(RTN_EINVAL, "Q_host, R_host and QN_host are required");
  DiCost cost;
  for (int i = 0; i < 4; ++i) {
    cost.Q[i] = Q_host[i];
    cost.QN[i] = QN_host[i];
    if (!std::isfinite(cost.Q[i]) || !std::isfinite(cost.QN[i])) return failf(RTN_EINVAL, "Q or Q_N is not finite");
  }
  cost.R = R_host[0];
  if (!(cost.R > 0.0) || !std::isfinite(cost.R)) return failf(RTN_EINVAL, "R must be positive and finite");
  if (n_nodes == 0) return RTN_OK;
  if (!x || !u || !xN || !x0) return failf(RTN_EINVAL, "x, u, xN and x0 must be device pointers");
  if (!du || !dx || !dxN) return failf(RTN_EINVAL, "du, dx and dxN must be device pointers");
  std::vector<int32_t> off(offsets_host ? offsets_host : nullptr, offsets_host ? offsets_host + n_inst + 1 : nullptr);
  if (!offsets_host) off = {0, n_nodes};
  int max_h = 0;
  for (int i = 0; i < n_inst; ++i) {
    if (off[i + 1] - off[i] > kDiMaxHorizon)
      return failf(RTN_ENOTSUP, "instance %d has %d nodes; at most %d per instance", i, off[i + 1] - off[i],
                   kDiMaxHorizon);
    max_h = std::max(max_h, off[i + 1] - off[i]);
  }
  hipStream_t st = (hipStream_t)stream;
  rtn_di_model* m = const_cast<rtn_di_model*>(model);
  // instance offsets and the nominal-only case use a model-independent holder
  static thread_local rtn_di_model* nominal = nullptr;
  rtn_di_model* h = m ? m : (nominal ? nominal : (nominal = new (std::nothrow) rtn_di_model()));
  if (!h) return failf(RTN_ENOMEM, "host allocation");
  if (m && (s = ensure_ws(m, n_nodes, st))) return s;
  if (h->off_host != off) {
    h->drop_graphs();
    DI_TRY(hipStreamSynchronize(st));
    if (h->d_off && h->off_host.size() < off.size()) {
      (void)hipFree(h->d_off);
      h->d_off = nullptr;
    }
    if (!h->d_off) {
      hipError_t e = hipMalloc((void**)&h->d_off, off.size() * 4);
      if (e != hipSuccess) return failf(RTN_ENOMEM, "offsets: %s", hipGetErrorString(e));
    }
    DI_TRY(hipMemcpy(h->d_off, off.data(), off.size() * 4, hipMemcpyHostToDevice));
    h->off_host = off;
  }
  const bool fused = m && m->fused && di_fused_fits(m->H, max_h);
  float* y = m ? m->yJ : nullptr;
  float* J = m ? m->yJ + (size_t)2 * n_nodes : nullptr;
  auto enqueue = [&](hipStream_t q) -> hipError_t {
    if (fused) {
      ProfScope ps("di_fused_small", q);
      return launch_di_fused(n_inst, h->d_off, m->L, m->H, m->act, m->fused, m->fused_off, dt, cost, x, u, xN, x0,
                             x_ref, du, dx, dxN, A, B, x_next, q);
    }
    if (m) {
      hipError_t e = enqueue_network(m, n_nodes, x, y, J, q);
      if (e != hipSuccess) return e;
    }
    ProfScope ps("di_rti", q);
    return launch_di_rti(n_inst, h->d_off, dt, cost, x, u, xN, x0, x_ref, y, J, du, dx, dxN, A, B, x_next, q);
  };
  // a single launch (the one-workgroup path, or the nominal model alone) gains
  // nothing from a graph
  if (profiling_on() || fused || !m) {
    DI_TRY(enqueue(st));
    return RTN_OK;
  }
  // one captured graph per distinct argument set (offsets are fixed between
  // uploads: a change above drops the graphs)
  uint64_t key[24] = {};
  uint32_t dtb;
  memcpy(&dtb, &dt, 4);
  const void* ptrs[12] = {x, u, xN, x0, x_ref, du, dx, dxN, A, B, x_next, y};
  key[0] = (uint64_t)n_nodes | ((uint64_t)n_inst << 32);
  key[1] = dtb;
  for (int i = 0; i < 12; ++i) key[2 + i] = (uint64_t)(uintptr_t)ptrs[i];
  for (int i = 0; i < 4; ++i) memcpy(&key[14 + i], &cost.Q[i], 8);
  for (int i = 0; i < 4; ++i) memcpy(&key[18 + i], &cost.QN[i], 8);
  memcpy(&key[22], &cost.R, 8);
  rtn_di_model::Graph* hit = nullptr;
  for (auto& g : h->graphs)
    if (!memcmp(g.key, key, sizeof key)) hit = &g;
  if (!hit) {
    if (!h->cap_stream) DI_TRY(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    DI_TRY(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue(h->cap_stream);
    hipError_t e2 = hipStreamEndCapture(h->cap_stream, &graph);
    if (e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return hip_fail(e, "capturing rtn_di_rti");
    }
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    if (h->graphs.size() >= 8) {
      size_t old = 0;
      for (size_t i = 1; i < h->graphs.size(); ++i)
        if (h->graphs[i].last_use < h->graphs[old].last_use) old = i;
      (void)hipGraphExecDestroy(h->graphs[old].exec);
      h->graphs.erase(h->graphs.begin() + old);
    }
    rtn_di_model::Graph g;
    memcpy(g.key, key, sizeof key);
    g.exec = exec;
    g.last_use = 0;
    h->graphs.push_back(g);
    hit = &h->graphs.back();
  }
  hit->last_use = ++h->clock;
  DI_TRY(hipGraphLaunch(hit->exec, st));
  return RTN_OK;
}

}  // extern "C"
