// C ABI of the library: argument validation, model ownership and dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/rtn.h"
#include "mlp_chain.h"
#include "model.h"
#include "profiler.h"
#include "tune.h"

using namespace rtn;

namespace {

thread_local std::string g_err;

rtn_status fail(rtn_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

}  // namespace

rtn_status rtn::failf(rtn_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

rtn_status rtn::hip_fail(hipError_t e, const char* what) {
  return fail(RTN_EHIP, "%s: %s", what, hipGetErrorString(e));
}

rtn_status rtn::inval(const char* fmt, const char* arg) { return fail(RTN_EINVAL, fmt, arg); }

#define HIP_TRY(expr)                                   \
  do {                                                  \
    hipError_t _e = (expr);                             \
    if (_e != hipSuccess) return hip_fail(_e, #expr);   \
  } while (0)

// ---------------------------------------------------------------------------
// model object

static bool width_supported(int w) { return w == 64 || w == 128 || w == 256 || w == 512 || w == 1024; }

static rtn_status check_desc(const rtn_mlp_desc* d) {
  if (!d) return fail(RTN_EINVAL, "desc is NULL");
  if (d->input < RTN_INPUT_FULL || d->input > RTN_INPUT_VB_U) return fail(RTN_EINVAL, "unknown input variant %d", d->input);
  const int din = d->input == RTN_INPUT_FULL ? kDin : (d->input == RTN_INPUT_VB ? 3 : 7);
  const int dout = d->input == RTN_INPUT_FULL ? kDout : 3;
  if (d->d_in != din) return fail(RTN_EINVAL, "d_in must be %d for this input variant (got %d)", din, d->d_in);
  if (d->d_out != dout) return fail(RTN_EINVAL, "d_out must be %d for this input variant (got %d)", dout, d->d_out);
  if (d->n_hidden < 1 || d->n_hidden > kMaxHidden)
    return fail(RTN_EINVAL, "n_hidden must be in [1, 16] (got %d)", d->n_hidden);
  if (d->activation != RTN_ACT_SILU && d->activation != RTN_ACT_IDENTITY)
    return fail(RTN_EINVAL, "unknown activation %d", d->activation);
  if (d->width <= 0) return fail(RTN_EINVAL, "width must be positive (got %d)", d->width);
  if (!width_supported(d->width)) return fail(RTN_ENOTSUP, "width %d not supported (64, 128, 256, 512, 1024)", d->width);
  return RTN_OK;
}

// Training and the exact / second-order linearisations work on the full
// residual network only.
static rtn_status full_only(const Model* m, const char* what) {
  if (m->input != RTN_INPUT_FULL)
    return fail(RTN_ENOTSUP, "%s is implemented for the full residual network (input RTN_INPUT_FULL) only", what);
  return RTN_OK;
}

int64_t rtn::Model::layer_fan_in(int l) const { return l == 0 ? desc.d_in : desc.width; }
int64_t rtn::Model::layer_fan_out(int l) const { return l == desc.n_hidden ? desc.d_out : desc.width; }

static int64_t count_params(const rtn_mlp_desc& d) {
  int64_t n = 0;
  for (int l = 0; l <= d.n_hidden; ++l) {
    int64_t fi = l == 0 ? d.d_in : d.width, fo = l == d.n_hidden ? d.d_out : d.width;
    n += fo * fi + fo;
  }
  return n;
}

rtn::Model::~Model() {
  drop_graphs();
  if (cap_stream) (void)hipStreamDestroy(cap_stream);
  for (void* p : allocs) (void)hipFree(p);
}

void rtn::Model::drop_graphs() {
  for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
  graphs.clear();
}

rtn_status rtn::Model::alloc(void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes ? bytes : 16);
  if (e != hipSuccess) return fail(RTN_ENOMEM, "hipMalloc(%zu bytes): %s", bytes, hipGetErrorString(e));
  allocs.push_back(*p);
  return RTN_OK;
}

void rtn::Model::release(void* p) {
  if (!p) return;
  for (size_t i = 0; i < allocs.size(); ++i)
    if (allocs[i] == p) {
      allocs.erase(allocs.begin() + i);
      break;
    }
  (void)hipFree(p);
}

// Internal column of user first-layer column c: v_B -> slots 0..2, u -> slots 10..13.
int rtn::Model::in_col(int c) const {
  if (input == RTN_INPUT_FULL) return c;
  return c < 3 ? c : 10 + (c - 3);
}

std::vector<float> rtn::Model::expand(const float* user) const {
  std::vector<float> out((size_t)n_params, 0.f);
  int64_t uo = 0;
  for (int l = 0; l <= L; ++l) {
    const int64_t fo = layer_fan_out(l), fi = layer_fan_in(l);
    const int64_t ufi = l == 0 ? user_desc.d_in : fi, ufo = l == L ? user_desc.d_out : fo;
    for (int64_t r = 0; r < ufo; ++r)
      for (int64_t c = 0; c < ufi; ++c) out[w_off[l] + r * fi + (l == 0 ? in_col((int)c) : c)] = user[uo + r * ufi + c];
    uo += ufo * ufi;
    for (int64_t r = 0; r < ufo; ++r) out[b_off[l] + r] = user[uo + r];
    uo += ufo;
  }
  return out;
}

void rtn::Model::contract(const float* internal, float* user) const {
  int64_t uo = 0;
  for (int l = 0; l <= L; ++l) {
    const int64_t fo = layer_fan_out(l), fi = layer_fan_in(l);
    const int64_t ufi = l == 0 ? user_desc.d_in : fi, ufo = l == L ? user_desc.d_out : fo;
    for (int64_t r = 0; r < ufo; ++r)
      for (int64_t c = 0; c < ufi; ++c) user[uo + r * ufi + c] = internal[w_off[l] + r * fi + (l == 0 ? in_col((int)c) : c)];
    uo += ufo * ufi;
    for (int64_t r = 0; r < ufo; ++r) user[uo + r] = internal[b_off[l] + r];
    uo += ufo;
  }
}

rtn_status rtn::Model::init(const rtn_mlp_desc& d) {
  (void)num_cu();  // device query outside any stream capture
  // the variants are stored embedded in the full 14-input / 6-output layout
  // (zero columns and rows), so every network kernel sees the same shapes
  user_desc = d;
  input = d.input;
  desc = d;
  desc.d_in = kDin;
  desc.d_out = kDout;
  L = d.n_hidden;
  H = d.width;
  n_params = count_params(desc);
  int64_t off = 0;
  for (int l = 0; l <= L; ++l) {
    w_off[l] = off;
    off += layer_fan_out(l) * layer_fan_in(l);
    b_off[l] = off;
    off += layer_fan_out(l);
  }
  rtn_status s;
  if ((s = alloc((void**)&params, n_params * 4))) return s;
  if ((s = alloc((void**)&grad, n_params * 4))) return s;
  if ((s = alloc((void**)&adam_m, n_params * 4))) return s;
  if ((s = alloc((void**)&adam_v, n_params * 4))) return s;
  if ((s = alloc((void**)&scales, (3 * L + 2) * 4))) return s;
  if ((s = alloc((void**)&w_out_s, (size_t)kDout * H * 4))) return s;
  HIP_TRY(hipMemset(grad, 0, n_params * 4));
  HIP_TRY(hipMemset(adam_m, 0, n_params * 4));
  HIP_TRY(hipMemset(adam_v, 0, n_params * 4));
  HIP_TRY(hipMemset(scales, 0, (3 * L + 2) * 4));
  for (int p = 0; p < 3; ++p) {
    for (int l = 0; l <= L; ++l) {
      int MT, KS;
      size_t elems = pack_geometry(p, (int)layer_fan_out(l), (int)layer_fan_in(l), &MT, &KS);
      if ((s = alloc(&packed_fw[p][l], elems * elem_bytes(p)))) return s;
      if (l < L) {
        elems = pack_geometry(p, (int)layer_fan_in(l), (int)layer_fan_out(l), &MT, &KS);
        if ((s = alloc(&packed_rw[p][l], elems * elem_bytes(p)))) return s;
      }
    }
  }
  return RTN_OK;
}

int rtn::Model::elem_bytes(int prec) { return prec == P_FP32 ? 4 : prec == P_BF16 ? 2 : 1; }

NetView rtn::Model::view(int prec) const {
  NetView v;
  memset(&v, 0, sizeof v);
  v.L = L;
  v.act = desc.activation == RTN_ACT_SILU ? 0 : 1;
  v.input = input;
  for (int l = 0; l <= L; ++l) {
    v.fw[l] = packed_fw[prec][l];
    v.bias[l] = params + b_off[l];
    if (l < L) v.rw[l] = packed_rw[prec][l];
  }
  v.w_out = params + w_off[L];
  v.w_out_s = w_out_s;
  v.wscale = scales;
  v.ascale = scales + (L + 1);
  v.gscale = scales + 2 * (L + 1);
  return v;
}

// Refresh the packed copy of one precision (and, for fp8, the weight scales)
// from the fp32 master weights if they changed since it was made.
rtn_status rtn::Model::ensure_packed(int prec, hipStream_t st, bool rev) {
  if (rev && !wout_ok) {
    HIP_TRY(launch_reorder_out(params + w_off[L], H, w_out_s, st));
    wout_ok = true;
  }
  if (!pack_ok[prec]) {
    if (prec == P_FP8) {
      for (int l = 0; l <= L; ++l) {
        int fo = (int)layer_fan_out(l), fi = (int)layer_fan_in(l);
        HIP_TRY(hipMemsetAsync(scales + l, 0, 4, st));
        HIP_TRY(launch_amax(params + w_off[l], (long)fo * fi, scales + l, st));
      }
      HIP_TRY(launch_amax_to_scale(scales, L + 1, st));
      rpack_ok[prec] = false;  // packed with the scales just replaced
    }
    PackSpec fw[kMaxHidden + 1];
    for (int l = 0; l <= L; ++l) {
      int fo = (int)layer_fan_out(l), fi = (int)layer_fan_in(l);
      fw[l] = PackSpec{params + w_off[l], fi, fo, fi, 0, scales + l, packed_fw[prec][l]};
    }
    HIP_TRY(launch_pack_layers(prec, L + 1, fw, st));
    pack_ok[prec] = true;
  }
  if (rev && !rpack_ok[prec]) {
    PackSpec rw[kMaxHidden];
    for (int l = 0; l < L; ++l) {
      int fo = (int)layer_fan_out(l), fi = (int)layer_fan_in(l);
      rw[l] = PackSpec{params + w_off[l], fi, fi, fo, 1, scales + l, packed_rw[prec][l]};
    }
    HIP_TRY(launch_pack_layers(prec, L, rw, st));
    rpack_ok[prec] = true;
  }
  return RTN_OK;
}

rtn_status rtn::Model::repack(hipStream_t st) {
  invalidate_packs();
  for (int p = 0; p < 3; ++p) {
    rtn_status s = ensure_packed(p, st);
    if (s) return s;
  }
  return RTN_OK;
}

LatNet rtn::Model::lat_view() const {
  LatNet v{};
  v.L = L;
  v.H = H;
  v.act = desc.activation == RTN_ACT_SILU ? 0 : 1;
  v.input = input;
  for (int l = 0; l <= L; ++l) {
    v.W[l] = params + w_off[l];
    v.b[l] = params + b_off[l];
  }
  return v;
}

rtn_status rtn::Model::ensure_lat_workspace(int64_t n, hipStream_t st) {
  if (n <= lat_cap) return RTN_OK;
  drop_graphs();
  if (lat_ws) {
    HIP_TRY(hipStreamSynchronize(st));
    release(lat_ws);
    lat_ws = nullptr;
  }
  lat_cap = 0;
  rtn_status s = alloc((void**)&lat_ws, (size_t)n * H * (2 + 2 * 6) * 4);
  if (s) return s;
  lat_cap = n;
  return RTN_OK;
}

rtn_status rtn::Model::ensure_workspace(int64_t n, int64_t nrow_train, hipStream_t st) {
  (void)nrow_train;
  const size_t need = (size_t)L * n * H * 4;  // fp32 stash is the largest
  if (need > stash_bytes) {
    drop_graphs();
    if (stash) {
      HIP_TRY(hipStreamSynchronize(st));
      release(stash);
      stash = nullptr;
    }
    stash_bytes = 0;
    rtn_status s = alloc(&stash, need);
    if (s) return s;
    stash_bytes = need;
  }
  const size_t need_y = (size_t)n * (kDout + kDout * kDin) * 4;
  if (need_y > tmp_bytes) {
    drop_graphs();
    if (tmp) {
      HIP_TRY(hipStreamSynchronize(st));
      release(tmp);
      tmp = nullptr;
    }
    tmp_bytes = 0;
    rtn_status s = alloc((void**)&tmp, need_y);
    if (s) return s;
    tmp_bytes = need_y;
  }
  return RTN_OK;
}

extern "C" {

const char* rtn_version(void) { return "rtn-mi355x 0.1 (gfx950)"; }

const char* rtn_last_error(void) { return g_err.c_str(); }

rtn_status rtn_param_count(const rtn_mlp_desc* desc, int64_t* count) {
  rtn_status s = check_desc(desc);
  if (s) return s;
  if (!count) return fail(RTN_EINVAL, "count is NULL");
  *count = count_params(*desc);
  return RTN_OK;
}

rtn_status rtn_model_create(const rtn_mlp_desc* desc, const float* params_host, rtn_model** out) {
  if (!out) return fail(RTN_EINVAL, "out is NULL");
  *out = nullptr;
  rtn_status s = check_desc(desc);
  if (s) return s;
  if (!params_host) return fail(RTN_EINVAL, "params_host is NULL");
  Model* m = new (std::nothrow) Model();
  if (!m) return fail(RTN_ENOMEM, "host allocation of the model failed");
  if ((s = m->init(*desc))) {
    delete m;
    return s;
  }
  const std::vector<float> full = m->expand(params_host);
  hipError_t e = hipMemcpy(m->params, full.data(), m->n_params * 4, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    delete m;
    return hip_fail(e, "hipMemcpy(params)");
  }
  if ((s = m->repack(nullptr))) {
    delete m;
    return s;
  }
  e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) {
    delete m;
    return hip_fail(e, "hipStreamSynchronize");
  }
  *out = reinterpret_cast<rtn_model*>(m);
  return RTN_OK;
}

rtn_status rtn_model_destroy(rtn_model* model) {
  if (!model) return RTN_OK;
  (void)hipDeviceSynchronize();
  delete reinterpret_cast<Model*>(model);
  return RTN_OK;
}

rtn_status rtn_model_set_params(rtn_model* model, const float* params_host) {
  if (!model) return fail(RTN_EINVAL, "model is NULL");
  if (!params_host) return fail(RTN_EINVAL, "params_host is NULL");
  Model* m = reinterpret_cast<Model*>(model);
  HIP_TRY(hipDeviceSynchronize());
  const std::vector<float> full = m->expand(params_host);
  HIP_TRY(hipMemcpy(m->params, full.data(), m->n_params * 4, hipMemcpyHostToDevice));
  m->calibrated = false;  // activation and cotangent scales belong to the old weights
  rtn_status s = m->repack(nullptr);
  if (s) return s;
  HIP_TRY(hipStreamSynchronize(nullptr));
  return RTN_OK;
}

rtn_status rtn_model_get_params(rtn_model* model, float* params_host) {
  if (!model) return fail(RTN_EINVAL, "model is NULL");
  if (!params_host) return fail(RTN_EINVAL, "params_host is NULL");
  Model* m = reinterpret_cast<Model*>(model);
  HIP_TRY(hipDeviceSynchronize());
  std::vector<float> full((size_t)m->n_params);
  HIP_TRY(hipMemcpy(full.data(), m->params, m->n_params * 4, hipMemcpyDeviceToHost));
  m->contract(full.data(), params_host);
  return RTN_OK;
}

rtn_status rtn_model_calibrate(rtn_model* model, int32_t n, const float* x, const float* u, void* stream) {
  if (!model) return fail(RTN_EINVAL, "model is NULL");
  if (n <= 0) return fail(RTN_EINVAL, "calibration needs n >= 1 nodes (got %d)", n);
  if (!x || !u) return fail(RTN_EINVAL, "x and u must be device pointers");
  Model* m = reinterpret_cast<Model*>(model);
  hipStream_t st = (hipStream_t)stream;
  rtn_status s = m->ensure_workspace(n, 0, st);
  if (s) return s;
  const int L = m->L;
  float* a_amax = m->scales + (L + 1);
  float* g_amax = m->scales + 2 * (L + 1);
  HIP_TRY(hipMemsetAsync(a_amax, 0, (2 * L + 1) * 4, st));
  if ((s = m->ensure_packed(P_FP32, st))) return s;
  NetView v = m->view(P_FP32);
  float* y = m->tmp;
  float* J = m->tmp + (size_t)n * kDout;
  HIP_TRY(launch_mlp_forward(P_FP32, m->H, v, n, x, u, nullptr, m->stash, y, a_amax, st));
  HIP_TRY(launch_mlp_reverse(P_FP32, m->H, v, n, m->stash, J, g_amax, st));
  HIP_TRY(launch_amax_to_scale(a_amax, 2 * L + 1, st));
  HIP_TRY(hipStreamSynchronize(st));
  m->calibrated = true;
  return RTN_OK;
}

rtn_status rtn_model_get_scales(const rtn_model* model, float* scales_host, int32_t* n_scales) {
  if (!model) return fail(RTN_EINVAL, "model is NULL");
  const Model* m = reinterpret_cast<const Model*>(model);
  if (n_scales) *n_scales = 3 * m->L + 2;
  if (scales_host) {
    rtn_status s = const_cast<Model*>(m)->ensure_packed(P_FP8, nullptr);  // current weight scales
    if (s) return s;
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(scales_host, m->scales, (3 * m->L + 2) * 4, hipMemcpyDeviceToHost));
    if (!m->calibrated)
      for (int i = m->L + 1; i < 3 * m->L + 2; ++i) scales_host[i] = 0.f;
  }
  return RTN_OK;
}

}  // extern "C"

// validation shared by the batched entry points
rtn_status rtn::check_offsets(int32_t n_inst, const int32_t* offsets, int32_t n_nodes) {
  if (n_nodes < 0) return fail(RTN_EINVAL, "n_nodes must be >= 0 (got %d)", n_nodes);
  if (n_inst < 1) return fail(RTN_EINVAL, "n_inst must be >= 1 (got %d)", n_inst);
  if (!offsets) {
    if (n_inst != 1) return fail(RTN_EINVAL, "offsets_host is NULL but n_inst = %d (must be 1)", n_inst);
    return RTN_OK;
  }
  if (offsets[0] != 0) return fail(RTN_EINVAL, "offsets[0] must be 0 (got %d)", offsets[0]);
  for (int i = 0; i < n_inst; ++i)
    if (offsets[i + 1] <= offsets[i])
      return fail(RTN_EINVAL, "instance %d has no nodes (offsets[%d]=%d, offsets[%d]=%d)", i, i, offsets[i], i + 1,
                  offsets[i + 1]);
  if (offsets[n_inst] != n_nodes)
    return fail(RTN_EINVAL, "offsets[n_inst] = %d but n_nodes = %d", offsets[n_inst], n_nodes);
  return RTN_OK;
}

extern "C" rtn_status rtn_linearize(const rtn_model* model, int32_t prec, const rtn_quad* quad, float dt,
                                    int32_t n_inst, const int32_t* offsets_host, int32_t n_nodes, const float* x,
                                    const float* u, float* x_next, float* A, float* B, float* f_D, float* J_D,
                                    uint8_t* status, void* stream) {
  if (!quad) return fail(RTN_EINVAL, "quad is NULL");
  if (!(dt > 0.f) || !std::isfinite(dt)) return fail(RTN_EINVAL, "dt must be positive and finite");
  if (!(quad->mass > 0.f) || !(quad->Jx > 0.f) || !(quad->Jy > 0.f) || !(quad->Jz > 0.f))
    return fail(RTN_EINVAL, "quad mass and inertia must be positive");
  rtn_status s = check_offsets(n_inst, offsets_host, n_nodes);
  if (s) return s;
  if (model && prec != RTN_FP32 && prec != RTN_BF16 && prec != RTN_FP8)
    return fail(RTN_EINVAL, "unknown precision %d", prec);
  if (n_nodes == 0) return RTN_OK;
  if (!x || !u) return fail(RTN_EINVAL, "x and u must be device pointers");
  if (!x_next || !A || !B) return fail(RTN_EINVAL, "x_next, A and B must be device pointers");
  Model* m = const_cast<Model*>(reinterpret_cast<const Model*>(model));
  if (m && prec == RTN_FP8 && !m->calibrated)
    return fail(RTN_EINVAL, "RTN_FP8 needs rtn_model_calibrate first");
  hipStream_t st = (hipStream_t)stream;
  QuadConst qc{quad->mass, quad->Jx, quad->Jy, quad->Jz, quad->arm, quad->c_tau, quad->g};
  if (!m) {
    if (f_D) HIP_TRY(hipMemsetAsync(f_D, 0, (size_t)n_nodes * kDout * 4, st));
    if (J_D) HIP_TRY(hipMemsetAsync(J_D, 0, (size_t)n_nodes * kDout * kDin * 4, st));
    ProfScope ps("rk4_linearize", st);
    HIP_TRY(launch_rk4_linearize(n_nodes, qc, dt, x, u, nullptr, nullptr, x_next, A, B, status, st));
    return RTN_OK;
  }
  if ((s = m->ensure_workspace(n_nodes, 0, st))) return s;
  float* y = f_D ? f_D : m->tmp;
  float* J = J_D ? J_D : m->tmp + (size_t)n_nodes * kDout;
  if (rtn_status sp = m->ensure_packed(prec, st)) return sp;
  const NetView v = m->view(prec);
  // tile shapes and workgroup counts: the tuned choice for this size class,
  // timed here on first use unless tuning is off or the stream is being captured
  TuneChoice tc;
  const TuneKey tk{prec, m->H, m->L, tune_size_class(n_nodes)};
  const LatNet lv = m->lat_view();
  const bool lat_ok = prec == RTN_FP32 && n_nodes <= kLatMaxNodes;
  if (lat_ok && (s = m->ensure_lat_workspace(n_nodes, st))) return s;
  float* lat_act = m->lat_ws;
  float* lat_g = lat_ok ? m->lat_ws + (size_t)2 * n_nodes * m->H : nullptr;
  if (!tune_lookup(tk, &tc) && tune_enabled()) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(st, &cs));
    if (cs == hipStreamCaptureStatusNone) {
      HIP_TRY(tune_run(prec, m->H, v, n_nodes, x, u, m->stash, y, J, lat_ok ? &lv : nullptr, lat_act, lat_g, st,
                       &tc));
      tune_store(tk, tc);
    }
  }
  if (tc.path == 1 && !lat_ok) tc = TuneChoice();  // an entry of this size class made for fewer nodes
  auto enqueue = [&](hipStream_t q) -> hipError_t {
    hipError_t e;
    if (tc.path == 1 && lat_fused_fits(lv)) {  // small network: value, Jacobian and RK4 in one launch
      const FusedRk4 rk{qc, dt, x_next, A, B, status};
      ProfScope ps("lat_fused_rk4", q);
      return launch_lat_fused(lv, n_nodes, x, u, y, J, q, &rk);
    }
    if (tc.path == 1) {
      const bool tail = lat_tail_fits(lv);  // J_D, y and RK4 in one launch after the layers
      {
        ProfScope ps("lat_forward", q);
        if ((e = launch_lat_forward(lv, n_nodes, x, u, lat_act, static_cast<float*>(m->stash), tail ? nullptr : y,
                                    q)) != hipSuccess)
          return e;
      }
      {
        ProfScope ps("lat_reverse", q);
        if ((e = launch_lat_reverse(lv, n_nodes, static_cast<float*>(m->stash), lat_g, tail ? nullptr : J, q)) !=
            hipSuccess)
          return e;
      }
      if (tail) {
        const FusedRk4 rk{qc, dt, x_next, A, B, status};
        ProfScope ps("lat_tail_rk4", q);
        return launch_lat_tail(lv, n_nodes, lat_act, lat_g, x, u, y, J, rk, q);
      }
      ProfScope ps("rk4_lanes", q);
      return launch_rk4_lanes(n_nodes, qc, dt, x, u, y, J, x_next, A, B, status, q, m->input);
    }
    {
      ProfScope ps("mlp_forward_chain", q);
      if ((e = launch_mlp_forward(prec, m->H, v, n_nodes, x, u, nullptr, m->stash, y, nullptr, q, nullptr,
                                  tc.fwd)) != hipSuccess)
        return e;
    }
    {
      ProfScope ps("mlp_reverse_chain", q);
      if ((e = launch_mlp_reverse(prec, m->H, v, n_nodes, m->stash, J, nullptr, q, tc.rev)) != hipSuccess) return e;
    }
    ProfScope ps("rk4_linearize", q);
    return launch_rk4_linearize(n_nodes, qc, dt, x, u, y, J, x_next, A, B, status, q, m->input);
  };
  // The launches are captured once per distinct argument set into a HIP
  // graph (on a private stream) and replayed as one graph launch on the caller's
  // stream.  Profiling, or RTN_NO_GRAPH=1, uses plain launches.
  static const bool no_graph = [] {
    const char* e = getenv("RTN_NO_GRAPH");
    return e && e[0] == '1';
  }();
  // A single launch (the fused small-network path) gains nothing from a graph.
  if (no_graph || profiling_on() || (tc.path == 1 && lat_fused_fits(lv))) {
    HIP_TRY(enqueue(st));
    return RTN_OK;
  }
  uint32_t qbits[7];
  memcpy(qbits, &qc, sizeof qbits);
  uint32_t dtb;
  memcpy(&dtb, &dt, 4);
  const uint64_t key[16] = {(uint64_t)prec | ((uint64_t)n_nodes << 8), (uint64_t)(uintptr_t)x, (uint64_t)(uintptr_t)u,
                            (uint64_t)(uintptr_t)x_next, (uint64_t)(uintptr_t)A, (uint64_t)(uintptr_t)B,
                            (uint64_t)(uintptr_t)y, (uint64_t)(uintptr_t)J, (uint64_t)(uintptr_t)status,
                            (uint64_t)(uintptr_t)m->stash, ((uint64_t)qbits[0] << 32) | qbits[1],
                            ((uint64_t)qbits[2] << 32) | qbits[3], ((uint64_t)qbits[4] << 32) | qbits[5],
                            ((uint64_t)qbits[6] << 32) | dtb,
                            (uint64_t)tc.fwd.variant | ((uint64_t)(uint32_t)tc.fwd.grid << 8) |
                                ((uint64_t)tc.rev.variant << 40) | ((uint64_t)tc.path << 48),
                            (uint64_t)(uint32_t)tc.rev.grid};
  Model::GraphEntry* hit = nullptr;
  for (auto& g : m->graphs)
    if (!memcmp(g.key, key, sizeof key)) hit = &g;
  if (!hit) {
    if (!m->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&m->cap_stream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(m->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue(m->cap_stream);
    hipError_t e2 = hipStreamEndCapture(m->cap_stream, &graph);
    if (e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return hip_fail(e, "capturing rtn_linearize");
    }
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    if (m->graphs.size() >= 8) {  // bounded cache: evict the least recently used
      size_t old = 0;
      for (size_t i = 1; i < m->graphs.size(); ++i)
        if (m->graphs[i].last_use < m->graphs[old].last_use) old = i;
      (void)hipGraphExecDestroy(m->graphs[old].exec);
      m->graphs.erase(m->graphs.begin() + old);
    }
    Model::GraphEntry g;
    memcpy(g.key, key, sizeof key);
    g.exec = exec;
    g.last_use = 0;
    m->graphs.push_back(g);
    hit = &m->graphs.back();
  }
  hit->last_use = ++m->graph_clock;
  HIP_TRY(hipGraphLaunch(hit->exec, st));
  return RTN_OK;
}

extern "C" rtn_status rtn_riccati(int32_t n_inst, const int32_t* offsets_host, int32_t n_nodes, const float* A,
                                  const float* B, const double* c, const double* Q_host, const double* R_host,
                                  const double* QN_host, const double* q, const double* r, const double* qN,
                                  double* K, double* kff, double* P, void* stream) {
  rtn_status s = check_offsets(n_inst, offsets_host, n_nodes);
  if (s) return s;
  if (!Q_host || !R_host || !QN_host) return fail(RTN_EINVAL, "Q_host, R_host and QN_host are required");
  for (int i = 0; i < 13 * 13; ++i)
    if (!std::isfinite(Q_host[i]) || !std::isfinite(QN_host[i])) return fail(RTN_EINVAL, "Q or Q_N is not finite");
  for (int i = 0; i < 16; ++i)
    if (!std::isfinite(R_host[i])) return fail(RTN_EINVAL, "R is not finite");
  if (n_nodes == 0) return RTN_OK;
  if (!A || !B) return fail(RTN_EINVAL, "A and B must be device pointers");
  if (!K || !kff) return fail(RTN_EINVAL, "K and kff must be device pointers");
  hipStream_t st = (hipStream_t)stream;
  // constants and instance ranges travel in one stream-ordered scratch block
  const size_t nd = 13 * 13 + 16 + 13 * 13;
  std::vector<char> host(nd * 8 + (size_t)(n_inst + 1) * 4);
  memcpy(host.data(), Q_host, 169 * 8);
  memcpy(host.data() + 169 * 8, R_host, 16 * 8);
  memcpy(host.data() + 185 * 8, QN_host, 169 * 8);
  int32_t* off = reinterpret_cast<int32_t*>(host.data() + nd * 8);
  if (offsets_host) {
    memcpy(off, offsets_host, (size_t)(n_inst + 1) * 4);
  } else {
    off[0] = 0;
    off[1] = n_nodes;
  }
  void* dev = nullptr;
  hipError_t e = hipMallocAsync(&dev, host.size(), st);
  if (e != hipSuccess) return fail(RTN_ENOMEM, "hipMallocAsync(%zu bytes): %s", host.size(), hipGetErrorString(e));
  e = hipMemcpyAsync(dev, host.data(), host.size(), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    const double* d = reinterpret_cast<const double*>(dev);
    ProfScope ps("riccati", st);
    e = launch_riccati(n_inst, reinterpret_cast<const int*>((char*)dev + nd * 8), d, d + 169, d + 185, A, B, c, q, r,
                       qN, K, kff, P, st);
  }
  // the pageable source is copied before hipMemcpyAsync returns; free when the kernel is done
  hipError_t e2 = hipFreeAsync(dev, st);
  if (e != hipSuccess) return hip_fail(e, "rtn_riccati");
  if (e2 != hipSuccess) return hip_fail(e2, "hipFreeAsync");
  return RTN_OK;
}

extern "C" rtn_status rtn_linearize_second(const rtn_model* model, int32_t prec, const rtn_quad* quad, float dt,
                                           int32_t n_inst, const int32_t* offsets_host, int32_t n_nodes,
                                           const float* x, const float* u, float* x_next, float* A, float* B,
                                           float* f_D, float* J_D, float* H_D, void* stream) {
  if (!model) return fail(RTN_EINVAL, "model is NULL (the second-order step needs a network)");
  if (!quad) return fail(RTN_EINVAL, "quad is NULL");
  if (!(dt > 0.f) || !std::isfinite(dt)) return fail(RTN_EINVAL, "dt must be positive and finite");
  if (!(quad->mass > 0.f) || !(quad->Jx > 0.f) || !(quad->Jy > 0.f) || !(quad->Jz > 0.f))
    return fail(RTN_EINVAL, "quad mass and inertia must be positive");
  rtn_status s = check_offsets(n_inst, offsets_host, n_nodes);
  if (s) return s;
  if (prec != RTN_FP32) return fail(RTN_ENOTSUP, "the second-order step is implemented in fp32 only");
  if (n_nodes == 0) return RTN_OK;
  if (!x || !u || !x_next || !A || !B) return fail(RTN_EINVAL, "x, u, x_next, A and B must be device pointers");
  Model* m = const_cast<Model*>(reinterpret_cast<const Model*>(model));
  if ((s = full_only(m, "rtn_linearize_second"))) return s;
  hipStream_t st = (hipStream_t)stream;
  QuadConst qc{quad->mass, quad->Jx, quad->Jy, quad->Jz, quad->arm, quad->c_tau, quad->g};
  const LatNet lv = m->lat_view();
  const int H = m->H, L = m->L;
  const int C = n_nodes < 4096 ? n_nodes : 4096;  // nodes per chunk
  // scratch per chunk: act [2][C][H], act' and act'' [L][C][H] each, cotangents [2][6C][H],
  // adjoints [L-1][6C][H], tangents [2][14C][H]; outputs the caller did not ask for
  const size_t per = (size_t)C * H;
  const size_t nfl = per * (2 + 2 * L + 12 + 6 * (L > 1 ? L - 1 : 0) + 28) +
                     (f_D ? 0 : (size_t)C * kDout) + (J_D ? 0 : (size_t)C * kDout * kDin) +
                     (H_D ? 0 : (size_t)C * kDout * kDin * kDin);
  void* dev = nullptr;
  hipError_t e = hipMallocAsync(&dev, nfl * 4, st);
  if (e != hipSuccess) return fail(RTN_ENOMEM, "hipMallocAsync(%zu bytes): %s", nfl * 4, hipGetErrorString(e));
  float* act = static_cast<float*>(dev);
  float* sp = act + 2 * per;
  float* spp = sp + (size_t)L * per;
  float* g = spp + (size_t)L * per;
  float* adj = g + 12 * per;
  float* tan = adj + 6 * per * (L > 1 ? L - 1 : 0);
  float* extra = tan + 28 * per;
  float* yw = f_D ? nullptr : extra;
  extra += f_D ? 0 : (size_t)C * kDout;
  float* Jw = J_D ? nullptr : extra;
  extra += J_D ? 0 : (size_t)C * kDout * kDin;
  float* Hw = H_D ? nullptr : extra;
  for (int c0 = 0; c0 < n_nodes && e == hipSuccess; c0 += C) {
    const int nc = n_nodes - c0 < C ? n_nodes - c0 : C;
    const float* xc = x + (size_t)c0 * kNx;
    const float* uc = u + (size_t)c0 * kNu;
    float* y = f_D ? f_D + (size_t)c0 * kDout : yw;
    float* J = J_D ? J_D + (size_t)c0 * kDout * kDin : Jw;
    float* Hd = H_D ? H_D + (size_t)c0 * kDout * kDin * kDin : Hw;
    ProfScope ps("linearize_second", st);
    if ((e = launch_lat_forward(lv, nc, xc, uc, act, sp, y, st, spp)) != hipSuccess) break;
    if ((e = launch_lat_reverse(lv, nc, sp, g, J, st, L > 1 ? adj : nullptr)) != hipSuccess) break;
    for (int l = 0; l < L && e == hipSuccess; ++l) {
      if (l >= 1 && (e = launch_lat_tangent(lv, nc, l, sp, tan, st)) != hipSuccess) break;
      e = launch_hess_accumulate(lv, nc, l, tan, adj, spp, Hd, l > 0, st);
    }
    if (e != hipSuccess) break;
    e = launch_rk4_quadratic(nc, qc, dt, xc, uc, y, J, Hd, x_next + (size_t)c0 * kNx, A + (size_t)c0 * kNx * kNx,
                             B + (size_t)c0 * kNx * kNu, st);
  }
  hipError_t e2 = hipFreeAsync(dev, st);
  if (e != hipSuccess) return hip_fail(e, "rtn_linearize_second");
  if (e2 != hipSuccess) return hip_fail(e2, "hipFreeAsync");
  return RTN_OK;
}

extern "C" rtn_status rtn_riccati_box(int32_t n_inst, const int32_t* offsets_host, int32_t n_nodes, const float* A,
                                      const float* B, const double* c, const double* Q_host, const double* R_host,
                                      const double* QN_host, const double* q, const double* r, const double* qN,
                                      const double* dx0, const double* du_lo, const double* du_hi, double rho,
                                      int32_t max_iter, double tol, double* du, double* dx, double* dxN,
                                      int32_t* iters, double* resid, void* stream) {
  rtn_status s = check_offsets(n_inst, offsets_host, n_nodes);
  if (s) return s;
  if (!Q_host || !R_host || !QN_host) return fail(RTN_EINVAL, "Q_host, R_host and QN_host are required");
  for (int i = 0; i < 13 * 13; ++i)
    if (!std::isfinite(Q_host[i]) || !std::isfinite(QN_host[i])) return fail(RTN_EINVAL, "Q or Q_N is not finite");
  for (int i = 0; i < 16; ++i)
    if (!std::isfinite(R_host[i])) return fail(RTN_EINVAL, "R is not finite");
  if (!(rho > 0.0) || !std::isfinite(rho)) return fail(RTN_EINVAL, "rho must be positive and finite");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(RTN_EINVAL, "tol must be positive and finite");
  if (max_iter < 1) return fail(RTN_EINVAL, "max_iter must be at least 1 (got %d)", max_iter);
  if (n_nodes == 0) return RTN_OK;
  if (!A || !B || !dx0 || !du_lo || !du_hi) return fail(RTN_EINVAL, "A, B, dx0, du_lo and du_hi must be device pointers");
  if (!du) return fail(RTN_EINVAL, "du must be a device pointer");
  hipStream_t st = (hipStream_t)stream;
  // one stream-ordered scratch block: Q, R + rho I, Q_N | offsets | K, kff, P, ADMM state
  const size_t nd = 169 + 16 + 169;
  const size_t off_bytes = ((size_t)(n_inst + 1) * 4 + 15) / 16 * 16;
  const size_t per_node = 52 + 4 + 169 + kBoxWsDoubles;
  std::vector<char> host(nd * 8 + off_bytes);
  double* hd = reinterpret_cast<double*>(host.data());
  memcpy(hd, Q_host, 169 * 8);
  for (int i = 0; i < 16; ++i) hd[169 + i] = R_host[i] + ((i % 5 == 0) ? rho : 0.0);
  memcpy(hd + 185, QN_host, 169 * 8);
  int32_t* off = reinterpret_cast<int32_t*>(host.data() + nd * 8);
  if (offsets_host) {
    memcpy(off, offsets_host, (size_t)(n_inst + 1) * 4);
  } else {
    off[0] = 0;
    off[1] = n_nodes;
  }
  const size_t bytes = host.size() + (size_t)n_nodes * per_node * 8;
  void* dev = nullptr;
  hipError_t e = hipMallocAsync(&dev, bytes, st);
  if (e != hipSuccess) return fail(RTN_ENOMEM, "hipMallocAsync(%zu bytes): %s", bytes, hipGetErrorString(e));
  e = hipMemcpyAsync(dev, host.data(), host.size(), hipMemcpyHostToDevice, st);
  const double* d = reinterpret_cast<const double*>(dev);
  const int* doff = reinterpret_cast<const int*>(static_cast<char*>(dev) + nd * 8);
  double* K = reinterpret_cast<double*>(static_cast<char*>(dev) + host.size());
  double* kff = K + (size_t)n_nodes * 52;
  double* P = kff + (size_t)n_nodes * 4;
  double* ws = P + (size_t)n_nodes * 169;
  if (e == hipSuccess) {
    ProfScope ps("riccati", st);
    e = launch_riccati(n_inst, doff, d, d + 169, d + 185, A, B, c, q, r, qN, K, kff, P, st);
  }
  if (e == hipSuccess) {
    ProfScope ps("box_admm", st);
    e = launch_box_admm(n_inst, doff, A, B, c, d + 185, d + 169, q, r, qN, K, P, dx0, du_lo, du_hi, rho, tol,
                        max_iter, ws, du, dx, dxN, iters, resid, st);
  }
  hipError_t e2 = hipFreeAsync(dev, st);
  if (e != hipSuccess) return hip_fail(e, "rtn_riccati_box");
  if (e2 != hipSuccess) return hip_fail(e2, "hipFreeAsync");
  return RTN_OK;
}

extern "C" rtn_status rtn_lq_rollout(int32_t n_inst, const int32_t* offsets_host, int32_t n_nodes,
                                     const float* A, const float* B, const double* c, const double* K,
                                     const double* kff, const double* dx0, double* dx, double* du, double* dxN,
                                     void* stream) {
  rtn_status s = check_offsets(n_inst, offsets_host, n_nodes);
  if (s) return s;
  if (n_nodes == 0) return RTN_OK;
  if (!A || !B || !K || !kff || !dx0) return fail(RTN_EINVAL, "A, B, K, kff and dx0 must be device pointers");
  if (!du) return fail(RTN_EINVAL, "du must be a device pointer");
  hipStream_t st = (hipStream_t)stream;
  std::vector<int32_t> off((size_t)n_inst + 1);
  if (offsets_host) {
    memcpy(off.data(), offsets_host, off.size() * 4);
  } else {
    off[0] = 0;
    off[1] = n_nodes;
  }
  void* dev = nullptr;
  hipError_t e = hipMallocAsync(&dev, off.size() * 4, st);
  if (e != hipSuccess) return fail(RTN_ENOMEM, "hipMallocAsync(%zu bytes): %s", off.size() * 4, hipGetErrorString(e));
  e = hipMemcpyAsync(dev, off.data(), off.size() * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    ProfScope ps("lq_rollout", st);
    e = launch_lq_rollout(n_inst, static_cast<const int*>(dev), A, B, c, K, kff, dx0, dx, du, dxN, st);
  }
  hipError_t e2 = hipFreeAsync(dev, st);
  if (e != hipSuccess) return hip_fail(e, "rtn_lq_rollout");
  if (e2 != hipSuccess) return hip_fail(e2, "hipFreeAsync");
  return RTN_OK;
}

// ---------------------------------------------------------------------------
// autotuner

static rtn_status tune_key(int32_t prec, int32_t width, int32_t n_hidden, int32_t n_nodes, TuneKey* k) {
  if (prec != RTN_FP32 && prec != RTN_BF16 && prec != RTN_FP8) return fail(RTN_EINVAL, "unknown precision %d", prec);
  if (!width_supported(width)) return fail(RTN_EINVAL, "width %d has no kernels", width);
  if (n_hidden < 1 || n_hidden > kMaxHidden) return fail(RTN_EINVAL, "n_hidden must be in [1, 16] (got %d)", n_hidden);
  if (n_nodes < 1) return fail(RTN_EINVAL, "n_nodes must be positive (got %d)", n_nodes);
  *k = TuneKey{prec, width, n_hidden, tune_size_class(n_nodes)};
  return RTN_OK;
}

extern "C" rtn_status rtn_tune_mode(int32_t on) {
  if (on != 0 && on != 1) return fail(RTN_EINVAL, "tune mode must be 0 or 1 (got %d)", on);
  tune_set_enabled(on == 1);
  return RTN_OK;
}

extern "C" rtn_status rtn_tune_get(int32_t prec, int32_t width, int32_t n_hidden, int32_t n_nodes, int32_t* choice,
                                   float* ms) {
  TuneKey k;
  rtn_status s = tune_key(prec, width, n_hidden, n_nodes, &k);
  if (s) return s;
  if (!choice) return fail(RTN_EINVAL, "choice is NULL");
  TuneChoice c;
  if (!tune_lookup(k, &c)) return fail(RTN_EINVAL, "no tuned entry for this precision, width, depth and size");
  choice[0] = c.path;
  choice[1] = c.fwd.variant;
  choice[2] = c.fwd.grid;
  choice[3] = c.rev.variant;
  choice[4] = c.rev.grid;
  if (ms) {
    ms[0] = c.fwd_ms;
    ms[1] = c.rev_ms;
  }
  return RTN_OK;
}

extern "C" rtn_status rtn_tune_set(int32_t prec, int32_t width, int32_t n_hidden, int32_t n_nodes,
                                   const int32_t* choice) {
  TuneKey k;
  rtn_status s = tune_key(prec, width, n_hidden, n_nodes, &k);
  if (s) return s;
  if (!choice) return fail(RTN_EINVAL, "choice is NULL");
  TuneChoice c;
  c.path = choice[0];
  c.fwd.variant = choice[1];
  c.fwd.grid = choice[2];
  c.rev.variant = choice[3];
  c.rev.grid = choice[4];
  if (!tune_choice_valid(prec, width, c))
    return fail(RTN_EINVAL, "choice {%d, %d, %d, %d, %d} names a path, tile shape or workgroup count that does not exist",
                choice[0], choice[1], choice[2], choice[3], choice[4]);
  tune_store(k, c);
  return RTN_OK;
}

extern "C" rtn_status rtn_tune_save(const char* path) {
  if (!path) return fail(RTN_EINVAL, "path is NULL");
  if (tune_save(path) != 0) return fail(RTN_EINVAL, "cannot write %s", path);
  return RTN_OK;
}

extern "C" rtn_status rtn_tune_load(const char* path) {
  if (!path) return fail(RTN_EINVAL, "path is NULL");
  if (tune_load(path) < 0) return fail(RTN_EINVAL, "cannot read %s", path);
  return RTN_OK;
}

// ---------------------------------------------------------------------------
// training

rtn_status rtn::Model::ensure_train_workspace(int64_t batch, hipStream_t st) {
  if (batch <= tcap) return RTN_OK;
  HIP_TRY(hipStreamSynchronize(st));
  void* old[] = {tstash, hsave, ty, tdy, tdelta[0], tdelta[1], tpart};
  for (void* p : old) release(p);
  tstash = nullptr;
  hsave = ty = tdy = tdelta[0] = tdelta[1] = tpart = nullptr;
  tcap = 0;
  rtn_status s;
  if ((s = alloc(&tstash, (size_t)L * batch * H * 4))) return s;
  if ((s = alloc((void**)&hsave, (size_t)L * batch * H * 4))) return s;
  if ((s = alloc((void**)&ty, (size_t)batch * kDout * 4))) return s;
  if ((s = alloc((void**)&tdy, (size_t)batch * kDout * 4))) return s;
  for (int i = 0; i < 2; ++i)
    if ((s = alloc((void**)&tdelta[i], (size_t)batch * H * 4))) return s;
  // split-K partial tiles: the largest over the backward products
  long part = gemm_part_floats(kDout, H, (int)batch);
  for (int l = 0; l < L; ++l) {
    const int fi = l == 0 ? kDin : H;
    part = std::max(part, gemm_part_floats(H, fi, (int)batch));
    part = std::max(part, gemm_part_floats((int)batch, l == 0 ? kDin : H, H));
  }
  part = std::max(part, gemm_part_floats((int)batch, H, kDout));
  if ((s = alloc((void**)&tpart, (size_t)part * 4))) return s;
  tcap = batch;
  return RTN_OK;
}

static rtn_status train_forward(Model* m, int32_t prec, int32_t batch, const float* in, hipStream_t st) {
  rtn_status s = m->ensure_train_workspace(batch, st);
  if (s) return s;
  if (rtn_status sp = m->ensure_packed(prec, st, false)) return sp;
  NetView v = m->view(prec);
  ProfScope ps("mlp_forward_chain(train)", st);
  HIP_TRY(launch_mlp_forward(prec, m->H, v, batch, nullptr, nullptr, in, m->tstash, m->ty, nullptr, st, m->hsave));
  m->tin = in;
  m->tbatch = batch;
  m->tprec = prec;
  return RTN_OK;
}

// dL/dparams of the last forward for upstream gradient dy [batch][6], added to the
// gradient buffer (accumulate) or written over it; din optional.
static rtn_status train_backward(Model* m, const float* dy, float* din, hipStream_t st, int accumulate = 1) {
  const int B = m->tbatch, H = m->H, L = m->L, prec = m->tprec;
  const int gate_f32 = prec == P_FP32 ? 1 : 0;
  const size_t sb = (size_t)(prec == P_FP32 ? 4 : 2);
  const char* stash = static_cast<const char*>(m->tstash);
  ProfScope ps("train_backward", st);
  float* part = m->tpart;
  // output layer W_{L+1} (6 x H): dW = dy^T h_L, db = sum dy, delta_L = (dy W) * act'(a_L)
  HIP_TRY(launch_gemm(prec, kDout, H, B, dy, 1, kDout, m->hsave + (size_t)(L - 1) * B * H, H, 1,
                      m->grad + m->w_off[L], H, m->grad + m->b_off[L], accumulate, nullptr, 1, 0, part, st));
  HIP_TRY(launch_gemm(prec, B, H, kDout, dy, kDout, 1, m->params + m->w_off[L], H, 1, m->tdelta[0], H, nullptr, 0,
                      stash + (size_t)(L - 1) * B * H * sb, gate_f32, H, part, st));
  int cur = 0;
  for (int l = L - 1; l >= 0; --l) {  // weight W_{l+1}: fan_out H, fan_in (l == 0 ? 14 : H)
    const int fi = l == 0 ? kDin : H;
    const float* hin = l == 0 ? m->tin : m->hsave + (size_t)(l - 1) * B * H;
    const float* d = m->tdelta[cur];
    HIP_TRY(launch_gemm(prec, H, fi, B, d, 1, H, hin, fi, 1, m->grad + m->w_off[l], fi, m->grad + m->b_off[l],
                        accumulate, nullptr, 1, 0, part, st));
    if (l > 0) {
      HIP_TRY(launch_gemm(prec, B, H, H, d, H, 1, m->params + m->w_off[l], H, 1, m->tdelta[cur ^ 1], H, nullptr, 0,
                          stash + (size_t)(l - 1) * B * H * sb, gate_f32, H, part, st));
      cur ^= 1;
    } else if (din) {
      HIP_TRY(launch_gemm(prec, B, kDin, H, d, H, 1, m->params + m->w_off[0], kDin, 1, din, kDin, nullptr, 0, nullptr,
                          1, 0, part, st));
    }
  }
  return RTN_OK;
}

static rtn_status adam_update(Model* m, float lr, float b1, float b2, float eps, hipStream_t st) {
  m->adam_step += 1;
  const double t = (double)m->adam_step;
  const float bc1 = (float)(1.0 - std::pow((double)b1, t));
  const float bc2 = (float)(1.0 - std::pow((double)b2, t));
  {
    ProfScope ps("adam", st);
    HIP_TRY(launch_adam(m->n_params, m->params, m->grad, m->adam_m, m->adam_v, lr, b1, b2, eps, bc1, bc2, st));
  }
  m->invalidate_packs();  // packed copies are refreshed by the next call that needs one
  m->calibrated = false;  // fp8 activation and cotangent scales belong to the old weights
  return RTN_OK;
}

static rtn_status check_train_prec(int32_t prec) {
  if (prec != RTN_FP32 && prec != RTN_BF16) return fail(RTN_ENOTSUP, "training supports RTN_FP32 and RTN_BF16 (got %d)", prec);
  return RTN_OK;
}

static rtn_status check_adam(float lr, float b1, float b2, float eps) {
  if (!(lr > 0.f) || !(b1 >= 0.f && b1 < 1.f) || !(b2 >= 0.f && b2 < 1.f) || !(eps > 0.f))
    return fail(RTN_EINVAL, "Adam needs lr > 0, 0 <= beta1, beta2 < 1, eps > 0");
  return RTN_OK;
}

extern "C" {

rtn_status rtn_mlp_forward(rtn_model* model, int32_t prec, int32_t batch, const float* in, float* out, void* stream) {
  if (!model) return fail(RTN_EINVAL, "model is NULL");
  rtn_status s = check_train_prec(prec);
  if (s) return s;
  if (batch <= 0) return fail(RTN_EINVAL, "batch must be >= 1 (got %d)", batch);
  if (!in || !out) return fail(RTN_EINVAL, "in and out must be device pointers");
  Model* m = reinterpret_cast<Model*>(model);
  if (rtn_status sv = full_only(m, "rtn_mlp_forward")) return sv;
  hipStream_t st = (hipStream_t)stream;
  if ((s = train_forward(m, prec, batch, in, st))) return s;
  HIP_TRY(hipMemcpyAsync(out, m->ty, (size_t)batch * kDout * 4, hipMemcpyDeviceToDevice, st));
  return RTN_OK;
}

rtn_status rtn_mlp_backward(rtn_model* model, int32_t batch, const float* dout, float* din, void* stream) {
  if (!model) return fail(RTN_EINVAL, "model is NULL");
  Model* m = reinterpret_cast<Model*>(model);
  if (rtn_status sv = full_only(m, "rtn_mlp_backward")) return sv;
  if (m->tprec < 0 || m->tbatch != batch)
    return fail(RTN_EINVAL, "rtn_mlp_backward needs a preceding rtn_mlp_forward with the same batch (%d)", batch);
  if (!dout) return fail(RTN_EINVAL, "dout must be a device pointer");
  return train_backward(m, dout, din, (hipStream_t)stream);
}

rtn_status rtn_model_zero_grad(rtn_model* model, void* stream) {
  if (!model) return fail(RTN_EINVAL, "model is NULL");
  Model* m = reinterpret_cast<Model*>(model);
  if (rtn_status sv = full_only(m, "rtn_model_zero_grad")) return sv;
  HIP_TRY(hipMemsetAsync(m->grad, 0, m->n_params * 4, (hipStream_t)stream));
  return RTN_OK;
}

rtn_status rtn_model_get_grad(rtn_model* model, float* grad_host) {
  if (!model || !grad_host) return fail(RTN_EINVAL, "model and grad_host are required");
  Model* m = reinterpret_cast<Model*>(model);
  if (rtn_status sv = full_only(m, "rtn_model_get_grad")) return sv;
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(grad_host, m->grad, m->n_params * 4, hipMemcpyDeviceToHost));
  return RTN_OK;
}

rtn_status rtn_adam_step(rtn_model* model, float lr, float beta1, float beta2, float eps, void* stream) {
  if (!model) return fail(RTN_EINVAL, "model is NULL");
  rtn_status s = check_adam(lr, beta1, beta2, eps);
  if (s) return s;
  if ((s = full_only(reinterpret_cast<Model*>(model), "rtn_adam_step"))) return s;
  return adam_update(reinterpret_cast<Model*>(model), lr, beta1, beta2, eps, (hipStream_t)stream);
}

rtn_status rtn_train_step(rtn_model* model, int32_t prec, int32_t batch, const float* in, const float* target,
                          float lr, float beta1, float beta2, float eps, float* loss, void* stream) {
  if (!model) return fail(RTN_EINVAL, "model is NULL");
  rtn_status s = check_train_prec(prec);
  if (s) return s;
  if ((s = check_adam(lr, beta1, beta2, eps))) return s;
  if (batch <= 0) return fail(RTN_EINVAL, "batch must be >= 1 (got %d)", batch);
  if (!in || !target) return fail(RTN_EINVAL, "in and target must be device pointers");
  Model* m = reinterpret_cast<Model*>(model);
  if (rtn_status sv = full_only(m, "rtn_train_step")) return sv;
  hipStream_t st = (hipStream_t)stream;
  if ((s = train_forward(m, prec, batch, in, st))) return s;
  HIP_TRY(launch_mse(batch * kDout, m->ty, target, m->tdy, loss, st));
  // every weight and bias gradient is written by one product (no zeroing needed)
  if ((s = train_backward(m, m->tdy, nullptr, st, 0))) return s;
  return adam_update(m, lr, beta1, beta2, eps, st);
}

rtn_status rtn_model_get_adam(rtn_model* model, float* m_host, float* v_host, int64_t* step) {
  if (!model) return fail(RTN_EINVAL, "model is NULL");
  Model* m = reinterpret_cast<Model*>(model);
  if (rtn_status sv = full_only(m, "rtn_model_get_adam")) return sv;
  HIP_TRY(hipDeviceSynchronize());
  if (m_host) HIP_TRY(hipMemcpy(m_host, m->adam_m, m->n_params * 4, hipMemcpyDeviceToHost));
  if (v_host) HIP_TRY(hipMemcpy(v_host, m->adam_v, m->n_params * 4, hipMemcpyDeviceToHost));
  if (step) *step = m->adam_step;
  return RTN_OK;
}

rtn_status rtn_model_set_adam(rtn_model* model, const float* m_host, const float* v_host, int64_t step) {
  if (!model) return fail(RTN_EINVAL, "model is NULL");
  if (step < 0) return fail(RTN_EINVAL, "step must be >= 0");
  Model* m = reinterpret_cast<Model*>(model);
  if (rtn_status sv = full_only(m, "rtn_model_set_adam")) return sv;
  HIP_TRY(hipDeviceSynchronize());
  if (m_host) HIP_TRY(hipMemcpy(m->adam_m, m_host, m->n_params * 4, hipMemcpyHostToDevice));
  if (v_host) HIP_TRY(hipMemcpy(m->adam_v, v_host, m->n_params * 4, hipMemcpyHostToDevice));
  m->adam_step = step;
  return RTN_OK;
}

}  // extern "C"

extern "C" rtn_status rtn_linearize_exact(const rtn_model* model, int32_t prec, const rtn_quad* quad, float dt,
                                          int32_t n_inst, const int32_t* offsets_host, int32_t n_nodes,
                                          const float* x, const float* u, float* x_next, float* A, float* B,
                                          void* stream) {
  if (!model) return fail(RTN_EINVAL, "model is NULL (the exact linearisation needs a network)");
  if (!quad) return fail(RTN_EINVAL, "quad is NULL");
  if (!(dt > 0.f) || !std::isfinite(dt)) return fail(RTN_EINVAL, "dt must be positive and finite");
  rtn_status s = check_offsets(n_inst, offsets_host, n_nodes);
  if (s) return s;
  if (prec != RTN_FP32 && prec != RTN_BF16 && prec != RTN_FP8) return fail(RTN_EINVAL, "unknown precision %d", prec);
  if (n_nodes == 0) return RTN_OK;
  if (!x || !u || !x_next || !A || !B) return fail(RTN_EINVAL, "x, u, x_next, A and B must be device pointers");
  Model* m = const_cast<Model*>(reinterpret_cast<const Model*>(model));
  if ((s = full_only(m, "rtn_linearize_exact"))) return s;
  if (prec == RTN_FP8 && !m->calibrated) return fail(RTN_EINVAL, "RTN_FP8 needs rtn_model_calibrate first");
  hipStream_t st = (hipStream_t)stream;
  if ((s = m->ensure_workspace(n_nodes, 0, st))) return s;
  if (n_nodes > m->exact_cap) {
    HIP_TRY(hipStreamSynchronize(st));
    m->release(m->exact_ws);
    m->exact_ws = nullptr;
    m->exact_cap = 0;
    if ((s = m->alloc((void**)&m->exact_ws, (size_t)n_nodes * (3 * 13 + 2 * 17 * 13) * 4))) return s;
    m->exact_cap = n_nodes;
  }
  const size_t n13 = (size_t)n_nodes * 13, n17 = (size_t)n_nodes * 17 * 13;
  float* xs = m->exact_ws;
  float* kp = xs + n13;
  float* kacc = kp + n13;
  float* dkp = kacc + n13;
  float* dacc = dkp + n17;
  float* y = m->tmp;
  float* J = m->tmp + (size_t)n_nodes * kDout;
  QuadConst qc{quad->mass, quad->Jx, quad->Jy, quad->Jz, quad->arm, quad->c_tau, quad->g};
  if (rtn_status sp = m->ensure_packed(prec, st)) return sp;
  const NetView v = m->view(prec);
  for (int stage = 0; stage < 4; ++stage) {
    const float* xin = stage == 0 ? x : xs;
    {
      ProfScope ps("mlp_forward_chain", st);
      HIP_TRY(launch_mlp_forward(prec, m->H, v, n_nodes, xin, u, nullptr, m->stash, y, nullptr, st));
    }
    {
      ProfScope ps("mlp_reverse_chain", st);
      HIP_TRY(launch_mlp_reverse(prec, m->H, v, n_nodes, m->stash, J, nullptr, st));
    }
    ProfScope ps("rk4_exact_stage", st);
    HIP_TRY(launch_rk4_exact_stage(n_nodes, stage, qc, dt, x, u, y, J, xs, kp, kacc, dkp, dacc, x_next, A, B, st));
  }
  return RTN_OK;
}
