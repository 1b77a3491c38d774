// The model object behind rtn_model*: everything it owns lives in device memory
// allocated by the library and is freed by rtn_model_destroy.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/rtn.h"
#include "mlp_chain.h"

namespace rtn {

struct Model {
  rtn_mlp_desc desc{};       // internal layout: d_in 14, d_out 6
  rtn_mlp_desc user_desc{};  // as created (the variants have 3 or 7 inputs, 3 outputs)
  int input = RTN_INPUT_FULL;
  int L = 0, H = 0;
  int64_t n_params = 0;
  int64_t w_off[kMaxHidden + 1] = {}, b_off[kMaxHidden + 1] = {};
  float* params = nullptr;  // fp32 master copy, layout of rtn_param_count
  float* grad = nullptr;
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  int64_t adam_step = 0;
  // per-precision operand copies in MFMA fragment order
  void* packed_fw[3][kMaxHidden + 1] = {};
  void* packed_rw[3][kMaxHidden] = {};
  // fp8 scales: weights [0, L], forward operands [L+1, 2L+1], reverse operands [2L+2, 3L+1]
  float* scales = nullptr;
  float* w_out_s = nullptr;  // W_{L+1} with each row in stash order
  bool calibrated = false;
  // packed copies are refreshed lazily, per precision, after the master weights change
  bool pack_ok[3] = {false, false, false};   // forward copies (and fp8 weight scales)
  bool rpack_ok[3] = {false, false, false};  // reverse copies
  bool wout_ok = false;
  // workspace (grown on demand)
  void* stash = nullptr;
  size_t stash_bytes = 0;
  float* tmp = nullptr;
  size_t tmp_bytes = 0;
  // training workspace (grown on demand): stash and activations of the last
  // rtn_mlp_forward, its batch and precision, output, dL/dy, two delta buffers
  void* tstash = nullptr;
  float* hsave = nullptr;
  float* ty = nullptr;
  float* tdy = nullptr;
  float* tdelta[2] = {nullptr, nullptr};
  float* tpart = nullptr;  // split-K partial tiles of the backward products
  const float* tin = nullptr;
  int64_t tcap = 0;
  int32_t tbatch = 0, tprec = -1;
  // captured rtn_linearize launch sequences, replayed on the caller's stream
  struct GraphEntry {
    uint64_t key[16];
    hipGraphExec_t exec;
    uint64_t last_use;
  };
  std::vector<GraphEntry> graphs;
  uint64_t graph_clock = 0;
  hipStream_t cap_stream = nullptr;
  void drop_graphs();
  float* exact_ws = nullptr;  // exact linearisation: xs, kp, kacc [n][13]; dkp, dacc [n][17][13]
  int64_t exact_cap = 0;
  float* lat_ws = nullptr;  // small-batch path: activations [2][n][H], cotangents [2][6n][H]
  int64_t lat_cap = 0;
  std::vector<void*> allocs;

  ~Model();
  rtn_status init(const rtn_mlp_desc& d);
  rtn_status alloc(void** p, size_t bytes);
  void release(void* p);
  rtn_status repack(hipStream_t st);  // mark every packed copy stale and refresh all three
  void invalidate_packs() {
    for (int p = 0; p < 3; ++p) pack_ok[p] = rpack_ok[p] = false;
    wout_ok = false;
  }
  // rev = false: only what a forward pass reads (the training forward)
  rtn_status ensure_packed(int prec, hipStream_t st, bool rev = true);
  rtn_status ensure_workspace(int64_t n, int64_t nrow_train, hipStream_t st);
  NetView view(int prec) const;
  int in_col(int c) const;
  std::vector<float> expand(const float* user) const;         // user parameter layout -> internal
  void contract(const float* internal, float* user) const;    // internal -> user layout
  LatNet lat_view() const;
  rtn_status ensure_lat_workspace(int64_t n, hipStream_t st);
  rtn_status ensure_train_workspace(int64_t batch, hipStream_t st);
  int64_t layer_fan_in(int l) const;
  int64_t layer_fan_out(int l) const;
  static int elem_bytes(int prec);
};

rtn_status hip_fail(hipError_t e, const char* what);
rtn_status failf(rtn_status code, const char* fmt, ...);  // set the thread's error message, return code
rtn_status inval(const char* fmt, const char* arg);
rtn_status check_offsets(int32_t n_inst, const int32_t* offsets, int32_t n_nodes);

}  // namespace rtn
