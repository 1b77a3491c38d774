// Tile autotuner of the layer-chain kernels.
//
// For each (precision, width, depth, size class) the first rtn_linearize call
// times every valid (tile variant, workgroup count) candidate of the forward
// and the reverse kernel on the call's own inputs and keeps the fastest; later
// calls (and graphs captured from them) use the kept choice.  The table lives
// in the process and can be saved to / loaded from a text file.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mlp_chain.h"

namespace rtn {

struct TuneKey {
  int prec, H, L, size_class;  // size_class = floor(log2(rows of the forward))
};

// path 0: layer-chain kernels with the fwd/rev shapes; path 1: the small-batch
// per-layer kernels (fp32 only; fwd/rev unused).
struct TuneChoice {
  int path = 0;
  ChainCfg fwd, rev;
  float fwd_ms = 0.f, rev_ms = 0.f;  // measured when tuned (0 when set by hand)
};

int tune_size_class(int n);
bool tune_enabled();
void tune_set_enabled(bool on);
bool tune_lookup(const TuneKey& k, TuneChoice* c);
void tune_store(const TuneKey& k, const TuneChoice& c);
// Validate a choice against the kernels that exist for (prec, H).
bool tune_choice_valid(int prec, int H, const TuneChoice& c);
// Time the candidates on stream st (synchronises it) and return the fastest.
// x, u, y, J, stash as for the linearisation launches; lat (nullable) adds the
// small-batch path with its workspace lat_act [2][n][H], lat_g [2][6n][H].
hipError_t tune_run(int prec, int H, const NetView& net, int n, const float* x, const float* u, void* stash, float* y,
                    float* J, const LatNet* lat, float* lat_act, float* lat_g, hipStream_t st, TuneChoice* out);
// Largest batch for which the small-batch path is a tuning candidate.
constexpr int kLatMaxNodes = 4096;
// Text persistence: one line per key,
// "prec H L class path fwd_variant fwd_grid rev_variant rev_grid fwd_ms rev_ms".
int tune_save(const char* path);  // 0 ok, -1 error
int tune_load(const char* path);  // entries read, -1 error

}  // namespace rtn
