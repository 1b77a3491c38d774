// Tile autotuner of the layer-chain kernels (see tune.h).
#include "tune.h"

#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <utility>
#include <vector>

namespace rtn {

namespace {

struct Entry {
  TuneKey k;
  TuneChoice c;
};

std::mutex g_mu;
std::vector<Entry> g_table;
bool g_loaded_env = false;
int g_enabled = -1;  // -1: not yet read from the environment

bool same(const TuneKey& a, const TuneKey& b) {
  return a.prec == b.prec && a.H == b.H && a.L == b.L && a.size_class == b.size_class;
}

// RTN_TUNE_FILE names a table that is read before the first lookup and
// rewritten after every new tuning result.
const char* env_file() {
  const char* f = getenv("RTN_TUNE_FILE");
  return f && f[0] ? f : nullptr;
}

void load_env_locked();
int load_locked(const char* path);
int save_locked(const char* path);

void load_env_locked() {
  if (g_loaded_env) return;
  g_loaded_env = true;
  if (const char* f = env_file()) (void)load_locked(f);
}

void store_locked(const TuneKey& k, const TuneChoice& c) {
  for (auto& e : g_table)
    if (same(e.k, k)) {
      e.c = c;
      return;
    }
  g_table.push_back({k, c});
}

int load_locked(const char* path) {
  FILE* f = fopen(path, "r");
  if (!f) return -1;
  int count = 0;
  char line[256];
  while (fgets(line, sizeof line, f)) {
    TuneKey k;
    TuneChoice c;
    if (line[0] == '#') continue;
    if (sscanf(line, "%d %d %d %d %d %d %d %d %d %f %f", &k.prec, &k.H, &k.L, &k.size_class, &c.path,
               &c.fwd.variant, &c.fwd.grid, &c.rev.variant, &c.rev.grid, &c.fwd_ms, &c.rev_ms) == 11 &&
        tune_choice_valid(k.prec, k.H, c)) {
      store_locked(k, c);
      ++count;
    }
  }
  fclose(f);
  return count;
}

int save_locked(const char* path) {
  FILE* f = fopen(path, "w");
  if (!f) return -1;
  fprintf(f, "# prec width n_hidden size_class path fwd_variant fwd_grid rev_variant rev_grid fwd_ms rev_ms\n");
  for (const auto& e : g_table)
    fprintf(f, "%d %d %d %d %d %d %d %d %d %.6f %.6f\n", e.k.prec, e.k.H, e.k.L, e.k.size_class, e.c.path,
            e.c.fwd.variant, e.c.fwd.grid, e.c.rev.variant, e.c.rev.grid, e.c.fwd_ms, e.c.rev_ms);
  return fclose(f) == 0 ? 0 : -1;
}

// Workgroup counts worth trying for `blocks` row blocks when `resident` fit on
// the chip at once: one or two full rounds of resident workgroups, and one
// workgroup per block (no persistence) -- each capped at the block count.
std::vector<int> grid_candidates(int blocks, int resident) {
  std::vector<int> out;
  const int cand[3] = {resident, 2 * resident, blocks};
  for (int g : cand) {
    if (g > blocks) g = blocks;
    if (g <= 0) continue;
    bool dup = false;
    for (int o : out) dup = dup || o == g;
    if (!dup) out.push_back(g);
  }
  return out;
}

}  // namespace

int tune_size_class(int n) {
  int c = 0;
  while (n > 1) {
    n >>= 1;
    ++c;
  }
  return c;
}

bool tune_enabled() {
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_enabled < 0) {
    const char* e = getenv("RTN_TUNE");
    g_enabled = (e && e[0] == '0') ? 0 : 1;
  }
  return g_enabled == 1;
}

void tune_set_enabled(bool on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_enabled = on ? 1 : 0;
}

bool tune_lookup(const TuneKey& k, TuneChoice* c) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_env_locked();
  for (const auto& e : g_table)
    if (same(e.k, k)) {
      *c = e.c;
      return true;
    }
  return false;
}

void tune_store(const TuneKey& k, const TuneChoice& c) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_env_locked();
  store_locked(k, c);
  if (const char* f = env_file()) (void)save_locked(f);
}

bool tune_choice_valid(int prec, int H, const TuneChoice& c) {
  if (prec < P_FP32 || prec > P_FP8) return false;
  if (c.path != 0 && c.path != 1) return false;
  if (c.path == 1 && prec != P_FP32) return false;
  if (c.fwd.grid < 0 || c.rev.grid < 0) return false;
  if (c.fwd.variant < 0 || c.fwd.variant >= kChainVariants) return false;
  if (c.rev.variant < 0 || c.rev.variant >= kChainVariants) return false;
  ChainGeom g;
  g.valid = 0;
  (void)chain_geometry(prec, H, 0, c.fwd.variant, 0, &g);
  if (!g.valid) return false;
  g.valid = 0;
  (void)chain_geometry(prec, H, 1, c.rev.variant, 0, &g);
  return g.valid != 0;
}

int tune_save(const char* path) {
  std::lock_guard<std::mutex> lk(g_mu);
  return save_locked(path);
}

int tune_load(const char* path) {
  std::lock_guard<std::mutex> lk(g_mu);
  return load_locked(path);
}

hipError_t tune_run(int prec, int H, const NetView& net, int n, const float* x, const float* u, void* stash, float* y,
                    float* J, const LatNet* lat, float* lat_act, float* lat_g, hipStream_t st, TuneChoice* out) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t err = hipEventCreate(&e0);
  if (err == hipSuccess) err = hipEventCreate(&e1);
  // Time of one candidate: one untimed launch, then three timed rounds of `reps`
  // back-to-back launches (reps from a first timed launch: more for short kernels);
  // the median round's average is kept, so one disturbed round (a clock change, a
  // neighbour on the device) cannot make a slow candidate look fast or a fast one slow.
  auto time_launch = [&](auto&& launch, float* ms) -> hipError_t {
    hipError_t e = launch();
    if (e != hipSuccess) return e;
    auto round = [&](int reps, float* t) -> hipError_t {
      hipError_t r;
      if ((r = hipEventRecord(e0, st)) != hipSuccess) return r;
      for (int i = 0; i < reps; ++i)
        if ((r = launch()) != hipSuccess) return r;
      if ((r = hipEventRecord(e1, st)) != hipSuccess) return r;
      if ((r = hipEventSynchronize(e1)) != hipSuccess) return r;
      if ((r = hipEventElapsedTime(t, e0, e1)) != hipSuccess) return r;
      *t /= (float)reps;
      return hipSuccess;
    };
    float t0 = 0.f;
    if ((e = round(1, &t0)) != hipSuccess) return e;
    const int reps = t0 > 20.f ? 1 : (t0 > 2.f ? 2 : 6);
    float t[3];
    for (int k = 0; k < 3; ++k)
      if ((e = round(reps, &t[k])) != hipSuccess) return e;
    if (t[0] > t[1]) std::swap(t[0], t[1]);
    if (t[1] > t[2]) std::swap(t[1], t[2]);
    if (t[0] > t[1]) std::swap(t[0], t[1]);
    *ms = t[1];
    return hipSuccess;
  };
  TuneChoice best;
  float best_f = 1e30f, best_r = 1e30f;
  for (int rev = 0; rev < 2 && err == hipSuccess; ++rev) {
    for (int v = 0; v < kChainVariants && err == hipSuccess; ++v) {
      ChainGeom g;
      g.valid = 0;
      (void)chain_geometry(prec, H, rev, v, 0, &g);
      if (!g.valid) continue;  // no such shape at this width
      if ((err = chain_geometry(prec, H, rev, v, 1, &g)) != hipSuccess) break;
      const long rows = rev ? 6L * n : (long)n;
      const int blocks = (int)((rows + g.rows - 1) / g.rows);
      const int resident = (g.resident_per_cu > 0 ? g.resident_per_cu : 1) * num_cu();
      for (int grid : grid_candidates(blocks, resident)) {
        ChainCfg cfg;
        cfg.variant = v;
        cfg.grid = grid;
        float ms = 0.f;
        if (!rev)
          err = time_launch([&] { return launch_mlp_forward(prec, H, net, n, x, u, nullptr, stash, y, nullptr, st,
                                                            nullptr, cfg); }, &ms);
        else
          err = time_launch([&] { return launch_mlp_reverse(prec, H, net, n, stash, J, nullptr, st, cfg); }, &ms);
        if (err != hipSuccess) break;
        if (!rev && ms < best_f) {
          best_f = ms;
          best.fwd = cfg;
        }
        if (rev && ms < best_r) {
          best_r = ms;
          best.rev = cfg;
        }
      }
    }
  }
  best.fwd_ms = best_f;
  best.rev_ms = best_r;
  // the small-batch per-layer path against the best chain pair
  if (err == hipSuccess && lat && prec == P_FP32 && n <= kLatMaxNodes) {
    float lf = 0.f, lr = 0.f;
    float* sp = static_cast<float*>(stash);
    if (lat_fused_fits(*lat)) {  // one launch for value and Jacobian (the form rtn_linearize runs)
      err = time_launch([&] { return launch_lat_fused(*lat, n, x, u, y, J, st); }, &lf);
    } else {
      err = time_launch([&] { return launch_lat_forward(*lat, n, x, u, lat_act, sp, y, st); }, &lf);
      if (err == hipSuccess) err = time_launch([&] { return launch_lat_reverse(*lat, n, sp, lat_g, J, st); }, &lr);
    }
    if (err == hipSuccess && lf + lr < best_f + best_r) {
      best = TuneChoice();
      best.path = 1;
      best.fwd_ms = lf;
      best.rev_ms = lr;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (err != hipSuccess) return err;
  *out = best;
  return hipSuccess;
}

}  // namespace rtn
