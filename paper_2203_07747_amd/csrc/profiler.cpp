// Per-kernel timing records (see rtn_profile_enable in include/rtn.h).
#include "profiler.h"

#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/rtn.h"

namespace rtn {
namespace {

struct Rec {
  const char* name;
  hipEvent_t a, b;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t get_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

}  // namespace

bool profiling_on() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_on;
}

ProfScope::ProfScope(const char* name, hipStream_t st) : st_(st) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on || g_recs.size() >= 65536) return;
  Rec r{name, get_event(), get_event()};
  if (!r.a || !r.b) return;
  if (hipEventRecord(r.a, st) != hipSuccess) return;
  slot_ = (int)g_recs.size();
  g_recs.push_back(r);
}

ProfScope::~ProfScope() {
  if (slot_ < 0) return;
  std::lock_guard<std::mutex> lk(g_mu);
  (void)hipEventRecord(g_recs[slot_].b, st_);
}

}  // namespace rtn

using namespace rtn;

extern "C" rtn_status rtn_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = on != 0;
  return RTN_OK;
}

extern "C" rtn_status rtn_profile_read(rtn_kernel_time* out, int32_t max_entries, int32_t* n_entries) {
  if (!n_entries) return RTN_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  std::vector<rtn_kernel_time> agg;
  for (const Rec& r : g_recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) ms = -1.f;
    size_t i = 0;
    for (; i < agg.size(); ++i)
      if (!strncmp(agg[i].name, r.name, sizeof agg[i].name)) break;
    if (i == agg.size()) {
      rtn_kernel_time t;
      memset(&t, 0, sizeof t);
      strncpy(t.name, r.name, sizeof t.name - 1);
      agg.push_back(t);
    }
    agg[i].calls += 1;
    if (ms >= 0) agg[i].total_ms += ms;
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  *n_entries = (int32_t)agg.size();
  if (out)
    for (int i = 0; i < (int)agg.size() && i < max_entries; ++i) out[i] = agg[i];
  return RTN_OK;
}
