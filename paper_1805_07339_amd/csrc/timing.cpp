// Per-kernel HIP-event timing for diagnostics and the benchmark's roofline
// figures (scn_timing_* in scn.h).
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

namespace scn {

namespace {
struct Rec {
  std::string name;
  int ev0, ev1;
  double units;
};
std::mutex g_mu;
bool g_on = false;
std::vector<hipEvent_t> g_pool;
size_t g_next = 0;
std::vector<Rec> g_recs;
int64_t g_dropped = 0;

void destroy_pool() {
  for (hipEvent_t e : g_pool) (void)hipEventDestroy(e);
  g_pool.clear();
  g_next = 0;
  g_recs.clear();
}
}  // namespace

bool timing_on() { return g_on; }

int timing_begin(const char* name, hipStream_t s, double units) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on) return -1;
  if (g_next + 2 > g_pool.size()) {
    ++g_dropped;
    return -1;
  }
  Rec r{name, (int)g_next, (int)g_next + 1, units};
  g_next += 2;
  if (hipEventRecord(g_pool[r.ev0], s) != hipSuccess) return -1;
  g_recs.push_back(r);
  return (int)g_recs.size() - 1;
}

void timing_end(int id, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (id < 0 || id >= (int)g_recs.size()) return;
  (void)hipEventRecord(g_pool[g_recs[id].ev1], s);
}

}  // namespace scn

using namespace scn;

extern "C" {

scn_status scn_timing_enable(int32_t enable, int32_t max_launches) {
  clear_error();
  std::lock_guard<std::mutex> lk(g_mu);
  destroy_pool();
  g_dropped = 0;
  g_on = false;
  if (!enable) return SCN_OK;
  if (max_launches < 1 || max_launches > (1 << 22)) {
    set_error("max_launches must be in [1, 4194304]");
    return SCN_EINVAL;
  }
  g_pool.resize((size_t)2 * max_launches);
  for (auto& e : g_pool) {
    hipError_t err = hipEventCreate(&e);
    if (err != hipSuccess) {
      g_pool.clear();
      return hip_fail(err, "hipEventCreate");
    }
  }
  g_on = true;
  return SCN_OK;
}

scn_status scn_timing_reset(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_next = 0;
  g_recs.clear();
  g_dropped = 0;
  return SCN_OK;
}

scn_status scn_timing_read(const char* kernel, double* total_ms, int64_t* launches) {
  clear_error();
  if (!kernel || !total_ms || !launches) {
    set_error("NULL argument");
    return SCN_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  double tot = 0.0;
  int64_t n = 0;
  for (const Rec& r : g_recs) {
    if (r.name != kernel) continue;
    SCN_HIP(hipEventSynchronize(g_pool[r.ev1]), "hipEventSynchronize");
    float ms = 0.f;
    SCN_HIP(hipEventElapsedTime(&ms, g_pool[r.ev0], g_pool[r.ev1]), "hipEventElapsedTime");
    tot += ms;
    ++n;
  }
  *total_ms = tot;
  *launches = n;
  if (g_dropped) {
    set_error("timing pool exhausted; some launches were not recorded");
    return SCN_ENOSPACE;
  }
  return SCN_OK;
}

scn_status scn_timing_units(const char* kernel, double* units) {
  clear_error();
  if (!kernel || !units) {
    set_error("NULL argument");
    return SCN_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  double u = 0.0;
  for (const Rec& r : g_recs)
    if (r.name == kernel) u += r.units;
  *units = u;
  if (g_dropped) {
    set_error("timing pool exhausted; some launches were not recorded");
    return SCN_ENOSPACE;
  }
  return SCN_OK;
}

}  // extern "C"
