// Plan upload cache: the row/pair tables a call needs on the device are
// copied into the head of the caller's workspace once and reused by later
// calls with the same plan and workspace (so steady-state calls, and calls
// captured into a HIP graph after a first eager call, enqueue kernels only).
#include <cstring>
#include <deque>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "common.hpp"

namespace scn {

namespace {
std::mutex g_mu;
std::unordered_map<const void*, std::vector<uint8_t>> g_cache;
// Host copies handed to hipMemcpyAsync stay alive here until enough newer
// uploads have happened that the stream must have consumed them; pageable
// copies are staged before hipMemcpyAsync returns, this only guards against
// a runtime that reads the source later.
std::deque<std::vector<uint8_t>> g_retired;
}  // namespace

scn_status upload_plan(void* ws, const void* bytes, size_t n, hipStream_t stream) {
  if (n == 0) return SCN_OK;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_cache.find(ws);
  if (it != g_cache.end() && it->second.size() == n && std::memcmp(it->second.data(), bytes, n) == 0)
    return SCN_OK;
  std::vector<uint8_t> copy((const uint8_t*)bytes, (const uint8_t*)bytes + n);
  SCN_HIP(hipMemcpyAsync(ws, copy.data(), n, hipMemcpyHostToDevice, stream), "plan upload");
  if (it != g_cache.end()) g_retired.push_back(std::move(it->second));
  while (g_retired.size() > 64) g_retired.pop_front();
  g_cache[ws] = std::move(copy);
  return SCN_OK;
}

void forget_plan(const void* ws) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_cache.find(ws);
  if (it != g_cache.end()) {
    g_retired.push_back(std::move(it->second));
    g_cache.erase(it);
  }
}

}  // namespace scn
