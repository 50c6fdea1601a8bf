// Plan upload: the row/pair tables a call needs on the device are copied
// into the head of the caller's workspace by every call made outside graph
// capture (the copy is ordered on the call's stream).  A call captured into
// a HIP graph records no copy: its kernels read the tables that the last
// eager call left in the same workspace, so a capture is accepted only when
// exactly these plan bytes were the last ones uploaded to this workspace.
#include <cstring>
#include <deque>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "common.hpp"

namespace scn {

namespace {
std::mutex g_mu;
// the last plan uploaded to each workspace (what a captured call may rely on)
std::unordered_map<const void*, std::vector<uint8_t>> g_last;
// Host copies handed to hipMemcpyAsync stay alive here until enough newer
// uploads have happened that the stream must have consumed them; pageable
// copies are staged before hipMemcpyAsync returns, this only guards against
// a runtime that reads the source later.
std::deque<std::vector<uint8_t>> g_retired;
}  // namespace

scn_status upload_plan(void* ws, const void* bytes, size_t n, hipStream_t stream) {
  if (n == 0) return SCN_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  SCN_HIP(hipStreamIsCapturing(stream, &cs), "stream capture query");
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_last.find(ws);
  if (cs != hipStreamCaptureStatusNone) {
    const bool same = it != g_last.end() && it->second.size() == n && std::memcmp(it->second.data(), bytes, n) == 0;
    if (cs == hipStreamCaptureStatusActive && same) return SCN_OK;
    set_error("a call captured into a graph needs its plan already in the workspace: make the same call "
              "eagerly (outside capture) on this workspace first");
    return SCN_EINVAL;
  }
  std::vector<uint8_t> copy((const uint8_t*)bytes, (const uint8_t*)bytes + n);
  SCN_HIP(hipMemcpyAsync(ws, copy.data(), n, hipMemcpyHostToDevice, stream), "plan upload");
  if (it != g_last.end()) g_retired.push_back(std::move(it->second));
  while (g_retired.size() > 64) g_retired.pop_front();
  g_last[ws] = std::move(copy);
  return SCN_OK;
}

void forget_plan(const void* ws) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_last.find(ws);
  if (it != g_last.end()) {
    g_retired.push_back(std::move(it->second));
    g_last.erase(it);
  }
}

}  // namespace scn
