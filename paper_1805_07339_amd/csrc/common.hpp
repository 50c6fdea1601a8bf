// Shared device/host helpers for libscn's HIP sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "plan.hpp"

namespace scn {

// Map a HIP error to SCN_EHIP with a message naming the failing step.
inline scn_status hip_fail(hipError_t e, const char* what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return SCN_EHIP;
}

#define SCN_HIP(call, what)                          \
  do {                                               \
    hipError_t _e = (call);                          \
    if (_e != hipSuccess) return ::scn::hip_fail(_e, what); \
  } while (0)

#define SCN_LAUNCHED(what)                                   \
  do {                                                       \
    hipError_t _e = hipGetLastError();                       \
    if (_e != hipSuccess) return ::scn::hip_fail(_e, what);  \
  } while (0)

// Upload `bytes` to the start of `ws` unless exactly these bytes were the
// last plan uploaded there.  The copy is ordered on `stream`.
scn_status upload_plan(void* ws, const void* bytes, size_t n, hipStream_t stream);
void forget_plan(const void* ws);

// Optional per-kernel timing (diagnostics): while enabled, launches wrapped
// in a KernelTimer are bracketed by HIP events recorded on their stream.
// Events come from a pool created when timing is enabled.
bool timing_on();
int timing_begin(const char* name, hipStream_t s, double units = 0.0);  // returns a record id or -1
void timing_end(int id, hipStream_t s);

// Workgroups are dispatched round-robin over the chip's 8 XCDs (workgroup b
// runs on XCD b mod 8), each with its own L2.  xcd_block(b, n) renumbers the
// n workgroups of a launch so that each XCD receives one contiguous range of
// logical block ids: neighbouring tiles, which share halo rows or columns,
// then run on the same XCD and meet in its L2 instead of being fetched from
// HBM once per XCD.  A bijection of [0, n) for any n.
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t n) {
  const uint32_t per = n / kXcds, rem = n % kXcds, x = b % kXcds;
  return x * per + min(x, rem) + b / kXcds;
}

struct KernelTimer {
  int id;
  hipStream_t s;
  // `units`: work units of the launch (the Jacobi passes record pixels x
  // pairs, so that a benchmark can form algorithmic bytes per launch)
  KernelTimer(const char* name, hipStream_t st, double units = 0.0)
      : id(timing_on() ? timing_begin(name, st, units) : -1), s(st) {}
  ~KernelTimer() {
    if (id >= 0) timing_end(id, s);
  }
};

}  // namespace scn
