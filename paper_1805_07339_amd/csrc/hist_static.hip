// scn_hist_static: HIST (Sec. 5.1.2) for callers that cannot allocate
// device memory.  It runs the same kernels as scn_hist; the only scratch
// those kernels use, the table of sampled row numbers that scn_hist stages in
// the caller's workspace, lives here in a fixed device array instead.
//
// The array is a file-scope __device__ variable: each GPU the library runs on
// holds its own copy, at its own address, from module load until the process
// ends.  Host code never passes the array's name to a kernel or a copy (on
// the host that name is only a stand-in, not a device address); it looks up
// each device's address once with hipGetSymbolAddress and uses that.
#include <hip/hip_runtime.h>

#include <mutex>

#include "common.hpp"

namespace scn {
scn_status launch_hist(const scn_table& t, const int64_t* rows_dev, int64_t m, uint32_t* hist, hipStream_t s);
}  // namespace scn

using namespace scn;

constexpr int64_t kStaticRows = SCN_HIST_STATIC_MAX_ROWS;  // 65,536 rows = 512 KiB per GPU

static __device__ __align__(256) int64_t scratch[kStaticRows];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
int64_t* g_ptr[kMaxDevices] = {};  // per device: address of that device's `scratch`

// Address of the current device's copy of `scratch` (looked up on the first
// call made with that device current), or nullptr with the error set.
int64_t* device_scratch() {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    hip_fail(e, "hipGetDevice");
    return nullptr;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device ordinal beyond the supported range");
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
      return nullptr;
    }
    g_ptr[dev] = static_cast<int64_t*>(p);
  }
  return g_ptr[dev];
}

}  // namespace

extern "C" scn_status scn_hist_static(const scn_job* job, uint32_t* hist, scn_stream_t stream) {
  clear_error();
  Resolved r;
  scn_status st = resolve_flat(job, &r);
  if (st != SCN_OK) return st;
  const int64_t m = (int64_t)r.rows.size();
  if (m > kStaticRows) {
    set_error("scn_hist_static takes at most SCN_HIST_STATIC_MAX_ROWS (65536) sampled rows; use scn_hist with a "
              "workspace for more");
    return SCN_ENOSPACE;
  }
  if (m == 0) return SCN_OK;
  if (!hist) { set_error("hist output is NULL"); return SCN_EINVAL; }
  int64_t* rows_dev = device_scratch();
  if (!rows_dev) return SCN_EHIP;
  hipStream_t s = (hipStream_t)stream;
  // the row table overwrites the whole prefix the kernels read; nothing else
  // in the array is read, so no clearing is needed
  st = upload_plan(rows_dev, r.rows.data(), r.rows.size() * sizeof(int64_t), s);
  if (st != SCN_OK) return st;
  return launch_hist(*job->table, rows_dev, m, hist, s);
}
