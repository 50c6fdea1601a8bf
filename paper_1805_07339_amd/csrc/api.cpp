// extern "C" entry points of libscn (declared and documented in scn.h).
#include <hip/hip_runtime.h>

#include <vector>

#include "common.hpp"
#include "flow_plan.hpp"

namespace scn {
scn_status launch_hist(const scn_table& t, const int64_t* rows_dev, int64_t m, uint32_t* hist, hipStream_t s);
scn_status launch_hist_diff(const uint32_t* hist, const int32_t* slots_dev, int64_t n_pairs, uint32_t threshold,
                            uint32_t* diff, uint8_t* cut, hipStream_t s);
scn_status launch_convert(const scn_table& t, const int64_t* rows_dev, int64_t m, int32_t out_w, int32_t out_h,
                          int32_t fmt, uint8_t* out, hipStream_t s);
scn_status run_flow(const FlowPlan& plan, const scn_flow_params& p, void* ws, hipStream_t s);
size_t surrogate_ws_bytes(int32_t op, const scn_job* jobs, int32_t n_jobs, const scn_flow_params* p);
}  // namespace scn

using namespace scn;

extern "C" {

const char* scn_version(void) { return "scn 0.1 gfx950"; }

const char* scn_last_error(void) { return last_error(); }

void scn_ws_forget(const void* ws) { forget_plan(ws); }

int64_t scn_count_rows(const scn_job* job) {
  clear_error();
  Resolved r;
  scn_status st = resolve_flat(job, &r);
  return st != SCN_OK ? (int64_t)st : (int64_t)r.rows.size();
}

int64_t scn_count_pairs(const scn_job* job) {
  clear_error();
  Resolved r;
  scn_status st = resolve_flat(job, &r);
  return st != SCN_OK ? (int64_t)st : (int64_t)r.pairs.size();
}

size_t scn_workspace_bytes(int32_t op, const scn_job* jobs, int32_t n_jobs, const scn_flow_params* p) {
  clear_error();
  if (!jobs || n_jobs < 1) {
    set_error("jobs is NULL or n_jobs < 1");
    return 0;
  }
  if (op == SCN_OP_CONVERT || op == SCN_OP_HIST) {
    if (n_jobs != 1) {
      set_error("convert and hist take exactly one job");
      return 0;
    }
    Resolved r;
    if (resolve_flat(&jobs[0], &r) != SCN_OK) return 0;
    return hist_ws_bytes((int64_t)r.rows.size());
  }
  if (op == SCN_OP_HIST_DIFF) {
    if (n_jobs != 1) {
      set_error("hist diff takes exactly one job");
      return 0;
    }
    Resolved r;
    if (resolve_flat(&jobs[0], &r) != SCN_OK) return 0;
    return hist_diff_ws_bytes((int64_t)r.pair_slots.size());
  }
  if (op == SCN_OP_FLOW) {
    FlowPlan plan;
    if (build_flow_plan(jobs, n_jobs, p, nullptr, /*ws_bytes=*/0, &plan) != SCN_OK) return 0;
    return plan.ws_needed;
  }
  if (op == SCN_OP_SURROGATE || op == SCN_OP_SURROGATE_GRADS || op == SCN_OP_SURROGATE_INFER)
    return surrogate_ws_bytes(op, jobs, n_jobs, p);
  set_error("unknown op");
  return 0;
}

scn_status scn_hist(const scn_job* job, uint32_t* hist, void* ws, size_t ws_bytes, scn_stream_t stream) {
  clear_error();
  Resolved r;
  scn_status st = resolve_flat(job, &r);
  if (st != SCN_OK) return st;
  const int64_t m = (int64_t)r.rows.size();
  if (m == 0) return SCN_OK;
  if (!hist) { set_error("hist output is NULL"); return SCN_EINVAL; }
  if (!ws) { set_error("workspace is NULL"); return SCN_EINVAL; }
  if (ws_bytes < hist_ws_bytes(m)) { set_error("workspace too small for hist"); return SCN_ENOSPACE; }
  hipStream_t s = (hipStream_t)stream;
  st = upload_plan(ws, r.rows.data(), r.rows.size() * sizeof(int64_t), s);
  if (st != SCN_OK) return st;
  return launch_hist(*job->table, (const int64_t*)ws, m, hist, s);
}

scn_status scn_space_map(const scn_job* job, int32_t mode, int64_t* map) {
  clear_error();
  Resolved r;
  scn_status st = resolve_flat(job, &r);
  if (st != SCN_OK) return st;
  if (mode != SCN_SPACE_NULL && mode != SCN_SPACE_REPEAT) {
    set_error("mode must be SCN_SPACE_NULL or SCN_SPACE_REPEAT");
    return SCN_EINVAL;
  }
  const int64_t n = job->table->n_frames;
  if (n > 0 && !map) { set_error("map is NULL"); return SCN_EINVAL; }
  for (int64_t t = 0; t < n; ++t) map[t] = -1;
  const int64_t p = (int64_t)r.pairs.size();
  for (int64_t k = 0; k < p; ++k) {
    const int64_t at = r.pairs[(size_t)k].first;  // strictly increasing in k
    if (mode == SCN_SPACE_NULL) {
      map[at] = k;
    } else {
      const int64_t end = k + 1 < p ? r.pairs[(size_t)(k + 1)].first : n;
      for (int64_t t = at; t < end; ++t) map[t] = k;
    }
  }
  return SCN_OK;
}

scn_status scn_hist_diff(const scn_job* job, const uint32_t* hist, uint32_t threshold, uint32_t* diff, uint8_t* cut,
                         void* ws, size_t ws_bytes, scn_stream_t stream) {
  clear_error();
  Resolved r;
  scn_status st = resolve_flat(job, &r);
  if (st != SCN_OK) return st;
  if (job->sampling->stencil != SCN_STENCIL_AFTER) {
    set_error("hist diff needs the stencil after sampling (HIST has no output for unsampled rows)");
    return SCN_EINVAL;
  }
  const int64_t p = (int64_t)r.pair_slots.size();
  const scn_table& t = *job->table;
  if ((int64_t)t.width * t.height > kHistDiffMaxPixels) {
    set_error("frame too large for 32-bit histogram distances");
    return SCN_EUNSUPPORTED;
  }
  if (p == 0) return SCN_OK;
  if (!hist || !diff) { set_error("hist or diff is NULL"); return SCN_EINVAL; }
  if (!ws) { set_error("workspace is NULL"); return SCN_EINVAL; }
  if (ws_bytes < hist_diff_ws_bytes(p)) { set_error("workspace too small for hist diff"); return SCN_ENOSPACE; }
  std::vector<int32_t> slots((size_t)(2 * p));
  for (int64_t k = 0; k < p; ++k) {
    slots[(size_t)(2 * k)] = r.pair_slots[(size_t)k].first;
    slots[(size_t)(2 * k + 1)] = r.pair_slots[(size_t)k].second;
  }
  hipStream_t s = (hipStream_t)stream;
  st = upload_plan(ws, slots.data(), slots.size() * sizeof(int32_t), s);
  if (st != SCN_OK) return st;
  return launch_hist_diff(hist, (const int32_t*)ws, p, threshold, diff, cut, s);
}

scn_status scn_sample_convert(const scn_job* job, int32_t out_w, int32_t out_h, int32_t fmt, uint8_t* out, void* ws,
                              size_t ws_bytes, scn_stream_t stream) {
  clear_error();
  Resolved r;
  scn_status st = resolve_flat(job, &r);
  if (st != SCN_OK) return st;
  if (fmt != SCN_RGB24 && fmt != SCN_GRAY8) { set_error("fmt must be SCN_RGB24 or SCN_GRAY8"); return SCN_EINVAL; }
  if (out_w < 1 || out_h < 1 || out_w > (1 << 15) || out_h > (1 << 15)) {
    set_error("out_w and out_h must be in [1, 32768]");
    return SCN_EINVAL;
  }
  const int64_t m = (int64_t)r.rows.size();
  if (m == 0) return SCN_OK;
  if (!out) { set_error("output is NULL"); return SCN_EINVAL; }
  if (!ws) { set_error("workspace is NULL"); return SCN_EINVAL; }
  if (ws_bytes < hist_ws_bytes(m)) { set_error("workspace too small for convert"); return SCN_ENOSPACE; }
  hipStream_t s = (hipStream_t)stream;
  st = upload_plan(ws, r.rows.data(), r.rows.size() * sizeof(int64_t), s);
  if (st != SCN_OK) return st;
  return launch_convert(*job->table, (const int64_t*)ws, m, out_w, out_h, fmt, out, s);
}

scn_status scn_flow(const scn_job* jobs, int32_t n_jobs, const scn_flow_params* p, float* const* flow, void* ws,
                    size_t ws_bytes, scn_stream_t stream) {
  clear_error();
  FlowPlan plan;
  scn_status st = build_flow_plan(jobs, n_jobs, p, flow, ws_bytes, &plan);
  if (st != SCN_OK) return st;
  if (plan.total_pairs == 0) return SCN_OK;
  if (!ws) { set_error("workspace is NULL"); return SCN_EINVAL; }
  if (ws_bytes < plan.ws_min) { set_error("workspace too small for flow"); return SCN_ENOSPACE; }
  return run_flow(plan, *p, ws, (hipStream_t)stream);
}

}  // extern "C"
