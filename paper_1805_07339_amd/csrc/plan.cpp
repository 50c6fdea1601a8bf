#include "plan.hpp"

#include <limits>

namespace scn {

namespace {
thread_local std::string g_err;
}

void set_error(const std::string& msg) { g_err = msg; }
void clear_error() { g_err.clear(); }
const char* last_error() { return g_err.c_str(); }

scn_status check_table(const scn_table* t) {
  if (!t) { set_error("table is NULL"); return SCN_EINVAL; }
  if (t->n_frames < 0) { set_error("table n_frames < 0"); return SCN_EINVAL; }
  if (t->width < 2 || t->height < 2) { set_error("table width/height must be >= 2"); return SCN_EINVAL; }
  if ((t->width & 1) || (t->height & 1)) {
    set_error("NV12 width and height must be even");
    return SCN_EUNSUPPORTED;
  }
  if (t->pitch < t->width) { set_error("table pitch < width"); return SCN_EINVAL; }
  const int64_t need = (int64_t)t->pitch * (t->height + t->height / 2);
  if (t->frame_bytes < need) { set_error("table frame_bytes < pitch * height * 3/2"); return SCN_EINVAL; }
  if (t->n_frames > 0 && !t->frames) { set_error("table frames pointer is NULL"); return SCN_EINVAL; }
  if (t->backed_first < 0 || t->backed_count < 0 ||
      (t->backed_count > 0 && t->backed_first > t->n_frames - t->backed_count)) {
    set_error("table backed rows must lie inside [0, n_frames)");
    return SCN_EINVAL;
  }
  if (t->width > (1 << 15) || t->height > (1 << 15)) {
    set_error("frame dimensions above 32768 are not supported");
    return SCN_EUNSUPPORTED;
  }
  // kernels address a frame with 32-bit byte offsets and 24-bit row products
  if (t->pitch > (1 << 20) || need > ((int64_t)1 << 31)) {
    set_error("table pitch above 2^20 bytes or frames above 2 GiB are not supported");
    return SCN_EUNSUPPORTED;
  }
  return SCN_OK;
}

scn_status resolve(const scn_job* job, std::vector<Slice>* out) {
  out->clear();
  if (!job || !job->sampling) { set_error("job or sampling is NULL"); return SCN_EINVAL; }
  scn_status st = check_table(job->table);
  if (st != SCN_OK) return st;
  const scn_sampling& s = *job->sampling;
  const int64_t n = job->table->n_frames;
  if (s.stencil != SCN_STENCIL_AFTER && s.stencil != SCN_STENCIL_BEFORE) {
    set_error("stencil must be SCN_STENCIL_AFTER or SCN_STENCIL_BEFORE");
    return SCN_EINVAL;
  }
  switch (s.kind) {
    case SCN_STRIDE: {
      if (s.step < 1) { set_error("stride step must be >= 1"); return SCN_EINVAL; }
      if (s.start < 0 || s.stop > n || s.start > s.stop) {
        set_error("stride needs 0 <= start <= stop <= n_frames");
        return SCN_EINVAL;
      }
      // count first (no overflow: 0 <= start <= stop), rows as start + i * step
      const int64_t count = s.stop > s.start ? (s.stop - s.start - 1) / s.step + 1 : 0;
      if (count > kMaxRows) { set_error("sampling selects more than 2^31 - 1 rows"); return SCN_EUNSUPPORTED; }
      Slice sl;
      sl.rows.reserve((size_t)count);
      for (int64_t i = 0; i < count; ++i) sl.rows.push_back(s.start + i * s.step);
      out->push_back(std::move(sl));
      return SCN_OK;
    }
    case SCN_GATHER: {
      if (s.n < 0 || (s.n > 0 && !s.idx)) { set_error("gather list is NULL or n < 0"); return SCN_EINVAL; }
      if (s.n > kMaxRows) { set_error("sampling selects more than 2^31 - 1 rows"); return SCN_EUNSUPPORTED; }
      Slice sl;
      sl.rows.reserve((size_t)s.n);
      for (int64_t i = 0; i < s.n; ++i) {
        const int64_t r = s.idx[i];
        if (r < 0 || r >= n) { set_error("gather row out of range"); return SCN_EINVAL; }
        if (i > 0 && r <= s.idx[i - 1]) { set_error("gather rows must be strictly increasing"); return SCN_EINVAL; }
        sl.rows.push_back(r);
      }
      out->push_back(std::move(sl));
      return SCN_OK;
    }
    case SCN_RANGE: {
      if (s.n < 0 || (s.n > 0 && !s.idx)) { set_error("range list is NULL or n < 0"); return SCN_EINVAL; }
      if (s.n > kMaxRows) { set_error("sampling selects more than 2^31 - 1 rows"); return SCN_EUNSUPPORTED; }
      // validate every window and bound the total before materialising rows
      int64_t prev_end = 0, total = 0;
      for (int64_t i = 0; i < s.n; ++i) {
        const int64_t b = s.idx[2 * i], e = s.idx[2 * i + 1];
        if (b < prev_end || e < b || b < 0 || e > n) {
          set_error("ranges must be half-open, ascending, disjoint and within the table");
          return SCN_EINVAL;
        }
        total += e - b;  // windows are disjoint inside [0, n): no overflow
        if (total > kMaxRows) { set_error("sampling selects more than 2^31 - 1 rows"); return SCN_EUNSUPPORTED; }
        prev_end = e;
      }
      for (int64_t i = 0; i < s.n; ++i) {
        const int64_t b = s.idx[2 * i], e = s.idx[2 * i + 1];
        Slice sl;
        sl.rows.reserve((size_t)(e - b));
        for (int64_t r = b; r < e; ++r) sl.rows.push_back(r);
        out->push_back(std::move(sl));
      }
      return SCN_OK;
    }
    default:
      set_error("unknown sampling kind");
      return SCN_EINVAL;
  }
}

scn_status resolve_flat(const scn_job* job, Resolved* out) {
  std::vector<Slice> sl;
  scn_status st = resolve(job, &sl);
  if (st != SCN_OK) return st;
  out->rows.clear();
  out->pairs.clear();
  out->pair_slots.clear();
  out->pair_slice.clear();
  const bool before = job->sampling->stencil == SCN_STENCIL_BEFORE;
  const int64_t n = job->table->n_frames;
  int32_t slice = -1;
  for (const Slice& s : sl) {
    ++slice;
    const int32_t base = (int32_t)out->rows.size();
    for (size_t i = 0; i < s.rows.size(); ++i) {
      out->rows.push_back(s.rows[i]);
      if (before) {
        // stencil on the original sequence: (s, s+1); the successor is not
        // a sampled row, so it has no slot in the row order
        if (s.rows[i] + 1 < n) {
          out->pairs.emplace_back(s.rows[i], s.rows[i] + 1);
          out->pair_slots.emplace_back(base + (int32_t)i, -1);
          out->pair_slice.push_back(slice);
        }
      } else if (i + 1 < s.rows.size()) {
        out->pairs.emplace_back(s.rows[i], s.rows[i + 1]);
        out->pair_slots.emplace_back(base + (int32_t)i, base + (int32_t)i + 1);
        out->pair_slice.push_back(slice);
      }
    }
  }
  if (out->rows.size() > (size_t)std::numeric_limits<int32_t>::max()) {
    set_error("too many sampled rows");
    return SCN_EUNSUPPORTED;
  }
  // every row a call reads (sampled rows, and the successors of the
  // before-sampling stencil) must be backed by memory
  const scn_table& t = *job->table;
  if (t.backed_count > 0) {
    const int64_t lo = t.backed_first, hi = t.backed_first + t.backed_count;
    auto backed = [&](int64_t r) { return r >= lo && r < hi; };
    for (int64_t r : out->rows)
      if (!backed(r)) { set_error("a sampled row is outside the table's backed rows"); return SCN_EINVAL; }
    for (const auto& pr : out->pairs)
      if (!backed(pr.first) || !backed(pr.second)) {
        set_error("a flow pair reads a row outside the table's backed rows");
        return SCN_EINVAL;
      }
  }
  return SCN_OK;
}

std::vector<LevelDim> level_dims(int32_t w, int32_t h, int32_t levels) {
  std::vector<LevelDim> d;
  d.push_back({w, h});
  for (int32_t l = 1; l < levels; ++l) {
    const LevelDim& p = d.back();
    d.push_back({(p.w + 1) / 2, (p.h + 1) / 2});
  }
  return d;
}

scn_status check_flow_params(const scn_flow_params* p, const scn_table* t) {
  if (!p) { set_error("flow params are NULL"); return SCN_EINVAL; }
  if (p->levels < 1 || p->levels > 12) { set_error("levels must be in [1, 12]"); return SCN_EINVAL; }
  if (p->iters < 0 || p->iters > 100000) { set_error("iters must be in [0, 100000]"); return SCN_EINVAL; }
  if (p->solver == SCN_SOLVER_FARNEBACK) {
    if (p->fb_poly_n != 2) { set_error("Farneback: only fb_poly_n = 2 (5x5 expansion) is supported"); return SCN_EUNSUPPORTED; }
    if (!(p->fb_sigma >= 0.5f && p->fb_sigma <= 8.0f)) { set_error("Farneback: fb_sigma must be in [0.5, 8]"); return SCN_EINVAL; }
    if (p->fb_win < 0 || p->fb_win > 8) { set_error("Farneback: fb_win must be in [0, 8]"); return SCN_EINVAL; }
    if (!(p->fb_lambda > 0.0f) || p->fb_lambda > 1e6f) { set_error("Farneback: fb_lambda must be in (0, 1e6]"); return SCN_EINVAL; }
    if (p->warm_packet >= 2) { set_error("Farneback: the temporal warm start applies to Horn-Schunck only"); return SCN_EINVAL; }
    if (p->warm_packet < 0) { set_error("warm_packet must be in [0, 2^20]"); return SCN_EINVAL; }
  } else if (p->solver != SCN_SOLVER_HS) {
    set_error("solver must be SCN_SOLVER_HS or SCN_SOLVER_FARNEBACK");
    return SCN_EINVAL;
  }
  if (p->solver == SCN_SOLVER_HS && (!(p->alpha > 0.0f) || p->alpha > 1e6f)) {
    set_error("alpha must be in (0, 1e6]");
    return SCN_EINVAL;
  }
  if (p->sweeps_per_pass < 0 || p->sweeps_per_pass > 63) {
    set_error("sweeps_per_pass must be in [0, 63]");
    return SCN_EINVAL;
  }
  if (p->tile_variant < 0 || p->tile_variant > 18) { set_error("tile_variant must be in [0, 18]"); return SCN_EINVAL; }
  if (p->warm_packet < 0 || p->warm_packet > (1 << 20)) {
    set_error("warm_packet must be in [0, 2^20]");
    return SCN_EINVAL;
  }
  if (p->warm_packet >= 2 && (p->warm_iters < 0 || p->warm_iters > 100000)) {
    set_error("warm_iters must be in [0, 100000]");
    return SCN_EINVAL;
  }
  if (t) {
    auto d = level_dims(t->width, t->height, p->levels);
    if (d.back().w < 2 || d.back().h < 2) {
      set_error("coarsest pyramid level would be smaller than 2x2");
      return SCN_EUNSUPPORTED;
    }
  }
  return SCN_OK;
}

size_t hist_ws_bytes(int64_t m) { return align_up((size_t)m * sizeof(int64_t)) + kAlign; }
size_t hist_diff_ws_bytes(int64_t p) { return align_up((size_t)p * 2 * sizeof(int32_t)) + kAlign; }

}  // namespace scn
