#include "flow_plan.hpp"

#include <algorithm>
#include <cstring>
#include <map>
#include <unordered_map>

namespace scn {

namespace {

struct PairRef {
  int32_t job;
  int64_t r1, r2;
  float* out;
  uint8_t* fb;
  float* resid;
  const float* init;
  int32_t pos;
};

size_t warm_extra(int32_t, int32_t) { return kWarmPairBytes; }

size_t chunk_scratch(const FlowGroup& g, int64_t frames, int64_t pairs) {
  return align_up((size_t)frames * g.pyr_floats * sizeof(float)) +
         align_up((size_t)pairs * g.pair_floats * sizeof(float)) + align_up((size_t)pairs * g.extra_pair_bytes);
}

}  // namespace

size_t chunk_pyr_bytes(const FlowGroup& g, const FlowChunk& c) {
  return align_up((size_t)c.n_frames * g.pyr_floats * sizeof(float));
}
size_t chunk_pairs_bytes(const FlowGroup& g, const FlowChunk& c) {
  return align_up((size_t)c.n_pairs * g.pair_floats * sizeof(float));
}

scn_status build_flow_plan(const scn_job* jobs, int32_t n_jobs, const scn_flow_params* p, float* const* flow,
                           size_t ws_bytes, FlowPlan* plan, ExtraPairBytes extra, uint8_t* const* fell_back,
                           float* const* residual) {
  *plan = FlowPlan();
  if (!jobs || n_jobs < 1) { set_error("jobs is NULL or n_jobs < 1"); return SCN_EINVAL; }
  scn_status st = check_flow_params(p, nullptr);
  if (st != SCN_OK) return st;
  plan->levels = p->levels;
  plan->solver = p->solver;
  const bool fb = p->solver == SCN_SOLVER_FARNEBACK;
  if (fb && extra) { set_error("the surrogate's fallback runs the Horn-Schunck solver only"); return SCN_EUNSUPPORTED; }
  const bool warm = p->warm_packet >= 2;
  if (warm && extra) { set_error("the warm start applies to scn_flow only"); return SCN_EINVAL; }
  if (warm) extra = warm_extra;

  std::map<std::pair<int32_t, int32_t>, int32_t> group_of;
  std::vector<std::vector<PairRef>> gpairs;
  for (int32_t j = 0; j < n_jobs; ++j) {
    Resolved r;
    st = resolve_flat(&jobs[j], &r);
    if (st != SCN_OK) return st;
    const scn_table& t = *jobs[j].table;
    st = check_flow_params(p, &t);
    if (st != SCN_OK) return st;
    if (r.pairs.empty()) continue;
    if (flow && !flow[j]) { set_error("flow output of a job with pairs is NULL"); return SCN_EINVAL; }
    auto key = std::make_pair(t.width, t.height);
    auto it = group_of.find(key);
    int32_t gi;
    if (it == group_of.end()) {
      gi = (int32_t)plan->groups.size();
      group_of[key] = gi;
      FlowGroup g;
      g.w = t.width;
      g.h = t.height;
      g.dims = level_dims(t.width, t.height, p->levels);
      g.lvl_off.assign(p->levels, 0);
      size_t off = 0;
      for (int32_t l = 1; l < p->levels; ++l) {  // levels >= 1 are FP64: two floats per pixel
        g.lvl_off[l] = off;
        off += (size_t)2 * g.dims[l].w * g.dims[l].h;
      }
      const size_t n0 = (size_t)t.width * t.height;
      g.exp_off = off;
      g.pyr_floats = off + (fb ? (size_t)kFbExpPlanes * n0 : 0);
      g.pair_floats = (size_t)(fb ? kFbPairPlanes : kPairPlanes) * n0;
      g.extra_pair_bytes = extra ? extra(t.width, t.height) : 0;
      plan->groups.push_back(g);
      gpairs.emplace_back();
    } else {
      gi = it->second;
    }
    const size_t fsz = (size_t)2 * t.width * t.height;
    int64_t run = 0;  // index of the pair within its slice
    for (size_t k = 0; k < r.pairs.size(); ++k) {
      run = (k > 0 && r.pair_slice[k] == r.pair_slice[k - 1]) ? run + 1 : 0;
      const int32_t pos = warm ? (int32_t)(run % p->warm_packet) : 0;
      const float* init = (pos > 0 && flow) ? flow[j] + (k - 1) * fsz : nullptr;
      gpairs[gi].push_back(PairRef{j, r.pairs[k].first, r.pairs[k].second, flow ? flow[j] + k * fsz : nullptr,
                                   (fell_back && fell_back[j]) ? fell_back[j] + k : nullptr,
                                   (residual && residual[j]) ? residual[j] + k : nullptr, init, pos});
    }
  }

  int64_t total = 0;
  for (auto& v : gpairs) total += (int64_t)v.size();
  plan->total_pairs = total;
  const size_t plan_reserved = align_up((2 * sizeof(FrameDesc) + sizeof(PairDesc)) * (size_t)total + 256);
  plan->scratch_off = plan_reserved;
  size_t need = 0, min_need = 0;
  for (size_t gi = 0; gi < plan->groups.size(); ++gi) {
    FlowGroup& g = plan->groups[gi];
    g.total_pairs = (int64_t)gpairs[gi].size();
    // full-group size counts distinct frames
    std::unordered_map<int64_t, int32_t> seen;
    for (auto& pr : gpairs[gi]) {
      seen[((int64_t)pr.job << 40) ^ pr.r1];
      seen[((int64_t)pr.job << 40) ^ pr.r2];
    }
    need = std::max(need, chunk_scratch(g, (int64_t)seen.size(), g.total_pairs));
    min_need = std::max(min_need, chunk_scratch(g, 2, 1));
  }
  plan->ws_needed = plan_reserved + need;
  plan->ws_min = plan_reserved + min_need;
  if (total == 0) return SCN_OK;
  const size_t avail = (ws_bytes == 0) ? need : (ws_bytes > plan_reserved ? ws_bytes - plan_reserved : 0);
  if (ws_bytes != 0 && ws_bytes < plan->ws_min) return SCN_OK;  // caller reports SCN_ENOSPACE

  // Chunk each group and lay out the descriptor tables.
  std::vector<uint8_t>& pb = plan->plan_bytes;
  for (size_t gi = 0; gi < plan->groups.size(); ++gi) {
    FlowGroup& g = plan->groups[gi];
    const std::vector<PairRef>& prs = gpairs[gi];
    size_t i = 0;
    while (i < prs.size()) {
      std::unordered_map<int64_t, int32_t> slot;
      std::vector<FrameDesc> fds;
      std::vector<PairDesc> pds;
      while (i < prs.size()) {
        const PairRef& pr = prs[i];
        const int64_t k1 = ((int64_t)pr.job << 40) ^ pr.r1, k2 = ((int64_t)pr.job << 40) ^ pr.r2;
        const int64_t nf = (int64_t)fds.size() + (slot.count(k1) ? 0 : 1) + (slot.count(k2) ? 0 : 1);
        if (!pds.empty() && chunk_scratch(g, nf, (int64_t)pds.size() + 1) > avail) break;
        const scn_table& t = *jobs[pr.job].table;
        auto get = [&](int64_t key, int64_t row) {
          auto it = slot.find(key);
          if (it != slot.end()) return it->second;
          const int32_t s = (int32_t)fds.size();
          slot[key] = s;
          fds.push_back(FrameDesc{t.frames + row * t.frame_bytes, (int64_t)t.pitch});
          return s;
        };
        PairDesc d;
        d.f1 = get(k1, pr.r1);
        d.f2 = get(k2, pr.r2);
        d.out = pr.out;
        d.fb = pr.fb;
        d.resid = pr.resid;
        d.init = pr.init;
        d.pos = pr.pos;
        d.pad_ = 0;
        pds.push_back(d);
        ++i;
      }
      FlowChunk c;
      for (const PairDesc& d : pds) c.max_pos = std::max(c.max_pos, d.pos);
      c.n_frames = (int64_t)fds.size();
      c.n_pairs = (int64_t)pds.size();
      c.frames_off = pb.size();
      pb.resize(pb.size() + fds.size() * sizeof(FrameDesc));
      std::memcpy(pb.data() + c.frames_off, fds.data(), fds.size() * sizeof(FrameDesc));
      c.pairs_off = pb.size();
      pb.resize(pb.size() + pds.size() * sizeof(PairDesc));
      std::memcpy(pb.data() + c.pairs_off, pds.data(), pds.size() * sizeof(PairDesc));
      g.chunks.push_back(c);
    }
  }
  if (pb.size() > plan_reserved) {
    set_error("internal: flow plan exceeds its reserved region");
    return SCN_EINVAL;
  }
  return SCN_OK;
}

}  // namespace scn
