// Host planning of a batched Horn-Schunck FLOW call: pair lists, per-frame
// pyramid slots (each sampled frame's pyramid is built once and shared by
// the pairs that use it -- Sec. 4.2 of the Scanner paper computes only the
// required elements, once), grouping by resolution, chunking to the
// workspace, and the device descriptor tables.  No HIP dependency.
#pragma once

#include <cstdint>
#include <vector>

#include "plan.hpp"

namespace scn {

// Device-visible descriptors (uploaded into the workspace's plan region).
struct FrameDesc {
  const uint8_t* y;  // level-0 luma plane (device)
  int64_t pitch;     // bytes per luma row
};
struct PairDesc {
  int32_t f1, f2;    // frame slots (within the chunk)
  float* out;        // [2][H][W] output (device); the training target for gradient calls
  uint8_t* fb;       // surrogate path: fell-back flag of this pair (device, may be NULL)
  float* resid;      // surrogate path: gate residual of this pair (device, may be NULL)
  const float* init; // warm start: the predecessor's output flow [2][H][W] (device; NULL for a cold pair)
  int32_t pos;       // warm start: position in its work packet (0: cold)
  int32_t pad_;
};

struct FlowChunk {
  int64_t n_frames = 0, n_pairs = 0;
  int32_t max_pos = 0;                   // warm start: largest packet position among the chunk's pairs
  size_t frames_off = 0, pairs_off = 0;  // offsets of the descriptor arrays in the plan region
};

struct FlowGroup {
  int32_t w = 0, h = 0;
  std::vector<LevelDim> dims;      // per level
  std::vector<size_t> lvl_off;     // float offset of level l (l >= 1, FP64 values) inside one frame's slot
  size_t pyr_floats = 0;           // floats per frame slot: pyramid levels 1..L-1 (+ Farneback expansion planes)
  size_t exp_off = 0;              // Farneback: float offset of the 5 expansion planes inside a frame slot
  size_t pair_floats = 0;          // floats per pair scratch (8 planes of level-0 size; 4 for Farneback)
  size_t extra_pair_bytes = 0;     // additional per-pair scratch (surrogate path)
  int64_t total_pairs = 0;
  std::vector<FlowChunk> chunks;
};

struct FlowPlan {
  std::vector<uint8_t> plan_bytes;  // uploaded to ws[0 .. plan_bytes.size())
  size_t scratch_off = 0;           // start of the reused scratch region in ws
  size_t ws_needed = 0;             // bytes for the fastest schedule (one chunk per group)
  size_t ws_min = 0;                // smallest workable workspace
  int64_t total_pairs = 0;
  int32_t levels = 0;
  int32_t solver = 0;               // SCN_SOLVER_*
  std::vector<FlowGroup> groups;
};

// Per-pair scratch planes (each of level-0 size): coefficient planes a, b, c,
// the warped second image, and two (u, v) ping-pong buffers.  Farneback pairs
// hold only the two (u, v) buffers (planes 0-3); their frames hold the five
// expansion planes (A11, A22, A12, b1, b2) of the level being solved after
// the pyramid.
enum : int32_t { kPlaneA = 0, kPlaneB = 1, kPlaneC = 2, kPlaneW = 3, kPlaneU0 = 4, kPlaneV0 = 5, kPlaneU1 = 6,
                 kPlaneV1 = 7, kPairPlanes = 8 };
enum : int32_t { kFbPairPlanes = 4, kFbExpPlanes = 5 };

// Build the plan.  flow may be NULL (sizing only).  ws_bytes = 0 plans one
// chunk per group (that plan's scratch size is ws_needed); otherwise pairs
// are chunked so that scratch fits in ws_bytes.
// extra_pair_bytes(w, h) adds per-pair scratch for the surrogate path (NULL:
// none); fell_back / residual are optional per-job surrogate outputs.
typedef size_t (*ExtraPairBytes)(int32_t w, int32_t h);
scn_status build_flow_plan(const scn_job* jobs, int32_t n_jobs, const scn_flow_params* p, float* const* flow,
                           size_t ws_bytes, FlowPlan* plan, ExtraPairBytes extra = nullptr,
                           uint8_t* const* fell_back = nullptr, float* const* residual = nullptr);

// Per-pair scratch of the warm-start schedule: step masks, frame marks, the
// active-pair list and its length (with alignment slack).
constexpr size_t kWarmPairBytes = 1024;

// Scratch layout of one chunk (offsets from the start of the scratch region).
size_t chunk_pyr_bytes(const FlowGroup& g, const FlowChunk& c);
size_t chunk_pairs_bytes(const FlowGroup& g, const FlowChunk& c);

}  // namespace scn
