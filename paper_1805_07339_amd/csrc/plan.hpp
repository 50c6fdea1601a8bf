// Host-side planning for libscn: validation, sampling resolution, pair
// lists and workspace layouts.  Plain C++17 with no HIP dependency, so the
// same code builds into a host-only test library.
#pragma once

#include <cstddef>
#include <cstdint>
#include <limits>
#include <string>
#include <vector>

#include "scn.h"

namespace scn {

// Thread-local error reporting shared by every entry point.
void set_error(const std::string& msg);
void clear_error();
const char* last_error();

struct Slice {
  std::vector<int64_t> rows;
};

// Validate a table; returns SCN_OK or an error (message set).
scn_status check_table(const scn_table* t);

// Resolve a sampling spec into slices of sampled rows (Sec. 3.2 sampling and
// slicing).  STRIDE and GATHER give one slice; each RANGE window is a slice.
scn_status resolve(const scn_job* job, std::vector<Slice>* out);

// Flattened rows (HIST/convert output order) and the S[0,1] pairs: after
// sampling, consecutive sampled rows of each slice; before sampling, (s, s+1)
// for each sampled row s with s+1 < n_frames.
struct Resolved {
  std::vector<int64_t> rows;                    // M sampled rows, output order
  std::vector<std::pair<int64_t, int64_t>> pairs;  // P pairs of table rows
  std::vector<std::pair<int32_t, int32_t>> pair_slots;  // indices into rows of each pair (-1: not a sampled row)
  std::vector<int32_t> pair_slice;                       // slice of each pair
};
scn_status resolve_flat(const scn_job* job, Resolved* out);

// Most rows one sampling may select (row positions are int32 on the device).
constexpr int64_t kMaxRows = std::numeric_limits<int32_t>::max();

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x, size_t a = kAlign) { return (x + a - 1) / a * a; }

// Pyramid level sizes: level 0 = (w, h), level l+1 = ceil(level l / 2).
struct LevelDim {
  int32_t w, h;
};
std::vector<LevelDim> level_dims(int32_t w, int32_t h, int32_t levels);
scn_status check_flow_params(const scn_flow_params* p, const scn_table* t);

// Workspace layouts -------------------------------------------------------
// HIST / convert: [plan: int64 rows[M]]
size_t hist_ws_bytes(int64_t m);
// HIST diff: [plan: int32 pair positions[P][2]]
size_t hist_diff_ws_bytes(int64_t p);
// Largest frame area whose histogram distances (at most 6 w h) fit 32 bits.
constexpr int64_t kHistDiffMaxPixels = 0xFFFFFFFFLL / 6;

// FLOW: see flow_layout() in flow planning (flow_plan.hpp).

}  // namespace scn
