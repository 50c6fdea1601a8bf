// Host-only driver for the planner under AddressSanitizer and
// UndefinedBehaviorSanitizer: resolves sampling specs (valid, adversarial and
// invalid) and builds flow plans, checking the counts and status codes.  Built
// with g++ from plan.cpp and flow_plan.cpp alone (no HIP), by the CPU test
// suite.  Exit status 0 = every check passed.
#include <cstdint>
#include <cstdio>
#include <limits>
#include <vector>

#include "flow_plan.hpp"
#include "plan.hpp"

using namespace scn;

static int g_fail = 0;
#define CHECK(c)                                                  \
  do {                                                            \
    if (!(c)) {                                                   \
      std::printf("FAIL line %d: %s (%s)\n", __LINE__, #c, last_error()); \
      ++g_fail;                                                   \
    }                                                             \
  } while (0)

static scn_table table(int64_t n, int32_t w = 64, int32_t h = 48) {
  static uint8_t dummy[16];
  scn_table t{};
  t.frames = dummy;  // never dereferenced by the planner
  t.width = w;
  t.height = h;
  t.pitch = w;
  t.frame_bytes = (int64_t)w * h * 3 / 2;
  t.n_frames = n;
  return t;
}

static scn_status resolve_spec(const scn_table& t, scn_sampling s, Resolved* r) {
  scn_job j{&t, &s};
  return resolve_flat(&j, r);
}

static scn_sampling stride(int64_t start, int64_t step, int64_t stop) {
  scn_sampling s{};
  s.kind = SCN_STRIDE;
  s.start = start;
  s.step = step;
  s.stop = stop;
  return s;
}

int main() {
  const int64_t kI64 = std::numeric_limits<int64_t>::max();
  Resolved r;
  // STRIDE: ordinary, empty, and a step so large that start + step overflows
  scn_table t = table(2400);
  CHECK(resolve_spec(t, stride(0, 24, 2400), &r) == SCN_OK && r.rows.size() == 100 && r.pairs.size() == 99);
  CHECK(resolve_spec(t, stride(5, 1, 5), &r) == SCN_OK && r.rows.empty() && r.pairs.empty());
  CHECK(resolve_spec(t, stride(1, kI64, 2), &r) == SCN_OK && r.rows.size() == 1 && r.rows[0] == 1);
  CHECK(resolve_spec(t, stride(2399, kI64 - 5, 2400), &r) == SCN_OK && r.rows.size() == 1);
  CHECK(resolve_spec(t, stride(0, 0, 10), &r) == SCN_EINVAL);
  CHECK(resolve_spec(t, stride(-1, 1, 10), &r) == SCN_EINVAL);
  CHECK(resolve_spec(t, stride(0, 1, 2401), &r) == SCN_EINVAL);
  // a huge table: the row count is refused before any row is materialised
  scn_table big = table(int64_t(1) << 40);
  CHECK(resolve_spec(big, stride(0, 1, int64_t(1) << 40), &r) == SCN_EUNSUPPORTED);
  CHECK(resolve_spec(big, stride(0, int64_t(1) << 20, int64_t(1) << 40), &r) == SCN_OK &&
        r.rows.size() == (size_t(1) << 20));
  // GATHER: valid, unsorted, duplicate, out of range, absurd length
  std::vector<int64_t> idx = {1, 5, 9, 2399};
  scn_sampling g{};
  g.kind = SCN_GATHER;
  g.idx = idx.data();
  g.n = (int64_t)idx.size();
  CHECK(resolve_spec(t, g, &r) == SCN_OK && r.rows.size() == 4 && r.pairs.size() == 3);
  g.stencil = SCN_STENCIL_BEFORE;  // the last table row has no successor
  CHECK(resolve_spec(t, g, &r) == SCN_OK && r.pairs.size() == 3 && r.pairs[2].second == 10);
  g.stencil = SCN_STENCIL_AFTER;
  std::vector<int64_t> bad = {3, 3};
  g.idx = bad.data();
  g.n = 2;
  CHECK(resolve_spec(t, g, &r) == SCN_EINVAL);
  bad = {5, 2};
  CHECK(resolve_spec(t, g, &r) == SCN_EINVAL);
  bad = {0, 2400};
  CHECK(resolve_spec(t, g, &r) == SCN_EINVAL);
  g.n = int64_t(1) << 33;  // refused before the list is read
  CHECK(resolve_spec(t, g, &r) == SCN_EUNSUPPORTED);
  // RANGE: windows are slices; overlapping, reversed, too long
  std::vector<int64_t> win = {10, 14, 20, 23};
  scn_sampling rg{};
  rg.kind = SCN_RANGE;
  rg.idx = win.data();
  rg.n = 2;
  CHECK(resolve_spec(t, rg, &r) == SCN_OK && r.rows.size() == 7 && r.pairs.size() == 5);
  win = {0, 5, 4, 8};
  CHECK(resolve_spec(t, rg, &r) == SCN_EINVAL);
  win = {5, 3, 6, 7};
  CHECK(resolve_spec(t, rg, &r) == SCN_EINVAL);
  std::vector<int64_t> huge = {0, int64_t(1) << 40};
  rg.idx = huge.data();
  rg.n = 1;
  CHECK(resolve_spec(big, rg, &r) == SCN_EUNSUPPORTED);
  // backed windows: rows 100 .. 139 of a 2400-row table
  scn_table win_t = table(2400);
  win_t.backed_first = 100;
  win_t.backed_count = 40;
  CHECK(resolve_spec(win_t, stride(100, 3, 140), &r) == SCN_OK);
  CHECK(resolve_spec(win_t, stride(99, 3, 140), &r) == SCN_EINVAL);
  std::vector<int64_t> inner = {100, 140};
  rg.idx = inner.data();
  rg.n = 1;
  CHECK(resolve_spec(win_t, rg, &r) == SCN_OK && r.pairs.size() == 39);
  rg.stencil = SCN_STENCIL_BEFORE;  // pair (139, 140) reads the unbacked row 140
  CHECK(resolve_spec(win_t, rg, &r) == SCN_EINVAL);
  rg.stencil = SCN_STENCIL_AFTER;
  std::vector<int64_t> gout = {100, 200};
  g.idx = gout.data();
  g.n = 2;
  CHECK(resolve_spec(win_t, g, &r) == SCN_EINVAL);
  win_t.backed_count = 2301;  // extends past n_frames
  CHECK(resolve_spec(win_t, stride(100, 3, 140), &r) == SCN_EINVAL);
  win_t.backed_count = -1;
  CHECK(resolve_spec(win_t, stride(100, 3, 140), &r) == SCN_EINVAL);
  // flow plans: sizing, chunking into a small workspace, uneven jobs
  scn_flow_params p{};
  p.levels = 4;
  p.alpha = 10.f;
  p.iters = 50;
  scn_table a = table(200, 320, 240), b = table(50, 640, 480);
  scn_sampling sa = stride(0, 7, 200), sb = stride(0, 1, 50);
  scn_job jobs[2] = {{&a, &sa}, {&b, &sb}};
  FlowPlan plan;
  CHECK(build_flow_plan(jobs, 2, &p, nullptr, 0, &plan) == SCN_OK && plan.total_pairs == 28 + 49);
  const size_t need = plan.ws_needed, mn = plan.ws_min;
  CHECK(mn > 0 && mn <= need);
  FlowPlan small;
  CHECK(build_flow_plan(jobs, 2, &p, nullptr, mn, &small) == SCN_OK && small.total_pairs == plan.total_pairs);
  size_t chunks = 0;
  for (const FlowGroup& grp : small.groups) chunks += grp.chunks.size();
  CHECK(chunks > 2);
  p.levels = 13;
  CHECK(build_flow_plan(jobs, 2, &p, nullptr, 0, &plan) == SCN_EINVAL);
  p.levels = 4;
  p.iters = -1;
  CHECK(build_flow_plan(jobs, 2, &p, nullptr, 0, &plan) == SCN_EINVAL);
  std::printf("%s: %d failure(s)\n", g_fail ? "FAILED" : "ok", g_fail);
  return g_fail ? 1 : 0;
}
