// Admission of the band reduction's panel kernels (eig2.hip) across streams.  The workgroups of a
// panel kernel wait for each other, so panel kernels that may run at the same time must fit the
// GPU together.  Each stream keeps one record: an event recorded after its latest panel kernel
// (waiting for it waits for all of that stream's panel kernels, which run in order) and a bound
// on the grid of whichever of them may still run.  A new panel kernel waits, on the GPU, for the
// earliest records of other streams until its grid and the remaining ones fit.  Waits point
// only at launches made before, so they form no cycle.  Host-only, so that it is checked on the
// CPU (tests/panel_admission_test.cpp).
#pragma once

#include <algorithm>
#include <vector>

namespace mfq_panel {

struct Record {
  long wgs = 0;  // grid bound of the stream's panel kernels that may still run; 0: all finished
  long seq = 0;  // order of the latest launch
};

// Records of other streams (unfinished ones) to wait for, earliest first, before a launch of
// `wgs` workgroups on a GPU that holds `cap` at once.
inline std::vector<int> waits_for(const std::vector<Record> &others, long wgs, long cap) {
  std::vector<int> order;
  long sum = wgs;
  for (int i = 0; i < (int)others.size(); ++i)
    if (others[i].wgs > 0) {
      order.push_back(i);
      sum += others[i].wgs;
    }
  std::sort(order.begin(), order.end(), [&](int a, int b) { return others[a].seq < others[b].seq; });
  std::vector<int> wait;
  for (int i : order) {
    if (sum <= cap) break;
    wait.push_back(i);
    sum -= others[i].wgs;
  }
  return wait;
}

// The stream's record after a launch of `wgs` workgroups: an earlier panel kernel that may still
// be running keeps its grid in the bound (the grids of one reduction shrink panel by panel).
inline long recorded_wgs(long old_wgs, bool old_finished, long wgs) {
  return old_finished ? wgs : std::max(old_wgs, wgs);
}

}  // namespace mfq_panel
