// Schedule of a group run (mfq_run_group for contexts above the fused kernel's size): which
// contexts the group graph advances in the next round, by how many pairs of steps, and which
// take a single step on their own.  Host-only, so that it is checked on the CPU
// (tests/group_schedule_test.cpp).
#pragma once

#include <algorithm>
#include <cstdint>
#include <vector>

namespace mfq_group {

// Steps of a context before its next stop: its last step, or the next step index that is a
// multiple of `every` (0: no observations).
inline int64_t steps_to_stop(int64_t left, int64_t step, int every) {
  int64_t s = left;
  if (every > 0) s = std::min<int64_t>(s, every - step % every);
  return s;
}

struct Round {
  std::vector<int> members;  // advanced by the group graph, 2 * pairs steps each
  int64_t pairs = 0;
  std::vector<int> singles;  // one step each, on their own stream
};

// The next round: every context with two or more steps before its stop joins the graph, which is
// replayed as often as the nearest of their stops allows (so no member passes one); contexts one
// step from their stop take that step alone.  An empty round (no members, no singles) means every
// context is done.
inline Round plan_round(const std::vector<int64_t> &left, const std::vector<int64_t> &step,
                        const std::vector<int> &every) {
  Round r;
  for (size_t k = 0; k < left.size(); ++k) {
    const int64_t s = steps_to_stop(left[k], step[k], every[k]);
    if (s >= 2) {
      r.members.push_back((int)k);
      r.pairs = r.pairs == 0 ? s / 2 : std::min(r.pairs, s / 2);
    } else if (left[k] > 0) {
      r.singles.push_back((int)k);
    }
  }
  return r;
}

}  // namespace mfq_group
