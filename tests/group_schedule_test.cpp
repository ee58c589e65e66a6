// Host-only checks of the group run's schedule (built and run by test_group_schedule.py):
// random groups of contexts with uneven step counts, starting steps and observation
// schedules are advanced round by round as mfq_run_group does, and every context must end at
// its last step, observe exactly at the multiples of its obs_every in between, and never be
// carried past one by the group graph.
#include <cstdio>
#include <random>
#include <vector>

#include "../paper_2508_18468_amd/csrc/group_schedule.h"

using namespace mfq_group;

static int failures = 0;
#define CHECK(c)                                                         \
  do {                                                                   \
    if (!(c)) {                                                          \
      std::printf("FAIL line %d: %s\n", __LINE__, #c);                   \
      ++failures;                                                        \
    }                                                                    \
  } while (0)

static void run_case(std::mt19937 &rng, int n) {
  std::vector<int64_t> left(n), step(n), start(n), total(n);
  std::vector<int> every(n);
  std::vector<std::vector<int64_t>> observed(n);
  for (int k = 0; k < n; ++k) {
    total[k] = left[k] = rng() % 41;
    start[k] = step[k] = rng() % 23;
    every[k] = (rng() % 3 == 0) ? 0 : 1 + (int)(rng() % 7);
  }
  int rounds = 0;
  int64_t most = 0;
  for (int k = 0; k < n; ++k) most += left[k];
  for (;;) {
    const Round r = plan_round(left, step, every);
    if (r.members.empty() && r.singles.empty()) break;
    CHECK(++rounds <= most + 1);
    if (rounds > most + 1) return;
    CHECK(r.members.empty() == (r.pairs == 0));
    std::vector<int> moved(n, 0);
    for (int k : r.members) {
      // the graph never carries a context past its stop
      CHECK(2 * r.pairs <= steps_to_stop(left[k], step[k], every[k]));
      for (int64_t s = step[k] + 1; s < step[k] + 2 * r.pairs; ++s) CHECK(every[k] == 0 || s % every[k] != 0);
      step[k] += 2 * r.pairs;
      left[k] -= 2 * r.pairs;
      moved[k] = 1;
    }
    for (int k : r.singles) {
      CHECK(!moved[k]);
      CHECK(left[k] > 0 && steps_to_stop(left[k], step[k], every[k]) == 1);
      ++step[k];
      --left[k];
      moved[k] = 1;
    }
    for (int k = 0; k < n; ++k)
      if (moved[k] && every[k] > 0 && step[k] % every[k] == 0) observed[k].push_back(step[k]);
  }
  for (int k = 0; k < n; ++k) {
    CHECK(left[k] == 0);
    CHECK(step[k] == start[k] + total[k]);
    std::vector<int64_t> want;
    if (every[k] > 0)
      for (int64_t s = start[k] + 1; s <= start[k] + total[k]; ++s)
        if (s % every[k] == 0) want.push_back(s);
    CHECK(observed[k] == want);
  }
}

int main() {
  std::mt19937 rng(12345);
  for (int it = 0; it < 20000; ++it) run_case(rng, 1 + (int)(rng() % 8));
  // a lone context with no steps plans an empty round
  {
    const Round r = plan_round({0}, {5}, {3});
    CHECK(r.members.empty() && r.singles.empty() && r.pairs == 0);
  }
  // two pairs before an observation at step 8, from step 4 with ten steps left
  {
    const Round r = plan_round({10, 9}, {4, 0}, {4, 0});
    CHECK(r.members.size() == 2 && r.pairs == 2 && r.singles.empty());
  }
  if (failures) {
    std::printf("%d failures\n", failures);
    return 1;
  }
  std::printf("all passed\n");
  return 0;
}
