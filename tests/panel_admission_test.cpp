// Host-only checks of the panel kernels' admission across streams (built and run by
// test_panel_admission.py).  A model GPU holds `cap` workgroups; a panel kernel completes only
// once all of its workgroups have been resident together (they wait for each other), and a
// placed workgroup keeps its slot until its kernel completes.  Streams issue shrinking panel
// kernels in random interleavings with the GPU progressing in between; the admission of
// panel_admission.h must never leave the model stuck.  Two weaker rules serve as controls and
// must get stuck in some interleavings: no admission, and a record that keeps only the latest
// launch's grid (an earlier, larger kernel of that stream may still be running).
#include <cstdio>
#include <random>
#include <vector>

#include "../paper_2508_18468_amd/csrc/panel_admission.h"

using namespace mfq_panel;

static int failures = 0;
#define CHECK(c)                                                         \
  do {                                                                   \
    if (!(c)) {                                                          \
      std::printf("FAIL line %d: %s\n", __LINE__, #c);                   \
      ++failures;                                                        \
    }                                                                    \
  } while (0)

enum Rule { ADMISSION, NO_ADMISSION, LATEST_ONLY };

struct Kernel {
  int stream, wgs;
  std::vector<std::pair<int, int>> deps;  // (stream, kernel index in that stream) to complete first
  int placed = 0;
  bool done = false;
};

struct Model {
  int cap, free_slots;
  std::vector<std::vector<Kernel>> ks;  // per stream, in launch order
  std::mt19937 &rng;
  Model(int c, int streams, std::mt19937 &r) : cap(c), free_slots(c), ks(streams), rng(r) {}
  bool complete(int s, int i) const { return i < 0 || ks[s][i].done; }
  bool dispatchable(int s, int i) const {
    const Kernel &k = ks[s][i];
    if (k.done || (i > 0 && !ks[s][i - 1].done)) return false;
    for (auto d : k.deps)
      if (!complete(d.first, d.second)) return false;
    return true;
  }
  // one step of progress: place workgroups, or complete a fully placed kernel; false if stuck
  bool step() {
    std::vector<std::pair<int, int>> place, finish;
    for (int s = 0; s < (int)ks.size(); ++s)
      for (int i = 0; i < (int)ks[s].size(); ++i) {
        if (!dispatchable(s, i)) continue;
        const Kernel &k = ks[s][i];
        if (k.placed < k.wgs && free_slots > 0) place.push_back({s, i});
        if (k.placed == k.wgs) finish.push_back({s, i});
      }
    if (place.empty() && finish.empty()) return false;
    const size_t pick = rng() % (place.size() + finish.size());
    if (pick < place.size()) {
      Kernel &k = ks[place[pick].first][place[pick].second];
      const int n = 1 + (int)(rng() % (unsigned)std::min(k.wgs - k.placed, free_slots));
      k.placed += n;
      free_slots -= n;
    } else {
      Kernel &k = ks[finish[pick - place.size()].first][finish[pick - place.size()].second];
      k.done = true;
      free_slots += k.placed;
    }
    return true;
  }
  bool all_done() const {
    for (auto &v : ks)
      for (auto &k : v)
        if (!k.done) return false;
    return true;
  }
};

// One trial; returns true if the model got stuck.
static bool trial(std::mt19937 &rng, Rule rule) {
  const int cap = 64, streams = 2 + (int)(rng() % 3);
  Model gpu(cap, streams, rng);
  // each stream: one or two reductions of shrinking panel grids, each at most 3/4 of cap
  std::vector<std::vector<int>> todo(streams);
  for (int s = 0; s < streams; ++s) {
    const int reductions = 1 + (int)(rng() % 2);
    for (int r = 0; r < reductions; ++r) {
      int g = 8 + (int)(rng() % 41);  // up to 48
      const int panels = 2 + (int)(rng() % 6);
      for (int p = 0; p < panels && g > 0; ++p) {
        todo[s].push_back(g);
        g -= 1 + (int)(rng() % 12);
      }
    }
  }
  std::vector<Record> rec(streams);
  long seq = 0;
  std::vector<size_t> next(streams, 0);
  for (;;) {
    std::vector<int> ready;
    for (int s = 0; s < streams; ++s)
      if (next[s] < todo[s].size()) ready.push_back(s);
    if (ready.empty()) break;
    // the GPU progresses a little between host launches
    for (int q = (int)(rng() % 4); q > 0; --q) gpu.step();
    const int s = ready[rng() % ready.size()];
    const int wgs = todo[s][next[s]++];
    Kernel k{s, wgs, {}, 0, false};
    // the host's view: a record is finished when that stream's latest kernel has completed
    auto latest = [&](int t) { return (int)gpu.ks[t].size() - 1; };
    std::vector<Record> others;
    std::vector<int> who;
    for (int t = 0; t < streams; ++t) {
      if (t == s) continue;
      if (gpu.complete(t, latest(t))) rec[t].wgs = 0;
      if (rec[t].wgs == 0) continue;
      others.push_back(rec[t]);
      who.push_back(t);
    }
    if (rule != NO_ADMISSION)
      for (int i : waits_for(others, wgs, cap)) k.deps.push_back({who[i], latest(who[i])});
    const bool finished = gpu.complete(s, latest(s));
    rec[s].wgs = rule == LATEST_ONLY ? wgs : recorded_wgs(rec[s].wgs, finished, wgs);
    rec[s].seq = ++seq;
    gpu.ks[s].push_back(k);
  }
  while (!gpu.all_done())
    if (!gpu.step()) return true;
  return false;
}

int main() {
  std::mt19937 rng(2024);
  int stuck[3] = {0, 0, 0};
  const int trials = 20000;
  for (int r = 0; r < 3; ++r)
    for (int t = 0; t < trials; ++t) stuck[r] += trial(rng, (Rule)r);
  std::printf("stuck: admission %d, no admission %d, latest grid only %d (of %d)\n", stuck[ADMISSION],
              stuck[NO_ADMISSION], stuck[LATEST_ONLY], trials);
  CHECK(stuck[ADMISSION] == 0);
  CHECK(stuck[NO_ADMISSION] > 0);
  CHECK(stuck[LATEST_ONLY] > 0);
  // waits_for: earliest first, only as many as needed, finished records ignored
  {
    std::vector<Record> o(3);
    o[0] = {40, 5};
    o[1] = {30, 2};
    o[2] = {0, 1};
    std::vector<int> w = waits_for(o, 30, 64);  // 30 + 40 + 30 = 100: wait for seq 2 (30) and 5 (40)
    CHECK(w.size() == 2 && w[0] == 1 && w[1] == 0);
    w = waits_for(o, 10, 64);  // 80: the earliest (30) suffices
    CHECK(w.size() == 1 && w[0] == 1);
    CHECK(waits_for(o, 0, 70).empty());
    CHECK(recorded_wgs(40, false, 10) == 40 && recorded_wgs(40, true, 10) == 10);
  }
  if (failures) {
    std::printf("%d failures\n", failures);
    return 1;
  }
  std::printf("all passed\n");
  return 0;
}
