// Host-only checks of the serving engine's scheduling policy with a mock
// executor and a fake memory budget (built and run by test_engine_policy.py).
#include <cassert>
#include <cstdio>
#include <set>

#include "../paper_2508_18468_amd/csrc/engine_policy.h"

using namespace mfq_serving;

static int failures = 0;
#define CHECK(c)                                                         \
  do {                                                                   \
    if (!(c)) {                                                          \
      std::printf("FAIL line %d: %s\n", __LINE__, #c);                   \
      ++failures;                                                        \
    }                                                                    \
  } while (0)

// footprint: 100 units per slot plus 50 per group (shared propagator), scaled by L
static size_t fake_bytes(const ShapeKey &k, int cap) { return (size_t)k.Lx * (50 + 100 * (size_t)cap); }

static Job job(int Lx, int n_steps, int protocol = 1) {
  Job j;
  j.key.dim = 1;
  j.key.Lx = Lx;
  j.key.N = Lx / 2;
  j.key.protocol = protocol;
  j.gamma = 0.5;
  j.n_steps = n_steps;
  return j;
}

// Mock executor: applies actions, then advances every active group by its chunk,
// completing jobs; returns the number of completions.
static int run_round(Policy &p, std::set<int> &live, double &t) {
  for (const Action &a : p.plan()) {
    if (a.kind == Action::CREATE) { p.group_created(a.group); live.insert(a.group); }
    if (a.kind == Action::DESTROY) live.erase(a.group);
  }
  CHECK(p.bytes_in_use() <= p.budget());
  int done = 0;
  for (int gid : p.active_groups()) {
    const int k = p.chunk(gid, 1.0, 1000);
    CHECK(k >= 1);
    for (uint64_t jid : p.advanced(gid, k, 0.001 * k)) {
      p.record(jid, 0.0);
      const Job *j = p.job(jid);
      CHECK(j->steps_done <= j->n_steps);
      if (j->steps_done >= j->n_steps) { p.complete(jid, t); ++done; }
    }
  }
  t += 1.0;
  return done;
}

int main() {
  {  // admission by footprint, budget never exceeded, everything completes
    Policy p(64 * 1000, 4, fake_bytes);
    std::vector<uint64_t> ids;
    for (int i = 0; i < 20; ++i) ids.push_back(p.submit(job(i % 3 == 0 ? 128 : 64, 10 + 7 * i)));
    std::set<int> live;
    double t = 0;
    int done = 0;
    for (int r = 0; r < 400 && done < 20; ++r) done += run_round(p, live, t);
    CHECK(done == 20);
    for (uint64_t id : ids) CHECK(p.job(id)->state == DONE);
    CHECK(p.peak_bytes() <= 64 * 1000);
    run_round(p, live, t);
    CHECK(p.bytes_in_use() == 0);  // idle groups were destroyed
  }
  {  // continuous batching: a freed slot is refilled while the others keep running
    // (budget for exactly one group of two slots, so c cannot get a group of its own)
    Policy p(fake_bytes(job(64, 1).key, 2), 2, fake_bytes);
    const uint64_t a = p.submit(job(64, 5)), b = p.submit(job(64, 50)), c = p.submit(job(64, 5));
    std::set<int> live;
    double t = 0;
    auto acts = p.plan();
    int creates = 0;
    for (auto &x : acts) if (x.kind == Action::CREATE) { ++creates; p.group_created(x.group); }
    CHECK(creates == 1);  // capacity 2: a and b share a group, c waits for a slot
    CHECK(p.job(a)->state == ACTIVE && p.job(b)->state == ACTIVE && p.job(c)->state == QUEUED);
    const int g = p.job(a)->group;
    CHECK(p.chunk(g, 1.0, 1000) == Policy::PROBE_STEPS);  // step cost unknown: a probe chunk
    CHECK(p.advanced(g, Policy::PROBE_STEPS, 0.01).empty());
    for (uint64_t jid : p.advanced(g, p.chunk(g, 1.0, 1000), 0.01)) {
      const Job *j = p.job(jid);
      if (j->steps_done >= j->n_steps) p.complete(jid, 1.0);
    }
    CHECK(p.job(a)->state == DONE && p.job(b)->state == ACTIVE);
    CHECK(p.job(b)->steps_done == 5);  // the chunk stopped at a's completion
    auto acts2 = p.plan();
    bool admitted_c = false;
    for (auto &x : acts2) if (x.kind == Action::ADMIT && x.job == c) admitted_c = (x.group == g);
    CHECK(admitted_c);
    CHECK(p.job(c)->slot == p.job(a)->slot);
    CHECK(p.job(c)->steps_done == 0 && p.job(b)->steps_done == 5);
    (void)live;
    (void)t;
  }
  {  // the oldest queued job keeps memory priority; later jobs may only join free slots
    Policy p(100 * 1000, 4, fake_bytes);
    const uint64_t small1 = p.submit(job(64, 100));
    const uint64_t small1b = p.submit(job(64, 3));     // group of two slots: 64 * 250 = 16000
    auto acts = p.plan();
    for (auto &x : acts) if (x.kind == Action::CREATE) p.group_created(x.group);
    const int g = p.job(small1)->group;
    p.advanced(g, p.chunk(g, 1.0, 1000), 0.01);  // the probe chunk
    for (uint64_t jid : p.advanced(g, p.chunk(g, 1.0, 1000), 0.01))
      if (p.job(jid)->steps_done >= p.job(jid)->n_steps) p.complete(jid, 1.0);
    CHECK(p.job(small1b)->state == DONE);
    const uint64_t big = p.submit(job(600, 10));       // 600 * 150 = 90000: fits alone, not now
    const uint64_t small2 = p.submit(job(64, 10));     // fits the free slot of small1's group
    const uint64_t other = p.submit(job(96, 10));      // would need a new group: must wait
    p.plan();
    CHECK(p.job(small1)->state == ACTIVE);
    CHECK(p.job(big)->state == QUEUED);
    CHECK(p.job(small2)->state == ACTIVE);
    CHECK(p.job(other)->state == QUEUED);
    CHECK(p.bytes_in_use() <= 100 * 1000);
  }
  {  // a job that can never fit fails at submission
    Policy p(1000, 4, fake_bytes);
    const uint64_t huge = p.submit(job(4096, 10));
    CHECK(p.job(huge)->state == FAILED && p.job(huge)->error == -2);
    CHECK(p.queued() == 0);
  }
  {  // observations: chunks stop at every observation point of every job
    Policy p(1000000, 4, fake_bytes);
    Job j1 = job(64, 30);
    j1.obs_every = 7;
    Job j2 = job(64, 30);
    j2.obs_every = 10;
    const uint64_t a = p.submit(j1), b = p.submit(j2);
    for (auto &x : p.plan()) if (x.kind == Action::CREATE) p.group_created(x.group);
    const int g = p.job(a)->group;
    std::vector<int> stops;
    while (p.job(a)->state != DONE || p.job(b)->state != DONE) {
      const int k = p.chunk(g, 1.0, 1000);
      for (uint64_t jid : p.advanced(g, k, 0.01)) {
        p.record(jid, 1.0);
        const Job *j = p.job(jid);
        if (j->steps_done >= j->n_steps) p.complete(jid, 2.0);
      }
      stops.push_back(p.job(a)->steps_done);
      if (stops.size() > 100) break;
    }
    CHECK(p.job(a)->S.size() == 5);  // steps 7, 14, 21, 28 and the last (30)
    CHECK(p.job(b)->S.size() == 3);  // steps 10, 20, 30
  }
  {  // scheduling: shortest work to the next completion first, within the width budget
    Policy p(1 << 30, 1, fake_bytes);
    const uint64_t big = p.submit(job(512, 100)), mid = p.submit(job(128, 100));
    const uint64_t small = p.submit(job(64, 100)), tiny_late = p.submit(job(64, 10));
    for (auto &x : p.plan()) if (x.kind == Action::CREATE) p.group_created(x.group);
    const int gb = p.job(big)->group, gm = p.job(mid)->group, gs = p.job(small)->group;
    const int gt = p.job(tiny_late)->group;
    CHECK(p.next_completion_work(gt) < p.next_completion_work(gs));
    CHECK(p.next_completion_work(gs) < p.next_completion_work(gm));
    CHECK(p.next_completion_work(gm) < p.next_completion_work(gb));
    // a budget of one element: only the group nearest to a completion runs
    std::vector<int> one = p.schedule(1.0);
    CHECK(one.size() == 1 && one[0] == gt);
    // a budget that the two smallest groups (64 * 32 elements each) do not fill
    std::vector<int> some = p.schedule(64.0 * 32 * 2 + 1);
    CHECK(some.size() == 3 && some[0] == gt && some[1] == gs && some[2] == gm);
    // an unlimited budget runs everything, still in that order
    std::vector<int> all = p.schedule(1e30);
    CHECK(all.size() == 4 && all[3] == gb);
    // progress changes the order: with one step left the big job (about 1.1e9 flop) comes
    // before the untouched L=128 job (100 steps of 1.7e7), behind the L=64 one (2.1e8)
    p.advanced(gb, 99, 0.1);
    p.advanced(gt, 10, 0.1);
    p.complete(tiny_late, 1.0);
    std::vector<int> after = p.schedule(1e30);
    CHECK(after.size() == 3 && after[0] == gs && after[1] == gb && after[2] == gm);
  }
  {  // chunk sizes: a probe first, then about the round's wall time, never past a completion
    Policy p(1 << 30, 2, fake_bytes);
    const uint64_t fast = p.submit(job(64, 1000)), slow = p.submit(job(256, 1000));
    for (auto &x : p.plan()) if (x.kind == Action::CREATE) p.group_created(x.group);
    const int gf = p.job(fast)->group, gs = p.job(slow)->group;
    CHECK(p.chunk(gf, 0.02, 256) == Policy::PROBE_STEPS && p.chunk(gs, 0.02, 256) == Policy::PROBE_STEPS);
    CHECK(p.round_target({gf, gs}, 0.02) == 0.02);  // no cost known yet
    p.advanced(gf, 2, 0.002);                        // 1 ms per step
    p.advanced(gs, 2, 0.2);                          // 100 ms per step
    const double T = p.round_target({gf, gs}, 0.02);
    CHECK(T > 0.0999 && T < 0.1001);                 // the slow group's one step sets the round
    CHECK(p.chunk(gs, T, 256) == 1);
    CHECK(p.chunk(gf, T, 256) == 100);               // the fast group fills that time
    CHECK(p.chunk(gf, T, 64) == 64);                 // within the chunk cap
    CHECK(p.round_target({gf}, 0.02) == 0.02);
    p.advanced(gf, 995, 0.995);
    CHECK(p.chunk(gf, T, 256) == 3);                 // stops at the job's last step
  }
  std::printf(failures ? "policy checks: %d failures\n" : "policy checks: all passed\n", failures);
  return failures ? 1 : 0;
}
