// Scheduling policy of the serving engine: admission by device-memory
// footprint, continuous batching of jobs with the same shape into batch
// groups, and step chunking.  Pure C++ (no HIP), so that it can be exercised
// on a host without a GPU.
//
// A job is one trajectory request.  Jobs with the same shape key (lattice, N,
// protocol, precision, dt, seed) share a batch group: one library context
// whose trajectories are slots.  A job is admitted into a free slot of a group
// of its shape, or a new group is created for it if its footprint fits in the
// memory budget.  When a job completes its slot is freed and the next queued
// job of that shape takes it while the other slots keep running (continuous
// batching).  Groups left without jobs are destroyed and their memory is
// returned.  The oldest queued job has priority on memory: while it cannot be
// placed, no other job may create a group (no starvation of large jobs); jobs
// may still join free slots of existing groups.
#pragma once

#include <algorithm>
#include <cstdint>
#include <deque>
#include <functional>
#include <map>
#include <string>
#include <tuple>
#include <vector>

namespace mfq_serving {

struct ShapeKey {
  int dim = 1, Lx = 0, Ly = 1;
  double J = 1.0;
  int N = 0, protocol = 0, precision = 0;
  double dt = 0.05;
  uint64_t seed = 0;
  auto tie() const { return std::tie(dim, Lx, Ly, J, N, protocol, precision, dt, seed); }
  bool operator<(const ShapeKey &o) const { return tie() < o.tie(); }
  bool operator==(const ShapeKey &o) const { return tie() == o.tie(); }
};

enum JobState { QUEUED = 0, ACTIVE = 1, DONE = 2, FAILED = 3 };

struct Job {
  uint64_t id = 0;
  ShapeKey key;
  double gamma = 0.0;
  uint64_t uid = 0;
  int n_steps = 0, obs_every = 0;
  std::vector<int> region;
  double t_submit = 0.0, t_done = 0.0;
  JobState state = QUEUED;
  int group = -1, slot = -1;
  int steps_done = 0;
  std::vector<double> S;
  int error = 0;
};

struct Group {
  int id = -1;
  ShapeKey key;
  int capacity = 0;
  size_t bytes = 0;
  bool created = false, alive = true;
  std::vector<int64_t> slot_job;  // job id per slot, -1 when free
  double step_cost_s = 0.0;       // moving estimate of the wall time of one step
  int active() const {
    return (int)std::count_if(slot_job.begin(), slot_job.end(), [](int64_t j) { return j >= 0; });
  }
};

struct Action {
  enum Kind { CREATE, ADMIT, DESTROY } kind;
  int group;
  int slot;
  uint64_t job;
};

class Policy {
 public:
  using BytesFn = std::function<size_t(const ShapeKey &, int capacity)>;

  Policy(size_t budget, int max_slots, BytesFn bytes_of)
      : budget_(budget), max_slots_(std::max(1, max_slots)), bytes_of_(std::move(bytes_of)) {}

  // Queue a job; returns its id.  A job whose footprint alone exceeds the
  // budget fails at once with error -2 (out of memory).
  uint64_t submit(Job j) {
    j.id = next_id_++;
    j.state = QUEUED;
    if (bytes_of_(j.key, 1) > budget_) {
      j.state = FAILED;
      j.error = -2;
    } else {
      queue_.push_back(j.id);
    }
    jobs_[j.id] = std::move(j);
    return next_id_ - 1;
  }

  // Decide what to do now: destroy idle groups, create groups, admit jobs.
  std::vector<Action> plan() {
    std::vector<Action> out;
    // idle groups with no queued job of their shape go away
    for (Group &g : groups_) {
      if (!g.alive || !g.created || g.active() > 0) continue;
      bool wanted = false;
      for (uint64_t id : queue_)
        if (jobs_[id].key == g.key) { wanted = true; break; }
      if (!wanted) {
        g.alive = false;
        used_ -= g.bytes;
        out.push_back({Action::DESTROY, g.id, -1, 0});
      }
    }
    bool head_blocked = false;
    std::deque<uint64_t> still;
    for (uint64_t id : queue_) {
      Job &j = jobs_[id];
      int gi = -1, slot = -1;
      for (Group &g : groups_) {
        if (!g.alive || !(g.key == j.key)) continue;
        for (int s = 0; s < g.capacity; ++s)
          if (g.slot_job[s] < 0) { gi = g.id; slot = s; break; }
        if (gi >= 0) break;
      }
      if (gi < 0 && !head_blocked) {
        int want = 0;  // jobs of this shape still queued from here on
        bool seen = false;
        for (uint64_t q : queue_) {
          if (q == id) seen = true;
          if (seen && jobs_[q].key == j.key) ++want;
        }
        int cap = std::min(max_slots_, std::max(1, want));
        size_t bytes = bytes_of_(j.key, cap);
        while (cap > 1 && used_ + bytes > budget_) {
          cap /= 2;
          bytes = bytes_of_(j.key, cap);
        }
        if (used_ + bytes <= budget_) {
          Group g;
          g.id = (int)groups_.size();
          g.key = j.key;
          g.capacity = cap;
          g.bytes = bytes;
          g.slot_job.assign(cap, -1);
          used_ += bytes;
          peak_ = std::max(peak_, used_);
          groups_.push_back(g);
          out.push_back({Action::CREATE, g.id, -1, 0});
          gi = g.id;
          slot = 0;
        }
      }
      if (gi >= 0) {
        groups_[gi].slot_job[slot] = (int64_t)id;
        j.state = ACTIVE;
        j.group = gi;
        j.slot = slot;
        j.steps_done = 0;
        out.push_back({Action::ADMIT, gi, slot, id});
      } else {
        if (still.empty()) head_blocked = true;  // the oldest job keeps the memory priority
        still.push_back(id);
      }
    }
    queue_.swap(still);
    return out;
  }

  // The executor could not create group gid: its jobs go back to the queue
  // head (or fail if nothing else holds memory that could be freed).
  void group_failed(int gid, int error) {
    Group &g = groups_[gid];
    if (!g.alive) return;
    g.alive = false;
    used_ -= g.bytes;
    std::vector<uint64_t> back;
    for (int64_t jid : g.slot_job) {
      if (jid < 0) continue;
      Job &j = jobs_[(uint64_t)jid];
      j.group = j.slot = -1;
      if (live_groups() == 0) {
        j.state = FAILED;
        j.error = error;
      } else {
        j.state = QUEUED;
        back.push_back((uint64_t)jid);
      }
    }
    for (auto it = back.rbegin(); it != back.rend(); ++it) queue_.push_front(*it);
  }

  void group_created(int gid) { groups_[gid].created = true; }

  // Steps for group g to advance now: up to the next observation or
  // completion of any of its jobs, and about target_s of wall time.
  // A group whose step cost is not yet known advances PROBE_STEPS steps (one captured
  // step pair), so that a first chunk never holds a round for long.
  static constexpr int PROBE_STEPS = 2;
  int chunk(int gid, double target_s, int max_chunk) const {
    const Group &g = groups_[gid];
    int k = std::min(max_chunk, PROBE_STEPS);
    if (g.step_cost_s > 0.0) k = std::max(1, std::min(max_chunk, (int)(target_s / g.step_cost_s)));
    for (int64_t jid : g.slot_job) {
      if (jid < 0) continue;
      const Job &j = jobs_.at((uint64_t)jid);
      int next = j.n_steps - j.steps_done;
      if (j.obs_every > 0) next = std::min(next, j.obs_every - j.steps_done % j.obs_every);
      k = std::min(k, std::max(1, next));
    }
    return k;
  }

  // Wall time of a round that advances groups gids: every group takes at least one step,
  // so the round lasts at least the slowest known step; the others then fill that time
  // (at least target_s).
  double round_target(const std::vector<int> &gids, double target_s) const {
    double t = target_s;
    for (int gid : gids) t = std::max(t, groups_[gid].step_cost_s);
    return t;
  }

  // Group gid advanced by k steps: returns the jobs that reached an
  // observation point (including their last step).
  std::vector<uint64_t> advanced(int gid, int k, double wall_s) {
    Group &g = groups_[gid];
    const double per = wall_s / std::max(1, k);
    g.step_cost_s = g.step_cost_s > 0.0 ? 0.5 * (g.step_cost_s + per) : per;
    std::vector<uint64_t> obs;
    for (int64_t jid : g.slot_job) {
      if (jid < 0) continue;
      Job &j = jobs_[(uint64_t)jid];
      j.steps_done += k;
      const bool at_obs = j.obs_every > 0 && j.steps_done % j.obs_every == 0;
      if (at_obs || j.steps_done >= j.n_steps) obs.push_back(j.id);
    }
    return obs;
  }

  void record(uint64_t jid, double S) { jobs_[jid].S.push_back(S); }

  // Job finished at time t: its slot is freed for the next queued job.
  void complete(uint64_t jid, double t) {
    Job &j = jobs_[jid];
    j.state = DONE;
    j.t_done = t;
    if (j.group >= 0) groups_[j.group].slot_job[j.slot] = -1;
  }

  void fail_group_jobs(int gid, int error, double t) {
    Group &g = groups_[gid];
    for (int64_t &jid : g.slot_job) {
      if (jid < 0) continue;
      Job &j = jobs_[(uint64_t)jid];
      j.state = FAILED;
      j.error = error;
      j.t_done = t;
      jid = -1;
    }
  }

  std::vector<int> active_groups() const {
    std::vector<int> v;
    for (const Group &g : groups_)
      if (g.alive && g.created && g.active() > 0) v.push_back(g.id);
    return v;
  }

  // Work left for the job of group gid that will finish first, in flops at about
  // 8 L^3 per trajectory-step for N = L/2 (propagator 8 L^2 N, two Cholesky-QR
  // passes 16 L N^2).
  double next_completion_work(int gid) const {
    const Group &g = groups_[gid];
    const double L = (double)g.key.Lx * g.key.Ly, N = g.key.N;
    double best = -1.0;
    for (int64_t jid : g.slot_job) {
      if (jid < 0) continue;
      const Job &j = jobs_.at((uint64_t)jid);
      const double w = (double)(j.n_steps - j.steps_done) * (8.0 * L * L * N + 16.0 * L * N * N);
      if (best < 0.0 || w < best) best = w;
    }
    return best;
  }

  // Groups to advance now: active groups in order of the work left to their next
  // job completion (shortest first), taken until their combined width (trajectory
  // elements L * N * slots) reaches width_budget; at least one group.  Running the
  // shortest work first lowers the median latency of an overloaded queue, and the
  // width budget keeps enough groups in flight to occupy the device.
  std::vector<int> schedule(double width_budget) const {
    std::vector<int> act = active_groups();
    std::vector<std::pair<double, int>> order;
    for (int gid : act) order.push_back({next_completion_work(gid), gid});
    std::sort(order.begin(), order.end());
    std::vector<int> out;
    double width = 0.0;
    for (const auto &o : order) {
      if (!out.empty() && width >= width_budget) break;
      const Group &g = groups_[o.second];
      width += (double)g.key.Lx * g.key.Ly * g.key.N * g.capacity;
      out.push_back(o.second);
    }
    return out;
  }
  int live_groups() const {
    int n = 0;
    for (const Group &g : groups_) n += g.alive ? 1 : 0;
    return n;
  }

  const Job *job(uint64_t id) const {
    auto it = jobs_.find(id);
    return it == jobs_.end() ? nullptr : &it->second;
  }
  Job *job_mut(uint64_t id) {
    auto it = jobs_.find(id);
    return it == jobs_.end() ? nullptr : &it->second;
  }
  const Group &group(int gid) const { return groups_[gid]; }
  size_t bytes_in_use() const { return used_; }
  size_t peak_bytes() const { return peak_; }
  size_t queued() const { return queue_.size(); }
  size_t budget() const { return budget_; }

 private:
  size_t budget_, used_ = 0, peak_ = 0;
  int max_slots_;
  BytesFn bytes_of_;
  std::map<uint64_t, Job> jobs_;
  std::deque<uint64_t> queue_;
  std::vector<Group> groups_;
  uint64_t next_id_ = 1;
};

}  // namespace mfq_serving
