// Serving engine: a request loop that admits trajectory jobs of different
// lattices, sizes and protocols by device-memory footprint and advances them
// with continuous batching (engine_policy.h).  A worker thread owns the GPU
// work: every batch group is one library context with its own stream, so the
// groups' steps overlap on the device.  Each round advances the groups whose
// next job completion is nearest in work (shortest first, up to a combined
// width that occupies the device), each in chunks of about CHUNK_TARGET_S of
// wall time (or of the slowest step in the round, which the round lasts anyway),
// up to the next observation or completion of one of its jobs, after which
// finished slots are refilled from the queue.  A group's step cost is measured
// by events on its stream; a new group first advances a short probe chunk.
// Projective groups whose steps synchronise the stream (the blocked
// measurement) are issued last, each from a host thread of its own.
// Each job keeps its own random numbers (key = (seed, uid), counter = its own
// step index), so a job gives the same result alone and in any mix.  Groups of small
// lattices (state, Gram and factor in one CU's LDS, FP64) are advanced together: up to
// eight of them, of any sizes and protocols, share one launch of the fused kernel.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <system_error>
#include <thread>

#include "../../include/mfq.h"
#include "engine_policy.h"
#include "mfq_internal.h"

using namespace mfq_serving;

namespace {
constexpr double CHUNK_TARGET_S = 0.02;
constexpr int CHUNK_MAX = 256;
// Groups advanced together hold at least this many state elements (L * N per
// trajectory): 128 x 128-tile propagator products of ~2000 workgroups.
constexpr double WIDTH_BUDGET = 32.0 * 1024 * 1024;

// Device resources of one batch group: its library context, the stream it runs on and two
// events that time each chunk on that stream (the time a chunk took on the shared device,
// whatever order the worker collects the groups in).
struct GroupRes {
  mfq_ctx *c = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
};

void release(GroupRes &r) {
  if (r.c) mfq_destroy(r.c);
  if (r.e0) (void)hipEventDestroy(r.e0);
  if (r.e1) (void)hipEventDestroy(r.e1);
  if (r.s) (void)hipStreamDestroy(r.s);
  r = GroupRes{};
}
}  // namespace

struct mfq_engine {
  int device = 0;
  Policy policy;
  std::mutex m;
  std::condition_variable cv;
  std::thread worker;
  bool stop = false;
  std::map<int, GroupRes> res_of_group;
  std::string err;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  mfq_engine(int dev, size_t budget, int max_slots, Policy::BytesFn f)
      : device(dev), policy(budget, max_slots, std::move(f)) {}
  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

mfq_lattice lattice_of(const ShapeKey &k) {
  mfq_lattice l{};
  l.dim = k.dim;
  l.Lx = k.Lx;
  l.Ly = k.Ly;
  l.J = k.J;
  return l;
}

size_t footprint(const ShapeKey &k, int cap) {
  mfq_lattice l = lattice_of(k);
  size_t b = 0;
  if (mfq_workspace_bytes(&l, k.N, cap, k.precision, &b) != MFQ_OK) return (size_t)-1;
  return b;
}

mfq_status create_group(int device, const Group &g, GroupRes &r) {
  if (hipSetDevice(device) != hipSuccess || hipStreamCreate(&r.s) != hipSuccess ||
      hipEventCreate(&r.e0) != hipSuccess || hipEventCreate(&r.e1) != hipSuccess) {
    release(r);
    return MFQ_EDEVICE;
  }
  mfq_lattice l = lattice_of(g.key);
  std::vector<uint64_t> uids(g.capacity, 0);
  mfq_status st = mfq_create(device, r.s, &r.c);
  if (st == MFQ_OK)
    st = mfq_init_state(r.c, &l, g.key.N, g.capacity, uids.data(), nullptr, g.key.precision, nullptr, 0);
  if (st != MFQ_OK) release(r);
  return st;
}

void worker_loop(mfq_engine *e) {
  (void)hipSetDevice(e->device);
  while (true) {
    std::vector<Action> actions;
    {
      std::unique_lock<std::mutex> lk(e->m);
      if (e->stop) break;
      actions = e->policy.plan();
    }
    for (const Action &a : actions) {
      std::unique_lock<std::mutex> lk(e->m);
      const Group &g = e->policy.group(a.group);
      if (a.kind == Action::DESTROY) {
        auto it = e->res_of_group.find(a.group);
        if (it != e->res_of_group.end()) {
          release(it->second);
          e->res_of_group.erase(it);
        }
      } else if (a.kind == Action::CREATE) {
        GroupRes r;
        const mfq_status st = create_group(e->device, g, r);
        if (st != MFQ_OK) {
          e->policy.group_failed(a.group, st);
        } else {
          e->res_of_group[a.group] = r;
          e->policy.group_created(a.group);
        }
      } else {  // ADMIT
        auto it = e->res_of_group.find(a.group);
        const Job *j = e->policy.job(a.job);
        if (it != e->res_of_group.end() && j)
          mfq_reset_trajectory(it->second.c, a.slot, j->uid);
      }
    }
    std::vector<int> active;
    double target = CHUNK_TARGET_S;
    {
      std::unique_lock<std::mutex> lk(e->m);
      active = e->policy.schedule(WIDTH_BUDGET);
      if (active.empty()) {
        e->cv.wait_for(lk, std::chrono::milliseconds(5));
        continue;
      }
      target = e->policy.round_target(active, CHUNK_TARGET_S);
    }
    // one chunk per group, each on its own stream between its two events; then collect
    struct Run {
      int gid, k;
      GroupRes r;
      double t_start;  // host clock at issue (fallback timing)
      mfq_status st;
      const GroupRes *timer;  // whose events bracket this run (fused runs share the first's)
    };
    std::vector<Run> runs;
    struct Pending {
      int gid, k;
      GroupRes r;
      ShapeKey key;
      std::vector<double> gam;
      mfq_status st = MFQ_OK;
    };
    std::vector<Pending> fused, blocking;
    for (int gid : active) {
      std::unique_lock<std::mutex> lk(e->m);
      const Group &g = e->policy.group(gid);
      const int k = e->policy.chunk(gid, target, CHUNK_MAX);
      std::vector<double> gam(g.capacity, 0.0);
      for (int s = 0; s < g.capacity; ++s)
        if (g.slot_job[s] >= 0) gam[s] = e->policy.job((uint64_t)g.slot_job[s])->gamma;
      const GroupRes r = e->res_of_group[gid];
      const ShapeKey key = g.key;
      lk.unlock();
      const int L = key.Lx * (key.dim == 2 ? key.Ly : 1);
      if (key.precision == MFQ_FP64 && mfq::fused_fits(L, key.N, key.Lx, key.dim == 2 ? key.Ly : 1)) {
        fused.push_back({gid, k, r, key, std::move(gam)});
        continue;
      }
      // projective steps in the blocked form synchronise their stream inside mfq_step
      if (key.protocol == MFQ_PROJECTIVE && key.N >= mfq::PM_BLOCKED_MIN_N) {
        blocking.push_back({gid, k, r, key, std::move(gam)});
        continue;
      }
      const double t = e->now();
      (void)hipEventRecord(r.e0, r.s);
      const mfq_status st = mfq_step(r.c, key.protocol, gam.data(), key.dt, key.seed, k);
      (void)hipEventRecord(r.e1, r.s);
      runs.push_back({gid, k, r, t, st, nullptr});
    }
    // small lattices: one fused launch per (up to) FUSED_GROUP_MAX groups, on the first
    // group's stream
    for (size_t b0 = 0; b0 < fused.size(); b0 += mfq::FUSED_GROUP_MAX) {
      const size_t b1 = std::min(fused.size(), b0 + (size_t)mfq::FUSED_GROUP_MAX);
      std::vector<mfq_ctx *> cs;
      std::vector<mfq_run_args> as;
      for (size_t i = b0; i < b1; ++i) {
        const Pending &f = fused[i];
        cs.push_back(f.r.c);
        mfq_run_args a{};
        a.protocol = f.key.protocol;
        a.gamma = f.gam.data();
        a.dt = f.key.dt;
        a.seed = f.key.seed;
        a.n_steps = f.k;
        as.push_back(a);
      }
      const GroupRes &lead = fused[b0].r;
      const double t = e->now();
      (void)hipEventRecord(lead.e0, lead.s);
      const mfq_status st = mfq_run_group(cs.data(), as.data(), (int32_t)cs.size());
      (void)hipEventRecord(lead.e1, lead.s);
      for (size_t i = b0; i < b1; ++i) runs.push_back({fused[i].gid, fused[i].k, fused[i].r, t, st, &fused[b0].r});
    }
    // the synchronising groups go last, each from a host thread of its own, so that their
    // host round trips overlap one another and the groups already in flight
    {
      std::vector<std::thread> th;
      std::vector<double> t0(blocking.size());
      auto advance = [e, &blocking, &t0](size_t i) {
        Pending &b = blocking[i];
        (void)hipSetDevice(e->device);
        t0[i] = e->now();
        (void)hipEventRecord(b.r.e0, b.r.s);
        b.st = mfq_step(b.r.c, b.key.protocol, b.gam.data(), b.key.dt, b.key.seed, b.k);
        (void)hipEventRecord(b.r.e1, b.r.s);
      };
      th.reserve(blocking.size());
      for (size_t i = 0; i < blocking.size(); ++i) {
        try {
          th.emplace_back(advance, i);
        } catch (const std::system_error &) {  // no thread available: advance it here
          advance(i);
        }
      }
      for (std::thread &t : th) t.join();
      for (size_t i = 0; i < blocking.size(); ++i)
        runs.push_back({blocking[i].gid, blocking[i].k, blocking[i].r, t0[i], blocking[i].st, nullptr});
    }
    for (Run &r : runs) {
      mfq_status st = r.st != MFQ_OK ? r.st : mfq_synchronize(r.r.c);
      const GroupRes &tm = r.timer ? *r.timer : r.r;
      float ms = 0.0f;
      double wall = e->now() - r.t_start;
      if (st == MFQ_OK && hipEventElapsedTime(&ms, tm.e0, tm.e1) == hipSuccess) wall = 1e-3 * ms;
      std::unique_lock<std::mutex> lk(e->m);
      if (st != MFQ_OK) {
        e->policy.fail_group_jobs(r.gid, st, e->now());
        continue;
      }
      std::vector<uint64_t> obs = e->policy.advanced(r.gid, r.k, wall);
      const Group &g = e->policy.group(r.gid);
      // one entropy call per distinct region among the observing jobs
      std::vector<double> S(g.capacity, 0.0);
      std::vector<bool> done(obs.size(), false);
      for (size_t a = 0; a < obs.size(); ++a) {
        if (done[a]) continue;
        const Job *ja = e->policy.job(obs[a]);
        const std::vector<int> region = ja->region;
        lk.unlock();
        st = mfq_entropy(r.r.c, region.data(), (int32_t)region.size(), S.data());
        lk.lock();
        if (st != MFQ_OK) {
          e->policy.fail_group_jobs(r.gid, st, e->now());
          break;
        }
        for (size_t b = a; b < obs.size(); ++b) {
          Job *jb = e->policy.job_mut(obs[b]);
          if (done[b] || jb->region != region) continue;
          done[b] = true;
          e->policy.record(jb->id, S[jb->slot]);
          if (jb->steps_done >= jb->n_steps) e->policy.complete(jb->id, e->now());
        }
      }
    }
    e->cv.notify_all();
  }
}

}  // namespace

extern "C" {

mfq_status mfq_engine_create(int device, size_t hbm_budget_bytes, int32_t max_slots, mfq_engine **out) {
  if (!out || max_slots < 1) return MFQ_EINVAL;
  *out = nullptr;
  if (hbm_budget_bytes == 0) hbm_budget_bytes = (size_t)64 << 30;
  mfq_engine *e = new (std::nothrow) mfq_engine(device, hbm_budget_bytes, max_slots, footprint);
  if (!e) return MFQ_ENOMEM;
  e->worker = std::thread(worker_loop, e);
  *out = e;
  return MFQ_OK;
}

mfq_status mfq_engine_destroy(mfq_engine *e) {
  if (!e) return MFQ_OK;
  {
    std::unique_lock<std::mutex> lk(e->m);
    e->stop = true;
  }
  e->cv.notify_all();
  if (e->worker.joinable()) e->worker.join();
  for (auto &kv : e->res_of_group) release(kv.second);
  delete e;
  return MFQ_OK;
}

const char *mfq_engine_last_error(const mfq_engine *e) { return e ? e->err.c_str() : "null engine"; }

mfq_status mfq_engine_submit(mfq_engine *e, const mfq_job *job, uint64_t *job_id) {
  if (!e || !job || !job_id) return MFQ_EINVAL;
  const int L = job->lat.dim == 2 ? job->lat.Lx * job->lat.Ly : job->lat.Lx;
  const int N = job->N > 0 ? job->N : L / 2;
  const bool lat_ok = (job->lat.dim == 1 && job->lat.Lx >= 2 && job->lat.Lx % 2 == 0) ||
                      (job->lat.dim == 2 && job->lat.Lx >= 2 && job->lat.Ly >= 2 && job->lat.Lx % 2 == 0 &&
                       job->lat.Ly % 2 == 0);
  if (!lat_ok || 2 * N != L) {
    e->err = "jobs start from the Neel / checkerboard state: even sizes and N = L/2";
    return MFQ_EINVAL;
  }
  if ((job->protocol != MFQ_PROJECTIVE && job->protocol != MFQ_HOMODYNE) || !(job->gamma >= 0.0) ||
      !(job->dt > 0.0) || job->n_steps < 1 || job->obs_every < 0 ||
      (job->precision != MFQ_FP64 && job->precision != MFQ_FP32_BULK) || job->n_region < 0 ||
      job->n_region > L || (job->n_region > 0 && !job->region)) {
    e->err = "invalid job";
    return MFQ_EINVAL;
  }
  Job j;
  j.key.dim = job->lat.dim;
  j.key.Lx = job->lat.Lx;
  j.key.Ly = job->lat.dim == 2 ? job->lat.Ly : 1;
  j.key.J = job->lat.J;
  j.key.N = N;
  j.key.protocol = job->protocol;
  j.key.precision = job->precision;
  j.key.dt = job->dt;
  j.key.seed = job->seed;
  j.gamma = job->gamma;
  j.uid = job->uid;
  j.n_steps = job->n_steps;
  j.obs_every = job->obs_every;
  for (int i = 0; i < job->n_region; ++i) {
    if (job->region[i] < 0 || job->region[i] >= L || (i > 0 && job->region[i] <= job->region[i - 1])) {
      e->err = "region must be ascending site ids in [0, L)";
      return MFQ_EINVAL;
    }
    j.region.push_back(job->region[i]);
  }
  {
    std::unique_lock<std::mutex> lk(e->m);
    j.t_submit = e->now();
    *job_id = e->policy.submit(std::move(j));
  }
  e->cv.notify_all();
  return MFQ_OK;
}

mfq_status mfq_engine_poll(mfq_engine *e, uint64_t job_id, double *S_host, int32_t max_obs,
                           int32_t *n_obs, double *latency_s) {
  if (!e) return MFQ_EINVAL;
  std::unique_lock<std::mutex> lk(e->m);
  const Job *j = e->policy.job(job_id);
  if (!j) return MFQ_EINVAL;
  if (j->state == FAILED) return j->error ? j->error : MFQ_EDEVICE;
  if (j->state != DONE) return MFQ_PENDING;
  const int n = (int)j->S.size();
  if (n_obs) *n_obs = n;
  if (S_host)
    for (int i = 0; i < std::min(n, (int)max_obs); ++i) S_host[i] = j->S[i];
  if (latency_s) *latency_s = j->t_done - j->t_submit;
  return MFQ_OK;
}

mfq_status mfq_engine_wait(mfq_engine *e, uint64_t job_id, double timeout_s) {
  if (!e) return MFQ_EINVAL;
  std::unique_lock<std::mutex> lk(e->m);
  const auto deadline = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s);
  while (true) {
    const Job *j = e->policy.job(job_id);
    if (!j) return MFQ_EINVAL;
    if (j->state == DONE) return MFQ_OK;
    if (j->state == FAILED) return j->error ? j->error : MFQ_EDEVICE;
    if (e->cv.wait_until(lk, deadline) == std::cv_status::timeout) return MFQ_PENDING;
  }
}

mfq_status mfq_engine_stats(mfq_engine *e, mfq_engine_stats_t *out) {
  if (!e || !out) return MFQ_EINVAL;
  std::unique_lock<std::mutex> lk(e->m);
  std::memset(out, 0, sizeof(*out));
  out->bytes_in_use = e->policy.bytes_in_use();
  out->peak_bytes = e->policy.peak_bytes();
  out->budget_bytes = e->policy.budget();
  out->queued = (int64_t)e->policy.queued();
  out->groups = e->policy.live_groups();
  return MFQ_OK;
}

}  // extern "C"
