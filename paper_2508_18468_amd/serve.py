"""Served mix: a seeded Poisson stream of trajectory jobs through the library's
continuous-batching engine, reporting throughput and latency percentiles.

    python -m paper_2508_18468_amd.serve --jobs 64 --rate 20

Jobs are submitted at their arrival times (wall clock from the start of the
run); each job's latency is the time from submission to completion as
measured by the engine.  Throughput = sum over jobs of L*N*steps / wall time
of the whole window (first submission to last completion).
"""

import argparse
import json
import sys
import time

import numpy as np

from . import mfq
from .workloads import served_mix, HOMODYNE


def run(n_jobs=64, rate=20.0, n_steps=500, budget_gb=200.0, max_slots=8, seed=1, verbose=False, log=None):
    """Serve the first n_jobs arrivals; `log` (a callable taking a line) reports each completion
    as it is collected."""
    jobs = served_mix(n_jobs, rate, n_steps, seed)
    eng = mfq.Engine(hbm_budget_bytes=int(budget_gb * (1 << 30)), max_slots=max_slots)
    t0 = time.perf_counter()
    ids = []
    for j in jobs:
        delay = j.arrival - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        ids.append(eng.submit(j.dim, j.Lx, j.Ly, j.protocol, j.gamma, j.dt, j.n_steps, j.seed, j.uid,
                              j.region))
        if log:
            log(f"submitted job {j.job_id} at {time.perf_counter() - t0:.1f} s (L={j.L})")
    t_sub = time.perf_counter() - t0
    lat, work = [], 0.0
    pending = list(zip(jobs, ids))
    deadline = time.perf_counter() + 3600.0
    while pending:  # collect in completion order (each latency is the engine's own measure)
        still = []
        for j, i in pending:
            r = eng.poll(i)
            if r is None:
                still.append((j, i))
                continue
            S, latency = r
            lat.append(latency)
            work += j.L * (j.L // 2) * j.n_steps
            line = (f"job {j.job_id}: L={j.L} proto={'qsd' if j.protocol == HOMODYNE else 'pm'} "
                    f"gamma={j.gamma:.2f} S={S[-1]:.4f} latency={latency:.2f}s")
            if verbose:
                print(line, flush=True)
            if log:
                log(line)
        pending = still
        if pending:
            if time.perf_counter() > deadline:
                raise TimeoutError(f"{len(pending)} jobs not done after an hour")
            time.sleep(0.05)
    T = time.perf_counter() - t0
    st = eng.stats()
    eng.close()
    lat = np.array(lat)
    offered_flop = sum(8.33 * j.L ** 3 * j.n_steps for j in jobs)
    return {
        "jobs": n_jobs, "rate_jobs_per_s": rate, "steps_per_job": n_steps,
        "arrival_window_s": float(jobs[-1].arrival), "submission_s": t_sub, "wall_s": T,
        "throughput_LNsteps_per_s": work / T,
        "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                      "mean": float(lat.mean()), "max": float(lat.max())},
        "offered_flop_per_s_approx": offered_flop / max(float(jobs[-1].arrival), 1e-9),
        "engine": {"peak_bytes": st["peak_bytes"], "budget_bytes": st["budget_bytes"]},
        "max_slots": max_slots,
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=64)
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--max-slots", type=int, default=8)
    ap.add_argument("--verbose", action="store_true")
    a = ap.parse_args(argv)
    res = run(a.jobs, a.rate, a.steps, a.budget_gb, a.max_slots, verbose=a.verbose)
    print(json.dumps(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
