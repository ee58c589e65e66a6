"""Benchmark: monitored free-fermion trajectories on one MI355X.

Default line (the largest single-GPU workload, 160 x 160 torus of Sec. IV): L = 25600 sites,
N = 12800 particles, checkerboard start, homodyne protocol with gamma in {0.5, 1.0, 2.0} (one
trajectory each, advanced together), dt = 0.05, plain FP64 with the dense propagator.  A "step"
is one time step of the three trajectories: propagator GEMM U <- P U (8 L^2 N flop per
trajectory), fused Born probabilities + homodyne factor, both Cholesky-QR passes.  `--warmup`
untimed steps, then exactly `--steps` steps timed on the host clock between two device
synchronisations; value = 3 L N steps / time.  The mutual information of the strips
x in [0,40) and [80,120) (observed every 100 steps) is timed on its own after the window.

Extra legs in the same run (not `value`): the FP32-bulk propagator on the same torus with its
entropy error against FP64 taken at the end of the warm-up (outside both timed windows), the
L = 16384 ring with the dense FP64 propagator (the propagator GEMM the 50 %-of-peak target is
stated on), the 384-trajectory L = 1024 ring batch, and the CPU oracle on a bounded sample.

Other workloads: --workload ring1024_qsd | ring16384_pm | ring16384_qsd | ring1024_pm_ct |
served_mix.  served_mix submits the first --jobs arrivals of a seeded Poisson stream at --rate
jobs/s to the continuous-batching engine (default 32 at 0.25 jobs/s, a load the engine keeps up
with) and reports throughput beside the measured per-job latency distribution (p50, p99).
Prints one JSON line.
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 matrix peak
PEAK_FP32_TFLOPS = 157.3  # MI355X dense FP32 matrix peak
PEAK_HBM_GBS = 8000.0
COPY_BYTES = 1 << 30      # calibration copy for the HBM byte counters
GEMM_SRC = os.path.join(ROOT, "paper_2508_18468_amd", "csrc", "zgemm.hip")


def pmc_file(workload):
    return os.path.join(ROOT, "profiles", f"propagator_zgemm_{workload}_pmc.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_hash():
    with open(GEMM_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_from_profile(workload, n_traj):
    """HBM bytes per propagator launch from committed rocprofv3 FETCH_SIZE / WRITE_SIZE runs,
    scaled by the copy-kernel calibration; null unless taken on the current kernel source."""
    try:
        with open(pmc_file(workload)) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256") != source_hash() or d.get("n_traj") != n_traj:
        return None
    return d.get("hbm_bytes_per_launch")


def host_cores():
    """(threads the BLAS pool uses, CPU model, CPUs in the affinity mask)."""
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), None)
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = None
    return int(cores), model, affinity


def cpu_baseline_sample(w, n_sample, protocol, steps=2):
    """The oracle's own steps (numpy / LAPACK FP64) on the workload's lattice with n_sample
    particles (the first n_sample sites of the default filling), `steps` steps at the first
    rate.  Its cost per step is about 8 L^2 N (dense propagator product) + 8 L N^2 flop
    (Householder QR), so the full-filling step time is extrapolated by that count."""
    import oracle
    from oracle.trajectory import step as ostep
    lat = oracle.Lattice(w.dim, w.Lx, w.Ly if w.dim == 2 else 1)
    t_build = time.perf_counter()
    P = oracle.propagator(lat, w.dt)
    t_build = time.perf_counter() - t_build
    U = oracle.initial_state(lat.L, oracle.default_occupied(lat)[:n_sample])
    t0 = time.perf_counter()
    for n in range(1, steps + 1):
        U, _ = ostep(U, P, protocol, w.gammas[0], w.dt, w.seed, 0, n)
    t1 = (time.perf_counter() - t0) / steps
    flops = lambda N: 8.0 * lat.L * lat.L * N + 8.0 * lat.L * N * N
    t_full = t1 * flops(w.N) / flops(n_sample)
    cores, model, affinity = host_cores()
    return {"value": lat.L * n_sample / t1, "unit": "L*N*steps/s", "cores": cores, "kind": "oracle",
            "cpu_model": model, "cpus_available": affinity,
            "sample": f"{steps} oracle steps (rate {w.gammas[0]}) of the {w.name} lattice (L={lat.L}) "
                      f"with N'={n_sample} particles: {t1:.2f} s per trajectory-step; the dense "
                      f"propagator (built once in {t_build:.1f} s, not counted) dominates the step",
            "extrapolated_full_N": {"N": w.N, "s_per_trajectory_step": t_full,
                                    "value": lat.L * w.N / t_full,
                                    "note": "extrapolated by the flop count 8 L^2 N + 8 L N^2"}}


def cpu_baseline_ring1024(w, steps):
    """The oracle on 2 trajectories x `steps` steps per gamma (bounded sample)."""
    import oracle
    from oracle.trajectory import step as ostep, HOMODYNE
    lat = oracle.Lattice(1, w.Lx)
    P = oracle.propagator(lat, w.dt)
    occ = oracle.default_occupied(lat)
    t0 = time.perf_counter()
    n_ts = 0
    for gi, g in enumerate(w.gammas):
        for uid in w.uids(gi)[:2]:
            U = oracle.initial_state(lat.L, occ)
            for n in range(1, steps + 1):
                U, _ = ostep(U, P, HOMODYNE, g, w.dt, w.seed, uid, n)
                n_ts += 1
            oracle.entanglement_entropy(U, w.regions[0])
    dt = time.perf_counter() - t0
    cores, model, affinity = host_cores()
    return {"value": n_ts * w.L * w.N / dt, "unit": "L*N*steps/s", "cores": cores,
            "kind": "oracle", "cpu_model": model, "cpus_available": affinity,
            "sample": f"2 trajectories x {steps} steps per gamma ({n_ts} trajectory-steps) of the same "
                      f"L={w.L} homodyne workload plus one entropy each, numpy/LAPACK FP64; "
                      f"{dt:.1f} s wall"}


def pmc_workload(workload):
    """Short run for hardware-counter passes: 3 FP64 steps of the workload, then an
    elementwise multiply over COPY_BYTES (the calibration kernel for FETCH/WRITE_SIZE)."""
    import numpy as np
    import torch
    from paper_2508_18468_amd import mfq
    from paper_2508_18468_amd.workloads import ring_qsd_batched, torus_qsd
    if workload == "torus160_qsd":
        w = torus_qsd()
        uids = list(range(len(w.gammas)))
        gam = np.asarray(w.gammas)
        sim = mfq.Trajectories(2, w.Lx, w.Ly, n_traj=len(uids), uids=uids, device=0)
    else:
        w = ring_qsd_batched()
        uids = w.uids(0) + w.uids(1) + w.uids(2)
        gam = np.repeat(np.asarray(w.gammas), w.n_traj)
        sim = mfq.Trajectories(1, w.Lx, n_traj=len(uids), uids=uids, device=0)
    for k in range(3):
        sim.step(mfq.HOMODYNE, gam, w.dt, w.seed, 1)
        sim.synchronize()
        log(f"pmc workload: step {k + 1}/3")
    sim.close()
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    torch.mul(src, 2.0, out=dst)  # elementwise kernel: reads COPY_BYTES, writes COPY_BYTES
    torch.cuda.synchronize()
    print("pmc workload done")


def _pmc_rows(path):
    import csv
    out = []
    for r in csv.DictReader(open(path)):
        out.append((int(r.get("Dispatch_Id", 0)), r.get("Kernel_Name", ""), r.get("Counter_Name", ""),
                    float(r.get("Counter_Value", "nan"))))
    return out


def summarize_pmc(fetch_csv, write_csv, out_path, workload):
    """Per-launch HBM bytes of the propagator kernel from FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch), each scaled by what the counter reads for the calibration multiply."""
    from paper_2508_18468_amd.workloads import ring_qsd_batched, torus_qsd
    w = torus_qsd() if workload == "torus160_qsd" else ring_qsd_batched()
    B = len(w.gammas) * (1 if workload == "torus160_qsd" else w.n_traj)
    res = {}
    for label, path in (("fetch", fetch_csv), ("write", write_csv)):
        rows = _pmc_rows(path)
        prop = [v for (_, n, c, v) in rows if "propagator_zgemm_kernel" in n]
        copy = [v for (_, n, c, v) in rows if "elementwise" in n and "Mul" in n]
        copy_kib = copy[-1] if copy else None
        scale = COPY_BYTES / (copy_kib * 1024.0) if copy_kib else None
        res[label] = {"propagator_kib_per_dispatch": prop, "copy_kib": copy_kib, "scale": scale}
    f, wr = res["fetch"], res["write"]
    per_launch = None
    if f["propagator_kib_per_dispatch"] and wr["propagator_kib_per_dispatch"] and f["scale"] and wr["scale"]:
        fk = sum(f["propagator_kib_per_dispatch"]) / len(f["propagator_kib_per_dispatch"])
        wk = sum(wr["propagator_kib_per_dispatch"]) / len(wr["propagator_kib_per_dispatch"])
        per_launch = fk * 1024.0 * f["scale"] + wk * 1024.0 * wr["scale"]
    d = {"kernel": "propagator_zgemm_kernel", "workload": workload, "n_traj": B,
         "kernel_source_sha256": source_hash(), "copy_bytes": COPY_BYTES,
         "fetch": f, "write": wr, "hbm_bytes_per_launch": per_launch,
         "algorithmic_bytes_per_launch": 16.0 * (w.L * w.L + 2 * w.L * w.N * B)}
    with open(out_path, "w") as fo:
        json.dump(d, fo, indent=1)
    print(json.dumps(d))


def timed_steps(sim, protocol, gam, w, steps, label):
    """`steps` steps, one call each, timed on the host clock between device synchronisations,
    with per-phase HIP-event times on the library's stream.  Returns (seconds, phases)."""
    import torch
    sim.synchronize()
    torch.cuda.synchronize()
    sim.profile(True)
    t0 = time.perf_counter()
    for k in range(steps):
        sim.step(protocol, gam, w.dt, w.seed, 1)
        if steps <= 50 or (k + 1) % 10 == 0:
            sim.synchronize()
            log(f"  {label}: step {k + 1}/{steps}")
    sim.synchronize()
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    phases = sim.phase_times()
    sim.profile(False)
    return T, phases


def phase_per_step(phases, steps):
    return {k: v[0] / steps for k, v in phases.items()}


def gemm_roofline(phases, flops, peak, kernel, traffic=None):
    ms, n = phases["propagate"]
    if not n:
        return None
    avg_ms = ms / n
    tf = flops / (avg_ms * 1e-3) / 1e12
    return {"bound": "mfma", "achieved": tf, "peak": peak, "unit": "TFLOP/s", "frac": tf / peak,
            "traffic": traffic, "kernel": kernel, "algorithmic_flops_per_launch": flops,
            "avg_launch_ms": avg_ms}


def leg_ring16384(steps, warmup):
    """The L = 16384 ring (projective, gamma 0.2 and 1.0) with the dense FP64 propagator."""
    import numpy as np
    from paper_2508_18468_amd import mfq
    from paper_2508_18468_amd.workloads import ring_pm_large
    w = ring_pm_large()
    B = len(w.gammas)
    sim = mfq.Trajectories(1, w.Lx, n_traj=B, uids=[g * w.n_traj for g in range(B)], device=0)
    gam = np.asarray(w.gammas)
    log(f"{w.name}: {warmup} warm-up step(s), {steps} timed")
    sim.step(w.protocol, gam, w.dt, w.seed, warmup)
    T, ph = timed_steps(sim, w.protocol, gam, w, steps, w.name)
    sim.close()
    roof = gemm_roofline(ph, 8.0 * w.L * w.L * w.N * B, PEAK_FP64_TFLOPS, "propagator_zgemm_kernel")
    return {"workload": w.name, "L": w.L, "N": w.N, "n_traj": B, "gammas": list(w.gammas),
            "protocol": "projective", "precision": "fp64", "propagator": "dense",
            "steps_timed": steps, "warmup": warmup, "value": B * w.L * w.N * steps / T,
            "unit": "L*N*steps/s", "ms_per_step": T / steps * 1e3, "propagator_roofline": roof,
            "phase_ms_per_step": phase_per_step(ph, steps)}


def leg_ring1024(steps, warmup):
    """The 384-trajectory L = 1024 homodyne batch, FP64 dense propagator."""
    import numpy as np
    from paper_2508_18468_amd import mfq
    from paper_2508_18468_amd.workloads import ring_qsd_batched
    w = ring_qsd_batched()
    uids = w.uids(0) + w.uids(1) + w.uids(2)
    B = len(uids)
    gam = np.repeat(np.asarray(w.gammas), w.n_traj)
    sim = mfq.Trajectories(1, w.Lx, n_traj=B, uids=uids, device=0)
    log(f"{w.name}: {warmup} warm-up steps, {steps} timed")
    sim.step(mfq.HOMODYNE, gam, w.dt, w.seed, warmup)
    T, ph = timed_steps(sim, mfq.HOMODYNE, gam, w, steps, w.name)
    sim.close()
    roof = gemm_roofline(ph, 8.0 * w.L * w.L * w.N * B, PEAK_FP64_TFLOPS, "propagator_zgemm_kernel")
    return {"workload": w.name, "L": w.L, "N": w.N, "n_traj": B, "precision": "fp64",
            "steps_timed": steps, "warmup": warmup, "value": B * w.L * w.N * steps / T,
            "unit": "L*N*steps/s", "ms_per_step": T / steps * 1e3, "propagator_roofline": roof,
            "phase_ms_per_step": phase_per_step(ph, steps)}


def run_headline(args):
    """160 x 160 torus, FP64 dense propagator (value), then the extra legs."""
    import numpy as np
    from paper_2508_18468_amd import mfq
    from paper_2508_18468_amd.workloads import torus_qsd
    w = torus_qsd()
    B = len(w.gammas)
    uids = [g * w.n_traj for g in range(B)]
    gam = np.asarray(w.gammas, dtype=np.float64)
    A, Bs = w.mi
    steps, warm = args.steps, args.warmup

    log(f"{w.name}: L={w.L} N={w.N} trajectories={B} fp64 dense: {warm} warm-up steps, {steps} timed")
    sim = mfq.Trajectories(2, w.Lx, w.Ly, n_traj=B, uids=uids, device=0, precision=mfq.FP64)
    sim.set_propagator(mfq.PROP_DENSE)
    sim.step(mfq.HOMODYNE, gam, w.dt, w.seed, warm)
    S64_warm = sim.entropy(A)  # at step `warm`, outside the timed window
    T, ph = timed_steps(sim, mfq.HOMODYNE, gam, w, steps, "torus160 fp64")
    t1 = time.perf_counter()
    I2 = sim.mutual_info(A, Bs)
    t_I2 = time.perf_counter() - t1
    sim.close()
    value = B * w.L * w.N * steps / T
    flops = 8.0 * w.L * w.L * w.N * B
    roof = gemm_roofline(ph, flops, PEAK_FP64_TFLOPS, "propagator_zgemm_kernel",
                         traffic_from_profile(w.name, B))
    step_s = T / steps
    out = {
        "metric": "L*N*steps/s",
        "value": value,
        "unit": "L*N*steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "torus160_qsd: 2d 160x160 torus (L=25600, N=12800), periodic, NN hopping "
                               "J=1, checkerboard start, homodyne gamma {0.5,1.0,2.0} (one trajectory "
                               "each, advanced together), dt=0.05, dense FP64 propagator, Cholesky-QR2; "
                               "I2 of the strips x in [0,40) and [80,120) every 100 steps",
                   "L": w.L, "N": w.N, "n_traj": B, "gammas": list(w.gammas), "dt": w.dt,
                   "precision": "fp64", "propagator": "dense", "obs_every": w.obs_every,
                   "observations_timed": 0},
        "gemm_tflops": roof["achieved"] if roof else None,
        "roofline": roof,
        "phase_ms_per_step": phase_per_step(ph, steps),
        "observation": {"mutual_info_s": t_I2, "I2": [float(x) for x in I2],
                        "value_with_I2_every_100_steps": B * w.L * w.N / (step_s + t_I2 / w.obs_every),
                        "note": "no observation falls inside the timed window (every 100 steps); "
                                "the I2 time is measured after it and amortised here"},
        "traj_latency_s": {"p50": None, "p99": None,
                           "note": "the three trajectories of this batch finish together; the "
                                   "per-job latency distribution is measured by --workload served_mix"},
    }
    if not args.headline_only:
        # FP32-bulk propagator on the same torus (the precision the torus workload names)
        k32 = min(steps, 6)
        log(f"{w.name}: fp32-bulk: {warm} warm-up steps, {k32} timed")
        s32 = mfq.Trajectories(2, w.Lx, w.Ly, n_traj=B, uids=uids, device=0, precision=mfq.FP32_BULK)
        s32.step(mfq.HOMODYNE, gam, w.dt, w.seed, warm)
        S32_warm = s32.entropy(A)
        T32, ph32 = timed_steps(s32, mfq.HOMODYNE, gam, w, k32, "torus160 fp32-bulk")
        s32.close()
        # relative where S > 0 (a product state, warm-up 0, has S = 0: absolute there)
        rel = np.abs(S32_warm - S64_warm) / np.where(np.abs(S64_warm) > 0, np.abs(S64_warm), 1.0)
        r32 = gemm_roofline(ph32, flops, PEAK_FP32_TFLOPS, "propagator_delta_f32_kernel")
        v32 = B * w.L * w.N * k32 / T32
        out["fp32_bulk"] = {
            "value": v32, "unit": "L*N*steps/s", "ms_per_step": T32 / k32 * 1e3, "steps_timed": k32,
            "speedup_vs_fp64": v32 / value, "propagator_roofline": r32,
            "phase_ms_per_step": phase_per_step(ph32, k32),
            "rel_dS_vs_fp64": [float(x) for x in rel], "max_rel_dS_vs_fp64": float(rel.max()),
            "S_fp64": [float(x) for x in S64_warm], "rel_dS_at_step": warm,
            "rel_dS_region": "strip x in [0,40), all y (6400 sites)",
            "note": "S of strip A after the warm-up steps in FP64 and in FP32-bulk from the same "
                    "start and draws, both outside the timed windows; target |dS|/S <= 1e-4"}
        out["ring16384_fp64_dense"] = leg_ring16384(min(steps, 3), 1)
        out["ring1024_qsd_batched"] = leg_ring1024(steps, warm)
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle sample")
        from oracle.trajectory import HOMODYNE
        out["cpu_baseline"] = cpu_baseline_sample(w, args.cpu_particles, HOMODYNE)
    print(json.dumps(out))


def run_ring1024(args):
    """The 384-trajectory ring L = 1024 homodyne batch as its own line."""
    from paper_2508_18468_amd.workloads import ring_qsd_batched
    w = ring_qsd_batched()
    leg = leg_ring1024(args.steps, args.warmup)
    B = leg["n_traj"]
    roof = leg["propagator_roofline"]
    if roof:
        roof["traffic"] = traffic_from_profile(w.name, B)
    out = {"metric": "L*N*steps/s", "value": leg["value"], "unit": "L*N*steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": leg["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "ring1024_qsd: 1d ring L=1024 N=512, Neel start, homodyne gamma "
                                  "{0.1,0.3,1.0} x 128 trajectories batched, dt=0.05",
                      "L": w.L, "N": w.N, "n_traj": B, "dt": w.dt, "precision": "fp64"},
           "roofline": roof, "phase_ms_per_step": leg["phase_ms_per_step"]}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_ring1024(w, args.cpu_steps)
    print(json.dumps(out))


def run_large(args):
    """The large ring shapes (one trajectory per gamma, batched): exactly `steps` timed steps
    after `warmup`, per-phase times, then every observation of the workload timed on its own."""
    import numpy as np
    from paper_2508_18468_amd import mfq
    from paper_2508_18468_amd.workloads import ring_pm_large, ring_qsd_large
    w = {"ring16384_pm": ring_pm_large, "ring16384_qsd": ring_qsd_large}[args.workload]()
    prec_name = args.precision or "fp64"
    precision = mfq.FP64 if prec_name == "fp64" else mfq.FP32_BULK
    B = len(w.gammas)
    uids = [g * w.n_traj for g in range(B)]
    sim = mfq.Trajectories(w.dim, w.Lx, w.Ly, n_traj=B, uids=uids, device=0, precision=precision)
    factored = args.propagator == "factored"
    sim.set_propagator(mfq.PROP_FACTORED if factored else mfq.PROP_DENSE)
    rk4 = args.integrator == "rk4"
    sim.set_integrator(mfq.INTEGRATOR_RK4 if rk4 else mfq.INTEGRATOR_SPLIT)
    gam = np.asarray(w.gammas, dtype=np.float64)
    steps, warm = args.steps, args.warmup
    log(f"{w.name}: L={w.L} N={w.N} trajectories={B} {prec_name}: {warm} warm-up steps, {steps} timed")
    sim.step(w.protocol, gam, w.dt, w.seed, warm)
    T, phases = timed_steps(sim, w.protocol, gam, w, steps, w.name)
    band = sim.propagator_band()
    obs = {}
    for r in w.regions:
        t1 = time.perf_counter()
        S = sim.entropy(r)
        obs[f"S_l{len(r)}_s"] = time.perf_counter() - t1
        obs[f"S_l{len(r)}"] = [float(x) for x in S]
    sim.close()
    prop_ms, prop_n = phases["propagate"]
    per_launch_s = prop_ms / prop_n * 1e-3 if prop_n else None
    if (rk4 and w.protocol == 1) or factored:
        # memory-bound passes: RK4 = Born read (16 L N B bytes) + the first stage (reads U, writes
        # V: 32 L N B) + three stages that read U and V and write V' (48 L N B each); ring band =
        # one read and one write of U
        alg = (192.0 if rk4 and w.protocol == 1 else 32.0) * w.L * w.N * B
        achieved = alg / per_launch_s / 1e9 if per_launch_s else None
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS if achieved else None, "traffic": None,
                "kernel": "rk4 step" if rk4 and w.protocol == 1 else "ring band stencil",
                "algorithmic_bytes_per_launch": alg}
    else:
        peak = PEAK_FP64_TFLOPS if precision == mfq.FP64 else PEAK_FP32_TFLOPS
        roof = gemm_roofline(phases, 8.0 * w.L * w.L * w.N * B, peak, "propagator")
    value = B * w.L * w.N * steps / T
    out = {"metric": "L*N*steps/s", "value": value, "unit": "L*N*steps/s",
           "n_gpus": 1, "steps": steps, "warmup": warm, "ms_per_step": T / steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": w.name, "L": w.L, "N": w.N, "n_traj": B, "propagator": args.propagator,
                      "band": band if factored else None, "gammas": list(w.gammas),
                      "protocol": "projective" if w.protocol == 0 else "homodyne",
                      "dt": w.dt, "precision": prec_name, "integrator": args.integrator,
                      "hours_per_trajectory_to_t_eq_L": (T / steps / B) * (w.L / w.dt) / 3600.0},
           "roofline": roof,
           "phase_ms_per_step": phase_per_step(phases, steps),
           "observations": obs}
    if w.name == "ring16384_qsd":
        # the paper's one measured rate: a homodyne trajectory at L = 16384 over t in [0, L] in
        # about 130 h on one A100, i.e. 9.4e7 L*N*steps/s (other hardware: context only)
        out["paper_context"] = {"a100_L_N_steps_per_s": 9.4e7, "ratio": value / 9.4e7}
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle sample")
        out["cpu_baseline"] = cpu_baseline_sample(w, args.cpu_particles, w.protocol)
    print(json.dumps(out))


def run_continuous(args):
    """Continuous-time projective protocol on the ring1024_pm_ct workload: `steps` event slots
    (one event per trajectory each) after `warmup`, timed on the host clock around the slots and
    per kernel with HIP events on the library's stream."""
    import numpy as np
    from paper_2508_18468_amd import mfq
    from paper_2508_18468_amd.workloads import ring_pm_continuous
    w = ring_pm_continuous()
    uids = w.uids(0) + w.uids(1) + w.uids(2)
    B = len(uids)
    gam = np.repeat(np.asarray(w.gammas), w.n_traj)
    sim = mfq.Trajectories(1, w.Lx, n_traj=B, uids=uids, device=0)
    sim.set_ct_block(args.ct_block)
    steps, warm = args.steps, args.warmup
    log(f"{w.name}: L={w.L} N={w.N} trajectories={B}: {warm} warm-up slots, {steps} timed")
    sim.ct_events(gam, w.seed, warm, reorth_every=args.reorth_every)
    sim.synchronize()
    sim.profile(True)
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        k = min(64, steps - done)
        sim.ct_events(gam, w.seed, k, reorth_every=args.reorth_every)
        sim.synchronize()
        done += k
        log(f"  {done}/{steps} slots")
    T = time.perf_counter() - t0
    phases = sim.phase_times()
    sim.profile(False)
    t = sim.times()
    sim.close()
    ev_ms = (phases["measure"][0] + phases["propagate"][0]) / steps
    if args.ct_block > 0:
        # per slot: the flush's products (8 L N (2K + 2K + K) flop per trajectory and block)
        # amortised over the block, the band pass over U once per block
        alg_flops = 8.0 * w.L * w.N * 5 * B
        achieved = alg_flops / (ev_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None,
                "kernel": f"deferred events, blocks of {args.ct_block}",
                "algorithmic_flops_per_slot": alg_flops}
    else:
        alg_bytes = 48.0 * w.L * w.N * B  # U read by the GEMV, read and written by the stencil pass
        achieved = alg_bytes / (ev_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                "kernel": "event slot (draw, GEMV, stencil + rank-1 update)",
                "algorithmic_bytes_per_slot": alg_bytes}
    out = {"metric": "L*N*events/s", "value": B * w.L * w.N * steps / T, "unit": "L*N*events/s",
           "n_gpus": 1, "steps": steps, "warmup": warm, "ms_per_step": T / steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": w.name, "L": w.L, "N": w.N, "n_traj": B, "gammas": list(w.gammas),
                      "protocol": "projective, continuous time", "reorth_every": args.reorth_every,
                      "ct_block": args.ct_block, "mean_clock_after": float(np.mean(t))},
           "roofline": roof,
           "phase_ms_per_step": phase_per_step(phases, steps)}
    print(json.dumps(out))


def run_served(args):
    """The served mix through the continuous-batching engine: the first `jobs` arrivals of the
    seeded Poisson stream at `rate` jobs/s, per-job latency from arrival to completion."""
    from paper_2508_18468_amd import serve
    log(f"served_mix: {args.jobs} jobs at {args.rate} jobs/s, {args.job_steps} steps each")
    r = serve.run(args.jobs, args.rate, args.job_steps, verbose=False, log=log)
    out = {"metric": "L*N*steps/s", "value": r["throughput_LNsteps_per_s"], "unit": "L*N*steps/s",
           "n_gpus": 1, "steps": args.job_steps, "warmup": 0, "ms_per_step": None,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"served_mix: first {args.jobs} arrivals of a seeded Poisson stream "
                                  f"({args.rate} jobs/s), 1d L in {{256..4096}} or 2d side in "
                                  "{16,32,48,64}, protocol 50/50, gamma ~ U(0.1,2), dt=0.05",
                      "jobs": args.jobs, "rate_jobs_per_s": args.rate, "steps_per_job": args.job_steps},
           "traj_latency_s": r["latency_s"], "served": r}
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-steps", type=int, default=20, help="ring1024_qsd: oracle steps per trajectory")
    ap.add_argument("--cpu-particles", type=int, default=400,
                    help="large workloads: particles of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="torus line only, without the extra legs (for profiler runs)")
    ap.add_argument("--pmc-workload", action="store_true",
                    help="short run for rocprofv3 --pmc passes (3 steps + calibration multiply)")
    ap.add_argument("--summarize-pmc", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "OUT_JSON"))
    ap.add_argument("--workload", default="torus160_qsd",
                    choices=["torus160_qsd", "ring1024_qsd", "ring16384_pm", "ring16384_qsd",
                             "ring1024_pm_ct", "served_mix"])
    ap.add_argument("--integrator", default="split", choices=["split", "rk4"],
                    help="large ring workloads: split step (default) or the paper's RK4")
    ap.add_argument("--ct-block", type=int, default=32,
                    help="ring1024_pm_ct: deferred events per block (0: event by event)")
    ap.add_argument("--reorth-every", type=int, default=256,
                    help="ring1024_pm_ct: Cholesky-QR after every this many event slots (0: never)")
    ap.add_argument("--propagator", default="dense", choices=["dense", "factored"],
                    help="large ring workloads: dense GEMM (default) or banded form")
    ap.add_argument("--precision", default=None, choices=["fp64", "fp32_bulk"],
                    help="large ring workloads (default fp64)")
    ap.add_argument("--jobs", type=int, default=32, help="served_mix: arrivals")
    ap.add_argument("--rate", type=float, default=0.25,
                    help="served_mix: mean arrivals per second (0.25: a load the engine sustains; "
                         "20: the overload window)")
    ap.add_argument("--job-steps", type=int, default=500, help="served_mix: steps per job")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc, args.workload)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: trajectories shard across GPUs with no communication, "
              "so a multi-GPU run is not measured here; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    if args.pmc_workload:
        pmc_workload(args.workload)
        return
    if args.workload == "torus160_qsd":
        run_headline(args)
    elif args.workload == "ring1024_qsd":
        run_ring1024(args)
    elif args.workload == "ring1024_pm_ct":
        run_continuous(args)
    elif args.workload == "served_mix":
        run_served(args)
    else:
        run_large(args)


if __name__ == "__main__":
    main()
