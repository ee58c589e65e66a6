"""Seeded synthetic workloads (inputs only; no arithmetic of the method).

Shared by the test suite, the benchmark and the serving driver to build the
inputs that both the GPU library and the CPU oracle consume.  The paper
(arXiv:2508.18468) runs on no external dataset: a workload is fully defined
by lattice, filling, initial state, protocol, gamma, dt, seeds and the
observation schedule.  Shapes follow the paper's runs: 1d rings up to
L = 16384 (Sec. III), the 160 x 160 torus (Sec. IV), dt = 0.05 (Appendix A).

Trajectory uid = gamma_index * n_traj + t keys the random numbers, so a
trajectory draws the same numbers alone, in a batch or in a served mix.
"""

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

PROJECTIVE = 0
HOMODYNE = 1


@dataclass
class Workload:
    name: str
    dim: int
    Lx: int
    Ly: int
    protocol: int
    gammas: Tuple[float, ...]
    dt: float
    n_steps: int
    n_traj: int                   # per gamma
    seed: int = 0
    obs_every: int = 0
    regions: List[List[int]] = field(default_factory=list)
    mi: Optional[Tuple[List[int], List[int]]] = None

    @property
    def L(self):
        return self.Lx * (self.Ly if self.dim == 2 else 1)

    @property
    def N(self):
        return self.L // 2

    def uids(self, gamma_index):
        return [gamma_index * self.n_traj + t for t in range(self.n_traj)]


def interval(a, b):
    return list(range(a, b))


def strip(Lx, Ly, x0, x1):
    """Sites with x in [x0, x1) and any y, site id i = x + Lx*y (sorted)."""
    return sorted(x + Lx * y for y in range(Ly) for x in range(x0, x1))


def ring_pm_small():
    """1d ring L=64, N=32, projective gamma=0.5, dt=0.05, 400 steps, 16 trajectories,
    seed 0, S of A = [0, 32) every 10 steps."""
    return Workload("ring64_pm", 1, 64, 1, PROJECTIVE, (0.5,), 0.05, 400, 16, 0, 10,
                    [interval(0, 32)])


def ring_qsd_batched():
    """1d ring L=1024, N=512, homodyne gamma in {0.1, 0.3, 1.0}, dt=0.05, 2000 steps,
    128 trajectories per gamma, S of A = [0, 512) every 100 steps."""
    return Workload("ring1024_qsd", 1, 1024, 1, HOMODYNE, (0.1, 0.3, 1.0), 0.05, 2000, 128,
                    0, 100, [interval(0, 512)])


def ring_pm_continuous():
    """1d ring L=1024, N=512, continuous-time projective protocol (Poisson waiting times,
    total rate gamma N), gamma in {0.1, 0.3, 1.0}, 128 trajectories per gamma, seed 0,
    run to t = L/2 (the paper's stopping rule); n_steps = event slots timed."""
    return Workload("ring1024_pm_ct", 1, 1024, 1, PROJECTIVE, (0.1, 0.3, 1.0), 0.0, 200, 128, 0,
                    0, [interval(0, 512)])


def ring_pm_large():
    """1d ring L=16384, N=8192, projective gamma in {0.2, 1.0}, dt=0.05, 4L steps,
    S for l in {L/16, L/8, L/4, L/2}."""
    L = 16384
    return Workload("ring16384_pm", 1, L, 1, PROJECTIVE, (0.2, 1.0), 0.05, 4 * L, 1, 0,
                    L // 8, [interval(0, L // 16), interval(0, L // 8), interval(0, L // 4),
                             interval(0, L // 2)])


def ring_qsd_large():
    """1d ring L=16384, N=8192, homodyne gamma in {0.2, 1.0} (one trajectory each), dt=0.05,
    run to t = L (327680 steps; the shape of the paper's longest homodyne timing), S for
    l in {L/16, L/8, L/4, L/2}."""
    L = 16384
    return Workload("ring16384_qsd", 1, L, 1, HOMODYNE, (0.2, 1.0), 0.05, 20 * L, 1, 0,
                    L // 8, [interval(0, L // 16), interval(0, L // 8), interval(0, L // 4),
                             interval(0, L // 2)])


def torus_qsd():
    """2d 160x160 torus, homodyne gamma in {0.5, 1.0, 2.0}, dt=0.05; mutual information
    of the strips x in [0,40) and x in [80,120) (all y)."""
    S = 160
    return Workload("torus160_qsd", 2, S, S, HOMODYNE, (0.5, 1.0, 2.0), 0.05, 50, 1, 0, 100,
                    [], (strip(S, S, 0, 40), strip(S, S, 80, 120)))


@dataclass
class Job:
    """One served trajectory request."""
    job_id: int
    arrival: float
    dim: int
    Lx: int
    Ly: int
    protocol: int
    gamma: float
    dt: float
    n_steps: int
    seed: int
    uid: int
    region: List[int]

    @property
    def L(self):
        return self.Lx * (self.Ly if self.dim == 2 else 1)


def served_mix(n_jobs=256, rate=20.0, n_steps=500, seed=1):
    """Poisson stream (mean `rate` jobs/s): 1d L uniform over {256..4096}, 2d side uniform
    over {16, 32, 48, 64}, protocol 50/50, gamma ~ U(0.1, 2.0), dt = 0.05, S of the
    left half at the end.  Dimension 1d/2d chosen 50/50."""
    rng = np.random.Generator(np.random.Philox(key=np.array([seed, 0], dtype=np.uint64)))
    t = 0.0
    jobs = []
    for j in range(n_jobs):
        t += rng.exponential(1.0 / rate)
        if rng.random() < 0.5:
            L = int(rng.choice([256, 512, 1024, 2048, 4096]))
            dim, Lx, Ly = 1, L, 1
            region = interval(0, L // 2)
        else:
            s = int(rng.choice([16, 32, 48, 64]))
            dim, Lx, Ly = 2, s, s
            region = strip(s, s, 0, s // 2)
        proto = PROJECTIVE if rng.random() < 0.5 else HOMODYNE
        gamma = float(rng.uniform(0.1, 2.0))
        jobs.append(Job(j, t, dim, Lx, Ly, proto, gamma, 0.05, n_steps, 0, 1000000 + j, region))
    return jobs
