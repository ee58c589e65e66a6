"""Long-time ensemble means of the GPU trajectories against what the physics fixes exactly:
the projective protocol's mean map (the outcome-averaged update of Eq. (A1)/(A2) is linear in
C) and the dephasing Lindblad limit of the homodyne protocol (Eq. (A4) unravels it).  The
expected means come from the oracle's side (propagator and closed forms written there); the
ensembles are thousands of GPU trajectories in one batch.

Criterion.  Per independent entry of the mean C (upper triangle i <= j, real and imaginary parts;
C is Hermitian) z = |mean - exact| / SE.  The 3-standard-error bar is applied per entry the way it
holds for a correct ensemble: the number of entries beyond 3 SE may not exceed the 0.999 quantile
of the binomial count with p = 0.0027 (what chance gives), and no entry may lie beyond 4.5 SE (the
largest of a few hundred comparisons of a correct ensemble exceeds 4.5 SE with probability below
0.2 %, whereas a single 3 SE bound on the largest of them would fail most correct runs)."""

import numpy as np
import pytest

from oracle import Lattice
from gpu_common import make_sim
from test_oracle_statistics import pm_mean_map, lindblad, ct_mean_map

pytestmark = pytest.mark.gpu

PM, QSD = 0, 1


def _gpu_ensemble(L, protocol, gamma, dt, n_steps, n_traj, seed):
    sim = make_sim(1, L, n_traj=n_traj, uids=list(range(n_traj)))
    sim.step(protocol, [gamma] * n_traj, dt, seed, n_steps)
    U, _ = sim.get_state()
    sim.close()
    Cs = U @ np.conj(U.transpose(0, 2, 1))
    se = (Cs.real.std(axis=0, ddof=1) + 1j * Cs.imag.std(axis=0, ddof=1)) / np.sqrt(n_traj)
    return Cs.mean(axis=0), se


def _check(mean, se, ref, label):
    from scipy.stats import binom
    upper = np.triu(np.ones(mean.shape, dtype=bool))
    zs = []
    for part in (np.real, np.imag):
        d, e = np.abs(part(mean) - part(ref))[upper], part(se)[upper]
        ok = e > 1e-10                 # entries that vanish by symmetry in every trajectory
        assert d[~ok].max(initial=0.0) < 1e-10
        zs.append(d[ok] / e[ok])
    z = np.concatenate(zs)
    allowed = int(binom.ppf(0.999, z.size, 0.0027))
    n3 = int((z > 3).sum())
    print(f"  {label}: max z = {z.max():.2f}, beyond 3 SE: {n3} of {z.size} (chance allows {allowed})",
          flush=True)
    assert z.max() < 4.5
    assert n3 <= allowed


def test_projective_mean_map_on_gpu():
    """Ring L=16, gamma=4 (q = 0.2 per site and step), 40 steps, 4096 trajectories."""
    L, gamma, dt, n = 16, 4.0, 0.05, 40
    mean, se = _gpu_ensemble(L, PM, gamma, dt, n, 4096, seed=9)
    ref = pm_mean_map(Lattice(1, L), gamma, dt, n)
    _check(mean, se, ref, "projective mean map")


def test_homodyne_dephasing_limit_on_gpu():
    """Ring L=8, gamma=1, dt=0.01, 60 steps, 1000 trajectories (the O(gamma dt) bias of the
    split step stays below the statistical error at this count)."""
    L, gamma, dt, n = 8, 1.0, 0.01, 60
    mean, se = _gpu_ensemble(L, QSD, gamma, dt, n, 1000, seed=13)
    ref = lindblad(Lattice(1, L), gamma, n * dt)
    _check(mean, se, ref, "homodyne dephasing limit")


def test_continuous_time_mean_map_on_gpu():
    """Ring L=16, N=8, continuous-time projective protocol, gamma = 0.5 (total rate 4), 6 events
    per trajectory, 4096 trajectories: the mean C against the exact mean map of the waiting-time
    average and the outcome-averaged single-site projection."""
    L, gamma, n_ev, n_traj = 16, 0.5, 6, 4096
    sim = make_sim(1, L, n_traj=n_traj, uids=list(range(n_traj)))
    sim.ct_events([gamma] * n_traj, 21, n_ev)
    U, _ = sim.get_state()
    sim.close()
    Cs = U @ np.conj(U.transpose(0, 2, 1))
    se = (Cs.real.std(axis=0, ddof=1) + 1j * Cs.imag.std(axis=0, ddof=1)) / np.sqrt(n_traj)
    _check(Cs.mean(axis=0), se, ct_mean_map(Lattice(1, L), gamma, L // 2, n_ev),
           "continuous-time mean map")
