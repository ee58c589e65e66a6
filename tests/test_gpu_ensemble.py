"""Long-time ensemble means of the GPU trajectories against what the physics fixes exactly:
the projective protocol's mean map (the outcome-averaged update of Eq. (A1)/(A2) is linear in
C) and the dephasing Lindblad limit of the homodyne protocol (Eq. (A4) unravels it).  The
expected means come from the oracle's side (propagator and closed forms written there); the
ensembles are thousands of GPU trajectories in one batch.  Criterion: every entry of the mean C
within 4.5 standard errors (about 3 SE per entry over the L^2 entries of each matrix)."""

import numpy as np
import pytest

from oracle import Lattice
from gpu_common import make_sim
from test_oracle_statistics import pm_mean_map, lindblad, _z

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


def test_projective_mean_map_on_gpu():
    """Ring L=16, gamma=4 (q = 0.2 per site and step), 40 steps, 4096 trajectories."""
    L, gamma, dt, n = 16, 4.0, 0.05, 40
    mean, se = _gpu_ensemble(L, PM, gamma, dt, n, 4096, seed=9)
    ref = pm_mean_map(Lattice(1, L), gamma, dt, n)
    z = _z(mean, se, ref)
    print(f"  projective mean map: max z = {z:.2f}", flush=True)
    assert z < 4.5


def test_homodyne_dephasing_limit_on_gpu():
    """Ring L=8, gamma=1, dt=0.01, 60 steps, 1000 trajectories (the O(gamma dt) bias of the
    split step stays below the statistical error at this count)."""
    L, gamma, dt, n = 8, 1.0, 0.01, 60
    mean, se = _gpu_ensemble(L, QSD, gamma, dt, n, 1000, seed=13)
    ref = lindblad(Lattice(1, L), gamma, n * dt)
    z = _z(mean, se, ref)
    print(f"  homodyne dephasing limit: max z = {z:.2f}", flush=True)
    assert z < 4.5
