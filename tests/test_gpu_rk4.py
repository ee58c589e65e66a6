"""Homodyne steps integrated by RK4 on the GPU (mfq_set_integrator(MFQ_INTEGRATOR_RK4))
against the oracle's RK4 step (Appendix A, Eq. (A4) with its exponent frozen over the step).

Tolerance.  The oracle forms the four RK4 stages with dense L x L products and re-orthonormalises
by Householder QR; the GPU evaluates the same polynomial in Horner form with a nearest-neighbour
stencil and Cholesky-QR2.  Both round each entry of a step to a few eps (|A| <= 4 J dt + |dW| +
gamma dt < 1 here), so after n steps the correlation matrices differ by a few n eps: C to 1e-11,
S to 1e-9.  The RK4 and split-step states differ by O(dt^2) per step (the diagonal is taken
before rather than after the free evolution), far above that bar, so the tests also show that the
integrator switch takes effect.
"""

import numpy as np
import pytest

import oracle
from oracle.rk4 import run_rk4
from gpu_common import make_sim, corr

pytestmark = pytest.mark.gpu

HOMODYNE = 1


def _oracle_states(dim, Lx, Ly, uids, gammas, dt, seed, n_steps):
    lat = oracle.Lattice(dim, Lx, Ly if dim == 2 else 1)
    U0 = oracle.initial_state(lat.L, oracle.default_occupied(lat))
    return [run_rk4(lat, U0, g, dt, seed, u, n_steps) for u, g in zip(uids, gammas)]


@pytest.mark.parametrize("dim,Lx,Ly,gammas,dt,n_steps", [
    (1, 64, 1, [0.1, 1.0, 3.0], 0.05, 20),
    (1, 200, 1, [0.5, 2.0], 0.05, 15),      # ragged row tiles
    (1, 96, 1, [1.0], 0.1, 12),             # the paper's largest step
    (2, 8, 6, [0.5, 1.5], 0.05, 15),
    (2, 12, 2, [1.0], 0.05, 10),            # Ly = 2: the two y neighbours coincide
])
def test_rk4_matches_oracle(dim, Lx, Ly, gammas, dt, n_steps):
    from paper_2508_18468_amd import mfq
    B, seed = len(gammas), 13
    uids = [2 + 3 * b for b in range(B)]
    sim = make_sim(dim, Lx, Ly, n_traj=B, uids=uids)
    sim.set_integrator(mfq.INTEGRATOR_RK4)
    for n in range(n_steps):
        sim.step(HOMODYNE, gammas, dt, seed)
    want = _oracle_states(dim, Lx, Ly, uids, gammas, dt, seed, n_steps)
    U, _ = sim.get_state()
    L = sim.L
    region = list(range(L // 2)) if dim == 1 else sorted(x + Lx * y for y in range(Ly)
                                                          for x in range(Lx // 2))
    S = sim.entropy(region)
    for b in range(B):
        assert np.abs(corr(U[b]) - corr(want[b])).max() <= 1e-11
        assert np.abs(U[b].conj().T @ U[b] - np.eye(sim.N)).max() <= 1e-12
        assert abs(S[b] - oracle.entanglement_entropy(want[b], region)) <= 1e-9
    # the split step gives a visibly different state from the same draws
    split = make_sim(dim, Lx, Ly, n_traj=B, uids=uids)
    for n in range(n_steps):
        split.step(HOMODYNE, gammas, dt, seed)
    Us, _ = split.get_state()
    assert max(np.abs(corr(Us[b]) - corr(U[b])).max() for b in range(B)) > 1e-6
    sim.close()
    split.close()


def test_rk4_graph_replay_run_path_and_switching():
    from paper_2508_18468_amd import mfq
    gam = [0.4, 1.2]
    a = make_sim(1, 64, n_traj=2)
    b = make_sim(1, 64, n_traj=2)
    for s in (a, b):
        s.set_integrator(mfq.INTEGRATOR_RK4)
    a.step(HOMODYNE, gam, 0.05, 3, 9)            # graph replay of step pairs
    for _ in range(9):
        b.step(HOMODYNE, gam, 0.05, 3, 1)
    Ua, _ = a.get_state()
    Ub, _ = b.get_state()
    assert np.array_equal(Ua, Ub)
    # mfq_run under RK4 takes the per-phase kernels (AUTO) and refuses the fused path
    c = make_sim(1, 64, n_traj=2)
    c.set_integrator(mfq.INTEGRATOR_RK4)
    S_run = c.run(HOMODYNE, gam, 0.05, 3, 9, obs_every=9, region=list(range(32)))
    Uc, _ = c.get_state()
    assert np.array_equal(Uc, Ua)
    assert np.allclose(S_run[-1], a.entropy(list(range(32))), atol=0.0, rtol=0.0)
    c.set_path(mfq.PATH_FUSED)
    with pytest.raises(Exception):
        c.run(HOMODYNE, gam, 0.05, 3, 2, obs_every=0)
    # back to the split step: identical to a context that never used RK4
    a.set_integrator(mfq.INTEGRATOR_SPLIT)
    d = make_sim(1, 64, n_traj=2)
    U9, st = a.get_state()
    d.set_state(U9, st)
    a.step(HOMODYNE, gam, 0.05, 3, 4)
    d.step(HOMODYNE, gam, 0.05, 3, 4)
    assert np.array_equal(a.get_state()[0], d.get_state()[0])
    with pytest.raises(Exception):
        a.set_integrator(7)
    for s in (a, b, c, d):
        s.close()


def test_rk4_full_size_batch():
    """The 384-trajectory ring L = 1024 workload under RK4: 6 steps, two sampled trajectories
    against the oracle; orthonormality of every 16th trajectory."""
    from paper_2508_18468_amd import mfq
    from paper_2508_18468_amd.workloads import ring_qsd_batched
    w = ring_qsd_batched()
    uids = w.uids(0) + w.uids(1) + w.uids(2)
    gam = np.repeat(np.asarray(w.gammas), w.n_traj)
    sim = mfq.Trajectories(1, w.Lx, n_traj=len(uids), uids=uids, device=0)
    sim.set_integrator(mfq.INTEGRATOR_RK4)
    sim.step(HOMODYNE, gam, w.dt, w.seed, 6)
    U, _ = sim.get_state()
    for t in (5, 300):
        want = _oracle_states(1, w.Lx, 1, [uids[t]], [gam[t]], w.dt, w.seed, 6)[0]
        assert np.abs(corr(U[t]) - corr(want)).max() <= 1e-11
    for t in range(0, len(uids), 16):
        assert np.abs(U[t].conj().T @ U[t] - np.eye(w.N)).max() <= 1e-12
    sim.close()
