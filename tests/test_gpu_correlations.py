"""C(r) of Eq. (2) and G_AB of Eq. (5) on the GPU (reduction epilogues of the C = U U^+
products) against the oracle on the same trajectories, and at full size through identities
that hold at any size: the sum rule sum_r n_r C(r) = -(N - sum_i p_i^2) (C^2 = C) and
G_{A, complement} = sum over the spectrum of C_A of l (1 - l).

Tolerance: C(r) and G_AB are sums of |C_ij|^2 with |C_ij| <= 1 accumulated in FP64 from
products of K = N terms; 1e-12 absolute per entry for the parity cases (each |C_ij|^2 carries
a few N eps of error and the averages divide by the pair count), 1e-9 relative for the full-size
identities.
"""

import numpy as np
import pytest

import oracle
from gpu_common import OracleBatch, make_sim

pytestmark = pytest.mark.gpu

PM, QSD = 0, 1


@pytest.mark.parametrize("L,protocol,gamma,tile", [(64, PM, 1.0, 0), (200, QSD, 0.8, 0),
                                                    (512, PM, 0.5, 0), (320, QSD, 1.5, 1),
                                                    (384, PM, 2.0, 2)])
def test_density_correlation_matches_oracle(L, protocol, gamma, tile):
    """Rings of 64 .. 512 sites (ragged 200 and 320 for the tile edges), three trajectories,
    12 steps; default, 64x64 and 128x128 tiles."""
    from paper_2508_18468_amd import mfq
    dt, seed, uids = 0.05, 4, [2, 5, 9]
    gams = [gamma, 0.5 * gamma, 2.0 * gamma]
    sim = make_sim(1, L, n_traj=3, uids=uids)
    if tile:
        mfq.mfq_set_tuning(sim.ctx, mfq.PATH_LAUNCHES, tile)
    ob = OracleBatch(1, L, 1, dt, uids)
    for n in range(12):
        sim.step(protocol, gams, dt, seed)
        ob.step(protocol, gams, seed)
    Cr = sim.density_correlation()
    A = list(range(0, L // 4))
    B = list(range(L // 2, L // 2 + L // 8)) + [L - 1]
    G = sim.particle_covariance(A, B)
    for t in range(3):
        ref = oracle.density_correlation(ob.U[t])
        assert np.abs(Cr[t] - ref).max() <= 1e-12, (t, np.abs(Cr[t] - ref).max())
        assert abs(G[t] - oracle.particle_covariance(ob.U[t], A, B)) <= 1e-12
    sim.close()


def test_particle_covariance_torus_matches_oracle():
    """2d 12 x 8 torus, homodyne: G between the strips x in [0, 3) and [6, 9) (all y)."""
    Lx, Ly, dt, seed, uids = 12, 8, 0.05, 7, [0, 1]
    sim = make_sim(2, Lx, Ly, n_traj=2, uids=uids)
    ob = OracleBatch(2, Lx, Ly, dt, uids)
    for n in range(10):
        sim.step(QSD, [1.0, 3.0], dt, seed)
        ob.step(QSD, [1.0, 3.0], seed)
    A = sorted(x + Lx * y for y in range(Ly) for x in range(0, 3))
    B = sorted(x + Lx * y for y in range(Ly) for x in range(6, 9))
    G = sim.particle_covariance(A, B)
    for t in range(2):
        assert abs(G[t] - oracle.particle_covariance(ob.U[t], A, B)) <= 1e-12
    with pytest.raises(Exception):
        sim.particle_covariance(A, A[:3])  # overlapping regions are rejected
    with pytest.raises(Exception):
        sim.density_correlation()          # C(r) is defined on rings only
    sim.close()


def test_long_ring_identities_full_size():
    """1d ring L=16384, N=8192, two projective steps (gamma 0.2, 1.0): the sum rule of C(r)
    and the number variance of a half chain against its spectrum."""
    import time
    L = 16384
    sim = make_sim(1, L, n_traj=2)
    sim.step(PM, [0.2, 1.0], 0.05, 0, 2)
    t0 = time.perf_counter()
    Cr = sim.density_correlation()
    t1 = time.perf_counter()
    print(f"  C(r) at L=16384, 2 trajectories: {1e3 * (t1 - t0):.0f} ms", flush=True)
    p = sim.occupations()
    n_r = np.array([2 * L] * (L // 2 - 1) + [L], dtype=float)
    for t in range(2):
        want = -(L // 2 - (p[t] ** 2).sum())
        got = float((n_r * Cr[t]).sum())
        assert abs(got - want) <= 1e-9 * abs(want), (t, got, want)
        assert (Cr[t] <= 1e-15).all()
    A = list(range(L // 2))
    comp = list(range(L // 2, L))
    t0 = time.perf_counter()
    G = sim.particle_covariance(A, comp)
    print(f"  G_AB at L=16384 (8192 x 8192 sites): {1e3 * (time.perf_counter() - t0):.0f} ms", flush=True)
    lam = sim.region_spectrum(A)
    for t in range(2):
        want = float((lam[t] * (1.0 - lam[t])).sum())
        assert abs(G[t] - want) <= 1e-9 * want, (t, G[t], want)
    sim.close()


def test_correlation_buffer_survives_fused_runs():
    """Regression: growing the fused path's observation buffer must leave the correlation
    buffer of the same context alone.  C(r) before and after fused runs with observations,
    against the oracle on the same trajectories."""
    from paper_2508_18468_amd import mfq
    L, dt, seed, uids, gams = 64, 0.05, 5, [1, 2], [0.5, 1.5]
    sim = make_sim(1, L, n_traj=2, uids=uids)
    ob = OracleBatch(1, L, 1, dt, uids)
    sim.density_correlation()                    # allocates the correlation buffer
    sim.set_path(mfq.PATH_FUSED)
    region = list(range(L // 2))
    for n_steps, every in ((4, 2), (12, 1)):     # the second run needs a larger buffer
        sim.run(QSD, gams, dt, seed, n_steps, obs_every=every, region=region)
        for _ in range(n_steps):
            ob.step(QSD, gams, seed)
    Cr = sim.density_correlation()
    G = sim.particle_covariance(list(range(8)), list(range(32, 40)))
    for t in range(2):
        assert np.abs(Cr[t] - oracle.density_correlation(ob.U[t])).max() <= 1e-12
        assert abs(G[t] - oracle.particle_covariance(ob.U[t], list(range(8)), list(range(32, 40)))) <= 1e-12
    sim.close()
