"""GPU library vs CPU oracle, element by element on the same seeded inputs.

Tolerances (FP64 path): |dS| <= 1e-9 per trajectory, C = U U^+ to 1e-10,
invariants (U^+ U = 1, C^2 = C, Tr C = N) to 1e-10, Born probabilities to 1e-12,
projective outcomes identical (integer decisions taken in FP64 on both sides).
"""

import re

import numpy as np
import pytest

import oracle
from gpu_common import make_sim, OracleBatch, corr

pytestmark = pytest.mark.gpu

PM, QSD = 0, 1


@pytest.mark.parametrize("dim,Lx,Ly", [(1, 64, 1), (1, 100, 1), (2, 8, 6)])
def test_free_evolution(dim, Lx, Ly):
    sim = make_sim(dim, Lx, Ly, n_traj=3)
    ob = OracleBatch(dim, Lx, Ly, 0.05, [0, 1, 2])
    for _ in range(40):
        sim.step(QSD, 0.0, 0.05, 0)
        ob.step(QSD, [0.0] * 3, 0)
    U, n = sim.get_state()
    assert n == 40
    for t in range(3):
        assert np.abs(corr(U[t]) - corr(ob.U[t])).max() < 1e-12
        assert np.abs(np.conj(U[t].T) @ U[t] - np.eye(sim.N)).max() < 1e-12
    sim.close()


def test_homodyne_parity_every_step():
    L, B = 64, 16
    gam = np.linspace(0.1, 2.0, B)
    sim = make_sim(1, L, n_traj=B, uids=range(100, 100 + B))
    ob = OracleBatch(1, L, 1, 0.05, range(100, 100 + B))
    A = list(range(32))
    for n in range(1, 21):
        sim.step(QSD, gam, 0.05, 7)
        ob.step(QSD, gam, 7)
        S = sim.entropy(A)
        assert np.abs(S - ob.entropy(A)).max() <= 1e-9, n
        p = sim.occupations()
        for t in range(B):
            assert np.abs(p[t] - np.diag(corr(ob.U[t])).real).max() < 1e-12
    U, _ = sim.get_state()
    for t in range(B):
        C = corr(U[t])
        assert np.abs(C - corr(ob.U[t])).max() < 1e-10
        assert np.abs(C @ C - C).max() < 1e-10
        assert abs(np.trace(C).real - L // 2) < 1e-10
    sim.close()


def test_projective_small_ring_full_run():
    """1d ring L=64, N=32, projective gamma=0.5, dt=0.05, 400 steps, 16 trajectories, seed 0,
    S of A = [0, 32) every 10 steps: outcomes identical, |dS| <= 1e-9 at every sample."""
    from paper_2508_18468_amd.workloads import ring_pm_small
    w = ring_pm_small()
    B = w.n_traj
    uids = w.uids(0)
    gam = [w.gammas[0]] * B
    sim = make_sim(1, w.Lx, n_traj=B, uids=uids)
    ob = OracleBatch(1, w.Lx, 1, w.dt, uids)
    A = w.regions[0]
    assert np.abs(sim.entropy(A)).max() == 0.0
    n_events = 0
    for n in range(1, w.n_steps + 1):
        sim.step(PM, gam, w.dt, w.seed)
        ev_ref = ob.step(PM, gam, w.seed)
        ev_gpu = sim.pm_events()
        for t in range(B):
            assert [(e[0], e[2]) for e in ev_gpu[t]] == [(e[0], e[2]) for e in ev_ref[t]], (n, t)
            for a, b in zip(ev_gpu[t], ev_ref[t]):
                assert abs(a[1] - b[1]) < 1e-12
            n_events += len(ev_ref[t])
        if n % w.obs_every == 0:
            assert np.abs(sim.entropy(A) - ob.entropy(A)).max() <= 1e-9, n
    assert n_events > 5000
    sim.close()


@pytest.mark.parametrize("protocol,gamma", [(PM, 3.0), (QSD, 1.3)])
def test_ragged_sizes_and_regions(protocol, gamma):
    """L=200, N=100: partial Cholesky block (64 + 36), GEMM tiles with ragged tails,
    regions smaller and larger than N, non-contiguous, single-site, empty and full."""
    L, B = 200, 3
    sim = make_sim(1, L, n_traj=B, uids=[5, 9, 11])
    ob = OracleBatch(1, L, 1, 0.05, [5, 9, 11])
    gam = [gamma] * B
    for n in range(12):
        sim.step(protocol, gam, 0.05, 3)
        ob.step(protocol, gam, 3)
    rng = np.random.default_rng(0)
    regions = [list(range(100)), list(range(37)), sorted(rng.choice(L, 57, replace=False).tolist()),
               list(range(150)), sorted(rng.choice(L, 171, replace=False).tolist()), [77], [], list(range(L))]
    for r in regions:
        assert np.abs(sim.entropy(r) - ob.entropy(r)).max() <= 1e-9, len(r)
    U, _ = sim.get_state()
    for t in range(B):
        assert np.abs(corr(U[t]) - corr(ob.U[t])).max() < 1e-10
        assert np.abs(np.conj(U[t].T) @ U[t] - np.eye(100)).max() < 1e-12
    sim.close()


@pytest.mark.parametrize("protocol,gamma", [(PM, 4.0), (QSD, 2.0)])
def test_torus_parity_and_mutual_information(protocol, gamma):
    Lx, Ly, B = 8, 6, 4
    sim = make_sim(2, Lx, Ly, n_traj=B, uids=range(B))
    ob = OracleBatch(2, Lx, Ly, 0.05, range(B))
    gam = [gamma] * B
    A = sorted(x + Lx * y for y in range(Ly) for x in range(0, 2))
    Bq = sorted(x + Lx * y for y in range(Ly) for x in range(4, 6))
    for n in range(15):
        sim.step(protocol, gam, 0.05, 1)
        ob.step(protocol, gam, 1)
    I = sim.mutual_info(A, Bq)
    for t in range(B):
        ref = oracle.mutual_information(ob.U[t], A, Bq)
        assert abs(I[t] - ref) <= 3e-9
    sim.close()


def test_spectrum_parity():
    L, B = 96, 2
    sim = make_sim(1, L, n_traj=B, uids=[3, 4])
    ob = OracleBatch(1, L, 1, 0.05, [3, 4])
    for _ in range(30):
        sim.step(QSD, [0.3, 1.5], 0.05, 2)
        ob.step(QSD, [0.3, 1.5], 2)
    for r in (list(range(48)), list(range(20, 90)), list(range(0, 96, 3))):
        lam = sim.region_spectrum(r)
        for t in range(B):
            ref = oracle.region_spectrum(ob.U[t], r)
            assert np.abs(np.sort(lam[t]) - np.sort(ref)[-lam.shape[1]:]).max() < 1e-12
    sim.close()


def test_step_chunking_and_batch_invariance():
    L = 128
    a = make_sim(1, L, n_traj=4, uids=[0, 1, 2, 3])
    b = make_sim(1, L, n_traj=4, uids=[0, 1, 2, 3])
    c = make_sim(1, L, n_traj=1, uids=[2])
    g = [0.5, 1.0, 1.5, 2.0]
    a.step(PM, g, 0.05, 9, 10)
    for _ in range(10):
        b.step(PM, g, 0.05, 9, 1)
        c.step(PM, [1.5], 0.05, 9, 1)
    Ua, na = a.get_state()
    Ub, nb = b.get_state()
    Uc, _ = c.get_state()
    assert na == nb == 10
    assert np.array_equal(Ua, Ub)
    assert np.array_equal(Ua[2], Uc[0])
    for s in (a, b, c):
        s.close()


def test_checkpoint_roundtrip():
    L = 64
    a = make_sim(1, L, n_traj=2, uids=[7, 8])
    a.step(QSD, [0.7, 0.7], 0.05, 4, 5)
    U, n = a.get_state()
    a.step(QSD, [0.7, 0.7], 0.05, 4, 5)
    S1 = a.entropy(list(range(32)))
    b = make_sim(1, L, n_traj=2, uids=[7, 8])
    b.set_state(U, n)
    b.step(QSD, [0.7, 0.7], 0.05, 4, 5)
    assert np.array_equal(S1, b.entropy(list(range(32))))
    a.close()
    b.close()


def test_checkpoint_of_reset_slots_resumes_exactly():
    """A slot refilled by mfq_reset_trajectory (new uid, own step count restarting) survives a
    checkpoint: state, step, uids and step bases restored in a fresh context continue exactly
    as the uninterrupted context, for both protocols, and the refilled slot draws as a fresh
    trajectory of its uid (against the oracle)."""
    L, dt, seed = 64, 0.05, 9
    for proto, gam in ((QSD, [0.6, 1.1, 0.4]), (PM, [0.8, 1.5, 0.5])):
        a = make_sim(1, L, n_traj=3, uids=[3, 4, 5])
        a.step(proto, gam, dt, seed, 5)
        a.reset_trajectory(1, 77)
        a.step(proto, gam, dt, seed, 4)
        U, n = a.get_state()
        uid, base = a.get_slots()
        assert list(uid) == [3, 77, 5] and list(base) == [0, 5, 0]
        b = make_sim(1, L, n_traj=3, uids=[3, 4, 5])
        b.set_state(U, n)
        b.set_slots(uid, base)
        a.step(proto, gam, dt, seed, 6)
        b.step(proto, gam, dt, seed, 6)
        Ua, _ = a.get_state()
        Ub, _ = b.get_state()
        assert np.array_equal(Ua, Ub)
        # the refilled slot is a fresh trajectory of uid 77 after 10 of its own steps
        ob = OracleBatch(1, L, 1, dt, [77])
        for _ in range(10):
            ob.step(proto, [gam[1]], seed)
        assert np.abs(corr(Ub[1]) - corr(ob.U[0])).max() <= 1e-10
        with pytest.raises(Exception):
            b.set_slots(uid, [0, n + 100, 0])
        a.close()
        b.close()


def test_all_site_projection_gives_zero_entropy():
    L = 32
    sim = make_sim(1, L, n_traj=2, uids=[0, 1])
    for n in range(4):
        sim.step(PM, [25.0, 25.0], 0.05, 0)
        ev = sim.pm_events()
        for t in range(2):
            assert [e[0] for e in ev[t]] == list(range(L))
            assert sum(e[2] for e in ev[t]) == L // 2
        for r in (list(range(16)), [1, 4, 5, 30]):
            assert np.abs(sim.entropy(r)).max() < 1e-10
    sim.close()


def test_errors_are_reported():
    from paper_2508_18468_amd import mfq
    sim = make_sim(1, 16, n_traj=1)
    with pytest.raises(mfq.MfqError) as e:
        sim.entropy([3, 2])
    assert e.value.code == -1
    with pytest.raises(mfq.MfqError):
        sim.entropy([0, 16])
    with pytest.raises(mfq.MfqError):
        sim.step(PM, [-1.0], 0.05, 0)
    with pytest.raises(mfq.MfqError):
        sim.mutual_info([0, 1], [1, 2])
    sim.close()


def test_cholesky_breakdown_is_located():
    """A state with an exactly zero column (trajectory 1, column 5) gives an exactly zero pivot
    in the first Cholesky-QR pass (gamma = 0 keeps the column zero through the propagator and
    the homodyne factor); the error names the pass, trajectory, column and pivot, and the flag
    is cleared after it is reported."""
    from paper_2508_18468_amd import mfq
    sim = make_sim(1, 32, n_traj=3)
    U, st = sim.get_state()
    U[1, :, 5] = 0.0
    sim.set_state(U, st)
    sim.step(QSD, [0.0, 0.0, 0.0], 0.05, 0, 1)
    with pytest.raises(mfq.MfqError) as e:
        sim.get_state()
    assert e.value.code == -4
    msg = str(e.value)
    assert re.search(r"pass 1, trajectory 1, column 5, pivot -?0$", msg), msg
    sim.get_state()  # cleared
    sim.close()


def test_batched_homodyne_ring_full_size_sampled():
    """1d ring L=1024, N=512, homodyne gamma in {0.1, 0.3, 1.0} x 128 trajectories in one batch
    (the benchmark's launch configuration: steps in captured step-pair graphs), the first 20
    steps; three sampled trajectories (one per rate) checked against the oracle: |dS| <= 1e-9
    after steps 1, 2, 5, 10, 15 and 20, C to 1e-10 after step 20, Born probabilities to 1e-12."""
    from paper_2508_18468_amd.workloads import ring_qsd_batched
    w = ring_qsd_batched()
    uids = w.uids(0) + w.uids(1) + w.uids(2)
    gam = np.repeat(w.gammas, w.n_traj)
    sim = make_sim(1, w.Lx, n_traj=len(uids), uids=uids)
    sample = [5, 128 + 77, 256 + 127]
    ob = OracleBatch(1, w.Lx, 1, w.dt, uids)
    done = 0
    for target in (1, 2, 5, 10, 15, 20):
        sim.step(QSD, gam, w.dt, w.seed, target - done)
        for _ in range(target - done):
            ob.step(QSD, gam, w.seed, idx=sample)
        done = target
        S = sim.entropy(w.regions[0])
        ref = ob.entropy(w.regions[0], idx=sample)
        for t in sample:
            assert abs(S[t] - ref[t]) <= 1e-9, (target, t, S[t], ref[t])
    U, _ = sim.get_state()
    p = sim.occupations()
    for t in sample:
        assert np.abs(corr(U[t]) - corr(ob.U[t])).max() < 1e-10
        assert np.abs(p[t] - oracle.born_probabilities(ob.U[t])).max() <= 1e-12
    sim.close()


def test_strong_homodyne_uses_full_second_pass():
    """gamma*dt = 2: factors up to e^{+-6} make U far from orthonormal before the first
    Cholesky-QR pass, so the second pass fails the near-identity test and runs the full
    factorisation on the device; results still match the oracle's Householder QR."""
    L, B = 64, 4
    sim = make_sim(1, L, n_traj=B, uids=range(B))
    ob = OracleBatch(1, L, 1, 0.05, range(B))
    for n in range(6):
        sim.step(QSD, [40.0] * B, 0.05, 8)
        ob.step(QSD, [40.0] * B, 8)
    S = sim.entropy(list(range(32)))
    assert np.abs(S - ob.entropy(list(range(32)))).max() <= 1e-8
    U, _ = sim.get_state()
    for t in range(B):
        assert np.abs(np.conj(U[t].T) @ U[t] - np.eye(32)).max() < 1e-12
        assert np.abs(corr(U[t]) - corr(ob.U[t])).max() < 1e-9
    sim.close()


def test_orthonormality_after_certified_second_pass():
    """The second Cholesky-QR pass keeps U when its Gram certifies |U^+ U - I| <= 1e-13 entrywise
    (and applies the first-order or full factor otherwise): after homodyne and projective steps
    at weak and strong monitoring every trajectory is orthonormal to that accuracy (host check
    adds its own rounding, about L eps)."""
    L, B = 256, 4
    gam = [0.05, 0.5, 2.0, 6.0]
    sim = make_sim(1, L, n_traj=B)
    for protocol in (QSD, PM, QSD):
        sim.step(protocol, gam, 0.05, 3, 7)
        U, _ = sim.get_state()
        for t in range(B):
            dev = np.abs(U[t].conj().T @ U[t] - np.eye(L // 2)).max()
            assert dev <= 1e-13 + 4 * L * 2.2e-16, (protocol, t, dev)
    sim.close()


@pytest.mark.parametrize("dim,Lx,Ly", [(1, 260, 1), (1, 400, 1), (1, 600, 1), (2, 20, 20),
                                       (1, 1100, 1)])
def test_cholqr_split_sizes(dim, Lx, Ly):
    """Particle numbers N = 130, 200, 300, 200, 550 split the first Cholesky-QR pass's product at
    128, 128, 256, 128 and 512 columns, leaving right blocks of 2, 72, 44, 72 and 38 columns (the
    72-wide inverse assembled from a narrower last pair one level down); at N = 550 the Cholesky
    runs in two outer panels (512 rows, the rank-512 update of the last 38, a 38-row panel):
    strong homodyne steps, where the first pass does real work, against the oracle's
    Householder QR."""
    B = 2
    sim = make_sim(dim, Lx, Ly, n_traj=B, uids=[7, 8])
    ob = OracleBatch(dim, Lx, Ly, 0.05, [7, 8])
    gam = [2.0, 6.0]
    for n in range(5):
        sim.step(QSD, gam, 0.05, 21)
        ob.step(QSD, gam, 21)
    U, _ = sim.get_state()
    N = U.shape[2]
    for t in range(B):
        assert np.abs(U[t].conj().T @ U[t] - np.eye(N)).max() < 1e-12
        assert np.abs(corr(U[t]) - corr(ob.U[t])).max() < 1e-10
    sim.close()
