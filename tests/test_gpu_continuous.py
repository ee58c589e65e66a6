"""Continuous-time projective protocol on the GPU (mfq_ct_events) against the oracle's
event-by-event D-form run (Appendix A, PM protocol) on the same draws.

Each event is compared as it happens: the measured site and the outcome exactly (integer
decisions), the Born probability and the waiting time to rounding; the state through
C = U U^+ and the entanglement entropy.

Tolerance.  The GPU applies P(tau) as a stencil of 2w + 1 taps, a reflector from a sum over N
columns and a rank-1 update; the oracle an L x L conjugation, a dense Eq. (A1)/(A2) update
and an eigendecomposition.  Both are backward stable, so an event adds a few L eps to the
difference of the two correlation matrices and E events at most E L eps: 2e-11 for the
E <= 60 events on L <= 224 sites used here (|C_ij| <= 1).  p_j carries the same error;
tau = -ln(eta)/(gamma N) agrees to a few ulp.  S is compared to 1e-9.
"""

import numpy as np
import pytest

import oracle
from oracle.continuous import run_continuous
from gpu_common import make_sim, corr

pytestmark = pytest.mark.gpu


class OracleCT:
    """The same trajectories advanced event by event by the oracle."""

    def __init__(self, dim, Lx, Ly, uids, gammas, seed):
        self.lat = oracle.Lattice(dim, Lx, Ly if dim == 2 else 1)
        occ = oracle.default_occupied(self.lat)
        self.U = [oracle.initial_state(self.lat.L, occ) for _ in uids]
        self.t = [0.0 for _ in uids]
        self.uids, self.gammas, self.seed = list(uids), list(gammas), seed
        self.n = 0

    def slot(self, t_end=np.inf):
        """One event slot (index n + 1); returns the records (None where no event)."""
        self.n += 1
        recs = []
        for b, uid in enumerate(self.uids):
            out = run_continuous(self.lat, self.U[b], self.gammas[b], self.seed, uid, 1, t_end,
                                 first_event=self.n, t0=self.t[b])
            self.U[b], self.t[b] = out["U"], out["t"]
            recs.append(out["records"].get(self.n))
        return recs


def _check_slot(sim, orc, recs, tol_p=2e-11):
    site, outc, prob, tau = sim.ct_last_events()
    for b, r in enumerate(recs):
        if r is None:
            assert site[b] == -1 and outc[b] == -1
            continue
        t_o, j_o, p_o, o_o = r
        assert site[b] == j_o and outc[b] == o_o, (b, site[b], j_o, outc[b], o_o, prob[b], p_o)
        assert abs(prob[b] - p_o) <= tol_p
        assert abs(tau[b] - t_o) <= 1e-14 * t_o


def _check_state(sim, orc, tol=2e-11):
    U, _ = sim.get_state()
    for b in range(len(orc.uids)):
        assert np.abs(corr(U[b]) - corr(orc.U[b])).max() <= tol
        N = U[b].shape[1]
        assert np.abs(U[b].conj().T @ U[b] - np.eye(N)).max() <= 1e-12
    t = sim.times()
    assert np.allclose(t, orc.t, rtol=1e-13, atol=0.0)


@pytest.mark.parametrize("dim,Lx,Ly,gammas,n_events,reorth", [
    (1, 64, 1, [0.3, 1.0, 2.5], 60, 0),      # Bessel band
    (1, 16, 1, [0.05, 0.2, 1.0], 50, 0),     # band wider than the ring: plane-wave row
    (1, 200, 1, [0.7, 4.0], 30, 8),          # ragged row tiles, Cholesky-QR every 8 slots
    (1, 200, 1, [0.001, 0.7], 12, 0),        # bands wider than the LDS ring kernel takes
    (2, 8, 6, [0.5, 1.5], 40, 0),            # torus, full rows in both directions
    (2, 56, 4, [3.0, 10.0], 40, 5),          # torus, band along x (mostly), full along y
])
def test_events_match_oracle(dim, Lx, Ly, gammas, n_events, reorth):
    B, seed = len(gammas), 21
    uids = [3 + 5 * b for b in range(B)]
    sim = make_sim(dim, Lx, Ly, n_traj=B, uids=uids)
    orc = OracleCT(dim, Lx, Ly, uids, gammas, seed)
    outcomes = set()
    for e in range(n_events):
        sim.ct_events(gammas, seed, 1, reorth_every=reorth)
        recs = orc.slot()
        _check_slot(sim, orc, recs)
        outcomes.update(r[3] for r in recs)
    assert outcomes == {0, 1}
    _check_state(sim, orc)
    L = sim.L
    region = list(range(L // 2)) if dim == 1 else sorted(x + Lx * y for y in range(Ly)
                                                          for x in range(Lx // 2))
    S = sim.entropy(region)
    for b in range(B):
        assert abs(S[b] - oracle.entanglement_entropy(orc.U[b], region)) <= 1e-9
    sim.close()


def test_end_time_chunking_and_shared_step_counter():
    """Two projective steps, then event slots with an end time; one call of 40 slots equals 40
    calls of one slot bit for bit; the clocks stop past t_end and the records say so."""
    from paper_2508_18468_amd import mfq
    L, gammas, seed, uids, t_end = 32, [0.5, 2.0], 4, [1, 2], 0.4
    sims = [make_sim(1, L, n_traj=2, uids=uids) for _ in range(2)]
    orc = OracleCT(1, L, 1, uids, gammas, seed)
    pre = oracle.Lattice(1, L)
    P = oracle.propagator(pre, 0.05)
    for n in (1, 2):
        for s in sims:
            s.step(mfq.PROJECTIVE, gammas, 0.05, seed)
        for b in range(2):
            orc.U[b], _ = oracle.step(orc.U[b], P, oracle.trajectory.PROJECTIVE, gammas[b], 0.05, seed,
                                      uids[b], n)
    orc.n = 2
    sims[0].ct_events(gammas, seed, 40, t_end=t_end)
    for e in range(40):
        sims[1].ct_events(gammas, seed, 1, t_end=t_end)
        recs = orc.slot(t_end)
    _check_slot(sims[1], orc, recs)
    Ua, _ = sims[0].get_state()
    Ub, _ = sims[1].get_state()
    assert np.array_equal(Ua, Ub)
    assert np.array_equal(sims[0].times(), sims[1].times())
    t = sims[1].times()
    assert (t >= t_end).all() and all(r is None for r in recs)
    _check_state(sims[1], orc)
    # a checkpoint of state and clocks continues identically
    U, step = sims[1].get_state()
    sims[0].set_state(U, step)
    sims[0].set_times(t - 0.3)
    orc.t = list(t - 0.3)
    sims[0].ct_events(gammas, seed, 3, t_end=t_end)
    for e in range(3):
        recs = orc.slot(t_end)
    _check_state(sims[0], orc)
    for s in sims:
        s.close()


def test_invalid_arguments():
    sim = make_sim(1, 16, n_traj=2)
    with pytest.raises(Exception):
        sim.ct_events([1.0, 0.0], 1, 1)
    with pytest.raises(Exception):
        sim.ct_events([1.0, 1.0], 1, 1, t_end=float("nan"))
    with pytest.raises(Exception):
        sim.ct_events([1.0, 1.0], 1, -1)
    with pytest.raises(Exception):
        sim.set_times([0.0, float("inf")])
    site, outc, _, _ = sim.ct_last_events()
    assert (site == -1).all() and (outc == -1).all()
    sim.close()


def test_full_size_ring():
    """Ring L = 1024, N = 512, 8 trajectories: the first 3 slots of trajectory 0 against the
    oracle, then 300 slots checked through properties that hold at any size: the measured
    site holds exactly the outcome afterwards, columns stay orthonormal, clocks add up."""
    L, B, seed = 1024, 8, 6
    gammas = list(np.linspace(0.2, 2.0, B))
    uids = list(range(100, 100 + B))
    sim = make_sim(1, L, n_traj=B, uids=uids)
    orc = OracleCT(1, L, 1, uids[:1], gammas[:1], seed)
    for e in range(3):
        sim.ct_events(gammas, seed, 1)
        recs = orc.slot()
        site, outc, prob, tau = sim.ct_last_events()
        t_o, j_o, p_o, o_o = recs[0]
        assert site[0] == j_o and outc[0] == o_o and abs(prob[0] - p_o) <= 1e-10
    U, _ = sim.get_state()
    assert np.abs(corr(U[0]) - corr(orc.U[0])).max() <= 1e-10
    clock = sim.times()
    for e in range(300):
        sim.ct_events(gammas, seed, 1, reorth_every=64)
        if e % 50 == 49:
            site, outc, prob, tau = sim.ct_last_events()
            p = sim.occupations()
            assert ((prob >= -1e-12) & (prob <= 1 + 1e-12)).all()
            for b in range(B):
                assert abs(p[b, site[b]] - outc[b]) <= 1e-13
    t_end = sim.times()
    assert (t_end > clock).all()
    U, _ = sim.get_state()
    for b in range(B):
        assert np.abs(U[b].conj().T @ U[b] - np.eye(L // 2)).max() <= 1e-12
    sim.close()


@pytest.mark.parametrize("dim,Lx,Ly,gammas,n_slots,K,reorth,t_end", [
    (1, 64, 1, [0.3, 1.0, 2.5], 60, 1, 0, np.inf),
    (1, 64, 1, [0.3, 1.0, 2.5], 60, 16, 0, np.inf),
    (1, 200, 1, [0.7, 4.0], 40, 5, 8, np.inf),       # ragged tiles, Cholesky-QR inside blocks
    (1, 200, 1, [0.001, 0.7], 12, 64, 0, np.inf),    # wide bands
    (1, 32, 1, [0.5, 2.0], 40, 16, 0, 0.4),          # trajectories stop inside a block
    (2, 8, 6, [0.3, 1.5], 40, 16, 0, np.inf),        # torus: full rows along both directions
    (2, 96, 2, [0.05, 2.0], 30, 7, 9, np.inf),       # torus: band along x, Ly = 2, ragged tiles
    (2, 6, 6, [0.5, 1.0], 24, 8, 0, 0.5),            # torus: trajectories stop inside a block
])
def test_deferred_events_equal_event_by_event_and_oracle(dim, Lx, Ly, gammas, n_slots, K, reorth, t_end):
    """Blocks of K deferred events (one call of n_slots slots) against the same slots taken one
    by one and against the oracle: same last events, same clocks, C to 2e-11."""
    B, seed = len(gammas), 23
    uids = [4 + 3 * b for b in range(B)]
    blk = make_sim(dim, Lx, Ly, n_traj=B, uids=uids)
    one = make_sim(dim, Lx, Ly, n_traj=B, uids=uids)
    blk.set_ct_block(K)
    blk.ct_events(gammas, seed, n_slots, t_end=t_end, reorth_every=reorth)
    one.ct_events(gammas, seed, n_slots, t_end=t_end, reorth_every=reorth)
    orc = OracleCT(dim, Lx, Ly, uids, gammas, seed)
    for _ in range(n_slots):
        recs = orc.slot(t_end)
    _check_slot(blk, orc, recs)
    sb, ob, pb, tb = blk.ct_last_events()
    so, oo, po, to = one.ct_last_events()
    assert np.array_equal(sb, so) and np.array_equal(ob, oo)
    assert np.allclose(blk.times(), one.times(), rtol=1e-13, atol=0.0)
    Ub, _ = blk.get_state()
    Uo, _ = one.get_state()
    for b in range(B):
        assert np.abs(corr(Ub[b]) - corr(Uo[b])).max() <= 2e-11
    _check_state(blk, orc)
    blk.close()
    one.close()


def test_deferred_events_full_size():
    """Ring L = 1024, N = 512, 8 trajectories: 96 slots in blocks of 32 against the same slots
    one by one (C to 1e-10, identical last events); orthonormality kept."""
    L, B, seed = 1024, 8, 9
    gammas = list(np.linspace(0.1, 1.0, B))
    uids = list(range(40, 40 + B))
    blk = make_sim(1, L, n_traj=B, uids=uids)
    one = make_sim(1, L, n_traj=B, uids=uids)
    blk.set_ct_block(32)
    blk.ct_events(gammas, seed, 96)
    one.ct_events(gammas, seed, 96)
    assert np.array_equal(blk.ct_last_events()[0], one.ct_last_events()[0])
    assert np.array_equal(blk.ct_last_events()[1], one.ct_last_events()[1])
    Ub, _ = blk.get_state()
    Uo, _ = one.get_state()
    for b in range(B):
        assert np.abs(corr(Ub[b]) - corr(Uo[b])).max() <= 1e-10
        assert np.abs(Ub[b].conj().T @ Ub[b] - np.eye(L // 2)).max() <= 1e-12
    with pytest.raises(Exception):
        blk.set_ct_block(65)
    blk.close()
    one.close()
