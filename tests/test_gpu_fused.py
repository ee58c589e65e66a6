"""Fused single-launch trajectory path (mfq_run) against the oracle and against the
per-phase path."""

import time

import numpy as np
import pytest

import oracle
from gpu_common import make_sim, OracleBatch, corr

pytestmark = pytest.mark.gpu

PM, QSD = 0, 1


def test_fused_small_ring_projective_full_workload():
    """1d ring L=64, N=32, projective gamma=0.5, dt=0.05, 400 steps, 16 trajectories, seed 0:
    S of A=[0,32) after every 10th step from one launch; |dS| <= 1e-9 at all 40 samples."""
    from paper_2508_18468_amd import mfq
    from paper_2508_18468_amd.workloads import ring_pm_small
    w = ring_pm_small()
    uids = w.uids(0)
    B = len(uids)
    sim = make_sim(1, w.Lx, n_traj=B, uids=uids)
    sim.set_path(mfq.PATH_FUSED)
    t0 = time.perf_counter()
    S = sim.run(PM, [w.gammas[0]] * B, w.dt, w.seed, w.n_steps, w.obs_every, w.regions[0])
    t_fused = time.perf_counter() - t0
    assert S.shape == (40, B)
    lat = oracle.Lattice(1, w.Lx)
    P = oracle.propagator(lat, w.dt)
    ref = np.zeros((40, B))
    Uref = []
    for t, uid in enumerate(uids):
        out = oracle.run_trajectory(P, oracle.default_occupied(lat), 0, w.gammas[0], w.dt, w.seed, uid,
                                    w.n_steps, obs_every=w.obs_every, regions=[w.regions[0]])
        for k in range(40):
            ref[k, t] = out["S"][(k + 1) * w.obs_every][0]
        Uref.append(out["U"])
    assert np.abs(S - ref).max() <= 1e-9
    U, n = sim.get_state()
    assert n == w.n_steps
    for t in range(B):
        assert np.abs(corr(U[t]) - corr(Uref[t])).max() < 1e-10
    print(f"fused small-ring run: {t_fused*1e3:.1f} ms for {B} x {w.n_steps} steps + 40 observations")
    sim.close()


@pytest.mark.parametrize("dim,Lx,Ly,protocol,gamma,region", [
    (1, 64, 1, QSD, 0.7, list(range(32))),
    (2, 6, 6, QSD, 1.5, list(range(0, 36, 2))),
    (2, 6, 6, PM, 3.0, list(range(24))),       # region larger than N: U_A^+ U_A form
    (1, 40, 1, PM, 2.0, [0, 3, 4, 9, 17, 30]),
])
def test_fused_equals_launch_path(dim, Lx, Ly, protocol, gamma, region):
    from paper_2508_18468_amd import mfq
    B = 5
    a = make_sim(dim, Lx, Ly, n_traj=B, uids=range(B))
    b = make_sim(dim, Lx, Ly, n_traj=B, uids=range(B))
    a.set_path(mfq.PATH_FUSED)
    b.set_path(mfq.PATH_LAUNCHES)
    g = np.linspace(0.5, 1.5, B) * gamma
    Sa = a.run(protocol, g, 0.05, 4, 37, 5, region)
    Sb = b.run(protocol, g, 0.05, 4, 37, 5, region)
    assert Sa.shape == Sb.shape == (7, B)
    assert np.abs(Sa - Sb).max() <= 1e-10
    Ua, _ = a.get_state()
    Ub, _ = b.get_state()
    for t in range(B):
        assert np.abs(corr(Ua[t]) - corr(Ub[t])).max() < 1e-11
    if protocol == PM:
        ea, eb = a.pm_events(), b.pm_events()
        assert [[(e[0], e[2]) for e in x] for x in ea] == [[(e[0], e[2]) for e in x] for x in eb]
    a.close()
    b.close()


def test_fused_chunking_is_exact():
    from paper_2508_18468_amd import mfq
    a = make_sim(1, 48, n_traj=3, uids=[4, 5, 6])
    b = make_sim(1, 48, n_traj=3, uids=[4, 5, 6])
    a.set_path(mfq.PATH_FUSED)
    b.set_path(mfq.PATH_FUSED)
    Sa = a.run(QSD, [0.4, 0.8, 1.2], 0.05, 2, 60, 10, list(range(24)))
    Sb1 = b.run(QSD, [0.4, 0.8, 1.2], 0.05, 2, 25, 10, list(range(24)))
    Sb2 = b.run(QSD, [0.4, 0.8, 1.2], 0.05, 2, 35, 10, list(range(24)))
    assert np.array_equal(Sa, np.concatenate([Sb1, Sb2]))
    assert np.array_equal(a.get_state()[0], b.get_state()[0])
    a.close()
    b.close()


def test_fused_rejects_problems_that_do_not_fit():
    from paper_2508_18468_amd import mfq
    sim = make_sim(1, 512, n_traj=1)
    sim.set_path(mfq.PATH_FUSED)
    with pytest.raises(mfq.MfqError):
        sim.run(QSD, [1.0], 0.05, 0, 2)
    sim.set_path(mfq.PATH_AUTO)
    S = sim.run(QSD, [1.0], 0.05, 0, 4, 2, list(range(256)))
    assert S.shape == (2, 1)
    sim.close()


@pytest.mark.parametrize("path", ["fused", "launches"])
def test_small_ring_timing(path):
    """The small-ring workload on each path after a warm-up run, for the record."""
    from paper_2508_18468_amd import mfq
    from paper_2508_18468_amd.workloads import ring_pm_small
    w = ring_pm_small()
    uids = w.uids(0)
    times = []
    for rep in range(2):
        sim = make_sim(1, w.Lx, n_traj=len(uids), uids=uids)
        sim.set_path(mfq.PATH_FUSED if path == "fused" else mfq.PATH_LAUNCHES)
        t0 = time.perf_counter()
        S = sim.run(PM, [w.gammas[0]] * len(uids), w.dt, w.seed, w.n_steps, w.obs_every, w.regions[0])
        times.append(time.perf_counter() - t0)
        assert S.shape == (40, len(uids))
        t1 = time.perf_counter()
        sim.run(QSD, [1.0] * len(uids), w.dt, w.seed, 400)
        t_qsd = time.perf_counter() - t1
        sim.close()
    print(f"{path} small-ring run: {times[-1]*1e3:.1f} ms (first {times[0]*1e3:.1f} ms); "
          f"400 homodyne steps without observation: {t_qsd*1e3:.1f} ms")


def _group_members():
    """Three lattices of uneven size and protocol: ring 64 projective, ring 40 homodyne, torus
    6 x 6 homodyne (different rates, dt, seeds, step counts and observation schedules)."""
    return [
        dict(dim=1, Lx=64, Ly=1, uids=[3, 4, 5, 6], protocol=PM, gamma=[0.5, 0.5, 1.0, 2.0], dt=0.05,
             seed=1, n_steps=20, obs_every=5, region=list(range(32))),
        dict(dim=1, Lx=40, Ly=1, uids=[7, 8, 9], protocol=QSD, gamma=[0.3, 1.0, 2.5], dt=0.04, seed=2,
             n_steps=15, obs_every=3, region=list(range(0, 40, 3))),
        dict(dim=2, Lx=6, Ly=6, uids=[10, 11], protocol=QSD, gamma=[1.0, 0.2], dt=0.05, seed=3,
             n_steps=10, obs_every=0, region=None),
    ]


def test_group_launch_equals_separate_runs_and_oracle():
    """One launch for the three lattices equals each lattice run on its own (bitwise: same body,
    same draws) and the homodyne ring follows the oracle (|dS| <= 1e-9)."""
    from paper_2508_18468_amd import mfq
    members = _group_members()
    grouped = [make_sim(m["dim"], m["Lx"], m["Ly"], n_traj=len(m["uids"]), uids=m["uids"]) for m in members]
    for sim in grouped:
        sim.step(QSD, [0.4] * sim.n_traj, 0.05, 9, 2)        # a common prefix of per-phase steps
    S_grp = mfq.mfq_run_group(grouped, members)
    for m, sim, S in zip(members, grouped, S_grp):
        alone = make_sim(m["dim"], m["Lx"], m["Ly"], n_traj=len(m["uids"]), uids=m["uids"])
        alone.step(QSD, [0.4] * alone.n_traj, 0.05, 9, 2)
        alone.set_path(mfq.PATH_FUSED)
        S_alone = alone.run(m["protocol"], m["gamma"], m["dt"], m["seed"], m["n_steps"], m["obs_every"],
                            m["region"])
        assert S.shape == S_alone.shape and np.array_equal(S, S_alone)
        assert np.array_equal(sim.get_state()[0], alone.get_state()[0])
        assert sim.step_index() == 2 + m["n_steps"]
        alone.close()
    m = members[1]
    ob = OracleBatch(1, m["Lx"], 1, 0.05, m["uids"])
    for _ in range(2):
        ob.step(QSD, [0.4] * 3, 9)
    ob.dt, ob.P = m["dt"], oracle.propagator(oracle.Lattice(1, m["Lx"]), m["dt"])
    k = 0
    for n in range(3, 3 + m["n_steps"]):
        ob.step(QSD, m["gamma"], m["seed"])
        if n % m["obs_every"] == 0:
            assert np.abs(S_grp[1][k] - ob.entropy(m["region"])).max() <= 1e-9
            k += 1
    assert k == S_grp[1].shape[0]
    for sim in grouped:
        sim.close()


def test_group_launch_errors():
    from paper_2508_18468_amd import mfq
    members = _group_members()
    sims = [make_sim(m["dim"], m["Lx"], m["Ly"], n_traj=len(m["uids"]), uids=m["uids"]) for m in members]
    with pytest.raises(Exception):
        mfq.mfq_run_group([sims[0], sims[0]], [members[0], members[0]])   # repeated context
    big = make_sim(1, 1024, n_traj=1)
    with pytest.raises(Exception):
        mfq.mfq_run_group([sims[0], big], [members[0], dict(members[0], gamma=[0.5])])
    with pytest.raises(Exception):                                        # blocked projective form
        mfq.mfq_run_group([sims[1], big], [members[1], dict(members[0], gamma=[0.5], region=None, obs_every=0)])
    sims[1].set_integrator(mfq.INTEGRATOR_RK4)                            # RK4 is not fused: one graph
    assert [S.shape for S in mfq.mfq_run_group(sims[:2], members[:2])] == [(4, 4), (5, 3)]
    many = [make_sim(1, 16, n_traj=1, uids=[k]) for k in range(9)]
    spec = dict(protocol=PM, gamma=[0.5], dt=0.05, seed=0, n_steps=1)
    with pytest.raises(Exception):
        mfq.mfq_run_group(many, [spec] * 9)
    assert len(mfq.mfq_run_group(many[:8], [spec] * 8)) == 8
    for s in sims + many + [big]:
        s.close()


def _graph_members():
    """Lattices that do not fit the fused kernel: ring 160 homodyne (split step), ring 200 with
    100 particles projective (per-workgroup measurement, N < 128), torus 12 x 12 homodyne by the
    paper's RK4, ring 96 homodyne; uneven step counts and observation schedules."""
    return [
        dict(dim=1, Lx=160, Ly=1, uids=[1, 2, 3], protocol=QSD, gamma=[0.5, 1.0, 2.0], dt=0.05, seed=4,
             n_steps=11, obs_every=4, region=list(range(80)), rk4=False),
        dict(dim=1, Lx=200, Ly=1, uids=[4, 5], protocol=PM, gamma=[0.3, 1.0], dt=0.05, seed=5,
             n_steps=7, obs_every=3, region=list(range(0, 200, 2)), rk4=False),
        dict(dim=2, Lx=12, Ly=12, uids=[6, 7], protocol=QSD, gamma=[1.0, 0.4], dt=0.04, seed=6,
             n_steps=10, obs_every=0, region=None, rk4=True),
        dict(dim=1, Lx=96, Ly=1, uids=[8], protocol=QSD, gamma=[1.5], dt=0.05, seed=7,
             n_steps=9, obs_every=2, region=list(range(48)), rk4=False),
    ]


def _graph_sim(m):
    from paper_2508_18468_amd import mfq
    sim = make_sim(m["dim"], m["Lx"], m["Ly"], n_traj=len(m["uids"]), uids=m["uids"])
    sim.set_path(mfq.PATH_LAUNCHES)
    if m["rk4"]:
        sim.set_integrator(mfq.INTEGRATOR_RK4)
    sim.step(QSD, [0.4] * sim.n_traj, 0.05, 9, 3)   # an odd prefix: the group starts at odd steps
    return sim


def test_group_graph_equals_separate_runs_and_oracle():
    """Lattices above the fused kernel's size advance in one graph (two steps of each per
    replay, parallel branches): observations and states equal each lattice run alone (bitwise:
    same kernels, same draws), and the split-step ring follows the oracle (|dS| <= 1e-9)."""
    from paper_2508_18468_amd import mfq
    members = _graph_members()
    grouped = [_graph_sim(m) for m in members]
    S_grp = mfq.mfq_run_group(grouped, members)
    for m, sim, S in zip(members, grouped, S_grp):
        alone = _graph_sim(m)
        S_alone = alone.run(m["protocol"], m["gamma"], m["dt"], m["seed"], m["n_steps"], m["obs_every"],
                            m["region"])
        assert S.shape == S_alone.shape and np.array_equal(S, S_alone), m["Lx"]
        assert np.array_equal(sim.get_state()[0], alone.get_state()[0]), m["Lx"]
        assert sim.step_index() == 3 + m["n_steps"]
        alone.close()
    m = members[0]
    ob = OracleBatch(1, m["Lx"], 1, 0.05, m["uids"])
    for _ in range(3):
        ob.step(QSD, [0.4] * 3, 9)
    k = 0
    for n in range(4, 4 + m["n_steps"]):
        ob.step(QSD, m["gamma"], m["seed"])
        if n % m["obs_every"] == 0:
            assert np.abs(S_grp[0][k] - ob.entropy(m["region"])).max() <= 1e-9
            k += 1
    assert k == S_grp[0].shape[0] == 3
    for sim in grouped:
        sim.close()


def test_group_graph_timing():
    """Four lattices above the fused kernel's size, 40 homodyne steps each: one group graph
    against the lattices run one after another (printed; both paths give the same states)."""
    from paper_2508_18468_amd import mfq
    specs = [(1, 256, 1, 8), (1, 384, 1, 4), (2, 16, 16, 4), (1, 512, 1, 2)]
    times = {}
    states = {}
    for mode in ("alone", "group", "alone", "group"):
        sims = [make_sim(d, Lx, Ly, n_traj=b, uids=list(range(b))) for d, Lx, Ly, b in specs]
        members = [dict(protocol=QSD, gamma=[1.0] * s.n_traj, dt=0.05, seed=3, n_steps=40) for s in sims]
        for s in sims:
            s.set_path(mfq.PATH_LAUNCHES)
            s.step(QSD, [1.0] * s.n_traj, 0.05, 3, 2)
            s.synchronize()
        t0 = time.perf_counter()
        if mode == "group":
            mfq.mfq_run_group(sims, members)
        else:
            for s, sp in zip(sims, members):
                s.run(QSD, sp["gamma"], 0.05, 3, 40)
        for s in sims:
            s.synchronize()
        times[mode] = time.perf_counter() - t0
        states[mode] = [s.get_state()[0] for s in sims]
        for s in sims:
            s.close()
    for a, b in zip(states["alone"], states["group"]):
        assert np.array_equal(a, b)
    print(f"group graph: {times['group'] * 1e3:.1f} ms; one after another: {times['alone'] * 1e3:.1f} ms")
