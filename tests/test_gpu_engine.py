"""Serving engine: every job's result is the same alone and in the mix; admission
respects the memory budget."""

import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

PM, QSD = 0, 1


def _alone(dim, Lx, Ly, protocol, gamma, dt, n_steps, seed, uid, region, obs_every):
    from paper_2508_18468_amd import mfq
    sim = mfq.Trajectories(dim, Lx, Ly, n_traj=1, uids=[uid])
    sim.set_path(mfq.PATH_LAUNCHES)
    S = sim.run(protocol, [gamma], dt, seed, n_steps, obs_every, region)
    sim.close()
    return S[:, 0]


def _mix():
    rng = np.random.default_rng(3)
    jobs = []
    shapes = [(1, 32, 1), (1, 48, 1), (1, 64, 1), (1, 96, 1), (2, 6, 6), (2, 8, 8)]
    for i in range(18):
        dim, Lx, Ly = shapes[i % len(shapes)]
        L = Lx * (Ly if dim == 2 else 1)
        region = list(range(L // 2)) if dim == 1 else sorted(x + Lx * y for y in range(Ly) for x in range(Lx // 2))
        jobs.append(dict(dim=dim, Lx=Lx, Ly=Ly, protocol=int(rng.integers(2)), gamma=float(rng.uniform(0.1, 2.0)),
                         dt=0.05, n_steps=int(rng.choice([40, 60, 80])), seed=0, uid=5000 + i, region=region,
                         obs_every=20))
    return jobs


def test_engine_results_equal_alone():
    from paper_2508_18468_amd import mfq
    eng = mfq.Engine(max_slots=4)
    jobs = _mix()
    ids = []
    for j in jobs:
        ids.append(eng.submit(j["dim"], j["Lx"], j["Ly"], j["protocol"], j["gamma"], j["dt"], j["n_steps"],
                              j["seed"], j["uid"], j["region"], obs_every=j["obs_every"]))
        time.sleep(0.002)
    results = [eng.wait(i, 300) for i in ids]
    st = eng.stats()
    eng.close()
    for j, (S, lat) in zip(jobs, results):
        ref = _alone(j["dim"], j["Lx"], j["Ly"], j["protocol"], j["gamma"], j["dt"], j["n_steps"], j["seed"],
                     j["uid"], j["region"], j["obs_every"])
        assert S.shape == ref.shape == (j["n_steps"] // 20,)
        assert np.abs(S - ref).max() <= 1e-10, (j, S, ref)
        assert lat > 0
    assert st["peak_bytes"] <= st["budget_bytes"]


def test_engine_small_budget_serialises_groups():
    from paper_2508_18468_amd import mfq
    # room for one small group at a time
    lat = mfq.Lattice(1, 64, 1, 0, 1.0)
    one = mfq.mfq_workspace_bytes(lat, 32, 2)
    eng = mfq.Engine(hbm_budget_bytes=int(one * 1.5), max_slots=2)
    ids = [eng.submit(1, L, 1, QSD, 0.5, 0.05, 30, 0, 100 + k, list(range(L // 2)))
           for k, L in enumerate([64, 48, 64, 32, 48, 64])]
    res = [eng.wait(i, 300) for i in ids]
    st = eng.stats()
    eng.close()
    assert all(r[0].shape == (1,) for r in res)
    assert st["peak_bytes"] <= st["budget_bytes"]


def test_engine_rejects_job_larger_than_budget():
    from paper_2508_18468_amd import mfq
    eng = mfq.Engine(hbm_budget_bytes=1 << 20, max_slots=2)
    jid = eng.submit(1, 1024, 1, QSD, 0.5, 0.05, 10, 0, 1, list(range(512)))
    with pytest.raises(mfq.MfqError) as e:
        eng.wait(jid, 30)
    assert e.value.code == -2
    with pytest.raises(mfq.MfqError):
        eng.submit(1, 63, 1, QSD, 0.5, 0.05, 10, 0, 2, [0])  # odd L: no Neel state
    eng.close()


def test_served_jobs_at_mix_sizes_match_oracle():
    """Jobs of the served mix's own shapes (1d L = 256 and 512, 2d 16 x 16; both protocols, rates
    drawn in [0.1, 2.0]) submitted together with smaller filler jobs, so that they share the
    device with other groups; each job's final entropy against the CPU oracle run of the same
    job (seed, uid, rate), |dS| <= 1e-9."""
    import oracle
    from paper_2508_18468_amd import mfq
    rng = np.random.default_rng(11)
    shapes = [(1, 256, 1), (1, 512, 1), (2, 16, 16)]
    jobs = []
    for i, (dim, Lx, Ly) in enumerate(shapes * 2):
        L = Lx * Ly
        region = list(range(L // 2)) if dim == 1 else sorted(x + Lx * y for y in range(Ly) for x in range(Lx // 2))
        jobs.append(dict(dim=dim, Lx=Lx, Ly=Ly, protocol=PM if i < 3 else QSD,
                         gamma=float(rng.uniform(0.1, 2.0)), n_steps=int(rng.choice([24, 30])), uid=7000 + i,
                         region=region))
    fillers = [dict(dim=1, Lx=64, Ly=1, protocol=QSD, gamma=0.7, n_steps=200, uid=7100 + k,
                    region=list(range(32))) for k in range(4)]
    eng = mfq.Engine(max_slots=4)
    ids = []
    for j in fillers + jobs:
        ids.append(eng.submit(j["dim"], j["Lx"], j["Ly"], j["protocol"], j["gamma"], 0.05, j["n_steps"], 0,
                              j["uid"], j["region"]))
    res = [eng.wait(i, 300) for i in ids]
    eng.close()
    for j, (S, _) in zip(jobs, res[len(fillers):]):
        lat = oracle.Lattice(j["dim"], j["Lx"], j["Ly"])
        P = oracle.propagator(lat, 0.05)
        out = oracle.run_trajectory(P, oracle.default_occupied(lat), j["protocol"], j["gamma"], 0.05, 0,
                                    j["uid"], j["n_steps"])
        ref = oracle.entanglement_entropy(out["U"], j["region"])
        assert S.shape == (1,)
        assert abs(S[0] - ref) <= 1e-9, (j, S[0], ref)
