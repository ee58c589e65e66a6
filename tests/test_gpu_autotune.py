"""Autotuner of the execution form (mfq_autotune): the probes leave every trajectory as it
was (state, step index and events of the last step), the chosen configuration is one of the
candidates and reproduces the same trajectories, and a cached choice is applied without
probing.  Every tile choice gives the same results as the default one within rounding."""

import json

import numpy as np
import pytest

from gpu_common import make_sim, corr

pytestmark = pytest.mark.gpu

PM, QSD = 0, 1


@pytest.mark.parametrize("protocol,L,B", [(PM, 64, 16), (QSD, 256, 8)])
def test_autotune_restores_state_and_keeps_results(protocol, L, B, tmp_path):
    from paper_2508_18468_amd import mfq
    dt, seed = 0.05, 3
    gam = np.linspace(0.3, 1.2, B)
    a = make_sim(1, L, n_traj=B)
    b = make_sim(1, L, n_traj=B)
    for s in (a, b):
        s.step(protocol, gam, dt, seed, 7)
    Ua0, st0 = a.get_state()
    ev0 = a.pm_events()
    cache = str(tmp_path / "tune.json")
    res = a.autotune(protocol, gam, dt, seed, probe_steps=4, cache=cache)
    print(f"  tuned L={L} B={B}: {res}", flush=True)
    assert not res["cached"]
    assert (res["path"], res["tile"]) in [(mfq.PATH_LAUNCHES, t) for t in (0, 1, 2)] + [(mfq.PATH_FUSED, 0)]
    assert res["ms_per_step"] == min(res["candidate_ms"])
    Ua1, st1 = a.get_state()
    assert st1 == st0 and np.array_equal(Ua1, Ua0)
    assert a.pm_events() == ev0
    # continue both: the tuned context follows the untuned one within rounding
    region = list(range(L // 2))
    Sa = a.run(protocol, gam, dt, seed, 10, obs_every=5, region=region)
    Sb = b.run(protocol, gam, dt, seed, 10, obs_every=5, region=region)
    assert np.abs(Sa - Sb).max() <= 1e-10
    with open(cache) as f:
        assert len(json.load(f)) == 1
    c = make_sim(1, L, n_traj=B)
    again = c.autotune(protocol, gam, dt, seed, probe_steps=4, cache=cache)
    assert again["cached"] and again["path"] == res["path"] and again["tile"] == res["tile"]
    for s in (a, b, c):
        s.close()


@pytest.mark.parametrize("tile", [1, 2])
def test_tile_choices_agree(tile):
    """L=320 (N=160): the small- and large-tile variants of every contraction of a step, the
    propagator included, against the default choice."""
    from paper_2508_18468_amd import mfq
    L, B, dt, seed = 320, 3, 0.05, 5
    gam = [0.4, 1.0, 2.5]
    ref = make_sim(1, L, n_traj=B)
    alt = make_sim(1, L, n_traj=B)
    mfq.mfq_set_tuning(alt.ctx, mfq.PATH_LAUNCHES, tile)
    for protocol in (QSD, PM):
        ref.step(protocol, gam, dt, seed, 6)
        alt.step(protocol, gam, dt, seed, 6)
    Ur, _ = ref.get_state()
    Ua, _ = alt.get_state()
    for t in range(B):
        assert np.abs(corr(Ur[t]) - corr(Ua[t])).max() <= 1e-10
    r = list(range(0, L, 2))
    assert np.abs(ref.entropy(r) - alt.entropy(r)).max() <= 1e-10
    ref.close()
    alt.close()
