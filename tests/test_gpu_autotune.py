"""Autotuner of the execution form (mfq_autotune): the probes leave every trajectory as it
was (state, step index and events of the last step), the chosen configuration is one of the
candidates and reproduces the same trajectories, and a cached choice is applied without
probing.  Every tile choice gives the same results as the default one within rounding, and
both tile orders give bitwise the same results."""

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
    assert res["order"] in (mfq.ORDER_XCD, mfq.ORDER_LINEAR)
    assert res["ms_per_step"] == min(res["candidate_ms"])
    assert {(k["tile"], k["order"]) for k in res["candidates"] if k["path"] == mfq.PATH_LAUNCHES} == \
        {(t, o) for t in (0, 1, 2) for o in (0, 1)}
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
    assert again["order"] == res["order"] and again["pm_path"] == res["pm_path"]
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


def test_autotune_searches_the_projective_form(tmp_path):
    """Projective ring of 256 sites (N = 128, both measurement forms apply), four trajectories:
    both forms are probed, the choice is kept in the cache, and the tuned context follows an
    untuned one within rounding (the two forms give the same outcomes)."""
    from paper_2508_18468_amd import mfq
    L, B, dt, seed = 256, 4, 0.05, 11
    gam = [0.5, 1.0, 1.5, 2.0]
    a = make_sim(1, L, n_traj=B)
    b = make_sim(1, L, n_traj=B)
    cache = str(tmp_path / "tune.json")
    res = a.autotune(PM, gam, dt, seed, probe_steps=3, cache=cache)
    print(f"  tuned projective L={L}: {res}", flush=True)
    assert {k["pm_path"] for k in res["candidates"]} == {mfq.PM_WORKGROUP, mfq.PM_BLOCKED}
    assert res["pm_path"] in (mfq.PM_WORKGROUP, mfq.PM_BLOCKED)
    region = list(range(L // 2))
    Sa = a.run(PM, gam, dt, seed, 12, obs_every=4, region=region)
    Sb = b.run(PM, gam, dt, seed, 12, obs_every=4, region=region)
    assert np.abs(Sa - Sb).max() <= 1e-10
    assert [[(e[0], e[2]) for e in x] for x in a.pm_events()] == [[(e[0], e[2]) for e in x] for x in b.pm_events()]
    c = make_sim(1, L, n_traj=B)
    again = c.autotune(PM, gam, dt, seed, probe_steps=3, cache=cache)
    assert again["cached"] and again["pm_path"] == res["pm_path"] and again["order"] == res["order"]
    for s in (a, b, c):
        s.close()


@pytest.mark.parametrize("L,B", [(320, 3), (256, 9)])
def test_tile_orders_are_bitwise_equal(L, B):
    """The linear and the XCD-grouped workgroup -> tile orders run the same tiles with the same
    arithmetic: states and entropies agree bitwise over homodyne and projective steps (column
    panels grouped per XCD with 3 trajectories, batch entries with 9)."""
    from paper_2508_18468_amd import mfq
    dt, seed = 0.05, 2
    gam = np.linspace(0.4, 2.0, B)
    x = make_sim(1, L, n_traj=B)
    y = make_sim(1, L, n_traj=B)
    y.set_tile_order(mfq.ORDER_LINEAR)
    for protocol in (QSD, PM):
        x.step(protocol, gam, dt, seed, 5)
        y.step(protocol, gam, dt, seed, 5)
    Ux, nx = x.get_state()
    Uy, ny = y.get_state()
    assert nx == ny and np.array_equal(Ux, Uy)
    r = list(range(0, L, 3))
    assert np.array_equal(x.entropy(r), y.entropy(r))
    x.close()
    y.close()
