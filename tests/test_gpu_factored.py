"""Factored propagator (banded ring stencil, Kronecker factors on the torus) against the dense
propagator and the oracle on the same trajectories.  The band drops generating-row entries
below 1e-20 of the largest and the torus factors are exact, so states agree with the dense
form to rounding: C within 1e-12 after 20 steps, S within 1e-10, and the oracle parity bar
|dS| <= 1e-9 holds as for the dense form."""

import numpy as np
import pytest

from gpu_common import OracleBatch, make_sim, corr

pytestmark = pytest.mark.gpu

PM, QSD = 0, 1


def _pair(dim, Lx, Ly, B, uids):
    from paper_2508_18468_amd import mfq
    dense = make_sim(dim, Lx, Ly, n_traj=B, uids=uids)
    fact = make_sim(dim, Lx, Ly, n_traj=B, uids=uids)
    fact.set_propagator(mfq.PROP_FACTORED)
    return dense, fact


@pytest.mark.parametrize("dim,Lx,Ly,dt", [(1, 64, 1, 0.05), (1, 200, 1, 0.05), (1, 1024, 1, 0.05),
                                           (1, 96, 1, 0.6), (2, 12, 8, 0.05), (2, 16, 16, 0.3)])
def test_factored_equals_dense_and_oracle(dim, Lx, Ly, dt):
    B, uids, seed = 3, [1, 4, 7], 8
    gams = [0.3, 1.0, 2.5]
    dense, fact = _pair(dim, Lx, Ly, B, uids)
    ob = OracleBatch(dim, Lx, Ly, dt, uids) if Lx * Ly <= 256 else None
    L = Lx * Ly
    region = list(range(L // 2)) if dim == 1 else sorted(x + Lx * y for y in range(Ly)
                                                          for x in range(Lx // 2))
    for n in range(20):
        protocol = QSD if n % 2 == 0 else PM
        dense.step(protocol, gams, dt, seed)
        fact.step(protocol, gams, dt, seed)
        if ob is not None:
            ob.step(protocol, gams, seed)
    w = fact.propagator_band()
    print(f"  dim={dim} L={L} dt={dt}: band {w}", flush=True)
    if dim == 1:
        assert 0 <= w <= 128 and 2 * w + 1 <= L
    Ud, _ = dense.get_state()
    Uf, _ = fact.get_state()
    for t in range(B):
        assert np.abs(corr(Ud[t]) - corr(Uf[t])).max() <= 1e-12
    Sf = fact.entropy(region)
    assert np.abs(dense.entropy(region) - Sf).max() <= 1e-10
    if ob is not None:
        assert np.abs(Sf - ob.entropy(region)).max() <= 1e-9
    dense.close()
    fact.close()


def test_factored_graph_replay_and_chunking():
    """The torus factors keep the state in its buffer, the ring band alternates like the dense
    form: many steps in one call (graph replay) equal the same steps one by one."""
    from paper_2508_18468_amd import mfq
    for dim, Lx, Ly in ((2, 8, 8), (1, 128, 1)):
        a = make_sim(dim, Lx, Ly, n_traj=2)
        b = make_sim(dim, Lx, Ly, n_traj=2)
        for s in (a, b):
            s.set_propagator(mfq.PROP_FACTORED)
        a.step(QSD, [0.5, 1.5], 0.05, 2, 9)
        for _ in range(9):
            b.step(QSD, [0.5, 1.5], 0.05, 2, 1)
        Ua, _ = a.get_state()
        Ub, _ = b.get_state()
        assert np.array_equal(Ua, Ub)
        a.close()
        b.close()
