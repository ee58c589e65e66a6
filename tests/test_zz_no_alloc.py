"""mfq_density_correlation_noalloc: C(r) of Sec. II, Eq. (2), with the tile partials and bins
in the library's static per-GPU buffer instead of a device allocation.

It runs the same kernels as mfq_density_correlation, so the two agree bitwise; both are also
checked against the oracle (1e-12 absolute, the tolerance of the C(r) parity tests).  Two calls
in a row, the second on a smaller input, then a request above the buffer's limit (MFQ_ENOMEM,
nothing launched) followed by a call that fits.
"""

import numpy as np
import pytest

import oracle
from gpu_common import OracleBatch, make_sim

pytestmark = pytest.mark.gpu

PM, QSD = 0, 1


def _advance(L, protocol, gams, n_steps, uids, seed=11, dt=0.05):
    sim = make_sim(1, L, n_traj=len(uids), uids=uids)
    ob = OracleBatch(1, L, 1, dt, uids)
    for _ in range(n_steps):
        sim.step(protocol, gams, dt, seed)
        ob.step(protocol, gams, seed)
    return sim, ob


def _check(sim, ob):
    print(f"no-alloc C(r): L={sim.L} n_traj={sim.n_traj}", flush=True)
    got = sim.density_correlation_noalloc()
    ref = sim.density_correlation()
    assert np.array_equal(got, ref)
    for t in range(sim.n_traj):
        assert np.abs(got[t] - oracle.density_correlation(ob.U[t])).max() <= 1e-12


def test_noalloc_two_calls_second_smaller():
    big, ob_big = _advance(512, PM, [0.4, 0.8, 1.2, 1.6, 2.0, 2.4], 8, [3, 4, 5, 6, 7, 8])
    _check(big, ob_big)
    small, ob_small = _advance(200, QSD, [0.5, 1.0, 3.0], 10, [1, 2, 9])
    _check(small, ob_small)
    big.close()
    small.close()


def test_noalloc_rejects_requests_above_the_limit():
    from paper_2508_18468_amd import mfq
    # partials of the upper 64 x 64 tiles of a 1024 x 1024 product (136 tiles x 127 diagonals)
    # plus 512 bins per trajectory: 480 trajectories need 68.3 MB, above the 64 MiB buffer
    sim = make_sim(1, 1024, n_traj=480, N=1, occupied=[0])
    with pytest.raises(mfq.MfqError) as e:
        sim.density_correlation_noalloc()
    assert e.value.code == -2
    sim.close()
    small, ob_small = _advance(64, PM, [1.0, 2.0], 6, [0, 1])
    _check(small, ob_small)
    small.close()
