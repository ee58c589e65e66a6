"""Pins for the oracle's Philox4x64-10 and its uniform / normal conversions."""

import numpy as np
import pytest
from scipy import stats

from oracle.philox import philox4x64_10, u01, pm_uniforms, qsd_normals

CASES = [
    (0, 0, (1, 0, 0, 0)),
    (0, 5, (7, 3, 1, 0)),
    (0xDEADBEEFCAFEF00D, 0x0123456789ABCDEF, (12345, 678, 0, 0)),
    (2**64 - 1, 2**64 - 1, (2**64 - 2, 2**64 - 1, 2**64 - 1, 2**64 - 1)),
    (42, 1000017, (399, 63, 1, 0)),
]


@pytest.mark.parametrize("k0,k1,ctr", CASES)
def test_philox_matches_numpy(k0, k1, ctr):
    # numpy's Philox increments its counter before producing a block, so the
    # block of counter c is numpy's first output at counter c - 1.
    c = list(ctr)
    prev = c.copy()
    prev[0] = (prev[0] - 1) % 2**64
    assert c[0] != 0  # keep the decrement free of borrows in these cases
    g = np.random.Philox(key=np.array([k0, k1], dtype=np.uint64),
                         counter=np.array(prev, dtype=np.uint64))
    ref = g.random_raw(4)
    got = philox4x64_10(np.uint64(k0), np.uint64(k1), *[np.uint64(x) for x in c])
    assert [int(x) for x in got] == [int(x) for x in ref]


def test_philox_numpy_zero_counter_case():
    g = np.random.Philox(key=np.array([3, 9], dtype=np.uint64),
                         counter=np.array([0, 0, 0, 0], dtype=np.uint64))
    ref = g.random_raw(8)
    a = philox4x64_10(np.uint64(3), np.uint64(9), 1, 0, 0, 0)
    b = philox4x64_10(np.uint64(3), np.uint64(9), 2, 0, 0, 0)
    assert [int(x) for x in a] + [int(x) for x in b] == [int(x) for x in ref]


def test_philox_vectorised_equals_scalar():
    sites = np.arange(17, dtype=np.uint64)
    vec = philox4x64_10(7, 11, 5, sites, 1, 0)
    for i in range(17):
        sc = philox4x64_10(7, 11, 5, i, 1, 0)
        assert all(int(vec[w][i]) == int(sc[w]) for w in range(4))


def test_u01_open_interval_and_extremes():
    x = np.array([0, 2**64 - 1, 2**12 - 1, 2**63], dtype=np.uint64)
    u = u01(x)
    assert u[0] == 2.0 ** -53
    assert u[1] == 1.0 - 2.0 ** -53
    assert u[2] == u[0]
    assert u[3] == 0.5 + 2.0 ** -53
    assert np.all((u > 0) & (u < 1))


def test_uniforms_are_uniform():
    us = np.concatenate([pm_uniforms(0, uid, n, 256)[0] for uid in range(4) for n in range(1, 21)])
    assert stats.kstest(us, "uniform").pvalue > 1e-3
    assert abs(us.mean() - 0.5) < 4 * np.sqrt(1 / 12 / us.size)


def test_normals_are_standard_normal():
    z = np.concatenate([qsd_normals(0, uid, n, 256) for uid in range(4) for n in range(1, 21)])
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 4 / np.sqrt(z.size)
    assert abs(z.var() - 1) < 4 * np.sqrt(2 / z.size)


def test_streams_are_distinct():
    a = pm_uniforms(0, 0, 1, 64)[0]
    b = pm_uniforms(0, 1, 1, 64)[0]
    c = pm_uniforms(0, 0, 2, 64)[0]
    d = pm_uniforms(1, 0, 1, 64)[0]
    assert len({tuple(a), tuple(b), tuple(c), tuple(d)}) == 4
