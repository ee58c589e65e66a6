"""Pins of the oracle's RK4 homodyne step (Appendix A, Eq. (A4) integrated by RK4).

* Taylor remainder: one RK4 step of the linear equation is the degree-4 Taylor polynomial of
  exp(A), so |RK4(A) U - expm(A) U| <= |A|^5 e^|A| / 120 (spectral norms), against scipy expm,
  for the generator built from real draws (rings and a torus, dt = 0.05 and 0.2).
* Order: with gamma = 0 the one-step error of the generator's step against the plane-wave
  propagator falls by about 2^5 when dt halves.
* No hopping (J = 0): the step equals the split step's diagonal factor exp(xi + gamma (2p - 1) dt)
  (independently pinned against Fock space and the Lindblad limit) within the same bound.
* Free part: one RK4 step forward in dt and one in -dt return to U to O(dt^5).
"""

import numpy as np
import pytest
from scipy.linalg import expm

from oracle import Lattice, hopping_matrix, default_occupied, initial_state, propagator
from oracle.trajectory import qsd_update, reorthonormalize
from oracle.rk4 import generator, rk4_propagate, rk4_step, run_rk4


def _state(lat, seed=0):
    rng = np.random.default_rng(seed)
    N = lat.L // 2
    Z = rng.normal(size=(lat.L, N)) + 1j * rng.normal(size=(lat.L, N))
    return np.linalg.qr(Z)[0]


@pytest.mark.parametrize("lat", [Lattice(1, 12), Lattice(1, 30), Lattice(2, 4, 3)])
@pytest.mark.parametrize("dt,gamma", [(0.05, 1.0), (0.2, 0.5), (0.05, 4.0)])
def test_taylor_remainder_against_expm(lat, dt, gamma):
    U = _state(lat, 1)
    A = generator(U, hopping_matrix(lat), gamma, dt, 3, 7, 5)
    a = np.linalg.norm(A, 2)
    err = np.linalg.norm(rk4_propagate(U, A) - expm(A) @ U, 2)
    assert err <= a ** 5 * np.exp(a) / 120.0 * (1 + 1e-9) + 1e-14
    assert err >= 1e-4 * a ** 5 / 120.0       # a fourth-order method, not an exact one


def test_fourth_order_free_step():
    lat = Lattice(1, 16)
    H = hopping_matrix(lat)
    U = initial_state(16, default_occupied(lat))
    errs = []
    for dt in (0.2, 0.1, 0.05):
        A = generator(U, H, 0.0, dt, 1, 1, 1)   # gamma = 0: the free part of the generator
        errs.append(np.abs(rk4_propagate(U, A) - propagator(lat, dt) @ U).max())
    for e1, e2 in zip(errs, errs[1:]):
        assert 26.0 < e1 / e2 < 38.0


def test_no_hopping_equals_split_diagonal():
    lat = Lattice(1, 10, J=0.0)
    H = hopping_matrix(lat)
    U = _state(lat, 2)
    for gamma, dt in ((1.0, 0.05), (0.3, 0.2)):
        A = generator(U, H, gamma, dt, 5, 1, 3)
        got = rk4_propagate(U, A)
        want = qsd_update(U, gamma, dt, 5, 1, 3)   # exp of the same diagonal, rows scaled
        a = np.abs(np.diag(A)).max()
        assert np.abs(got - want).max() <= a ** 5 * np.exp(a) / 120.0 + 1e-15
        # after normalisation the steps agree to the same order
        assert np.abs(reorthonormalize(got) @ reorthonormalize(got).conj().T
                      - reorthonormalize(want) @ reorthonormalize(want).conj().T).max() \
            <= 4 * a ** 5 * np.exp(a) / 120.0 + 1e-14


def test_free_step_time_reversal():
    lat = Lattice(2, 4, 4)
    H = hopping_matrix(lat)
    U = _state(lat, 3)
    dt = 0.05
    back = rk4_propagate(rk4_propagate(U, -1j * dt * H), 1j * dt * H)
    a = np.linalg.norm(dt * H, 2)
    assert np.abs(back - U).max() <= 2 * a ** 5 * np.exp(a) / 120.0


def test_run_keeps_orthonormal_and_chunks():
    lat = Lattice(1, 20)
    U0 = initial_state(20, default_occupied(lat))
    U = run_rk4(lat, U0, 0.8, 0.05, 2, 4, 30)
    assert np.abs(U.conj().T @ U - np.eye(10)).max() < 1e-13
    V = run_rk4(lat, run_rk4(lat, U0, 0.8, 0.05, 2, 4, 12), 0.8, 0.05, 2, 4, 18, first_step=13)
    assert np.abs(U - V).max() == 0.0
    W = U0.copy()
    H = hopping_matrix(lat)
    for n in range(1, 31):
        W = rk4_step(W, H, 0.8, 0.05, 2, 4, n)
    assert np.abs(U - W).max() == 0.0
