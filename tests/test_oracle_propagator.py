"""Pins for the oracle's lattice and propagator exp(-i Ht dt)."""

import numpy as np
import pytest
from scipy import linalg, special

from oracle import Lattice, hopping_matrix, propagator, default_occupied


@pytest.mark.parametrize("lat", [Lattice(1, 8), Lattice(1, 64), Lattice(2, 4, 4),
                                 Lattice(2, 6, 4), Lattice(2, 4, 2)])
@pytest.mark.parametrize("dt", [0.05, 0.37])
def test_propagator_equals_expm(lat, dt):
    H = hopping_matrix(lat)
    ref = linalg.expm(-1j * dt * H)
    P = propagator(lat, dt)
    assert np.abs(P - ref).max() < 1e-13


@pytest.mark.parametrize("lat", [Lattice(1, 128), Lattice(2, 8, 6)])
def test_propagator_unitary_symmetric(lat):
    P = propagator(lat, 0.05)
    I = np.eye(lat.L)
    assert np.abs(P @ np.conj(P.T) - I).max() < 1e-14
    assert np.abs(P - P.T).max() < 1e-15


def test_propagator_bessel_entries():
    # exp(-i z cos k) = sum_n (-i)^n J_n(z) e^{ink}: P_{0,n} = (-i)^n J_n(2 J dt) for n << L
    L, dt = 256, 0.05
    P = propagator(Lattice(1, L), dt)
    for n in range(0, 9):
        ref = (-1j) ** n * special.jv(n, 2 * dt)
        assert abs(P[n, 0] - ref) < 1e-16 + 1e-13 * abs(ref)
        assert abs(P[0, n] - ref) < 1e-16 + 1e-13 * abs(ref)
    # |P_{0,1}| = J_1(0.1) at dt = 0.05, to ten digits
    assert abs(abs(P[0, 1]) - 0.0499375260) < 1e-9


def test_hopping_matrix_structure():
    H = hopping_matrix(Lattice(1, 10))
    assert np.allclose(H, H.T) and H.sum() == 20
    H2 = hopping_matrix(Lattice(2, 6, 4))
    assert np.allclose(H2, H2.T) and H2.sum() == 2 * 2 * 24
    # spectrum 2J (cos kx + cos ky)
    kx = 2 * np.pi * np.arange(6) / 6
    ky = 2 * np.pi * np.arange(4) / 4
    ref = np.sort((2 * np.cos(kx)[None, :] + 2 * np.cos(ky)[:, None]).ravel())
    assert np.abs(np.linalg.eigvalsh(H2) - ref).max() < 1e-12


def test_default_occupied():
    assert default_occupied(Lattice(1, 8)) == [0, 2, 4, 6]
    occ = default_occupied(Lattice(2, 4, 4))
    assert len(occ) == 8 and 0 in occ and 1 not in occ and 4 not in occ and 5 in occ
