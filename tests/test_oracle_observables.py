"""Pins for the oracle's entropy / mutual-information functions."""

import numpy as np

from oracle import (Lattice, propagator, default_occupied, initial_state, region_spectrum,
                    entropy_from_spectrum, entanglement_entropy, mutual_information,
                    correlation_matrix, run_trajectory)
from oracle.trajectory import HOMODYNE, PROJECTIVE
from fock import FockSim
from oracle import hopping_matrix


def _evolved(L=32, protocol=HOMODYNE, gamma=0.4, steps=80, uid=1):
    lat = Lattice(1, L)
    return run_trajectory(propagator(lat, 0.05), default_occupied(lat), protocol, gamma, 0.05,
                          0, uid, steps)["U"]


def test_neel_entropy_zero():
    lat = Lattice(1, 16)
    U = initial_state(16, default_occupied(lat))
    for r in ([0], list(range(8)), [1, 4, 9, 10]):
        assert entanglement_entropy(U, r) == 0.0


def test_entropy_of_known_spectra():
    assert entropy_from_spectrum([0.5]) == np.log(2)
    assert entropy_from_spectrum([0.0, 1.0, 1.0 + 1e-15, -1e-16]) == 0.0
    lam = np.array([0.1, 0.3, 0.75])
    ref = -(lam * np.log(lam) + (1 - lam) * np.log(1 - lam)).sum()
    assert abs(entropy_from_spectrum(lam) - ref) < 1e-15


def test_spectrum_identities_and_complement_pairing():
    U = _evolved()
    A = list(range(11))
    Ab = list(range(11, 32))
    la, lb = region_spectrum(U, A), region_spectrum(U, Ab)
    C = correlation_matrix(U)
    CA = C[np.ix_(A, A)]
    assert abs(la.sum() - np.trace(CA).real) < 1e-12
    assert abs((la ** 2).sum() - np.linalg.norm(CA) ** 2) < 1e-12
    assert la.min() > -1e-13 and la.max() < 1 + 1e-13
    # pure state: spectra of C_A and C_Abar agree on (0,1) after lambda -> 1 - lambda
    inner_a = np.sort(la[(la > 1e-9) & (la < 1 - 1e-9)])
    inner_b = np.sort(1 - lb[(lb > 1e-9) & (lb < 1 - 1e-9)])
    assert inner_a.size == inner_b.size and np.abs(inner_a - inner_b).max() < 1e-10


def test_entropy_bounds_and_mutual_information():
    U = _evolved(L=24, protocol=PROJECTIVE, gamma=1.0)
    for l in range(1, 24):
        s = entanglement_entropy(U, list(range(l)))
        assert -1e-14 <= s <= min(l, 24 - l) * np.log(2) + 1e-12
    A, B = list(range(0, 5)), list(range(10, 16))
    assert mutual_information(U, A, B) >= -1e-12


def test_mutual_information_matches_fock():
    lat = Lattice(1, 10)
    occ = default_occupied(lat)
    fs = FockSim(hopping_matrix(lat), occ)
    fs.set_evolution(0.05)
    from oracle.trajectory import step
    P = propagator(lat, 0.05)
    U = initial_state(10, occ)
    for n in range(1, 31):
        U, _ = step(U, P, HOMODYNE, 0.8, 0.05, 2, 4, n)
        fs.qsd_step(0.8, 0.05, 2, 4, n)
    A, B = [0, 1, 2], [5, 6, 8]
    ref = fs.entropy(A) + fs.entropy(B) - fs.entropy(sorted(A + B))
    assert abs(mutual_information(U, A, B) - ref) < 1e-10
    assert ref > 1e-3
