"""Pins of the oracle's correlation observables: C(r) of Eq. (2) and G_AB of Eq. (5).

* Fock-space brute force: the density covariance <n_i n_j> - <n_i><n_j> of the many-body
  state (computed from occupation bit strings, no Wick theorem) equals the Eq. (2) entry
  C_ij = -|C_ij|^2 for i != j, and -sum over A x B of it equals G_AB.
* Sum rule from C^2 = C: sum_{i != j} |C_ij|^2 = N - sum_i p_i^2, i.e. sum_r n_r C(r) =
  -(N - sum_i p_i^2) with n_r ordered pairs at ring distance r.
* Two sites: C(1) = -|a|^2 |b|^2 for the single orbital (a, b).
* G between a region and its complement is the number variance of the region,
  sum over the spectrum of C_A of l (1 - l).
* Product state: G_AB = 0 and C(r) = 0; symmetry G_AB = G_BA; additivity over a split of B.
"""

import numpy as np

from oracle import (Lattice, hopping_matrix, default_occupied, propagator, initial_state,
                    density_correlation, particle_covariance, correlation_matrix,
                    region_spectrum, born_probabilities)
from oracle.trajectory import step, PROJECTIVE, HOMODYNE
from fock import FockSim


def _evolved(L, protocol, gamma, n_steps, seed=3, uid=1):
    lat = Lattice(1, L)
    P = propagator(lat, 0.05)
    U = initial_state(L, default_occupied(lat))
    for n in range(1, n_steps + 1):
        U, _ = step(U, P, protocol, gamma, 0.05, seed, uid, n)
    return U


def test_density_covariance_matches_fock_space():
    L = 10
    lat = Lattice(1, L)
    occ = default_occupied(lat)
    fs = FockSim(hopping_matrix(lat), occ)
    fs.set_evolution(0.05)
    P = propagator(lat, 0.05)
    U = initial_state(L, occ)
    for n in range(1, 25):
        U, _ = step(U, P, HOMODYNE, 0.7, 0.05, 6, 2, n)
        fs.qsd_step(0.7, 0.05, 6, 2, n)
    w = np.abs(fs.psi) ** 2
    nn = (fs.occ * w[:, None]).T @ fs.occ   # <n_i n_j>
    n1 = w @ fs.occ
    cov = nn - np.outer(n1, n1)
    C = correlation_matrix(U)
    for i in range(L):
        for j in range(L):
            if i != j:
                assert abs(cov[i, j] - (-abs(C[i, j]) ** 2)) < 1e-11
    # C(r) as the average of the many-body covariance over pairs at ring distance r
    Cr = density_correlation(U)
    for r in range(1, L // 2 + 1):
        vals = [cov[i, j] for i in range(L) for j in range(L)
                if i != j and min(abs(i - j), L - abs(i - j)) == r]
        assert abs(Cr[r - 1] - np.mean(vals)) < 1e-11
    A, B = [0, 1, 2], [5, 7]
    assert abs(particle_covariance(U, A, B) + sum(cov[i, j] for i in A for j in B)) < 1e-11


def test_sum_rule():
    for protocol, gamma in ((PROJECTIVE, 2.0), (HOMODYNE, 1.0)):
        L = 24
        U = _evolved(L, protocol, gamma, 30)
        Cr = density_correlation(U)
        n_r = np.array([2 * L] * (L // 2 - 1) + [L], dtype=float)
        p = born_probabilities(U)
        assert abs((n_r * Cr).sum() + (L // 2 - (p ** 2).sum())) < 1e-10
        assert (Cr <= 1e-15).all()


def test_two_site_closed_form():
    rng = np.random.default_rng(0)
    z = rng.normal(size=2) + 1j * rng.normal(size=2)
    z /= np.linalg.norm(z)
    U = z[:, None]
    assert abs(density_correlation(U)[0] + abs(z[0]) ** 2 * abs(z[1]) ** 2) < 1e-15


def test_region_number_variance():
    L = 20
    U = _evolved(L, HOMODYNE, 1.5, 40)
    for A in (list(range(7)), [0, 3, 4, 9, 15]):
        comp = [i for i in range(L) if i not in A]
        lam = region_spectrum(U, A)
        assert abs(particle_covariance(U, A, comp) - float((lam * (1 - lam)).sum())) < 1e-11


def test_product_state_symmetry_additivity():
    L = 16
    lat = Lattice(1, L)
    U0 = initial_state(L, default_occupied(lat))
    assert particle_covariance(U0, [0, 1, 2], [8, 9]) == 0.0
    assert np.abs(density_correlation(U0)).max() == 0.0
    U = _evolved(L, PROJECTIVE, 1.0, 20)
    A, B1, B2 = [0, 2, 5], [8, 9], [12, 14, 15]
    g = particle_covariance(U, A, B1 + B2)
    assert abs(g - particle_covariance(U, B1 + B2, A)) < 1e-14
    assert abs(g - particle_covariance(U, A, B1) - particle_covariance(U, A, B2)) < 1e-14
