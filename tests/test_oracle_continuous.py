"""Pins of the continuous-time projective protocol of the oracle (Appendix A, PM protocol).

* Fock-space brute force with the same draws: the many-body state is evolved by
  exp(-i H tau) and multiplied by the projector n_j or 1 - n_j, and its correlation
  matrix (from operator matrix elements) equals the oracle's D after every event
  (L = 8 ring, 4 x 2 torus).
* The propagator from the eigendecomposition of H equals the plane-wave closed form
  for the same tau and obeys P(a) P(b) = P(a + b).
* Averaging the two outcomes with their Born weights gives the dephasing map at site j
  (D unchanged except that row and column j lose their off-diagonal entries); the
  printed minus sign of Eq. (A2) fails this.
* After every event D^2 = D, tr D = N, D_jj = outcome and row j is e_j or zero.
* An immediate second measurement of the same site repeats the first outcome.
* Waiting times: gamma N tau is Exp(1) (Kolmogorov-Smirnov, mean); sites are uniform.
* Stopping rule and the independence of the draws of event n from earlier events.
"""

import numpy as np
import pytest
from scipy import stats

from oracle import Lattice, hopping_matrix, default_occupied, initial_state, propagator
from oracle.continuous import (event_draws, waiting_time, evolution_operator, evolve,
                               measure_site, state_from_correlation, run_continuous)
from oracle.observables import correlation_matrix
from fock import FockSim
from dform import project_outcome0_as_printed


def _random_projector(L, N, seed):
    rng = np.random.default_rng(seed)
    Z = rng.normal(size=(L, N)) + 1j * rng.normal(size=(L, N))
    Q, _ = np.linalg.qr(Z)
    return Q @ np.conj(Q.T)


@pytest.mark.parametrize("lat,gamma,n_events", [(Lattice(1, 8), 0.8, 40),
                                                (Lattice(2, 4, 2), 1.3, 30)])
def test_events_match_fock_space(lat, gamma, n_events):
    occ = default_occupied(lat)
    fs = FockSim(hopping_matrix(lat), occ)
    U0 = initial_state(lat.L, occ)
    seed, uid = 11, 3
    out = run_continuous(lat, U0, gamma, seed, uid, n_events)
    # replay event by event against the many-body state
    H = hopping_matrix(lat)
    D = correlation_matrix(U0)
    N = len(occ)
    outcomes = set()
    for n in range(1, n_events + 1):
        tau, j, p, outcome = out["records"][n]
        _, j_draw, p_c = event_draws(seed, uid, n, lat.L)
        assert j == j_draw
        fs.evolve(tau)
        pf, of = fs.measure(j, p_c)
        assert abs(pf - p) < 1e-11 and of == outcome
        outcomes.add(outcome)
        D = evolve(D, H, tau)
        D, _, _ = measure_site(D, j, p_c)
        D = correlation_matrix(state_from_correlation(D, N))
        assert np.abs(fs.correlation() - D).max() < 1e-10
    assert outcomes == {0, 1}
    assert np.abs(out["D"] - D).max() < 1e-12


@pytest.mark.parametrize("lat", [Lattice(1, 12), Lattice(2, 4, 6)])
def test_evolution_operator_closed_form_and_group_law(lat):
    H = hopping_matrix(lat)
    for tau in (0.003, 0.7, 13.0):
        assert np.abs(evolution_operator(H, tau) - propagator(lat, tau)).max() < 1e-12
    a, b = 0.31, 1.27
    Pab = evolution_operator(H, a) @ evolution_operator(H, b)
    assert np.abs(Pab - evolution_operator(H, a + b)).max() < 1e-12


def test_outcome_average_is_dephasing():
    L, N = 10, 4
    D = _random_projector(L, N, 5)
    for j in range(L):
        p = D[j, j].real
        D1, p1, o1 = measure_site(D, j, 1e-300)      # p_c <= p: outcome 1
        D0, p0, o0 = measure_site(D, j, 1.0)         # p < 1 = p_c: outcome 0
        assert (o1, o0) == (1, 0) and p1 == p0 == p
        want = D.copy()
        want[j, :] = 0.0
        want[:, j] = 0.0
        want[j, j] = p
        assert np.abs(p * D1 + (1 - p) * D0 - want).max() < 1e-13
        # the printed minus sign of Eq. (A2) breaks the average (and D^2 = D)
        Dm = project_outcome0_as_printed(D, j)
        assert np.abs(p * D1 + (1 - p) * Dm - want).max() > 1e-3


def test_invariants_after_every_event():
    lat = Lattice(1, 16)
    occ = default_occupied(lat)
    H = hopping_matrix(lat)
    N = len(occ)
    D = correlation_matrix(initial_state(lat.L, occ))
    for n in range(1, 61):
        eta, j, p_c = event_draws(5, 9, n, lat.L)
        D = evolve(D, H, waiting_time(eta, 0.5, N))
        D, p, outcome = measure_site(D, j, p_c)
        U = state_from_correlation(D, N)
        assert np.abs(U.conj().T @ U - np.eye(N)).max() < 1e-12
        assert np.abs(U @ U.conj().T - D).max() < 1e-12
        assert np.abs(D @ D - D).max() < 1e-12
        assert abs(np.trace(D).real - N) < 1e-12
        assert D[j, j] == outcome
        assert np.abs(np.delete(D[j, :], j)).max() == 0.0
        D = U @ U.conj().T


def test_immediate_remeasurement_repeats():
    lat = Lattice(1, 4)
    occ = default_occupied(lat)
    out = run_continuous(lat, initial_state(4, occ), 1e9, 2, 7, 400)
    recs = [out["records"][n] for n in sorted(out["records"])]
    repeats = 0
    for (t0, j0, p0, o0), (t1, j1, p1, o1) in zip(recs, recs[1:]):
        assert t1 < 1e-7
        if j1 == j0:
            repeats += 1
            assert o1 == o0 and abs(p1 - o0) < 1e-12
    assert repeats > 50


def test_waiting_time_law_and_uniform_sites():
    L, N, gamma = 10, 5, 0.37
    n = np.arange(1, 20001)
    taus, sites = [], []
    for k in n:
        eta, j, _ = event_draws(8, 1, int(k), L)
        taus.append(waiting_time(eta, gamma, N))
        sites.append(j)
    x = gamma * N * np.asarray(taus)
    assert stats.kstest(x, "expon").pvalue > 1e-3
    assert abs(x.mean() - 1.0) < 4.0 / np.sqrt(len(x))
    counts = np.bincount(sites, minlength=L)
    assert counts.size == L and min(sites) >= 0 and max(sites) < L
    assert stats.chisquare(counts).pvalue > 1e-3


def test_stop_rule_and_event_indices():
    lat = Lattice(1, 12)
    U0 = initial_state(12, default_occupied(lat))
    full = run_continuous(lat, U0, 0.4, 3, 2, 200, t_end=1.5)
    keys = sorted(full["records"])
    assert keys == list(range(1, len(keys) + 1)) and len(keys) < 200
    t_last = sum(full["records"][k][0] for k in keys)
    assert abs(full["t"] - t_last) < 1e-12
    assert full["t"] >= 1.5 and full["t"] - full["records"][keys[-1]][0] < 1.5
    # two halves equal one run
    a = run_continuous(lat, U0, 0.4, 3, 2, 10)
    b = run_continuous(lat, a["U"], 0.4, 3, 2, 10, first_event=11, t0=a["t"])
    c = run_continuous(lat, U0, 0.4, 3, 2, 20)
    assert np.abs(b["D"] - c["D"]).max() < 1e-12 and abs(b["t"] - c["t"]) < 1e-12
