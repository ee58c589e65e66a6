"""Ensemble pins: exact mean maps of the projective protocol (discrete and continuous time) and
the dephasing limit of the homodyne protocol, plus planted mistakes that these pins must catch."""

import numpy as np
import pytest
from scipy import linalg

import oracle.trajectory as tr
from oracle import Lattice, hopping_matrix, propagator, default_occupied, initial_state, correlation_matrix


def _ensemble(lat, protocol, gamma, dt, n_steps, n_traj, seed=5):
    P = propagator(lat, dt)
    occ = default_occupied(lat)
    Cs = []
    for uid in range(n_traj):
        U = initial_state(lat.L, occ)
        for n in range(1, n_steps + 1):
            U, _ = tr.step(U, P, protocol, gamma, dt, seed, uid, n)
        Cs.append(correlation_matrix(U))
    Cs = np.array(Cs)
    se = (Cs.real.std(axis=0, ddof=1) + 1j * Cs.imag.std(axis=0, ddof=1)) / np.sqrt(n_traj)
    return Cs.mean(axis=0), se


def _z(mean, se, ref):
    # entries that vanish by symmetry in every trajectory have se ~ 0; floor it
    zr = np.abs(mean.real - ref.real) / np.maximum(se.real, 1e-10)
    zi = np.abs(mean.imag - ref.imag) / np.maximum(se.imag, 1e-10)
    return max(zr.max(), zi.max())


def pm_mean_map(lat, gamma, dt, n_steps):
    """Outcome-averaged projection is a martingale that zeroes row/column j off the
    diagonal; with independent selection (prob q) E[C'] = M o (P E[C] P^+),
    M_aa = 1, M_ab = (1-q)^2 (Appendix A updates averaged over the Born rule)."""
    P = propagator(lat, dt)
    q = min(gamma * dt, 1.0)
    M = np.full((lat.L, lat.L), (1 - q) ** 2)
    np.fill_diagonal(M, 1.0)
    C = correlation_matrix(initial_state(lat.L, default_occupied(lat)))
    for _ in range(n_steps):
        C = M * (P @ C @ np.conj(P.T))
    return C


def lindblad(lat, gamma, t):
    """dC/dt = -i[Ht, C] - gamma (C - diag C): mean dynamics of continuous monitoring of
    every n_i at rate gamma (the unravelling that Eq. (A4) implements)."""
    H = hopping_matrix(lat)
    L = lat.L
    I = np.eye(L)
    # vec(C) column-stacked: vec(H C) = (I kron H) vec C, vec(C H) = (H^T kron I) vec C
    G = -1j * (np.kron(I, H) - np.kron(H.T, I))
    offdiag = 1.0 - np.eye(L).ravel(order="F")
    G = G - gamma * np.diag(offdiag)
    C0 = correlation_matrix(initial_state(L, default_occupied(lat)))
    v = linalg.expm(G * t) @ C0.ravel(order="F")
    return v.reshape((L, L), order="F")


def ct_mean_map(lat, gamma, N, n_events):
    """Mean of C after n events of the continuous-time projective protocol.  Averaging one event
    over the waiting time tau ~ gamma N exp(-gamma N tau) maps the energy-basis entries X_ab of C
    to K_ab X_ab with K_ab = G / (G + i (e_a - e_b)), G = gamma N (the Laplace transform of
    exp(-i (e_a - e_b) tau)); averaging over the uniform site j and its Born outcome removes row
    and column j off the diagonal (the outcome-weighted mean of Eq. (A1) and Eq. (A2)), i.e.
    multiplies every off-diagonal entry by 1 - 2/L.  Both maps are linear, so
    E[C_n] = (M o R)^n (C_0)."""
    H = hopping_matrix(lat)
    eps, V = np.linalg.eigh(H)
    G = gamma * N
    K = G / (G + 1j * (eps[:, None] - eps[None, :]))
    L = lat.L
    M = np.full((L, L), 1.0 - 2.0 / L)
    np.fill_diagonal(M, 1.0)
    C = correlation_matrix(initial_state(L, default_occupied(lat)))
    for _ in range(n_events):
        C = M * (V @ (K * (V.T @ C @ V)) @ V.T)
    return C


def _ct_ensemble(lat, gamma, n_events, n_traj, seed=3):
    from oracle.continuous import run_continuous
    U0 = initial_state(lat.L, default_occupied(lat))
    Cs = np.array([correlation_matrix(run_continuous(lat, U0, gamma, seed, uid, n_events)["U"])
                   for uid in range(n_traj)])
    se = (Cs.real.std(axis=0, ddof=1) + 1j * Cs.imag.std(axis=0, ddof=1)) / np.sqrt(n_traj)
    return Cs.mean(axis=0), se


@pytest.mark.slow
def test_continuous_time_mean_map():
    lat = Lattice(1, 6)
    mean, se = _ct_ensemble(lat, 1.0, 4, 3000)
    assert _z(mean, se, ct_mean_map(lat, 1.0, 3, 4)) < 4.5
    # a total rate gamma L instead of gamma N (the other reading of the rate) is a different law
    assert _z(mean, se, ct_mean_map(lat, 2.0, 3, 4)) > 6


@pytest.mark.slow
def test_projective_mean_map():
    lat = Lattice(1, 8)
    mean, se = _ensemble(lat, tr.PROJECTIVE, 4.0, 0.05, 10, 600)
    ref = pm_mean_map(lat, 4.0, 0.05, 10)
    assert _z(mean, se, ref) < 4.5


@pytest.mark.slow
def test_homodyne_dephasing_limit():
    lat = Lattice(1, 8)
    dt, n = 0.01, 60
    mean, se = _ensemble(lat, tr.HOMODYNE, 1.0, dt, n, 600)
    ref = lindblad(lat, 1.0, n * dt)
    # O(gamma dt) discretisation bias is far below the statistical error here
    assert _z(mean, se, ref) < 4.5


@pytest.mark.slow
def test_planted_wrong_drift_sign_is_caught(monkeypatch):
    orig = tr.qsd_update

    def wrong(U, gamma, dt, seed, uid, n):
        p = tr.born_probabilities(U)
        xi = np.sqrt(gamma * dt) * tr.qsd_normals(seed, uid, n, U.shape[0])
        return np.exp(xi - gamma * (2.0 * p - 1.0) * dt)[:, None] * U

    monkeypatch.setattr(tr, "qsd_update", wrong)
    lat = Lattice(1, 8)
    mean, se = _ensemble(lat, tr.HOMODYNE, 1.0, 0.01, 60, 600)
    assert _z(mean, se, lindblad(lat, 1.0, 0.6)) > 6
    monkeypatch.setattr(tr, "qsd_update", orig)


@pytest.mark.slow
def test_planted_inverted_born_rule_is_caught(monkeypatch):
    orig = tr.pm_uniforms

    def flipped(seed, uid, n, L):
        a, b = orig(seed, uid, n, L)
        return a, 1.0 - b  # outcome 1 iff u > 1 - p: same law, must still pass

    monkeypatch.setattr(tr, "pm_uniforms", flipped)
    lat = Lattice(1, 8)
    mean, se = _ensemble(lat, tr.PROJECTIVE, 4.0, 0.05, 10, 600)
    assert _z(mean, se, pm_mean_map(lat, 4.0, 0.05, 10)) < 4.5

    def wrong_rule(seed, uid, n, L):
        a, b = orig(seed, uid, n, L)
        return a, np.full(L, 0.5)  # outcome decided by p >= 1/2: not the Born rule

    monkeypatch.setattr(tr, "pm_uniforms", wrong_rule)
    mean, se = _ensemble(lat, tr.PROJECTIVE, 4.0, 0.05, 10, 600)
    assert _z(mean, se, pm_mean_map(lat, 4.0, 0.05, 10)) > 6


def test_planted_conjugated_propagator_is_caught():
    """Entropies cannot see P -> conj(P); the free closed form of C does."""
    from test_oracle_dynamics import neel_free_closed_form
    lat = Lattice(1, 16)
    P = np.conj(propagator(lat, 0.05))
    U = initial_state(16, default_occupied(lat))
    for _ in range(20):
        U = P @ U
    err = np.abs(correlation_matrix(U) - neel_free_closed_form(lat, 1.0)).max()
    assert err > 1e-2
