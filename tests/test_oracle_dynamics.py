"""Physics pins for the oracle's trajectory step (projective and homodyne)."""

import numpy as np
import pytest

import oracle
from oracle import (Lattice, hopping_matrix, propagator, default_occupied, initial_state,
                    correlation_matrix, entanglement_entropy, run_trajectory)
from oracle.trajectory import PROJECTIVE, HOMODYNE, propagate, pm_measure, reorthonormalize, step
from fock import FockSim
import dform


def neel_free_closed_form(lat, t):
    """C(t) = P C0 P^+ for the Neel / checkerboard start, from the plane-wave closed form:
    C_ab = 1/2 delta_ab + 1/2 s_a (1/L) sum_k e^{ik(r_a - r_b)} e^{2 i eps_k t},
    s_a = (-1)^(x_a + y_a), eps_k = 2J(cos kx + cos ky); uses eps_{k+(pi,pi)} = -eps_k."""
    L = lat.L
    xs = np.array([i % lat.Lx for i in range(L)])
    ys = np.array([i // lat.Lx for i in range(L)])
    kx = 2 * np.pi * np.arange(lat.Lx) / lat.Lx
    if lat.dim == 1:
        K = [(k, 0.0) for k in kx]
    else:
        ky = 2 * np.pi * np.arange(lat.Ly) / lat.Ly
        K = [(a, b) for a in kx for b in ky]
    C = 0.5 * np.eye(L, dtype=np.complex128)
    dx = xs[:, None] - xs[None, :]
    dy = ys[:, None] - ys[None, :]
    acc = np.zeros((L, L), dtype=np.complex128)
    for (a, b) in K:
        eps = 2 * lat.J * (np.cos(a) + (np.cos(b) if lat.dim == 2 else 0.0))
        acc += np.exp(1j * (a * dx + b * dy)) * np.exp(2j * eps * t)
    s = (-1.0) ** (xs + ys)
    return C + 0.5 * s[:, None] * acc / L


def neel_free_entries(lat, t, a, b):
    """Entries C_ab(t) of neel_free_closed_form for site lists a, b, at any lattice size: the
    sum over k factorises, (1/L) sum_k e^{ik(r_a - r_b)} e^{2 i eps_k t} = f_x(dx) f_y(dy) with
    f(d) = (1/Lr) sum_m e^{i k_m d} e^{4 i J t cos k_m} on a ring of Lr sites (f_y = 1 in 1d)."""
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)

    def ring_table(Lr):
        m = np.arange(Lr)
        k = 2 * np.pi * m / Lr
        md = np.outer(np.arange(Lr), m) % Lr  # m d reduced first: accurate phases
        return (np.exp(2j * np.pi * md / Lr) * np.exp(4j * lat.J * t * np.cos(k))[None, :]).sum(axis=1) / Lr

    xa, ya, xb, yb = a % lat.Lx, a // lat.Lx, b % lat.Lx, b // lat.Lx
    val = ring_table(lat.Lx)[(xa - xb) % lat.Lx]
    if lat.dim == 2:
        val = val * ring_table(lat.Ly)[(ya - yb) % lat.Ly]
    s = (-1.0) ** (xa + ya)
    return 0.5 * (a == b) + 0.5 * s * val


@pytest.mark.parametrize("lat", [Lattice(1, 64), Lattice(2, 8, 6), Lattice(2, 10, 4)])
def test_free_entries_equal_full_closed_form(lat):
    t = 1.3
    C = neel_free_closed_form(lat, t)
    a, b = np.meshgrid(np.arange(lat.L), np.arange(lat.L), indexing="ij")
    E = neel_free_entries(lat, t, a.ravel(), b.ravel()).reshape(lat.L, lat.L)
    assert np.abs(E - C).max() < 1e-13


@pytest.mark.parametrize("lat", [Lattice(1, 64), Lattice(2, 8, 6)])
@pytest.mark.parametrize("protocol", [PROJECTIVE, HOMODYNE])
def test_free_evolution_closed_form(lat, protocol):
    dt, n = 0.05, 40
    P = propagator(lat, dt)
    out = run_trajectory(P, default_occupied(lat), protocol, 0.0, dt, 0, 0, n)
    C = correlation_matrix(out["U"])
    assert np.abs(C - neel_free_closed_form(lat, n * dt)).max() < 1e-12


def test_free_evolution_bessel_diagonal():
    # diagonal -> 1/2 + 1/2 (-1)^a J0(4Jt) while 4Jt << L
    from scipy import special
    lat = Lattice(1, 256)
    t = 3.7
    C = neel_free_closed_form(lat, t)
    ref = 0.5 + 0.5 * (-1.0) ** np.arange(256) * special.j0(4 * t)
    assert np.abs(np.diag(C).real - ref).max() < 1e-13


def _check_invariants(U, N, tol=1e-12):
    C = correlation_matrix(U)
    assert np.abs(C - np.conj(C.T)).max() < tol
    assert np.abs(C @ C - C).max() < tol
    assert abs(np.trace(C).real - N) < tol
    assert np.abs(np.conj(U.T) @ U - np.eye(N)).max() < tol
    lam = np.linalg.eigvalsh(C)
    assert lam.min() > -tol and lam.max() < 1 + tol


@pytest.mark.parametrize("protocol,gamma", [(PROJECTIVE, 2.0), (HOMODYNE, 1.0)])
def test_invariants_along_trajectory(protocol, gamma):
    lat = Lattice(1, 32)
    P = propagator(lat, 0.05)
    U = initial_state(32, default_occupied(lat))
    for n in range(1, 60):
        U, _ = step(U, P, protocol, gamma, 0.05, 3, 7, n)
        _check_invariants(U, 16)


@pytest.mark.parametrize("lat", [Lattice(1, 16), Lattice(2, 4, 4)])
def test_all_site_projection_gives_zero_entropy(lat):
    # gamma*dt >= 1: every site is measured every step -> product state
    P = propagator(lat, 0.05)
    U = initial_state(lat.L, default_occupied(lat))
    for n in range(1, 6):
        U, ev = step(U, P, PROJECTIVE, 25.0, 0.05, 0, 1, n)
        assert [e[0] for e in ev] == list(range(lat.L))
        assert sum(e[2] for e in ev) == lat.L // 2
        C = correlation_matrix(U)
        assert np.abs(C - np.diag(np.round(np.diag(C).real))).max() < 1e-12
        for region in ([0, 1, 2], list(range(lat.L // 2)), [1, 5, 6, 9]):
            assert abs(entanglement_entropy(U, region)) < 1e-10


def test_projection_matches_dform_updates():
    """Each U-form projection reproduces Eq. (A1) / sign-fixed Eq. (A2) on C."""
    lat = Lattice(1, 24)
    P = propagator(lat, 0.05)
    U = initial_state(24, default_occupied(lat))
    n_events = [0, 0]
    for n in range(1, 80):
        U = propagate(U, P)
        C = correlation_matrix(U)
        Un, events = pm_measure(U, 3.0, 0.05, 11, 2, n)
        for (j, p, outcome) in events:
            assert abs(C[j, j].real - p) < 1e-13
            C = dform.project_outcome1(C, j) if outcome == 1 else dform.project_outcome0(C, j)
            n_events[outcome] += 1
        assert np.abs(C - correlation_matrix(Un)).max() < 1e-12
        U = reorthonormalize(Un)
    assert min(n_events) > 10


def test_printed_sign_of_A2_is_not_a_projection():
    # two sites, one particle in (|10> + |01>)/sqrt2: outcome 0 on site 0 must give C_11 = 1
    U = np.array([[1.0], [1.0]], dtype=np.complex128) / np.sqrt(2)
    C = correlation_matrix(U)
    good = dform.project_outcome0(C, 0)
    bad = dform.project_outcome0_as_printed(C, 0)
    assert abs(good[1, 1] - 1.0) < 1e-15
    assert abs(bad[1, 1] - 0.0) < 1e-15
    assert np.abs(good @ good - good).max() < 1e-15
    assert abs(np.trace(bad).real) < 1e-15  # the printed sign loses the particle (Tr C = 0, not 1)


def _brute_force_compare(lat, protocol, gamma, n_steps, seed, uid, dt=0.05):
    L = lat.L
    occ = default_occupied(lat)
    H = hopping_matrix(lat)
    P = propagator(lat, dt)
    fs = FockSim(H, occ)
    fs.set_evolution(dt)
    U = initial_state(L, occ)
    regions = [list(range(L // 2)), [0], [1, 2, 5], list(range(1, L - 1, 2))]
    n_ev = 0
    for n in range(1, n_steps + 1):
        U, ev = step(U, P, protocol, gamma, dt, seed, uid, n)
        if protocol == PROJECTIVE:
            ev_f = fs.pm_step(gamma, dt, seed, uid, n)
            assert [(e[0], e[2]) for e in ev] == [(e[0], e[2]) for e in ev_f]
            for a, b in zip(ev, ev_f):
                assert abs(a[1] - b[1]) < 1e-12
            n_ev += len(ev)
        else:
            fs.qsd_step(gamma, dt, seed, uid, n)
        assert np.abs(np.diag(correlation_matrix(U)).real - fs.occupations()).max() < 1e-12
        if n % 5 == 0:
            assert np.abs(correlation_matrix(U) - fs.correlation()).max() < 1e-11
        for r in regions:
            assert abs(entanglement_entropy(U, r) - fs.entropy(r)) < 1e-10
    return n_ev


@pytest.mark.parametrize("L,seed", [(6, 0), (8, 1), (10, 2)])
def test_brute_force_projective_1d(L, seed):
    n_ev = _brute_force_compare(Lattice(1, L), PROJECTIVE, 4.0, 20, seed, 5)
    assert n_ev >= 10


@pytest.mark.parametrize("L,seed", [(6, 0), (8, 1), (10, 2)])
def test_brute_force_homodyne_1d(L, seed):
    _brute_force_compare(Lattice(1, L), HOMODYNE, 1.0, 20, seed, 5)


def test_brute_force_2d():
    lat = Lattice(2, 4, 2)
    assert _brute_force_compare(lat, PROJECTIVE, 4.0, 15, 3, 1) > 5
    _brute_force_compare(lat, HOMODYNE, 1.5, 15, 3, 1)


def test_sublattice_sign_flip_and_conjugation_invariance():
    """J -> -J (sublattice gauge) and P -> conj(P) leave every S and outcome unchanged."""
    for protocol, gamma in ((PROJECTIVE, 2.0), (HOMODYNE, 0.7)):
        outs = []
        for J, conj in ((1.0, False), (-1.0, False), (1.0, True)):
            lat = Lattice(1, 20, 1, J)
            P = propagator(lat, 0.05)
            if conj:
                P = np.conj(P)
            outs.append(run_trajectory(P, default_occupied(lat), protocol, gamma, 0.05, 4, 9, 50,
                                       obs_every=5, regions=[list(range(10)), [0, 3, 4, 11]]))
        for o in outs[1:]:
            for n in outs[0]["S"]:
                assert np.allclose(outs[0]["S"][n], o["S"][n], atol=1e-11, rtol=0)
            assert ([(e[0], e[2]) for v in outs[0]["events"].values() for e in v]
                    == [(e[0], e[2]) for v in o["events"].values() for e in v])


def test_pure_state_complement_symmetry():
    lat = Lattice(1, 40)
    P = propagator(lat, 0.05)
    out = run_trajectory(P, default_occupied(lat), HOMODYNE, 0.5, 0.05, 0, 3, 100)
    U = out["U"]
    A = [0, 1, 2, 3, 10, 11, 12, 30]
    Ab = [i for i in range(40) if i not in A]
    assert abs(entanglement_entropy(U, A) - entanglement_entropy(U, Ab)) < 1e-11
    assert abs(entanglement_entropy(U, list(range(20))) - entanglement_entropy(U, list(range(20, 40)))) < 1e-11


def test_reorthonormalize_keeps_C_and_fixes_gauge():
    rng = np.random.default_rng(0)
    A = rng.normal(size=(30, 12)) + 1j * rng.normal(size=(30, 12))
    Q = reorthonormalize(A)
    assert np.abs(np.conj(Q.T) @ Q - np.eye(12)).max() < 1e-14
    R = np.conj(Q.T) @ A
    assert np.abs(np.tril(R, -1)).max() < 1e-13
    assert np.all(np.diag(R).real > 0) and np.abs(np.diag(R).imag).max() < 1e-13
    Q2 = reorthonormalize(Q)
    assert np.abs(Q2 @ np.conj(Q2.T) - Q @ np.conj(Q.T)).max() < 1e-14
