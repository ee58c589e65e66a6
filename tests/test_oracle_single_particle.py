"""Hand-worked single-particle examples of one projective measurement (Appendix A, Eq. (A1) and
Eq. (A2) with the sign fixed), pinning both oracle forms of the projection: the Slater
determinant form (Householder projection of U) and the correlation-matrix form (D updates).

One particle in the state u (a unit column) has C = u u^+.  Measuring site j:
  outcome 1 (probability |u_j|^2) leaves the particle on j: C' = e_j e_j^+;
  outcome 0 leaves u with entry j removed and renormalised: C'_ab = u_a conj(u_b) / (1 - |u_j|^2)
  for a, b != j, and zero in row and column j.
The paper prints no worked example with numbers (its printed values are fit parameters of large
ensembles), so these closed forms, derived by hand, serve instead.
"""
import numpy as np
import pytest

from oracle.continuous import measure_site
from oracle.trajectory import _project_site


def _corr(U):
    return U @ U.conj().T


def _after(u, j, outcome):
    """Closed form of C after measuring site j with the given outcome (one particle)."""
    L = u.shape[0]
    if outcome == 1:
        C = np.zeros((L, L), complex)
        C[j, j] = 1.0
        return C
    w = u.copy()
    w[j] = 0.0
    w /= np.sqrt(1.0 - abs(u[j]) ** 2)
    return np.outer(w, w.conj())


def test_two_sites_symmetric_state():
    # u = (1, 1)/sqrt 2: p_0 = 1/2; outcome 0 on site 0 must put the particle on site 1
    u = np.array([1.0, 1.0], complex) / np.sqrt(2.0)
    D = np.outer(u, u.conj())
    D1, p, o = measure_site(D, 0, 0.0)  # u_out = 0 <= p: outcome 1
    assert o == 1 and abs(p - 0.5) < 1e-15
    assert np.abs(D1 - np.diag([1.0, 0.0])).max() < 1e-15
    D0, p, o = measure_site(D, 0, 1.0)  # u_out = 1 > p: outcome 0
    assert o == 0 and abs(p - 0.5) < 1e-15
    assert np.abs(D0 - np.diag([0.0, 1.0])).max() < 1e-15  # the printed sign of Eq. (A2) gives 0
    for outcome, ref in ((1, np.diag([1.0, 0.0])), (0, np.diag([0.0, 1.0]))):
        U = _project_site(u[:, None].copy(), 0, outcome)
        assert np.abs(_corr(U) - ref).max() < 1e-15


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("L", [2, 3, 5])
def test_one_particle_any_state(seed, L):
    rng = np.random.default_rng(seed)
    u = rng.normal(size=L) + 1j * rng.normal(size=L)
    u /= np.linalg.norm(u)
    D = np.outer(u, u.conj())
    for j in range(L):
        p = abs(u[j]) ** 2
        for outcome, p_c in ((1, 0.0), (0, 1.0)):
            ref = _after(u, j, outcome)
            Dn, pd, od = measure_site(D, j, p_c)
            assert od == outcome and abs(pd - p) < 1e-14
            assert np.abs(Dn - ref).max() < 1e-13, (j, outcome)
            U = _project_site(u[:, None].copy(), j, outcome)
            assert np.abs(_corr(U) - ref).max() < 1e-13, (j, outcome)
            assert abs(np.trace(Dn).real - 1.0) < 1e-13  # one particle before and after


def test_two_particles_product_of_sites():
    # particles on sites 0 and 2 of three (u = e_0, e_2): measuring site 1 gives outcome 0 with
    # probability 1 and changes nothing; measuring site 0 gives outcome 1 and changes nothing
    U = np.zeros((3, 2), complex)
    U[0, 0] = 1.0
    U[2, 1] = 1.0
    D = _corr(U)
    D1, p, o = measure_site(D, 1, 0.5)
    assert o == 0 and p == 0.0 and np.abs(D1 - D).max() == 0.0
    D0, p, o = measure_site(D, 0, 0.5)
    assert o == 1 and p == 1.0 and np.abs(D0 - D).max() == 0.0
    assert np.abs(_corr(_project_site(U.copy(), 1, 0)) - D).max() < 1e-15
