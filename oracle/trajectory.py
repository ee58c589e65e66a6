"""One quantum trajectory of the Gaussian (Slater-determinant) state (oracle).

TEST INFRASTRUCTURE.  State (Appendix A, wavefunction equation): an L x N
complex matrix U with U^+ U = 1; the correlation matrix is C = U U^+ (the
paper's D is its transpose, same spectrum).

A step n = 1, 2, ... does, in this order (the paper does not fix the order
inside a step; this reading is shared with the GPU library):

1. propagate      U <- P U                               (Appendix A)
2. Born probs     p_i = sum_k |U_ik|^2                   (Appendix A, <n_i>)
3a. projective    each site i measured iff u_sel(i) < min(gamma dt, 1); the
                  measured sites are projected one after another in ascending
                  order, each with its conditional Born probability
                  p = sum_k |U_ik|^2 of the current U; outcome 1 iff
                  u_out(i) <= p (Appendix A: "p_j >= p_c").  The projection
                  is done exactly on U (a Householder reflector that confines
                  row j to column 0, then column 0 := e_j for outcome 1, or
                  row j of column 0 zeroed and column 0 renormalised for
                  outcome 0); it reproduces Eq. (A1) and the sign-corrected
                  Eq. (A2) on C.
3b. homodyne      row i of U scaled by exp(xi_i + gamma (2 p_i - 1) dt) with
                  xi_i = sqrt(gamma dt) z_i, z_i ~ N(0,1)   (Eq. (A4), split
                  step: the diagonal factor is applied after the propagator
                  and uses p of the propagated U)
4. re-orthonormalise by Householder QR with a positive diagonal of R
                  (Appendix A: "QR decomposition" after each step).

Pinned by: Fock-space brute force with the same draws (L <= 10), the D-form
updates Eq. (A1)/(A2), the free-evolution closed form, the exact mean map of
the projective protocol and the dephasing (Lindblad) limit of the homodyne
protocol (tests/test_oracle_*.py).
"""

import numpy as np

from .philox import pm_uniforms, qsd_normals
from .observables import entanglement_entropy

PROJECTIVE = 0
HOMODYNE = 1


def initial_state(L, occupied):
    """U[:, k] = e_{occupied[k]} (occupied ascending)."""
    U = np.zeros((L, len(occupied)), dtype=np.complex128)
    for k, o in enumerate(occupied):
        U[o, k] = 1.0
    return U


def propagate(U, P):
    return P @ U


def born_probabilities(U):
    """p_i = <n_i> = sum_k |U_ik|^2 (Appendix A)."""
    return (U.real ** 2 + U.imag ** 2).sum(axis=1)


def _project_site(U, j, outcome):
    """Exact projection of the Slater determinant U onto n_j = outcome."""
    x = np.conj(U[j, :])
    nx = np.linalg.norm(x)
    if nx == 0.0:
        # row j empty: p_j = 0, only outcome 0 is possible and it is the identity
        return U
    ph = x[0] / abs(x[0]) if x[0] != 0 else 1.0
    beta = -ph * nx
    v = x.copy()
    v[0] -= beta
    # H = I - 2 v v^+ / (v^+ v) is Hermitian unitary with H x = beta e_0,
    # hence row j of U H is conj(beta) e_0^T.
    U = U - (U @ v)[:, None] * (2.0 / np.vdot(v, v).real) * np.conj(v)[None, :]
    U[j, 1:] = 0.0
    if outcome == 1:
        U[:, 0] = 0.0
        U[j, 0] = 1.0
    else:
        U[j, 0] = 0.0
        U[:, 0] /= np.linalg.norm(U[:, 0])
    return U


def pm_measure(U, gamma, dt, seed, uid, n):
    """Projective measurements of step n.  Returns (U, [(site, p, outcome), ...])."""
    L = U.shape[0]
    u_sel, u_out = pm_uniforms(seed, uid, n, L)
    q = min(gamma * dt, 1.0)
    events = []
    for j in range(L):
        if u_sel[j] < q:
            p = float((U[j, :].real ** 2 + U[j, :].imag ** 2).sum())
            outcome = 1 if u_out[j] <= p else 0
            U = _project_site(U, j, outcome)
            events.append((j, p, outcome))
    return U, events


def qsd_update(U, gamma, dt, seed, uid, n):
    """Homodyne diagonal factor of step n (Eq. (A4), split step)."""
    L = U.shape[0]
    p = born_probabilities(U)
    xi = np.sqrt(gamma * dt) * qsd_normals(seed, uid, n, L)
    f = np.exp(xi + gamma * (2.0 * p - 1.0) * dt)
    return f[:, None] * U


def reorthonormalize(U):
    """Householder QR (LAPACK via numpy), phases fixed so that diag(R) > 0."""
    Q, R = np.linalg.qr(U)
    d = np.diag(R)
    ph = np.where(d != 0, d / np.abs(d), 1.0)
    return Q * ph[None, :]


def step(U, P, protocol, gamma, dt, seed, uid, n):
    """Advance by one step (n is the 1-based index of the step being taken)."""
    U = propagate(U, P)
    events = []
    if protocol == PROJECTIVE:
        U, events = pm_measure(U, gamma, dt, seed, uid, n)
    else:
        U = qsd_update(U, gamma, dt, seed, uid, n)
    U = reorthonormalize(U)
    return U, events


def run_trajectory(P, occupied, protocol, gamma, dt, seed, uid, n_steps,
                   obs_every=0, regions=(), U0=None, first_step=1):
    """Run n_steps steps; observe S for each region at step 0 and every obs_every.

    Returns dict(U=final U, S={step: [S per region]}, events={step: events}).
    """
    L = P.shape[0]
    U = initial_state(L, occupied) if U0 is None else U0.copy()
    out = {"S": {}, "events": {}}
    if obs_every and first_step == 1:
        out["S"][0] = [entanglement_entropy(U, r) for r in regions]
    for n in range(first_step, first_step + n_steps):
        U, ev = step(U, P, protocol, gamma, dt, seed, uid, n)
        out["events"][n] = ev
        if obs_every and n % obs_every == 0:
            out["S"][n] = [entanglement_entropy(U, r) for r in regions]
    out["U"] = U
    return out
