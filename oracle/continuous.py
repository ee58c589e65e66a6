"""Continuous-time projective monitoring (Appendix A, PM protocol) -- oracle.

TEST INFRASTRUCTURE.  The protocol is taken in the paper's order, one event
at a time, on the L x L correlation matrix D:

1. waiting time   tau = -ln(eta) / (gamma N), eta uniform in (0, 1], N the
                  particle number (the printed formula lacks the minus sign;
                  ln(eta) <= 0, so the sign is restored; the total event rate
                  is gamma N as printed);
2. evolution      D <- exp(-i H tau) D exp(i H tau);
3. measurement    site j uniform over the L sites, p_j = D_jj, p_c uniform;
                  outcome 1 iff p_c <= p_j; Eq. (A1) for outcome 1 and
                  Eq. (A2) for outcome 0, whose rank-1 term enters with a plus
                  sign (the printed minus sign breaks D^2 = D);
4. state          the orthonormal U rebuilt from D: D = U S U^+ with
                  S = diag(1 .. 1, 0 .. 0) (for the Hermitian projector D this
                  decomposition is its eigendecomposition; U = the eigenvectors
                  of the N largest eigenvalues).
The clock t advances by tau at every event; a trajectory takes events while
t < t_end (the paper stops once t >= L/2).

Reading of the notation: the printed evolution exp(-iH tau) D exp(iH tau) is
that of C_ab = <c_b^+ c_a> = (U U^+)_ab, and Eqs. (A1)/(A2) keep their form
under transposition, so D here is C = U U^+ (the transpose of <c_a^+ c_b>).

Random numbers (a choice of this library): Philox4x64-10 with key
(seed, uid) and counter (n, 0, 2, 0) for event n = 1, 2, ... of a trajectory:
word 0 -> eta = u01(word 0), word 1 -> j = floor(word 1 * L / 2^64) (the high
64 bits of the 128-bit product, exact in integers), word 2 -> p_c = u01(word 2).

exp(-i H tau) comes from the eigendecomposition of the hopping matrix (LAPACK
eigh as a library primitive), valid for every tau.

Pinned by (tests/test_oracle_continuous.py): Fock-space brute force with the
same draws (many-body evolution and projection, L = 8 ring and 4 x 2 torus);
the plane-wave closed form of the propagator and its group law; the exact
mean of the two outcomes (the dephasing map at site j, which the printed sign
of Eq. (A2) violates); idempotency and trace after every event; repeatability
of an immediate second measurement of the same site; the exponential law of
the waiting times (mean 1/(gamma N), Kolmogorov-Smirnov) and the uniformity of
the selected sites; the stopping rule.
"""

import numpy as np

from .lattice import hopping_matrix
from .philox import philox4x64_10, u01, _mulhilo
from .observables import correlation_matrix

PURPOSE_CONTINUOUS = 2


def event_draws(seed, uid, n, L):
    """(eta, j, p_c) of event n of trajectory uid."""
    w = philox4x64_10(seed, uid, n, 0, PURPOSE_CONTINUOUS, 0)
    eta = float(u01(w[0]))
    hi, _ = _mulhilo(np.asarray(w[1], dtype=np.uint64), np.uint64(L))
    return eta, int(hi), float(u01(w[2]))


def waiting_time(eta, gamma, N):
    """Step 1: tau = -ln(eta) / (gamma N)."""
    return -np.log(eta) / (gamma * N)


def evolution_operator(H, tau):
    """exp(-i H tau) for the real symmetric hopping matrix H."""
    eps, V = np.linalg.eigh(H)
    return (V * np.exp(-1j * eps * tau)[None, :]) @ V.T


def evolve(D, H, tau):
    """Step 2: D <- exp(-i H tau) D exp(i H tau)."""
    P = evolution_operator(H, tau)
    return P @ D @ np.conj(P.T)


def measure_site(D, j, p_c):
    """Step 3: Born rule p_j = D_jj, outcome 1 iff p_c <= p_j, then Eq. (A1) / Eq. (A2)."""
    p = float(D[j, j].real)
    outcome = 1 if p_c <= p else 0
    L = D.shape[0]
    Dn = np.empty_like(D)
    for a in range(L):
        for b in range(L):
            if outcome == 1:
                if a == j and b == j:
                    Dn[a, b] = 1.0
                elif a == j or b == j:
                    Dn[a, b] = 0.0
                else:
                    Dn[a, b] = D[a, b] - D[a, j] * D[j, b] / D[j, j]
            else:
                if a == j or b == j:
                    Dn[a, b] = 0.0
                else:
                    Dn[a, b] = D[a, b] + D[a, j] * D[j, b] / (1.0 - D[j, j])
    return Dn, p, outcome


def state_from_correlation(D, N):
    """Step 4: U = the eigenvectors of D for its N largest eigenvalues (all 1 for a pure state)."""
    lam, V = np.linalg.eigh(D)
    return V[:, np.argsort(lam)[::-1][:N]]


def event(D, H, N, gamma, seed, uid, n):
    """One event (steps 1-4).  Returns (D, U, record) with record = (tau, j, p_j, outcome)."""
    L = D.shape[0]
    eta, j, p_c = event_draws(seed, uid, n, L)
    tau = waiting_time(eta, gamma, N)
    D = evolve(D, H, tau)
    D, p, outcome = measure_site(D, j, p_c)
    U = state_from_correlation(D, N)
    return correlation_matrix(U), U, (tau, j, p, outcome)


def run_continuous(lat, U0, gamma, seed, uid, n_events, t_end=np.inf, first_event=1, t0=0.0):
    """Events first_event .. first_event + n_events - 1 of one trajectory from state U0 at time t0.

    An event is taken only while t < t_end; events skipped that way still use up
    their index n (the draws of event n never depend on earlier events).
    Returns dict(U, D, t, records={n: (tau, j, p, outcome)}).
    """
    H = hopping_matrix(lat)
    N = U0.shape[1]
    U = U0.copy()
    D = correlation_matrix(U)
    t = t0
    records = {}
    for n in range(first_event, first_event + n_events):
        if not t < t_end:
            continue
        D, U, rec = event(D, H, N, gamma, seed, uid, n)
        t += rec[0]
        records[n] = rec
    return {"U": U, "D": D, "t": t, "records": records}
