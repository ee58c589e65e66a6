"""Entanglement observables of a Slater determinant (oracle, test infrastructure).

Sec. II: S_A = -sum_i [l_i ln l_i + (1 - l_i) ln(1 - l_i)] over the eigenvalues
l_i of the correlation matrix restricted to region A (the printed formula
drops the minus sign and the trace; this is the reading used).  Natural
logarithm, 0 ln 0 = 0, eigenvalues clamped to [0, 1].
Sec. IV: mutual information I_2 = S_A + S_B - S_{A u B}.
Sec. II, Eq. (2): density-density correlation C_ij = -D_ij D_ji = -|C_ij|^2 for
i != j (Wick's theorem), averaged over the pairs at distance r.
Sec. IV, Eq. (5): particle-number covariance G_AB = -sum_{i in A, j in B} C_ij.

C_A = U_A U_A^+ (rows of U in A); its spectrum equals that of the paper's
D restricted to A (D = C^T).  The eigenvalues come from LAPACK (numpy
eigvalsh), used as a library primitive.

Pinned by: Fock-space reduced density matrices (L <= 10), S(Neel) = 0,
S_A = S_complement for pure states, trace and Frobenius identities and the
particle-hole pairing of the two complementary spectra
(tests/test_oracle_observables.py); the correlation observables by the sum
rule sum_{i != j} |C_ij|^2 = N - sum_i p_i^2 (C^2 = C), the two-site closed form,
the Fock-space density covariance <n_i n_j> - <n_i><n_j>, and
G_{A, complement} = sum over the spectrum of C_A of l (1 - l)
(tests/test_oracle_correlations.py).
"""

import numpy as np


def correlation_matrix(U):
    """C = U U^+ (C_ab = <c_b^+ c_a>)."""
    return U @ np.conj(U.T)


def region_spectrum(U, region):
    """Eigenvalues of C_A = U_A U_A^+ (ascending)."""
    UA = U[np.asarray(region, dtype=np.int64), :]
    CA = UA @ np.conj(UA.T)
    return np.linalg.eigvalsh(CA)


def entropy_from_spectrum(lam):
    lam = np.clip(np.asarray(lam, dtype=np.float64), 0.0, 1.0)
    s = 0.0
    for x in lam:
        if 0.0 < x < 1.0:
            s -= x * np.log(x) + (1.0 - x) * np.log1p(-x)
    return float(s)


def entanglement_entropy(U, region):
    return entropy_from_spectrum(region_spectrum(U, region))


def mutual_information(U, A, B):
    AB = sorted(set(A) | set(B))
    return (entanglement_entropy(U, A) + entanglement_entropy(U, B)
            - entanglement_entropy(U, AB))


def ring_distance(i, j, L):
    d = abs(i - j) % L
    return min(d, L - d)


def density_correlation(U):
    """Eq. (2) on a 1d ring of L sites: C(r) for r = 1 .. L//2, the average of
    C_ij = -|C_ij|^2 over the ordered pairs (i, j), i != j, at ring distance r
    (one trajectory; the average over trajectories is taken by the caller)."""
    C = correlation_matrix(U)
    L = C.shape[0]
    total = np.zeros(L // 2 + 1)
    count = np.zeros(L // 2 + 1)
    for i in range(L):
        for j in range(L):
            if i == j:
                continue
            r = ring_distance(i, j, L)
            total[r] -= abs(C[i, j]) ** 2
            count[r] += 1
    return total[1:] / count[1:]


def particle_covariance(U, A, B):
    """Eq. (5): G_AB = -sum_{i in A, j in B} C_ij = sum |C_ij|^2 for disjoint A, B
    (minus the covariance of the particle numbers of A and B)."""
    C = correlation_matrix(U)
    g = 0.0
    for i in A:
        for j in B:
            g += abs(C[i, j]) ** 2
    return float(g)
