"""Entanglement observables of a Slater determinant (oracle, test infrastructure).

Sec. II: S_A = -sum_i [l_i ln l_i + (1 - l_i) ln(1 - l_i)] over the eigenvalues
l_i of the correlation matrix restricted to region A (the printed formula
drops the minus sign and the trace; this is the reading used).  Natural
logarithm, 0 ln 0 = 0, eigenvalues clamped to [0, 1].
Sec. IV: mutual information I_2 = S_A + S_B - S_{A u B}.

C_A = U_A U_A^+ (rows of U in A); its spectrum equals that of the paper's
D restricted to A (D = C^T).  The eigenvalues come from LAPACK (numpy
eigvalsh), used as a library primitive.

Pinned by: Fock-space reduced density matrices (L <= 10), S(Neel) = 0,
S_A = S_complement for pure states, trace and Frobenius identities and the
particle-hole pairing of the two complementary spectra
(tests/test_oracle_observables.py).
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
