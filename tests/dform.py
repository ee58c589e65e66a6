"""Correlation-matrix (D-form) updates of Appendix A (test-only second opinion).

Eq. (A1) (outcome 1 at site j) and Eq. (A2) (outcome 0) act directly on the
L x L correlation matrix.  Written here for C = U U^+ (C = D^T; the formulas
keep their form under transposition).  Eq. (A2) is printed with a minus sign
in front of the rank-1 term; the correct sign is plus (the rank-1 term of a
projection onto n_j = 0 is divided by 1 - C_jj, and its sign follows from
requiring C^2 = C).  The plus sign is used here.
"""

import numpy as np


def project_outcome1(C, j):
    Cn = C - np.outer(C[:, j], C[j, :]) / C[j, j]
    Cn[j, :] = 0.0
    Cn[:, j] = 0.0
    Cn[j, j] = 1.0
    return Cn


def project_outcome0(C, j):
    Cn = C + np.outer(C[:, j], C[j, :]) / (1.0 - C[j, j])
    Cn[j, :] = 0.0
    Cn[:, j] = 0.0
    return Cn


def project_outcome0_as_printed(C, j):
    """Eq. (A2) with the printed minus sign (used to show that it is wrong)."""
    Cn = C - np.outer(C[:, j], C[j, :]) / (1.0 - C[j, j])
    Cn[j, :] = 0.0
    Cn[:, j] = 0.0
    return Cn
