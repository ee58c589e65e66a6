"""Homodyne step with the paper's fourth-order Runge-Kutta integrator -- oracle.

TEST INFRASTRUCTURE.  Appendix A writes the homodyne step as
U(t + dt) ∝ exp(A) U(t) with the exponent of Eq. (A4),
    A = -i Ht dt + dW^t + (2 <n>_t - 1) gamma dt
(dW^t and <n>_t diagonal, taken at the start of the step), and integrates it with the
fourth-order Runge-Kutta method, followed by the QR re-orthonormalisation.  Reading: over
the step the exponent is frozen, so U(t + dt) is one classical RK4 step of the linear
equation dU/ds = (A / dt) U from s = 0 to s = dt:
    k1 = A U, k2 = A (U + k1/2), k3 = A (U + k2/2), k4 = A (U + k3),
    U(t + dt) = U + (k1 + 2 k2 + 2 k3 + k4) / 6.
dW_i = sqrt(gamma dt) z_i with the standard normals of the split step (Philox purpose 1,
site i, step n), <n_i>_t = sum_k |U_ik|^2 of the state entering the step.

Pinned by (tests/test_oracle_rk4.py): the Taylor remainder bound
|RK4 - expm(A)| <= |A|^5 e^|A| / 120 against scipy's expm; fourth-order convergence of the
free step against the plane-wave propagator (one-step error ratio 32 when dt halves); with
no hopping the step equals the split step's diagonal factor within the same remainder bound;
and the step's time reversal symmetry of the free part.
"""

import numpy as np

from .lattice import hopping_matrix
from .philox import qsd_normals
from .trajectory import born_probabilities, reorthonormalize


def generator(U, H, gamma, dt, seed, uid, n):
    """A = -i H dt + diag(dW + (2 p - 1) gamma dt) at the start of step n."""
    L = U.shape[0]
    p = born_probabilities(U)
    dW = np.sqrt(gamma * dt) * qsd_normals(seed, uid, n, L)
    return -1j * dt * H + np.diag(dW + (2.0 * p - 1.0) * gamma * dt)


def rk4_propagate(U, A):
    """One classical RK4 step of dU/ds = (A/dt) U over [0, dt]."""
    k1 = A @ U
    k2 = A @ (U + 0.5 * k1)
    k3 = A @ (U + 0.5 * k2)
    k4 = A @ (U + k3)
    return U + (k1 + 2.0 * k2 + 2.0 * k3 + k4) / 6.0


def rk4_step(U, H, gamma, dt, seed, uid, n):
    """Homodyne step n with the RK4 integrator, then QR (diag R > 0)."""
    return reorthonormalize(rk4_propagate(U, generator(U, H, gamma, dt, seed, uid, n)))


def run_rk4(lat, U0, gamma, dt, seed, uid, n_steps, first_step=1):
    """Steps first_step .. first_step + n_steps - 1 of one trajectory."""
    H = hopping_matrix(lat)
    U = U0.copy()
    for n in range(first_step, first_step + n_steps):
        U = rk4_step(U, H, gamma, dt, seed, uid, n)
    return U
