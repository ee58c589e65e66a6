"""Single-particle propagator P = exp(-i Ht dt) (oracle, test infrastructure).

Appendix A: between measurements the state evolves unitarily under H, and
for the homodyne protocol the coefficient matrix is advanced with
exp(-i Ht dt) (Eq. (A4) without its measurement terms).

Plane-wave closed form: Ht on the ring is diagonalised by k_m = 2 pi m / L with
eigenvalue 2J cos k_m, so
    P_ab = (1/L) sum_m exp(-2iJ dt cos k_m) exp(i k_m (a - b)),
a circulant; on the torus P = P_y (x) P_x for site order i = x + Lx*y.

Pinned by: scipy.linalg.expm of the hopping matrix, unitarity, symmetry and
the Bessel-function entries |P_{0,n}| = J_n(2J dt) for n << L
(tests/test_oracle_propagator.py).
"""

import numpy as np


def _ring_propagator(L, J, dt):
    k = 2.0 * np.pi * np.arange(L) / L
    phase = np.exp(-2j * J * dt * np.cos(k))
    d = np.arange(L)
    # column c_d = P_{d,0} = (1/L) sum_m phase_m exp(i k_m d); the integer product
    # m*d is reduced modulo L first so every plane-wave phase is accurate.
    md = np.outer(d, np.arange(L)) % L
    col = (phase[None, :] * np.exp(2j * np.pi * md / L)).sum(axis=1) / L
    a = np.arange(L)
    return col[(a[:, None] - a[None, :]) % L]


def propagator(lat, dt):
    """Dense complex128 L x L matrix exp(-i Ht dt)."""
    if lat.dim == 1:
        return _ring_propagator(lat.Lx, lat.J, dt)
    Px = _ring_propagator(lat.Lx, lat.J, dt)
    Py = _ring_propagator(lat.Ly, lat.J, dt)
    return np.kron(Py, Px)
