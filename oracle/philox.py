"""Philox4x64-10 counter-based generator (oracle side, test infrastructure).

Written from the published definition (J. Salmon, M. Moraes, R. Dror,
D. Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11): a 4-word
counter and a 2-word key, ten rounds of two 64x64->128-bit multiplies with
the multipliers M0, M1, the key bumped by the Weyl constants W0, W1 between
rounds.  Vectorised over numpy uint64 arrays; the 128-bit products are built
from 32-bit halves.

Draw layout (the paper does not say how its random numbers are produced;
this layout is a choice of this library, shared by oracle and GPU only by
specification, not by code):

* key     = (seed, trajectory uid)
* counter = (step n, site i, purpose, 0), purpose 0 = projective protocol
  (word 0 -> site-selection uniform, word 1 -> outcome uniform),
  purpose 1 = homodyne protocol (words 0, 1 -> Box-Muller normal).

Pinned by: known-answer tests against ``numpy.random.Philox`` (an
independent implementation of the same definition), plus uniformity and
normality checks (tests/test_oracle_rng.py).
"""

import numpy as np

_M0 = np.uint64(0xD2E7470EE14C6C93)
_M1 = np.uint64(0xCA5A826395121157)
_W0 = np.uint64(0x9E3779B97F4A7C15)
_W1 = np.uint64(0xBB67AE8584CAA73B)
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a, b):
    """Full 128-bit product of uint64 arrays: returns (hi, lo)."""
    a_lo, a_hi = a & _LO32, a >> _S32
    b_lo, b_hi = b & _LO32, b >> _S32
    t = a_lo * b_lo
    u = a_hi * b_lo + (t >> _S32)
    v = a_lo * b_hi + (u & _LO32)
    hi = a_hi * b_hi + (u >> _S32) + (v >> _S32)
    lo = a * b  # wraps modulo 2**64
    return hi, lo


def philox4x64_10(k0, k1, c0, c1, c2, c3):
    """Philox4x64 with 10 rounds.  All arguments broadcast as uint64 arrays.

    Returns a tuple of four uint64 arrays (the output block).
    """
    with np.errstate(over="ignore"):
        k0 = np.asarray(k0, dtype=np.uint64)
        k1 = np.asarray(k1, dtype=np.uint64)
        x0, x1, x2, x3 = np.broadcast_arrays(*[np.asarray(c, dtype=np.uint64)
                                               for c in (c0, c1, c2, c3)])
        x0, x1, x2, x3 = x0.copy(), x1.copy(), x2.copy(), x3.copy()
        for r in range(10):
            if r > 0:
                k0 = k0 + _W0
                k1 = k1 + _W1
            hi0, lo0 = _mulhilo(_M0, x0)
            hi1, lo1 = _mulhilo(_M1, x2)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return x0, x1, x2, x3


def u01(x):
    """Map a uint64 to a double in the open interval (0, 1): ((x>>12)+0.5)*2^-52.

    52 bits keep every value exactly representable (53 bits plus the half
    offset would round the largest input up to 1.0).
    """
    x = np.asarray(x, dtype=np.uint64)
    return ((x >> np.uint64(12)).astype(np.float64) + 0.5) * (2.0 ** -52)


def pm_uniforms(seed, uid, n, L):
    """Projective-protocol draws of step n: (u_select[L], u_outcome[L])."""
    w = philox4x64_10(seed, uid, n, np.arange(L, dtype=np.uint64), 0, 0)
    return u01(w[0]), u01(w[1])


def qsd_normals(seed, uid, n, L):
    """Homodyne-protocol standard normals z[L] of step n (Box-Muller, cos branch)."""
    w = philox4x64_10(seed, uid, n, np.arange(L, dtype=np.uint64), 1, 0)
    a, b = u01(w[0]), u01(w[1])
    return np.sqrt(-2.0 * np.log(a)) * np.cos(2.0 * np.pi * b)
