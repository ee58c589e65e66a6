"""Lattices and the single-particle hopping matrix (oracle, test infrastructure).

Sec. II: H = J sum_i (c_i^+ c_{i+1} + h.c.) on a ring with periodic boundary
conditions, J = 1; Sec. IV uses the same Hamiltonian on a square lattice.
Appendix A writes H = sum_ij Ht_ij c_i^+ c_j with Ht_ij = J on nearest-neighbour
bonds.  Site numbering (a choice of this library): i = x + Lx*y.

Initial state (Appendix A): the Neel state |1010...>, i.e. even sites
(0-based) occupied; on the square lattice the checkerboard x+y even (the
paper does not state the 2d start).

Pinned by: symmetry, bond count and spectrum 2J(cos kx + cos ky) checked in
tests/test_oracle_propagator.py.
"""

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Lattice:
    dim: int          # 1 or 2
    Lx: int
    Ly: int = 1
    J: float = 1.0

    @property
    def L(self):
        return self.Lx * (self.Ly if self.dim == 2 else 1)

    def site(self, x, y=0):
        return x + self.Lx * y


def hopping_matrix(lat):
    """Real symmetric L x L matrix Ht with Ht_ij = J for nearest neighbours (PBC)."""
    L = lat.L
    H = np.zeros((L, L))
    if lat.dim == 1:
        for i in range(L):
            H[i, (i + 1) % L] += lat.J
            H[(i + 1) % L, i] += lat.J
    else:
        for y in range(lat.Ly):
            for x in range(lat.Lx):
                i = lat.site(x, y)
                jx = lat.site((x + 1) % lat.Lx, y)
                jy = lat.site(x, (y + 1) % lat.Ly)
                H[i, jx] += lat.J
                H[jx, i] += lat.J
                H[i, jy] += lat.J
                H[jy, i] += lat.J
    return H


def default_occupied(lat):
    """Neel (1d) / checkerboard (2d) occupied sites, ascending."""
    if lat.dim == 1:
        return [i for i in range(lat.L) if i % 2 == 0]
    return sorted(lat.site(x, y) for y in range(lat.Ly) for x in range(lat.Lx)
                  if (x + y) % 2 == 0)
