"""Fock-space brute force for L <= 10 (test-only second opinion for the oracle).

The many-body state is a vector over occupation bit strings s (bit i = n_i)
in the fixed-N sector.  Jordan-Wigner convention: c_i^+ |s> carries the sign
(-1)^(number of occupied sites j < i); the basis state of sites j1 < ... < jN
is c_j1^+ ... c_jN^+ |vac>, so the Slater determinant of orbitals U has
amplitude det(U[{j1..jN}, :]) on it.

Dynamics (arXiv:2508.18468, Appendix A), with the same Philox draws as the
oracle:
* free evolution by exp(-i H dt), H = sum_ij Ht_ij c_i^+ c_j, built from its
  matrix elements and exponentiated by eigendecomposition;
* projective measurement of n_j: Born probability <n_j>, outcome 1 iff
  u_out <= p, state multiplied by the projector and renormalised;
* homodyne update: the diagonal operator exp(sum_i a_i n_i),
  a_i = xi_i + gamma (2<n_i> - 1) dt, then renormalisation.
Nothing here uses the single-particle (U-matrix) representation after the
initial state, so it shares no arithmetic with the oracle.
"""

import itertools

import numpy as np

from oracle.philox import pm_uniforms, qsd_normals


def _popcount(x):
    return bin(x).count("1")


class FockSim:
    def __init__(self, Ht, occupied):
        L = Ht.shape[0]
        N = len(occupied)
        self.L, self.N = L, N
        self.basis = [s for s in range(1 << L) if _popcount(s) == N]
        self.index = {s: k for k, s in enumerate(self.basis)}
        D = len(self.basis)
        H = np.zeros((D, D), dtype=np.complex128)
        for col, s in enumerate(self.basis):
            for i in range(L):
                for j in range(L):
                    if Ht[i, j] == 0.0 or not (s >> j) & 1:
                        continue
                    sign = -1 if _popcount(s & ((1 << j) - 1)) % 2 else 1
                    s1 = s ^ (1 << j)
                    if (s1 >> i) & 1:
                        continue
                    if _popcount(s1 & ((1 << i) - 1)) % 2:
                        sign = -sign
                    H[self.index[s1 | (1 << i)], col] += Ht[i, j] * sign
        self.H = H
        self.occ = np.array([[(s >> i) & 1 for i in range(L)] for s in self.basis],
                            dtype=np.float64)
        s0 = sum(1 << o for o in occupied)
        self.psi = np.zeros(D, dtype=np.complex128)
        self.psi[self.index[s0]] = 1.0

    def set_evolution(self, dt):
        w, V = np.linalg.eigh(self.H)
        self.E = (V * np.exp(-1j * w * dt)[None, :]) @ np.conj(V.T)

    def evolve(self, tau):
        """psi <- exp(-i H tau) psi for any tau (many-body eigendecomposition)."""
        if not hasattr(self, "_eig"):
            self._eig = np.linalg.eigh(self.H)
        w, V = self._eig
        self.psi = V @ (np.exp(-1j * w * tau) * (np.conj(V.T) @ self.psi))

    def measure(self, j, p_c):
        """Projective measurement of n_j: outcome 1 iff p_c <= <n_j>; projector, renormalise."""
        p = float((np.abs(self.psi) ** 2) @ self.occ[:, j])
        outcome = 1 if p_c <= p else 0
        mask = self.occ[:, j] if outcome == 1 else 1.0 - self.occ[:, j]
        self.psi = self.psi * mask
        self.psi /= np.linalg.norm(self.psi)
        return p, outcome

    def occupations(self):
        return (np.abs(self.psi) ** 2) @ self.occ

    def correlation(self):
        """C_ab = <c_b^+ c_a>, computed from operator matrix elements."""
        L = self.L
        C = np.zeros((L, L), dtype=np.complex128)
        for col, s in enumerate(self.basis):
            amp = self.psi[col]
            if amp == 0:
                continue
            for a in range(L):
                if not (s >> a) & 1:
                    continue
                sa = -1 if _popcount(s & ((1 << a) - 1)) % 2 else 1
                s1 = s ^ (1 << a)
                for b in range(L):
                    if (s1 >> b) & 1:
                        continue
                    sb = -1 if _popcount(s1 & ((1 << b) - 1)) % 2 else 1
                    t = s1 | (1 << b)
                    C[a, b] += np.conj(self.psi[self.index[t]]) * sa * sb * amp
        return C

    def pm_step(self, gamma, dt, seed, uid, n):
        self.psi = self.E @ self.psi
        u_sel, u_out = pm_uniforms(seed, uid, n, self.L)
        q = min(gamma * dt, 1.0)
        events = []
        for j in range(self.L):
            if u_sel[j] < q:
                p = float((np.abs(self.psi) ** 2) @ self.occ[:, j])
                outcome = 1 if u_out[j] <= p else 0
                mask = self.occ[:, j] if outcome == 1 else 1.0 - self.occ[:, j]
                self.psi = self.psi * mask
                self.psi /= np.linalg.norm(self.psi)
                events.append((j, p, outcome))
        return events

    def qsd_step(self, gamma, dt, seed, uid, n):
        self.psi = self.E @ self.psi
        p = self.occupations()
        xi = np.sqrt(gamma * dt) * qsd_normals(seed, uid, n, self.L)
        a = xi + gamma * (2.0 * p - 1.0) * dt
        self.psi = self.psi * np.exp(self.occ @ a)
        self.psi /= np.linalg.norm(self.psi)

    def _permuted_state(self, order):
        """Amplitudes after relabelling modes so that order[k] becomes mode k."""
        newlabel = {old: new for new, old in enumerate(order)}
        out = np.zeros(1 << self.L, dtype=np.complex128)
        for col, s in enumerate(self.basis):
            occ = [i for i in range(self.L) if (s >> i) & 1]
            new = [newlabel[i] for i in occ]
            # sign of the permutation that sorts the relabelled creation operators
            inv = sum(1 for x, y in itertools.combinations(new, 2) if x > y)
            t = sum(1 << m for m in new)
            out[t] = self.psi[col] * (-1 if inv % 2 else 1)
        return out

    def entropy(self, region):
        """Von Neumann entropy of the fermionic reduced state of `region`."""
        region = list(region)
        rest = [i for i in range(self.L) if i not in region]
        full = self._permuted_state(region + rest)
        nA = len(region)
        M = full.reshape(1 << (self.L - nA), 1 << nA)  # bits 0..nA-1 = region
        sv = np.linalg.svd(M, compute_uv=False)
        w = sv ** 2
        w = w[w > 1e-300]
        return float(-(w * np.log(w)).sum())
