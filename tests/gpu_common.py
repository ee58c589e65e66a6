"""Shared helpers of the GPU parity tests (no method arithmetic: the oracle computes
every expected value, the GPU library every result under test)."""

import numpy as np

import oracle
from oracle.trajectory import step as oracle_step


def make_sim(dim, Lx, Ly=1, n_traj=1, uids=None, N=None, occupied=None):
    from paper_2508_18468_amd import mfq
    return mfq.Trajectories(dim, Lx, Ly, N=N, n_traj=n_traj, uids=uids, occupied=occupied)


def oracle_lattice(dim, Lx, Ly=1):
    return oracle.Lattice(dim, Lx, Ly if dim == 2 else 1)


class OracleBatch:
    """The same trajectories advanced by the CPU oracle."""

    def __init__(self, dim, Lx, Ly, dt, uids, occupied=None):
        self.lat = oracle_lattice(dim, Lx, Ly)
        self.P = oracle.propagator(self.lat, dt)
        occ = oracle.default_occupied(self.lat) if occupied is None else list(occupied)
        self.U = [oracle.initial_state(self.lat.L, occ) for _ in uids]
        self.uids = list(uids)
        self.dt = dt
        self.n = 0

    def step(self, protocol, gammas, seed, idx=None):
        self.n += 1
        events = []
        for t in range(len(self.uids)):
            if idx is not None and t not in idx:
                events.append(None)
                continue
            self.U[t], ev = oracle_step(self.U[t], self.P, protocol, gammas[t], self.dt, seed,
                                        self.uids[t], self.n)
            events.append(ev)
        return events

    def entropy(self, region, idx=None):
        return np.array([oracle.entanglement_entropy(self.U[t], region) if (idx is None or t in idx)
                         else np.nan for t in range(len(self.uids))])


def corr(U):
    return U @ np.conj(U.T)
