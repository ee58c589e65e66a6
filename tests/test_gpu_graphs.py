"""Captured two-step HIP graphs replay exactly what direct launches compute.

Every replay is checked against the direct-launch result, with the program's own eager
work (entropies, occupations, state downloads, synchronisations) between replays."""

import numpy as np
import pytest

from gpu_common import make_sim

pytestmark = pytest.mark.gpu

PM, QSD = 0, 1


@pytest.mark.parametrize("protocol,gamma,L,B", [(QSD, 0.8, 96, 5), (PM, 2.0, 64, 4), (QSD, 1.0, 200, 3)])
def test_graph_replay_equals_direct(protocol, gamma, L, B):
    uids = list(range(10, 10 + B))
    direct = make_sim(1, L, n_traj=B, uids=uids)
    direct.use_graphs(False)
    graph = make_sim(1, L, n_traj=B, uids=uids)
    graph.use_graphs(True)
    g = [gamma] * B
    for rep, n in enumerate((6, 5, 2, 7)):
        direct.step(protocol, g, 0.05, 3, n)
        graph.step(protocol, g, 0.05, 3, n)
        Ud, nd = direct.get_state()
        Ug, ng = graph.get_state()
        assert nd == ng
        assert np.array_equal(Ud, Ug), rep
        assert np.array_equal(direct.entropy(list(range(L // 2))), graph.entropy(list(range(L // 2))))
        assert np.array_equal(direct.occupations(), graph.occupations())
        if protocol == PM:
            assert direct.pm_events() == graph.pm_events()
    direct.close()
    graph.close()


def test_graph_rebuilt_when_parameters_change():
    L, B = 64, 2
    a = make_sim(1, L, n_traj=B, uids=[1, 2])
    a.use_graphs(False)
    b = make_sim(1, L, n_traj=B, uids=[1, 2])
    for (proto, gam, dt, seed, n) in ((QSD, 0.5, 0.05, 1, 4), (QSD, 0.5, 0.05, 2, 4), (PM, 1.0, 0.05, 2, 4),
                                      (QSD, 0.9, 0.02, 2, 6), (QSD, 0.9, 0.02, 2, 3)):
        a.step(proto, [gam] * B, dt, seed, n)
        b.step(proto, [gam] * B, dt, seed, n)
        assert np.array_equal(a.get_state()[0], b.get_state()[0])
    a.close()
    b.close()
