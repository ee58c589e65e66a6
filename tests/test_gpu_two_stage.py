"""The two-stage reduction of region Grams (dense -> band of half-width 32 by block reflectors,
then bulge chasing; mfq_set_eig_path(MFQ_EIG_TWO_STAGE)) on states with a known spectrum, on
trajectories against the oracle, and against the one-stage reduction.

Tolerances as in test_gpu_fullsize.py: by Weyl's inequality each eigenvalue is within |dC|_2
of the exact one; the tests allow 200 n eps for a Gram of order n.  Against the oracle the
states themselves differ by rounding (C to 1e-11 after a few steps), so the spectra may differ
by that much.
"""

import numpy as np
import pytest

import oracle
from gpu_common import OracleBatch, make_sim
from test_gpu_fullsize import EPS, coupled_state, entropy_bound, h, known_state, spectrum_mix

pytestmark = pytest.mark.gpu

ONE, TWO = 1, 2


@pytest.mark.parametrize("l", [200, 333, 700])
def test_two_stage_known_spectrum(l):
    """Three trajectories, L=1400, N=700, random regions: 200 sites (six panels, the last
    with 8 rows), 333 and 700 (21 panels, the last with 28 rows)."""
    L, N, B = 1400, 700, 3
    rng = np.random.default_rng(l)
    region = sorted(rng.choice(L, l, replace=False).tolist())
    lams = [spectrum_mix(l, rng) for _ in range(B)]
    sim = make_sim(1, L, n_traj=B)
    sim.set_eig_path(TWO)
    sim.set_state(np.concatenate([known_state(L, N, region, lam, rng) for lam in lams]), 0)
    print(f"two-stage known spectrum: l={l}", flush=True)
    got = sim.region_spectrum(region)
    S = sim.entropy(region)
    delta = 200 * l * EPS
    for t in range(B):
        err = float(np.max(np.abs(np.sort(got[t]) - np.sort(lams[t]))))
        assert err <= delta, (t, err)
        assert abs(S[t] - h(lams[t]).sum()) <= entropy_bound(lams[t], delta)
    sim.close()


def test_two_stage_tiny_couplings():
    """Columns with entries of 1e-160 (subnormal squares), 1e-100, 1e-30 and 0.3 between the
    region halves, n = 650, four trajectories: the panel reflectors and the chase reflectors
    are formed from scaled vectors, so the spectrum stays exact."""
    half, B = 325, 4
    L, N = 4 * half + 64, 2 * half + 32
    rng = np.random.default_rng(7)
    A1 = list(range(0, half))
    A2 = list(range(L // 2, L // 2 + half))
    region = sorted(A1 + A2)
    sim = make_sim(1, L, n_traj=B, N=N, occupied=list(range(N)))
    sim.set_eig_path(TWO)
    lams, Us = [], []
    for t in range(B):
        lam = spectrum_mix(2 * half, rng)
        lams.append(lam)
        Us.append(coupled_state(L, N, A1, A2, lam, (1e-160, 1e-100, 1e-30, 0.3)[t], rng))
    sim.set_state(np.concatenate(Us), 0)
    got = sim.region_spectrum(region)
    for t in range(B):
        err = float(np.max(np.abs(np.sort(got[t]) - np.sort(lams[t]))))
        assert err <= 200 * len(region) * EPS, (t, err)
    sim.close()


def test_two_stage_product_state_is_exact():
    """The Neel state: C_A is diagonal with entries 0 and 1, every panel is zero (no
    reflector), and the spectrum comes out exactly, so S = 0 exactly."""
    L = 1400
    sim = make_sim(1, L, n_traj=2)
    sim.set_eig_path(TWO)
    region = list(range(0, 700))
    lam = sim.region_spectrum(region)
    assert np.array_equal(np.sort(lam[0]), np.repeat([0.0, 1.0], 350))
    assert np.array_equal(sim.entropy(region), np.zeros(2))
    sim.close()


def test_two_stage_trajectories_against_oracle():
    """Ring L=1200, N=600, two homodyne and two projective trajectories after 12 steps: region
    spectra of 600 and 460 sites from both reduction forms against the oracle's numpy eigvalsh
    of C_A, and the two forms against each other."""
    L, dt, seed, uids = 1200, 0.05, 5, [3, 8]
    gams = [0.5, 2.0]
    for protocol in (1, 0):
        sim = make_sim(1, L, n_traj=2, uids=uids)
        ob = OracleBatch(1, L, 1, dt, uids)
        for _ in range(12):
            sim.step(protocol, gams, dt, seed)
            ob.step(protocol, gams, seed)
        rng = np.random.default_rng(protocol)
        for region in (list(range(600)), sorted(rng.choice(L, 460, replace=False).tolist())):
            spec = {}
            for path in (ONE, TWO):
                sim.set_eig_path(path)
                spec[path] = np.sort(sim.region_spectrum(region), axis=1)
            for t in range(2):
                want = np.sort(oracle.region_spectrum(ob.U[t], region))
                for path in (ONE, TWO):
                    assert np.abs(spec[path][t] - want).max() <= 1e-11, (protocol, len(region), path)
                assert np.abs(spec[ONE][t] - spec[TWO][t]).max() <= 1e-11
        sim.close()


def test_two_stage_panel_forms_agree():
    """Sixteen trajectories of a 6400-site ring, region of 3200 sites: the first panels' grid
    (25 workgroups per matrix, 400 in all) exceeds three quarters of what the GPU holds at once,
    so they run as one launch per column, and the later panels (24 per matrix) run in the panel
    kernel; the spectra match the one-stage reduction (1e-11) after a few homodyne steps."""
    L, B = 6400, 16
    sim = make_sim(1, L, n_traj=B, uids=list(range(B)))
    sim.step(1, [0.5 + 0.1 * t for t in range(B)], 0.05, 3, 2)
    region = list(range(3200))
    spec = {}
    for path in (ONE, TWO):
        sim.set_eig_path(path)
        print(f"panel forms: eig path {path}", flush=True)
        spec[path] = np.sort(sim.region_spectrum(region), axis=1)
    assert np.abs(spec[ONE] - spec[TWO]).max() <= 1e-11
    assert np.all(spec[TWO] > -1e-12) and np.all(spec[TWO] < 1.0 + 1e-12)
    sim.close()


def test_two_stage_panel_kernels_on_two_streams():
    """Two contexts on two streams reduce 6400-site region Grams of six trajectories from two
    host threads at once: 300 panel-kernel workgroups each, more than the GPU holds for both, so
    a panel kernel of one stream waits on the GPU for the other's running one; both spectra
    match the one-stage reduction (1e-11)."""
    import threading
    import torch
    L, B = 12800, 6
    sims = []
    for k in range(2):
        with torch.cuda.stream(torch.cuda.Stream()):
            sims.append(make_sim(1, L, n_traj=B, uids=list(range(10 * k, 10 * k + B))))
    region = list(range(6400))
    ref = []
    for sim in sims:
        sim.step(1, [0.5] * B, 0.05, 3, 2)
        sim.set_eig_path(ONE)
        ref.append(np.sort(sim.region_spectrum(region), axis=1))
        sim.set_eig_path(TWO)
    print("panel kernels on two streams: one-stage references done", flush=True)
    out, errs = [None, None], []

    def work(k):
        try:
            out[k] = np.sort(sims[k].region_spectrum(region), axis=1)
        except Exception as ex:  # reported below
            errs.append(ex)

    threads = [threading.Thread(target=work, args=(k,)) for k in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errs, errs
    for k in range(2):
        assert np.abs(out[k] - ref[k]).max() <= 1e-11
    for sim in sims:
        sim.close()
