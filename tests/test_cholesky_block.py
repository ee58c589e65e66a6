"""The blocked Cholesky of a Cholesky-QR pass (Appendix A: QR after each step) on the CPU.

tests/cholesky_block_harness.cpp runs the device kernel's own diagonal-block code
(paper_2508_18468_amd/csrc/potrf_block.h) with every phase's 256 threads in three orders
(bitwise equal results: no intra-phase dependence, i.e. no missing barrier) and checks that
the four back-substitution lanes of a column agree bitwise; it is built with the address
and undefined-behaviour sanitizers (array bounds included).  Inputs:

* the Grams that the 384-trajectory ring L = 1024 homodyne batch with the RK4 integrator
  produces in its first six steps (oracle RK4 states before re-orthonormalisation, sampled
  trajectories of each rate), and the near-identity Grams of the second pass;
* ragged sizes (N = 130, 550: a last block narrower than 64, two outer panels);
* Grams with a known first breakdown (a repeated column, a NaN), whose reported column and
  pivot must be the first bad one.

R is checked against numpy's Cholesky factor and R^+ R = G, R^{-1} R = I.
"""

import os
import subprocess

import numpy as np
import pytest

import oracle
from oracle.rk4 import generator, rk4_propagate
from oracle.lattice import hopping_matrix
from oracle.trajectory import reorthonormalize

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("chol") / "cholesky_block_harness")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Wextra", "-Werror", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-o", exe,
                    os.path.join(ROOT, "tests", "cholesky_block_harness.cpp")], check=True)
    return exe


def run(harness, tmp_path, G):
    N = G.shape[0]
    fin, fout = str(tmp_path / "g.bin"), str(tmp_path / "r.bin")
    with open(fin, "wb") as f:
        np.int32(N).tofile(f)
        np.asfortranarray(G.astype(np.complex128)).T.ravel().tofile(f)  # column-major
    out = subprocess.run([harness, fin, fout], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    with open(fout, "rb") as f:
        first_bad = int(np.fromfile(f, np.int32, 1)[0])
        pivot = float(np.fromfile(f, np.float64, 1)[0])
        mism = int(np.fromfile(f, np.int32, 1)[0])
        R = np.fromfile(f, np.complex128, N * N).reshape(N, N).T
        Rinv = np.fromfile(f, np.complex128, N * N).reshape(N, N).T
    return first_bad, pivot, mism, R, Rinv


def check_factor(G, R, Rinv):
    N = G.shape[0]
    Gh = np.triu(G) + np.triu(G, 1).conj().T
    scale = np.abs(Gh).max()
    assert np.abs(R.conj().T @ R - Gh).max() <= 1e-13 * scale
    R_np = np.linalg.cholesky(Gh).conj().T
    cond = np.linalg.cond(R_np)
    assert np.abs(R - R_np).max() <= 1e-13 * cond * np.abs(R_np).max()
    assert np.abs(Rinv @ R - np.eye(N)).max() <= 1e-13 * cond
    assert np.abs(np.tril(Rinv, -1)).max() == 0.0


def rk4_grams(uid, gamma, n_steps=6, L=1024, dt=0.05, seed=0):
    """Pass-1 and pass-2 Grams of steps 1..n_steps of one RK4 trajectory (ring L, Neel)."""
    lat = oracle.Lattice(1, L)
    H = hopping_matrix(lat)
    U = oracle.initial_state(L, oracle.default_occupied(lat))
    out = []
    for n in range(1, n_steps + 1):
        V = rk4_propagate(U, generator(U, H, gamma, dt, seed, uid, n))
        G1 = V.conj().T @ V
        R1 = np.linalg.cholesky(G1).conj().T
        Q = np.linalg.solve(R1.T, V.T).T  # V R1^{-1}
        out.append((n, G1, Q.conj().T @ Q))
        U = reorthonormalize(V)
    return out


@pytest.mark.slow
@pytest.mark.parametrize("t", [0, 127, 128 + 5, 256 + 44, 383])
def test_rk4_batch_grams(harness, tmp_path, t):
    """Sampled trajectories of the three rates (0.1, 0.3, 1.0; uid = t) of the batch."""
    from paper_2508_18468_amd.workloads import ring_qsd_batched
    w = ring_qsd_batched()
    gamma = w.gammas[t // w.n_traj]
    for n, G1, G2 in rk4_grams(t, gamma, dt=w.dt, seed=w.seed):
        for G in (G1, G2):
            fb, _, mism, R, Rinv = run(harness, tmp_path, G)
            assert fb == -1 and mism == 0, (n, fb, mism)
            check_factor(G, R, Rinv)


@pytest.mark.parametrize("N", [64, 130, 550])
def test_ragged_sizes(harness, tmp_path, N):
    rng = np.random.default_rng(N)
    V = rng.standard_normal((2 * N, N)) + 1j * rng.standard_normal((2 * N, N))
    G = V.conj().T @ V
    fb, _, mism, R, Rinv = run(harness, tmp_path, G)
    assert fb == -1 and mism == 0
    check_factor(G, R, Rinv)


def test_first_breakdown_reported(harness, tmp_path):
    rng = np.random.default_rng(7)
    N = 200
    V = rng.standard_normal((400, N)) + 1j * rng.standard_normal((400, N))
    V[:, 70] = V[:, 3]                       # rank deficient from column 70 on
    fb, piv, mism, _, _ = run(harness, tmp_path, V.conj().T @ V)
    assert mism == 0
    assert fb == 70 and abs(piv) <= 1e-9 * np.abs(V).max() ** 2 * 400
    G = np.eye(N, dtype=np.complex128)
    G[150, 150] = np.nan
    fb, piv, _, _, _ = run(harness, tmp_path, G)
    assert fb == 150 and np.isnan(piv)
    G = np.eye(N, dtype=np.complex128)
    G[10, 10] = -1.0
    fb, piv, _, _, _ = run(harness, tmp_path, G)
    assert fb == 10 and piv == -1.0
