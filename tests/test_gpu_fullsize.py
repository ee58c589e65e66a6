"""Region spectra and entropies at the full sizes of the large workloads, on states whose
spectrum is known in closed form.

For a region A of l <= N sites and its complement, take orthonormal Fourier vectors a_k on A
(k < l) and b_k on the complement (k < N), and the orbitals
    u_k = sqrt(lam_k) a_k + sqrt(1 - lam_k) b_k   (k < l),   u_k = b_k   (l <= k < N).
They are orthonormal, and C_A = U_A U_A^+ = sum_k lam_k a_k a_k^+ has eigenvalues exactly
{lam_k}, so S_A = sum_k h(lam_k) (Sec. II entropy formula).  The Fourier index runs over a
random permutation of the region's sites, which makes C_A dense.

Tolerance: by Weyl's inequality each computed eigenvalue is within |dC|_2 of the exact one;
for a Gram with K = N terms and a Householder reduction of order n that is a few n * eps in
practice, and the test allows DELTA = 200 n eps (1.8e-10 at n = 8192).  The entropy may then
differ by at most sum_k max_{|x - lam_k| <= DELTA} |h(x) - h(lam_k)|, computed here.
"""

import numpy as np
import pytest

from gpu_common import make_sim

pytestmark = pytest.mark.gpu

EPS = 2.220446049250313e-16


def h(x):
    x = np.clip(x, 0.0, 1.0)
    out = np.zeros_like(x)
    m = (x > 0) & (x < 1)
    out[m] = -(x[m] * np.log(x[m]) + (1 - x[m]) * np.log1p(-x[m]))
    return out


def spectrum_mix(r, rng):
    """A quarter spread over (0, 1), the rest exponentially close to 0 or 1 (area-law-like)."""
    lam = np.empty(r)
    q = r // 4
    lam[:q] = rng.uniform(0.0, 1.0, q)
    x = rng.uniform(3.0, 34.0, r - q)
    near = np.exp(-x)
    side = rng.random(r - q) < 0.5
    lam[q:] = np.where(side, near, 1.0 - near)
    rng.shuffle(lam)
    return lam


def fourier_columns(sites, ncols, rng):
    n = len(sites)
    order = rng.permutation(n)
    s = order[:, None].astype(np.float64)
    k = np.arange(ncols, dtype=np.float64)[None, :]
    return np.exp(2j * np.pi * (s * k) / n) / np.sqrt(n)


def known_state(L, N, region, lam, rng):
    region = np.asarray(region)
    comp = np.setdiff1d(np.arange(L), region)
    r = len(lam)
    assert r == len(region) <= N <= len(comp)
    U = np.zeros((1, L, N), dtype=np.complex128)
    ext = np.zeros(N)
    ext[:r] = lam
    U[0][np.ix_(comp, np.arange(N))] = fourier_columns(comp, N, rng) * np.sqrt(1.0 - ext)[None, :]
    U[0][np.ix_(region, np.arange(r))] = fourier_columns(region, r, rng) * np.sqrt(lam)[None, :]
    return U


def entropy_bound(lam, delta):
    b = np.abs(h(lam + delta) - h(lam)) + np.abs(h(lam - delta) - h(lam))
    return float(b.sum())


def check_region(sim, L, N, region, seed):
    rng = np.random.default_rng(seed)
    lam = spectrum_mix(len(region), rng)
    sim.set_state(known_state(L, N, region, lam, rng), 0)
    n = len(region)
    delta = 200 * n * EPS
    got = np.sort(sim.region_spectrum(region)[0])
    want = np.sort(lam)
    err = float(np.max(np.abs(got - want)))
    print(f"  l={n}: max |d lambda| = {err:.2e} (allowed {delta:.1e})", flush=True)
    assert err <= delta
    S = sim.entropy(region)[0]
    S_exact = float(h(lam).sum())
    tol = entropy_bound(lam, delta)
    print(f"  l={n}: S = {S:.12f}, exact {S_exact:.12f}, |dS| = {abs(S - S_exact):.2e} "
          f"(allowed {tol:.1e})", flush=True)
    assert abs(S - S_exact) <= tol


@pytest.mark.parametrize("path", [1, 2])
def test_known_spectrum_ring_16384(path):
    """1d ring L=16384, N=8192 (the long-chain projective workload): contiguous regions of
    1024, 4096 and 8192 sites, with the one-stage (path 1) and the two-stage (path 2)
    reduction."""
    L, N = 16384, 8192
    sim = make_sim(1, L, n_traj=1)
    sim.set_eig_path(path)
    for l, seed in ((1024, 11), (4096, 12), (8192, 13)):
        check_region(sim, L, N, list(range(l)), seed)
    sim.close()


def test_known_spectrum_torus_160():
    """2d torus 160 x 160 (L=25600, N=12800): the union A u B of the strips x in [0, 40) and
    [80, 120), 12800 sites (the default form: two stages at this order)."""
    Lx = Ly = 160
    L, N = Lx * Ly, Lx * Ly // 2
    region = sorted(x + Lx * y for y in range(Ly) for x in list(range(0, 40)) + list(range(80, 120)))
    sim = make_sim(2, Lx, Ly, n_traj=1)
    check_region(sim, L, N, region, 21)
    sim.close()


def test_known_spectrum_batched_medium():
    """Three trajectories, L=1200, N=600: regions of 150 and 600 sites (batched grid-wide
    reduction, one wave per eigenvalue in the bisection)."""
    L, N, B = 1200, 600, 3
    sim = make_sim(1, L, n_traj=B)
    for l, seed in ((150, 31), (600, 32)):
        rng = np.random.default_rng(seed)
        region = sorted(rng.choice(L, l, replace=False).tolist())
        lams = [spectrum_mix(l, rng) for _ in range(B)]
        U = np.concatenate([known_state(L, N, region, lam, rng) for lam in lams])
        sim.set_state(U, 0)
        got = sim.region_spectrum(region)
        S = sim.entropy(region)
        delta = 200 * l * EPS
        for t in range(B):
            err = float(np.max(np.abs(np.sort(got[t]) - np.sort(lams[t]))))
            assert err <= delta, (l, t, err)
            assert abs(S[t] - h(lams[t]).sum()) <= entropy_bound(lams[t], delta)
    sim.close()


def coupled_state(L, N, A1, A2, lam, eps, rng):
    """Like known_state for the region A1 u A2 (|A1| = |A2| = l/2), but each pair of orbitals
    mixes a Fourier vector on A1 with one on A2 by the angle eps: C_A keeps the eigenvalues
    lam while its A1-A2 block is of order eps."""
    A1, A2 = np.asarray(A1), np.asarray(A2)
    region = np.concatenate([A1, A2])
    comp = np.setdiff1d(np.arange(L), region)
    h_ = len(A1)
    r = len(lam)
    assert r == 2 * h_ and len(A2) == h_ and r <= N <= len(comp)
    F1 = fourier_columns(A1, h_, rng)
    F2 = fourier_columns(A2, h_, rng)
    a = np.zeros((L, r), dtype=np.complex128)
    c, s_ = np.cos(eps), np.sin(eps)
    a[A1, :h_] = c * F1
    a[A2, :h_] = s_ * F2
    a[A1, h_:] = -s_ * F1
    a[A2, h_:] = c * F2
    U = np.zeros((1, L, N), dtype=np.complex128)
    ext = np.zeros(N)
    ext[:r] = lam
    U[0][np.ix_(comp, np.arange(N))] = fourier_columns(comp, N, rng) * np.sqrt(1.0 - ext)[None, :]
    U[0][:, :r] += a * np.sqrt(lam)[None, :]
    return U


@pytest.mark.parametrize("half", [40, 100])
def test_known_spectrum_with_tiny_couplings(half):
    """Householder reflectors formed from columns whose entries are ~1e-160 (their squares are
    subnormal): the spectrum must stay exact.  half=40: the in-LDS reduction (n = 80);
    half=100: the grid-wide reduction (n = 200)."""
    L, N = 4 * half + 64, 2 * half + 32
    rng = np.random.default_rng(half)
    A1 = list(range(0, half))
    A2 = list(range(L // 2, L // 2 + half))
    region = sorted(A1 + A2)
    sim = make_sim(1, L, n_traj=1, N=N, occupied=list(range(N)))
    for eps in (1e-160, 1e-100, 1e-30):
        lam = spectrum_mix(2 * half, rng)
        sim.set_state(coupled_state(L, N, A1, A2, lam, eps, rng), 0)
        got = np.sort(sim.region_spectrum(region)[0])
        err = float(np.max(np.abs(got - np.sort(lam))))
        assert err <= 200 * len(region) * EPS, (eps, err)
    sim.close()


def test_known_spectrum_blocked_reduction():
    """40 trajectories, L=1300, N=650, a random region of 650 sites: enough work for the
    blocked reduction (panels of 32 reflectors, the last panel ragged, then the 88-column block
    in LDS); every trajectory's spectrum and entropy against its known spectrum."""
    L, N, B, l = 1300, 650, 40, 650
    rng = np.random.default_rng(41)
    region = sorted(rng.choice(L, l, replace=False).tolist())
    lams = [spectrum_mix(l, rng) for _ in range(B)]
    U = np.concatenate([known_state(L, N, region, lam, rng) for lam in lams])
    sim = make_sim(1, L, n_traj=B)
    sim.set_state(U, 0)
    got = sim.region_spectrum(region)
    S = sim.entropy(region)
    delta = 200 * l * EPS
    for t in range(B):
        err = float(np.max(np.abs(np.sort(got[t]) - np.sort(lams[t]))))
        assert err <= delta, (t, err)
        assert abs(S[t] - h(lams[t]).sum()) <= entropy_bound(lams[t], delta)
    sim.close()


def test_known_spectrum_with_tiny_couplings_blocked():
    """The tiny-coupling states of the test above at n = 650 in a batch of 40 (the blocked
    reduction): reflectors of columns with entries ~1e-160 keep the spectrum exact."""
    half, B = 325, 40
    L, N = 4 * half + 64, 2 * half + 32
    rng = np.random.default_rng(half)
    A1 = list(range(0, half))
    A2 = list(range(L // 2, L // 2 + half))
    region = sorted(A1 + A2)
    sim = make_sim(1, L, n_traj=B, N=N, occupied=list(range(N)))
    lams, Us = [], []
    for t in range(B):
        eps = (1e-160, 1e-100, 1e-30, 0.3)[t % 4]
        lam = spectrum_mix(2 * half, rng)
        lams.append(lam)
        Us.append(coupled_state(L, N, A1, A2, lam, eps, rng))
    sim.set_state(np.concatenate(Us), 0)
    got = sim.region_spectrum(region)
    for t in range(B):
        err = float(np.max(np.abs(np.sort(got[t]) - np.sort(lams[t]))))
        assert err <= 200 * len(region) * EPS, (t, err)
    sim.close()


def test_known_spectrum_blocked_tiled_batch():
    """14 trajectories, L=2200, N=1100, a random region of 1100 sites: the blocked reduction with
    the tiled lower-triangle A v for trailing blocks of 1024 and more (ragged 64 x 64 tiles), then
    whole columns, a ragged last panel and the LDS tail; every spectrum and entropy against its
    known spectrum."""
    L, N, B, l = 2200, 1100, 14, 1100
    rng = np.random.default_rng(51)
    region = sorted(rng.choice(L, l, replace=False).tolist())
    lams = [spectrum_mix(l, rng) for _ in range(B)]
    U = np.concatenate([known_state(L, N, region, lam, rng) for lam in lams])
    sim = make_sim(1, L, n_traj=B)
    sim.set_eig_path(1)  # the one-stage form (the default takes two stages at this order)
    sim.set_state(U, 0)
    got = sim.region_spectrum(region)
    S = sim.entropy(region)
    delta = 200 * l * EPS
    for t in range(B):
        err = float(np.max(np.abs(np.sort(got[t]) - np.sort(lams[t]))))
        assert err <= delta, (t, err)
        assert abs(S[t] - h(lams[t]).sum()) <= entropy_bound(lams[t], delta)
    sim.close()
