"""Python binding of libmfq (ctypes).  Argument marshalling only.

Every function ``mfq_*`` here calls the C entry point of the same name in
``libmfq.so`` (declared in include/mfq.h).  Device memory for the workspace
comes from PyTorch (a uint8 CUDA tensor that the library borrows) and work is
ordered on PyTorch's current HIP stream.  There is no fallback: if the
library is not built, or no GPU is visible, the calls raise.
"""

import ctypes
import os

import numpy as np

PROJECTIVE = 0
HOMODYNE = 1
FP64 = 0
FP32_BULK = 1

MFQ_OK = 0
_ERRORS = {-1: "MFQ_EINVAL", -2: "MFQ_ENOMEM", -3: "MFQ_EDEVICE", -4: "MFQ_ENUMERIC", -5: "MFQ_ESTATE"}

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmfq.so")


class MfqError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRORS.get(code, code)}: {msg}")
        self.code = code


class Lattice(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("J", ctypes.c_double)]


class Job(ctypes.Structure):
    _fields_ = [("lat", Lattice), ("N", ctypes.c_int32), ("protocol", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("n_steps", ctypes.c_int32), ("obs_every", ctypes.c_int32),
                ("n_region", ctypes.c_int32), ("gamma", ctypes.c_double), ("dt", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("uid", ctypes.c_uint64), ("region", ctypes.c_void_p)]


class RunArgs(ctypes.Structure):
    _fields_ = [("protocol", ctypes.c_int32), ("gamma", ctypes.c_void_p), ("dt", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("n_steps", ctypes.c_int32), ("obs_every", ctypes.c_int32),
                ("region", ctypes.c_void_p), ("n_sites", ctypes.c_int32), ("S_host", ctypes.c_void_p),
                ("n_obs", ctypes.c_int32)]


TUNE_MAX_CANDIDATES = 16


class Tuning(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int32), ("tile", ctypes.c_int32), ("ms_per_step", ctypes.c_double),
                ("n_candidates", ctypes.c_int32), ("order", ctypes.c_int32), ("pm_path", ctypes.c_int32),
                ("reserved", ctypes.c_int32),
                ("candidate_ms", ctypes.c_double * TUNE_MAX_CANDIDATES),
                ("cand_path", ctypes.c_int32 * TUNE_MAX_CANDIDATES),
                ("cand_tile", ctypes.c_int32 * TUNE_MAX_CANDIDATES),
                ("cand_order", ctypes.c_int32 * TUNE_MAX_CANDIDATES),
                ("cand_pm", ctypes.c_int32 * TUNE_MAX_CANDIDATES)]


class EngineStats(ctypes.Structure):
    _fields_ = [("bytes_in_use", ctypes.c_uint64), ("peak_bytes", ctypes.c_uint64),
                ("budget_bytes", ctypes.c_uint64), ("queued", ctypes.c_int64), ("groups", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


MFQ_PENDING = 1
_lib = None

_SIGS = {
    "mfq_create": (ctypes.c_int32, [ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "mfq_destroy": (ctypes.c_int32, [ctypes.c_void_p]),
    "mfq_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "mfq_workspace_bytes": (ctypes.c_int32, [ctypes.POINTER(Lattice), ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "mfq_init_state": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Lattice), ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                        ctypes.c_void_p, ctypes.c_size_t]),
    "mfq_step": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_double,
                                  ctypes.c_uint64, ctypes.c_int32]),
    "mfq_entropy": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "mfq_region_spectrum": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                             ctypes.c_void_p]),
    "mfq_mutual_info": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.c_int32, ctypes.c_void_p]),
    "mfq_occupations": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p]),
    "mfq_pm_events": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p]),
    "mfq_ct_events": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32,
                                       ctypes.c_double, ctypes.c_int32]),
    "mfq_ct_last_events": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p]),
    "mfq_get_times": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p]),
    "mfq_set_ct_block": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "mfq_set_times": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p]),
    "mfq_get_state": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "mfq_set_state": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]),
    "mfq_get_slots": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "mfq_set_slots": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "mfq_synchronize": (ctypes.c_int32, [ctypes.c_void_p]),
    "mfq_profile": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "mfq_use_graphs": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "mfq_run": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_double,
                                 ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                 ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "mfq_set_path": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "mfq_set_pm_path": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "mfq_set_eig_path": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "mfq_autotune": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_double,
                                      ctypes.c_uint64, ctypes.c_int32, ctypes.c_void_p]),
    "mfq_set_tuning": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]),
    "mfq_set_tile_order": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "mfq_density_correlation": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p]),
    "mfq_density_correlation_noalloc": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p]),
    "mfq_set_propagator": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "mfq_set_integrator": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "mfq_run_group": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(RunArgs), ctypes.c_int32]),
    "mfq_propagator_band": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p]),
    "mfq_particle_covariance": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                                 ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "mfq_reset_trajectory": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64]),
    "mfq_engine_create": (ctypes.c_int32, [ctypes.c_int, ctypes.c_size_t, ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_void_p)]),
    "mfq_engine_destroy": (ctypes.c_int32, [ctypes.c_void_p]),
    "mfq_engine_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "mfq_engine_submit": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Job), ctypes.POINTER(ctypes.c_uint64)]),
    "mfq_engine_poll": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]),
    "mfq_engine_wait": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_double]),
    "mfq_engine_stats": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(EngineStats)]),
    "mfq_phase_times": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
}

PHASES = ("propagate", "measure", "reorth", "observe")

EXPORTED = tuple(_SIGS)


def lib():
    """Load libmfq.so (built in-tree by __graft_entry__.build()); raise if absent.

    PyTorch is imported first: its bundled HIP runtime carries the same soname as
    the one libmfq links against, so loading torch first makes both use one
    runtime (loading libmfq first would put two HIP runtimes in the process).
    """
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() first")
        import torch  # noqa: F401  (one HIP runtime per process, see above)
        l = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(l, name)
            f.restype = res
            f.argtypes = args
        _lib = l
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _i32(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.int32))


def _check(ctx, code):
    if code != MFQ_OK:
        msg = lib().mfq_last_error(ctx).decode() if ctx else ""
        raise MfqError(code, msg)


# ------------------------------------------------------------------ thin wrappers (same names)

def mfq_create(device=0, stream=None):
    out = ctypes.c_void_p()
    _check(None, lib().mfq_create(device, stream, ctypes.byref(out)))
    return out.value


def mfq_destroy(ctx):
    _check(None, lib().mfq_destroy(ctx))


def mfq_workspace_bytes(lat, N, n_traj, precision=FP64):
    b = ctypes.c_size_t()
    _check(None, lib().mfq_workspace_bytes(ctypes.byref(lat), N, n_traj, precision, ctypes.byref(b)))
    return b.value


def mfq_init_state(ctx, lat, N, n_traj, uids, occupied=None, precision=FP64, dev_ws=None, ws_bytes=0):
    u = np.ascontiguousarray(np.asarray(uids, dtype=np.uint64))
    assert u.size == n_traj
    occ = None if occupied is None else _i32(occupied)
    _check(ctx, lib().mfq_init_state(ctx, ctypes.byref(lat), N, n_traj, _ptr(u), _ptr(occ), precision,
                                     dev_ws, ws_bytes))


def mfq_step(ctx, protocol, gamma, dt, seed, n_steps=1):
    g = np.ascontiguousarray(np.asarray(gamma, dtype=np.float64))
    _check(ctx, lib().mfq_step(ctx, protocol, _ptr(g), float(dt), int(seed), int(n_steps)))


def mfq_entropy(ctx, region, n_traj):
    r = _i32(region)
    S = np.zeros(n_traj)
    _check(ctx, lib().mfq_entropy(ctx, _ptr(r), r.size, _ptr(S)))
    return S


def mfq_region_spectrum(ctx, region, n_traj, N):
    r = _i32(region)
    m = min(r.size, N)
    lam = np.zeros((n_traj, m))
    _check(ctx, lib().mfq_region_spectrum(ctx, _ptr(r), r.size, _ptr(lam)))
    return lam


def mfq_mutual_info(ctx, A, B, n_traj):
    a, b = _i32(A), _i32(B)
    I = np.zeros(n_traj)
    _check(ctx, lib().mfq_mutual_info(ctx, _ptr(a), a.size, _ptr(b), b.size, _ptr(I)))
    return I


def mfq_density_correlation(ctx, n_traj, L):
    """C(r) of Eq. (2), r = 1 .. L/2, per trajectory: an (n_traj, L//2) array."""
    Cr = np.zeros((n_traj, L // 2))
    _check(ctx, lib().mfq_density_correlation(ctx, _ptr(Cr)))
    return Cr


def mfq_density_correlation_noalloc(ctx, n_traj, L):
    """As mfq_density_correlation, with the library's per-GPU static buffer (no allocation)."""
    Cr = np.zeros((n_traj, L // 2))
    _check(ctx, lib().mfq_density_correlation_noalloc(ctx, _ptr(Cr)))
    return Cr


def mfq_particle_covariance(ctx, A, B, n_traj):
    a, b = _i32(A), _i32(B)
    G = np.zeros(n_traj)
    _check(ctx, lib().mfq_particle_covariance(ctx, _ptr(a), a.size, _ptr(b), b.size, _ptr(G)))
    return G


def mfq_occupations(ctx, n_traj, L):
    p = np.zeros((n_traj, L))
    _check(ctx, lib().mfq_occupations(ctx, _ptr(p)))
    return p


def mfq_pm_events(ctx, n_traj, max_events):
    cnt = np.zeros(n_traj, dtype=np.int32)
    sites = np.zeros((n_traj, max(max_events, 1)), dtype=np.int32)
    outc = np.zeros_like(sites)
    prob = np.zeros((n_traj, max(max_events, 1)))
    _check(ctx, lib().mfq_pm_events(ctx, max_events, _ptr(cnt), _ptr(sites), _ptr(outc), _ptr(prob)))
    return [[(int(sites[b, e]), float(prob[b, e]), int(outc[b, e])) for e in range(min(cnt[b], max_events))]
            for b in range(n_traj)]


def mfq_ct_events(ctx, gamma, seed, n_events, t_end=float("inf"), reorth_every=0):
    g = np.ascontiguousarray(gamma, dtype=np.float64)
    _check(ctx, lib().mfq_ct_events(ctx, _ptr(g), seed, n_events, float(t_end), reorth_every))


def mfq_ct_last_events(ctx, n_traj):
    site = np.zeros(n_traj, dtype=np.int32)
    outc = np.zeros(n_traj, dtype=np.int32)
    prob = np.zeros(n_traj)
    tau = np.zeros(n_traj)
    _check(ctx, lib().mfq_ct_last_events(ctx, _ptr(site), _ptr(outc), _ptr(prob), _ptr(tau)))
    return site, outc, prob, tau


def mfq_get_times(ctx, n_traj):
    t = np.zeros(n_traj)
    _check(ctx, lib().mfq_get_times(ctx, _ptr(t)))
    return t


def mfq_set_times(ctx, t):
    tt = np.ascontiguousarray(t, dtype=np.float64)
    _check(ctx, lib().mfq_set_times(ctx, _ptr(tt)))


def mfq_get_state(ctx, n_traj, L, N, contiguous=True):
    """(U, step); U[b] is L x N.  contiguous=False returns the transposed view of the
    column-major download (no second copy: large states)."""
    U = np.empty((n_traj, N, L), dtype=np.complex128)  # column-major L x N per trajectory
    step = ctypes.c_int64()
    _check(ctx, lib().mfq_get_state(ctx, _ptr(U), ctypes.byref(step)))
    V = U.transpose(0, 2, 1)
    return (np.ascontiguousarray(V) if contiguous else V), step.value


def mfq_set_state(ctx, U, step):
    Uc = np.ascontiguousarray(np.asarray(U, dtype=np.complex128).transpose(0, 2, 1))
    _check(ctx, lib().mfq_set_state(ctx, _ptr(Uc), int(step)))


def mfq_synchronize(ctx):
    _check(ctx, lib().mfq_synchronize(ctx))


PATH_AUTO, PATH_FUSED, PATH_LAUNCHES = 0, 1, 2
EIG_AUTO, EIG_ONE_STAGE, EIG_TWO_STAGE = 0, 1, 2


def mfq_run(ctx, protocol, gamma, dt, seed, n_steps, obs_every, region, n_traj, step_now):
    """Returns S as an (n_obs, n_traj) array."""
    g = np.ascontiguousarray(np.asarray(gamma, dtype=np.float64))
    r = _i32(region if region is not None else [])
    n_obs_expected = 0
    if obs_every > 0:
        n_obs_expected = (step_now + n_steps) // obs_every - step_now // obs_every
    S = np.zeros((max(n_obs_expected, 1), n_traj))
    n_obs = ctypes.c_int32()
    _check(ctx, lib().mfq_run(ctx, protocol, _ptr(g), float(dt), int(seed), int(n_steps), int(obs_every),
                              _ptr(r), r.size, _ptr(S), ctypes.byref(n_obs)))
    assert n_obs.value == n_obs_expected
    return S[:n_obs.value]


def mfq_run_group(sims, specs):
    """Several Trajectories objects advanced together (mfq_run_group): one fused launch when all
    fit the fused kernel, else one graph replayed for pairs of steps of all of them.  specs[k]:
    dict with protocol, gamma, dt, seed, n_steps and optionally obs_every, region.  Returns the
    list of S arrays (n_obs x n_traj) per context."""
    n = len(sims)
    ctxs = (ctypes.c_void_p * n)(*[s.ctx for s in sims])
    args = (RunArgs * n)()
    keep = []
    for k, (sim, sp) in enumerate(zip(sims, specs)):
        g = np.ascontiguousarray(np.broadcast_to(np.asarray(sp["gamma"], dtype=np.float64), (sim.n_traj,)))
        r = _i32(sp.get("region") or [])
        every = int(sp.get("obs_every", 0))
        step_now = sim.step_index()
        n_obs = (step_now + sp["n_steps"]) // every - step_now // every if every > 0 else 0
        S = np.zeros((max(n_obs, 1), sim.n_traj))
        keep += [g, r, S]
        args[k] = RunArgs(int(sp["protocol"]), g.ctypes.data, float(sp["dt"]), int(sp["seed"]),
                          int(sp["n_steps"]), every, r.ctypes.data if r.size else None, r.size,
                          S.ctypes.data, 0)
    code = lib().mfq_run_group(ctxs, args, n)
    if code != MFQ_OK:
        msgs = [lib().mfq_last_error(s.ctx).decode() for s in sims]
        raise MfqError(code, "; ".join(m for m in msgs if m))
    return [keep[3 * k + 2][:args[k].n_obs] for k in range(n)]


def mfq_reset_trajectory(ctx, slot, uid):
    _check(ctx, lib().mfq_reset_trajectory(ctx, int(slot), int(uid)))


TILE_AUTO, TILE_SMALL, TILE_LARGE = 0, 1, 2
ORDER_XCD, ORDER_LINEAR = 0, 1


def mfq_autotune(ctx, protocol, gamma, dt, seed, probe_steps):
    g = np.ascontiguousarray(np.asarray(gamma, dtype=np.float64))
    t = Tuning()
    _check(ctx, lib().mfq_autotune(ctx, int(protocol), _ptr(g), float(dt), int(seed), int(probe_steps),
                                   ctypes.byref(t)))
    n = t.n_candidates
    return {"path": t.path, "tile": t.tile, "order": t.order, "pm_path": t.pm_path,
            "ms_per_step": t.ms_per_step,
            "candidate_ms": [t.candidate_ms[i] for i in range(n)],
            "candidates": [{"path": t.cand_path[i], "tile": t.cand_tile[i], "order": t.cand_order[i],
                            "pm_path": t.cand_pm[i]} for i in range(n)]}


def mfq_set_tuning(ctx, path, tile):
    _check(ctx, lib().mfq_set_tuning(ctx, int(path), int(tile)))


def mfq_set_tile_order(ctx, order):
    _check(ctx, lib().mfq_set_tile_order(ctx, int(order)))


PROP_DENSE, PROP_FACTORED = 0, 1
INTEGRATOR_SPLIT, INTEGRATOR_RK4 = 0, 1


def mfq_set_propagator(ctx, form):
    _check(ctx, lib().mfq_set_propagator(ctx, int(form)))


def mfq_propagator_band(ctx):
    w = ctypes.c_int32()
    _check(ctx, lib().mfq_propagator_band(ctx, ctypes.byref(w)))
    return w.value


PM_AUTO, PM_WORKGROUP, PM_BLOCKED = 0, 1, 2


def mfq_set_pm_path(ctx, path):
    _check(ctx, lib().mfq_set_pm_path(ctx, int(path)))


def mfq_set_path(ctx, path):
    _check(ctx, lib().mfq_set_path(ctx, int(path)))


def mfq_use_graphs(ctx, enable):
    _check(ctx, lib().mfq_use_graphs(ctx, 1 if enable else 0))


def mfq_profile(ctx, enable):
    _check(ctx, lib().mfq_profile(ctx, 1 if enable else 0))


def mfq_phase_times(ctx):
    ms = np.zeros(len(PHASES))
    cnt = np.zeros(len(PHASES), dtype=np.int64)
    _check(ctx, lib().mfq_phase_times(ctx, _ptr(ms), _ptr(cnt)))
    return {ph: (float(ms[i]), int(cnt[i])) for i, ph in enumerate(PHASES)}


# ------------------------------------------------------------------ serving engine

class Engine:
    """Continuous-batching engine of the library (worker thread inside libmfq)."""

    def __init__(self, device=0, hbm_budget_bytes=0, max_slots=16):
        out = ctypes.c_void_p()
        _check(None, lib().mfq_engine_create(device, hbm_budget_bytes, max_slots, ctypes.byref(out)))
        self.h = out.value
        self._keep = {}

    def _err(self, code):
        if code not in (MFQ_OK, MFQ_PENDING):
            raise MfqError(code, lib().mfq_engine_last_error(self.h).decode())

    def submit(self, dim, Lx, Ly, protocol, gamma, dt, n_steps, seed, uid, region, obs_every=0,
               precision=FP64, J=1.0):
        r = _i32(region)
        j = Job(Lattice(dim, Lx, Ly if dim == 2 else 1, 0, J), 0, protocol, precision, n_steps, obs_every,
                r.size, float(gamma), float(dt), int(seed), int(uid), r.ctypes.data_as(ctypes.c_void_p))
        jid = ctypes.c_uint64()
        self._err(lib().mfq_engine_submit(self.h, ctypes.byref(j), ctypes.byref(jid)))
        return jid.value

    def poll(self, job_id, max_obs=4096):
        """None while pending, else (S array, latency seconds)."""
        S = np.zeros(max_obs)
        n = ctypes.c_int32()
        lat = ctypes.c_double()
        code = lib().mfq_engine_poll(self.h, job_id, _ptr(S), max_obs, ctypes.byref(n), ctypes.byref(lat))
        if code == MFQ_PENDING:
            return None
        self._err(code)
        return S[:n.value].copy(), lat.value

    def wait(self, job_id, timeout_s=600.0):
        code = lib().mfq_engine_wait(self.h, job_id, float(timeout_s))
        if code == MFQ_PENDING:
            raise TimeoutError(f"job {job_id} not done after {timeout_s} s")
        self._err(code)
        return self.poll(job_id)

    def stats(self):
        st = EngineStats()
        self._err(lib().mfq_engine_stats(self.h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in EngineStats._fields_ if f != "reserved"}

    def close(self):
        if getattr(self, "h", None):
            lib().mfq_engine_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ convenience object

class Trajectories:
    """n_traj trajectories of one lattice, resident in HBM, driven through the C ABI.

    The workspace is a PyTorch CUDA tensor; work runs on PyTorch's current stream.
    """

    def __init__(self, dim, Lx, Ly=1, N=None, n_traj=1, uids=None, occupied=None, J=1.0, device=0,
                 precision=FP64):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: libmfq runs only on the GPU")
        lib()
        self.lat = Lattice(dim, Lx, Ly if dim == 2 else 1, 0, J)
        self.L = Lx * (Ly if dim == 2 else 1)
        self.N = self.L // 2 if N is None else N
        self.n_traj = n_traj
        self.precision = precision
        self.uids = list(range(n_traj)) if uids is None else list(uids)
        self.device = device
        torch.cuda.set_device(device)
        self.stream = torch.cuda.current_stream(device)
        self.ctx = mfq_create(device, ctypes.c_void_p(self.stream.cuda_stream))
        nb = mfq_workspace_bytes(self.lat, self.N, n_traj, precision)
        self.ws = torch.empty(nb, dtype=torch.uint8, device=f"cuda:{device}")
        mfq_init_state(self.ctx, self.lat, self.N, n_traj, self.uids, occupied, precision,
                       ctypes.c_void_p(self.ws.data_ptr()), nb)

    def step(self, protocol, gamma, dt, seed, n_steps=1):
        g = np.broadcast_to(np.asarray(gamma, dtype=np.float64), (self.n_traj,))
        mfq_step(self.ctx, protocol, g, dt, seed, n_steps)

    def entropy(self, region):
        return mfq_entropy(self.ctx, region, self.n_traj)

    def region_spectrum(self, region):
        return mfq_region_spectrum(self.ctx, region, self.n_traj, self.N)

    def mutual_info(self, A, B):
        return mfq_mutual_info(self.ctx, A, B, self.n_traj)

    def occupations(self):
        return mfq_occupations(self.ctx, self.n_traj, self.L)

    def density_correlation(self):
        return mfq_density_correlation(self.ctx, self.n_traj, self.L)

    def density_correlation_noalloc(self):
        return mfq_density_correlation_noalloc(self.ctx, self.n_traj, self.L)

    def particle_covariance(self, A, B):
        return mfq_particle_covariance(self.ctx, A, B, self.n_traj)

    def pm_events(self, max_events=None):
        return mfq_pm_events(self.ctx, self.n_traj, self.L if max_events is None else max_events)

    def ct_events(self, gamma, seed, n_events, t_end=float("inf"), reorth_every=0):
        """Continuous-time projective protocol: n_events event slots (mfq_ct_events)."""
        g = np.broadcast_to(np.asarray(gamma, dtype=np.float64), (self.n_traj,))
        mfq_ct_events(self.ctx, g, seed, n_events, t_end, reorth_every)

    def set_ct_block(self, block):
        """Deferred continuous-time events (rings and tori): blocks of `block` events (0: one by one)."""
        _check(self.ctx, lib().mfq_set_ct_block(self.ctx, int(block)))

    def ct_last_events(self):
        """(site, outcome, p, tau) per trajectory for the latest event slot (site -1: none)."""
        return mfq_ct_last_events(self.ctx, self.n_traj)

    def times(self):
        return mfq_get_times(self.ctx, self.n_traj)

    def set_times(self, t):
        mfq_set_times(self.ctx, np.broadcast_to(np.asarray(t, dtype=np.float64), (self.n_traj,)))

    def get_state(self, contiguous=True):
        return mfq_get_state(self.ctx, self.n_traj, self.L, self.N, contiguous)

    def set_state(self, U, step):
        mfq_set_state(self.ctx, U, step)

    def get_slots(self):
        """(uids, step bases) of the trajectories (mfq_get_slots)."""
        uid = np.zeros(self.n_traj, dtype=np.uint64)
        base = np.zeros(self.n_traj, dtype=np.int64)
        _check(self.ctx, lib().mfq_get_slots(self.ctx, _ptr(uid), _ptr(base)))
        return uid, base

    def set_slots(self, uid, base):
        """Restore (uids, step bases) from a checkpoint (mfq_set_slots)."""
        u = np.ascontiguousarray(np.asarray(uid, dtype=np.uint64))
        b = np.ascontiguousarray(np.asarray(base, dtype=np.int64))
        _check(self.ctx, lib().mfq_set_slots(self.ctx, _ptr(u), _ptr(b)))
        self.uids = [int(x) for x in u]

    def synchronize(self):
        mfq_synchronize(self.ctx)

    def run(self, protocol, gamma, dt, seed, n_steps, obs_every=0, region=None):
        g = np.broadcast_to(np.asarray(gamma, dtype=np.float64), (self.n_traj,))
        return mfq_run(self.ctx, protocol, g, dt, seed, n_steps, obs_every, region, self.n_traj,
                       self.step_index())

    def step_index(self):
        step = ctypes.c_int64()
        _check(self.ctx, lib().mfq_get_state(self.ctx, None, ctypes.byref(step)))
        return step.value

    def reset_trajectory(self, slot, uid):
        mfq_reset_trajectory(self.ctx, slot, uid)
        self.uids[slot] = uid

    def set_path(self, path):
        mfq_set_path(self.ctx, path)

    def set_pm_path(self, path):
        mfq_set_pm_path(self.ctx, path)

    def set_eig_path(self, path):
        """EIG_AUTO, EIG_ONE_STAGE or EIG_TWO_STAGE (mfq_set_eig_path)."""
        _check(self.ctx, lib().mfq_set_eig_path(self.ctx, int(path)))

    def set_propagator(self, form):
        mfq_set_propagator(self.ctx, form)

    def set_integrator(self, integrator):
        """INTEGRATOR_SPLIT (default) or INTEGRATOR_RK4 for homodyne steps."""
        _check(self.ctx, lib().mfq_set_integrator(self.ctx, integrator))

    def propagator_band(self):
        return mfq_propagator_band(self.ctx)

    def autotune(self, protocol, gamma, dt, seed, probe_steps=4, cache=None):
        """Tune the execution form (mfq_autotune) or reuse a choice cached in the JSON file
        `cache` under a key of device architecture, lattice, N, batch, protocol and precision."""
        import json
        import os
        import torch
        props = torch.cuda.get_device_properties(self.device)
        arch = getattr(props, "gcnArchName", props.name)
        key = "|".join(str(x) for x in (arch, self.lat.dim, self.lat.Lx, self.lat.Ly, self.N,
                                         self.n_traj, protocol, self.precision))
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
        if key in table:
            t = table[key]
            mfq_set_tuning(self.ctx, t["path"], t["tile"])
            mfq_set_tile_order(self.ctx, t["order"])
            mfq_set_pm_path(self.ctx, t["pm_path"])
            return dict(t, cached=True)
        g = np.broadcast_to(np.asarray(gamma, dtype=np.float64), (self.n_traj,))
        res = mfq_autotune(self.ctx, protocol, g, dt, seed, probe_steps)
        if cache:
            table[key] = res
            os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
            with open(cache, "w") as f:
                json.dump(table, f, indent=1)
        return dict(res, cached=False)

    def set_tile_order(self, order):
        """GEMM workgroup -> tile order: ORDER_XCD (default) or ORDER_LINEAR (mfq_set_tile_order)."""
        mfq_set_tile_order(self.ctx, order)

    def use_graphs(self, enable=True):
        mfq_use_graphs(self.ctx, enable)

    def profile(self, enable=True):
        mfq_profile(self.ctx, enable)

    def phase_times(self):
        return mfq_phase_times(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            mfq_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
