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
    "mfq_get_state": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "mfq_set_state": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]),
    "mfq_synchronize": (ctypes.c_int32, [ctypes.c_void_p]),
    "mfq_profile": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "mfq_use_graphs": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "mfq_phase_times": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
}

PHASES = ("propagate", "measure", "reorth", "observe")

EXPORTED = tuple(_SIGS)


def lib():
    """Load libmfq.so (built in-tree by __graft_entry__.build()); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() first")
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


def mfq_get_state(ctx, n_traj, L, N):
    U = np.zeros((n_traj, N, L), dtype=np.complex128)  # column-major L x N per trajectory
    step = ctypes.c_int64()
    _check(ctx, lib().mfq_get_state(ctx, _ptr(U), ctypes.byref(step)))
    return np.ascontiguousarray(U.transpose(0, 2, 1)), step.value


def mfq_set_state(ctx, U, step):
    Uc = np.ascontiguousarray(np.asarray(U, dtype=np.complex128).transpose(0, 2, 1))
    _check(ctx, lib().mfq_set_state(ctx, _ptr(Uc), int(step)))


def mfq_synchronize(ctx):
    _check(ctx, lib().mfq_synchronize(ctx))


def mfq_use_graphs(ctx, enable):
    _check(ctx, lib().mfq_use_graphs(ctx, 1 if enable else 0))


def mfq_profile(ctx, enable):
    _check(ctx, lib().mfq_profile(ctx, 1 if enable else 0))


def mfq_phase_times(ctx):
    ms = np.zeros(len(PHASES))
    cnt = np.zeros(len(PHASES), dtype=np.int64)
    _check(ctx, lib().mfq_phase_times(ctx, _ptr(ms), _ptr(cnt)))
    return {ph: (float(ms[i]), int(cnt[i])) for i, ph in enumerate(PHASES)}


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

    def pm_events(self, max_events=None):
        return mfq_pm_events(self.ctx, self.n_traj, self.L if max_events is None else max_events)

    def get_state(self):
        return mfq_get_state(self.ctx, self.n_traj, self.L, self.N)

    def set_state(self, U, step):
        mfq_set_state(self.ctx, U, step)

    def synchronize(self):
        mfq_synchronize(self.ctx)

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
