"""Python binding of the CDUGKS C ABI (``include/cdugks.h``).

Argument marshalling only: every stage of a time step runs in the HIP kernels
of ``libcdugks.so``.  PyTorch supplies the device memory (arenas) and the
stream when a caller wants them; plain use needs only numpy.

The functions keep the C names (``cdugks_init``, ``cdugks_step``, ...); the
``Solver`` class wraps one context.  Loading fails loudly when the HIP library
has not been built -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; CDUGKS_LIBRARY may name another build of the same ABI
LIB_PATH = os.environ.get("CDUGKS_LIBRARY") or os.path.join(HERE, "libcdugks.so")

OK, PENDING = 0, 1
ERR_INVALID, ERR_NOMEM, ERR_DEVICE, ERR_NONPHYSICAL, ERR_TOO_LARGE, ERR_BUSY, ERR_UNKNOWN = -1, -2, -3, -4, -5, -6, -7
BC = {"periodic": 0, "outflow": 1, "dirichlet": 2}
RELAX = {"kn": 0, "mu": 1, "tau": 2}
QUAD = {"trapezoid": 0, "boole": 1}
STORE = {"f64": 0, "f32": 1, "f32_bf16tail": 2}
RECON = {"slopes_of_slopes": 0, "single_slope": 1}

ERROR_NAMES = {ERR_INVALID: "ERR_INVALID", ERR_NOMEM: "ERR_NOMEM", ERR_DEVICE: "ERR_DEVICE",
               ERR_NONPHYSICAL: "ERR_NONPHYSICAL", ERR_TOO_LARGE: "ERR_TOO_LARGE", ERR_BUSY: "ERR_BUSY",
               ERR_UNKNOWN: "ERR_UNKNOWN"}


class CdugksError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class cdugks_space(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int64 * 3), ("lo", ctypes.c_double * 3),
                ("hi", ctypes.c_double * 3), ("bc", ctypes.c_int * 3),
                ("dirichlet", ctypes.c_double * 30)]  # [3][2][5]: (rho, u_x, u_y, u_z, T)


class cdugks_velocity(ctypes.Structure):
    _fields_ = [("nv", ctypes.c_int64 * 3), ("vmin", ctypes.c_double * 3), ("vmax", ctypes.c_double * 3),
                ("quadrature", ctypes.c_int)]


class cdugks_params(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("Pr", ctypes.c_double), ("R", ctypes.c_double),
                ("omega", ctypes.c_double), ("relax_mode", ctypes.c_int), ("Kn", ctypes.c_double),
                ("L_ref", ctypes.c_double), ("rho_ref", ctypes.c_double), ("T_ref", ctypes.c_double),
                ("mu_ref", ctypes.c_double), ("tau", ctypes.c_double), ("cfl", ctypes.c_double),
                ("dt", ctypes.c_double), ("storage", ctypes.c_int), ("velocity_slices", ctypes.c_int),
                ("reconstruction", ctypes.c_int), ("face_tile", ctypes.c_int),
                ("accel", ctypes.c_double * 3)]


_lib = None
_DP = ctypes.POINTER(ctypes.c_double)


def load_library():
    """Load ``libcdugks.so``; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"CDUGKS HIP library not built: {LIB_PATH} is missing "
                          "(run __graft_entry__.build() or python -m paper_2208_09132_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t
    sig = {
        "cdugks_required_bytes": (ctypes.c_int, [ctypes.POINTER(cdugks_space), ctypes.POINTER(cdugks_velocity),
                                                 ctypes.POINTER(cdugks_params), ctypes.POINTER(sz)]),
        "cdugks_init": (ctypes.c_int, [ctypes.POINTER(cdugks_space), ctypes.POINTER(cdugks_velocity),
                                       ctypes.POINTER(cdugks_params), _DP, _DP, _DP, vp, vp, sz,
                                       ctypes.POINTER(vp)]),
        "cdugks_regrid": (ctypes.c_int, [vp, ctypes.POINTER(cdugks_space), ctypes.POINTER(cdugks_velocity),
                                         ctypes.POINTER(cdugks_params), vp, vp, sz, ctypes.POINTER(vp)]),
        "cdugks_fit_velocity": (ctypes.c_int, [ctypes.POINTER(cdugks_space), ctypes.POINTER(cdugks_params), _DP,
                                               _DP, _DP, ctypes.c_double, ctypes.c_int,
                                               ctypes.POINTER(cdugks_velocity)]),
        "cdugks_step": (ctypes.c_int, [vp, i64]),
        "cdugks_sync": (ctypes.c_int, [vp]),
        "cdugks_moments": (ctypes.c_int, [vp, _DP, _DP, _DP, ctypes.c_int]),
        "cdugks_conserved": (ctypes.c_int, [vp, _DP]),
        "cdugks_distributions": (ctypes.c_int, [vp, _DP, _DP]),
        "cdugks_distributions_noalloc": (ctypes.c_int, [vp, _DP, _DP]),
        "cdugks_info": (ctypes.c_int, [vp, _DP, _DP, ctypes.POINTER(i64)]),
        "cdugks_launch_info": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                              ctypes.POINTER(ctypes.c_int)]),
        "cdugks_storage_info": (ctypes.c_int, [vp, ctypes.POINTER(i64), ctypes.POINTER(sz)]),
        "cdugks_profile_phases": (ctypes.c_int, [vp, i64, _DP]),
        "cdugks_destroy": (None, [vp]),
        "cdugks_batch_create": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, ctypes.POINTER(vp)]),
        "cdugks_batch_step": (ctypes.c_int, [vp, i64]),
        "cdugks_batch_destroy": (None, [vp]),
        "cdugks_server_create": (ctypes.c_int, [sz, ctypes.c_int, ctypes.c_int, vp, ctypes.POINTER(vp)]),
        "cdugks_submit": (ctypes.c_int, [vp, ctypes.POINTER(cdugks_space), ctypes.POINTER(cdugks_velocity),
                                         ctypes.POINTER(cdugks_params), _DP, _DP, _DP, i64,
                                         ctypes.POINTER(ctypes.c_uint64)]),
        "cdugks_poll": (ctypes.c_int, [vp, ctypes.c_uint64, _DP, _DP, _DP, _DP, _DP]),
        "cdugks_server_destroy": (None, [vp]),
        "cdugks_autotune": (ctypes.c_int, [vp, ctypes.c_int]),
        "cdugks_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def last_error() -> str:
    return load_library().cdugks_last_error().decode()


def check(rc: int) -> int:
    if rc < 0:
        raise CdugksError(rc, last_error())
    return rc


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_DP)


def describe(prob: dict):
    """Build the three ABI structs from a workload dict (see workloads.py)."""
    D = int(prob["dim"])
    sp = cdugks_space()
    ve = cdugks_velocity()
    pa = cdugks_params()
    sp.dim = D
    for d in range(3):
        if d < D:
            sp.n[d] = int(prob["n"][d])
            sp.lo[d] = float(prob["lo"][d])
            sp.hi[d] = float(prob["hi"][d])
            sp.bc[d] = BC[prob["bc"][d]]
            if prob["bc"][d] == "dirichlet":
                # prob["dirichlet"][d] = [[rho, u_1..u_D, T] low side, [...] high side]
                for side in range(2):
                    st = [float(x) for x in prob["dirichlet"][d][side]]
                    row = [st[0]] + st[1:1 + D] + [0.0] * (3 - D) + [st[1 + D]]
                    for k in range(5):
                        sp.dirichlet[(d * 2 + side) * 5 + k] = row[k]
            ve.nv[d] = int(prob["nv"][d])
            ve.vmin[d] = float(prob["vmin"][d])
            ve.vmax[d] = float(prob["vmax"][d])
        else:
            sp.n[d] = 1
            sp.hi[d] = 1.0
            ve.nv[d] = 1
    ve.quadrature = QUAD[prob.get("quad", "trapezoid")]
    pa.gamma = float(prob.get("gamma", 5.0 / 3.0))
    pa.Pr = float(prob.get("Pr", 2.0 / 3.0))
    pa.R = float(prob.get("R", 0.5))
    pa.omega = float(prob.get("omega", 0.5))
    pa.relax_mode = RELAX[prob.get("relax", "kn")]
    pa.Kn = float(prob.get("Kn") or 0.0)
    pa.L_ref = float(prob.get("L_ref") or 0.0)
    pa.rho_ref = float(prob.get("rho_ref") or 0.0)
    pa.T_ref = float(prob.get("T_ref") or 0.0)
    pa.mu_ref = float(prob.get("mu_ref") or 0.0)
    pa.tau = float(prob.get("tau", math.inf))
    pa.cfl = float(prob.get("cfl", 0.5))
    pa.dt = float(prob.get("dt") or 0.0)
    pa.storage = STORE[prob.get("storage", "f64")]
    pa.reconstruction = RECON[prob.get("reconstruction", "slopes_of_slopes")]
    pa.velocity_slices = int(prob.get("velocity_slices", 0))
    pa.face_tile = int(prob.get("face_tile", 0))
    acc = prob.get("accel") or [0.0] * D
    for d in range(D):
        pa.accel[d] = float(acc[d])
    return sp, ve, pa


def _fields(prob: dict):
    D = int(prob["dim"])
    N = int(np.prod([prob["n"][d] for d in range(D)]))
    rho = np.ascontiguousarray(prob["rho"], dtype=np.float64).reshape(N)
    u = np.ascontiguousarray(prob["u"], dtype=np.float64).reshape(D * N)
    T = np.ascontiguousarray(prob["T"], dtype=np.float64).reshape(N)
    return D, N, rho, u, T


def cdugks_required_bytes(prob: dict) -> int:
    sp, ve, pa = describe(prob)
    out = ctypes.c_size_t(0)
    check(load_library().cdugks_required_bytes(ctypes.byref(sp), ctypes.byref(ve), ctypes.byref(pa),
                                               ctypes.byref(out)))
    return out.value


def cdugks_init(prob: dict, stream=None, arena=None, arena_bytes: int = 0):
    sp, ve, pa = describe(prob)
    _, _, rho, u, T = _fields(prob)
    h = ctypes.c_void_p()
    check(load_library().cdugks_init(ctypes.byref(sp), ctypes.byref(ve), ctypes.byref(pa), _ptr(rho), _ptr(u),
                                     _ptr(T), stream, arena, arena_bytes, ctypes.byref(h)))
    return h


def fit_velocity(prob: dict, rho, u, T, tol: float, quad: str = "trapezoid") -> dict:
    """cdugks_fit_velocity for prob's space and gas at the moments rho, u, T:
    returns prob with nv, vmin, vmax and quad replaced by the fitted grid."""
    sp, _, pa = describe(prob)
    D = int(prob["dim"])
    rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
    T = np.ascontiguousarray(T, dtype=np.float64).reshape(-1)
    ve = cdugks_velocity()
    check(load_library().cdugks_fit_velocity(ctypes.byref(sp), ctypes.byref(pa), _ptr(rho), _ptr(u), _ptr(T),
                                             float(tol), 1 if quad == "boole" else 0, ctypes.byref(ve)))
    return dict(prob, nv=[int(ve.nv[d]) for d in range(D)], vmin=[ve.vmin[d] for d in range(D)],
                vmax=[ve.vmax[d] for d in range(D)], quad=quad)


def cdugks_step(ctx, nsteps: int) -> None:
    check(load_library().cdugks_step(ctx, int(nsteps)))


def cdugks_sync(ctx) -> None:
    check(load_library().cdugks_sync(ctx))


def cdugks_destroy(ctx) -> None:
    load_library().cdugks_destroy(ctx)


def _torch_stream_handle():
    """Handle of torch's current stream; a fresh default-priority stream when
    that is the null stream (graphs are not captured on the null stream)."""
    import torch  # plumbing only
    st = torch.cuda.current_stream()
    if st.cuda_stream == 0:
        st = torch.cuda.Stream()
    return st, ctypes.c_void_p(st.cuda_stream)


class Solver:
    """One problem on the GPU.  ``use_torch`` takes the arena from a torch
    tensor and the stream from torch's current stream."""

    def __init__(self, prob: dict, use_torch: bool = False, stream=None):
        # stream: a hipStream_t handle (ctypes.c_void_p or int) or None
        self.prob = prob
        self.D, self.N, _, _, _ = _fields(prob)
        self.V = int(np.prod([prob["nv"][d] for d in range(self.D)]))
        self._arena = None
        self._stream = None
        self._batch = None  # the live Batch this solver belongs to, if any
        arena, nbytes = None, 0
        if use_torch:
            import torch
            nbytes = cdugks_required_bytes(prob)
            self._arena = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
            base = self._arena.data_ptr()
            arena = ctypes.c_void_p((base + 255) & ~255)
            if stream is None:
                self._stream, stream = _torch_stream_handle()
        self.ctx = cdugks_init(prob, stream=stream, arena=arena, arena_bytes=nbytes)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            b = getattr(self, "_batch", None)
            if b is not None and getattr(b, "h", None) is not None:
                # the library refuses too (the batch refers to this context)
                raise CdugksError(ERR_BUSY, "solver belongs to a live batch; close the batch first")
            cdugks_destroy(self.ctx)
            self.ctx = None
        self._arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1) -> None:
        cdugks_step(self.ctx, n)

    def sync(self) -> None:
        cdugks_sync(self.ctx)

    def moments(self):
        rho = np.zeros(self.N)
        u = np.zeros(self.D * self.N)
        T = np.zeros(self.N)
        check(load_library().cdugks_moments(self.ctx, _ptr(rho), _ptr(u), _ptr(T), 0))
        return rho, u.reshape(self.D, self.N), T

    def moments_device(self, rho_ptr: int, u_ptr: int, T_ptr: int) -> None:
        c = ctypes.cast
        check(load_library().cdugks_moments(self.ctx, c(rho_ptr, _DP), c(u_ptr, _DP), c(T_ptr, _DP), 1))

    def conserved(self):
        W = np.zeros(self.N * (self.D + 2))
        check(load_library().cdugks_conserved(self.ctx, _ptr(W)))
        return W.reshape(self.N, self.D + 2)

    def distributions(self):
        g = np.zeros(self.V * self.N)
        b = np.zeros(self.V * self.N)
        check(load_library().cdugks_distributions(self.ctx, _ptr(g), _ptr(b)))
        return g.reshape(self.V, self.N), b.reshape(self.V, self.N)

    def info(self):
        dt, t = ctypes.c_double(), ctypes.c_double()
        n = ctypes.c_int64()
        check(load_library().cdugks_info(self.ctx, ctypes.byref(dt), ctypes.byref(t), ctypes.byref(n)))
        return dt.value, t.value, n.value

    def regrid(self, prob: dict) -> "Solver":
        """A new solver for ``prob`` (this problem's cells, gas and storage
        form on another velocity grid) holding this solver's state carried to
        that grid by cdugks_regrid; this solver is unchanged."""
        sp, ve, pa = describe(prob)
        h = ctypes.c_void_p()
        check(load_library().cdugks_regrid(self.ctx, ctypes.byref(sp), ctypes.byref(ve), ctypes.byref(pa), None,
                                           None, 0, ctypes.byref(h)))
        s = Solver.__new__(Solver)
        s.prob = prob
        s.D, s.N, _, _, _ = _fields(prob)
        s.V = int(np.prod([prob["nv"][d] for d in range(s.D)]))
        s._arena, s._stream, s._batch = None, None, None
        s.ctx = h
        return s

    def launch_info(self):
        """(face-sum tile shape, 1-based; face-sum velocity slices; update
        velocity slices)."""
        t, fs, us = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        check(load_library().cdugks_launch_info(self.ctx, ctypes.byref(t), ctypes.byref(fs), ctypes.byref(us)))
        return t.value, fs.value, us.value

    def storage_info(self):
        """(velocity rows held in BF16, bytes of one state array)."""
        n, nb = ctypes.c_int64(), ctypes.c_size_t()
        check(load_library().cdugks_storage_info(self.ctx, ctypes.byref(n), ctypes.byref(nb)))
        return n.value, nb.value

    def profile_phases(self, nsteps: int):
        """Mean per-step kernel durations (ms) from HIP events on the context's
        stream: face sums, face closure, cell closure, update."""
        ms = np.zeros(4)
        check(load_library().cdugks_profile_phases(self.ctx, int(nsteps), _ptr(ms)))
        return ms

    def autotune(self, steps_per_trial: int = 4) -> None:
        check(load_library().cdugks_autotune(self.ctx, int(steps_per_trial)))

    @property
    def dt(self) -> float:
        return self.info()[0]


class Batch:
    """Several Solvers advanced together (one launch per kernel phase for the
    whole batch, graphs of chunk_steps steps).  All solvers must share a stream."""

    def __init__(self, solvers, chunk_steps: int = 100):
        self.solvers = list(solvers)
        arr = (ctypes.c_void_p * len(self.solvers))(*[sv.ctx.value for sv in self.solvers])
        h = ctypes.c_void_p()
        check(load_library().cdugks_batch_create(arr, len(self.solvers), int(chunk_steps), ctypes.byref(h)))
        self.h = h
        for sv in self.solvers:
            sv._batch = self

    def step(self, n: int) -> None:
        check(load_library().cdugks_batch_step(self.h, int(n)))

    def close(self) -> None:
        if getattr(self, "h", None) is not None:
            load_library().cdugks_batch_destroy(self.h)
            self.h = None
            for sv in self.solvers:
                if sv._batch is self:
                    sv._batch = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching solve server (host thread inside the library)."""

    def __init__(self, hbm_budget: int, max_active: int = 64, chunk_steps: int = 100, stream=None):
        h = ctypes.c_void_p()
        check(load_library().cdugks_server_create(int(hbm_budget), int(max_active), int(chunk_steps), stream,
                                                  ctypes.byref(h)))
        self.h = h
        self._shapes = {}

    def submit(self, prob: dict, nsteps: int) -> int:
        sp, ve, pa = describe(prob)
        D, N, rho, u, T = _fields(prob)
        t = ctypes.c_uint64()
        check(load_library().cdugks_submit(self.h, ctypes.byref(sp), ctypes.byref(ve), ctypes.byref(pa), _ptr(rho),
                                           _ptr(u), _ptr(T), int(nsteps), ctypes.byref(t)))
        self._shapes[t.value] = (D, N)
        return t.value

    def poll(self, ticket: int):
        """None while pending; else (rho, u, T, t_queue_s, t_service_s).  Raises
        CdugksError if the request failed."""
        D, N = self._shapes[ticket]
        rho, u, T = np.zeros(N), np.zeros(D * N), np.zeros(N)
        tq, ts = ctypes.c_double(), ctypes.c_double()
        rc = load_library().cdugks_poll(self.h, ctypes.c_uint64(ticket), _ptr(rho), _ptr(u), _ptr(T),
                                        ctypes.byref(tq), ctypes.byref(ts))
        if rc == PENDING:
            return None
        del self._shapes[ticket]
        check(rc)
        return rho, u.reshape(D, N), T, tq.value, ts.value

    def close(self) -> None:
        if getattr(self, "h", None) is not None:
            load_library().cdugks_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
