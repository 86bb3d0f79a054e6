"""ctypes wrapper of the FP64 CDUGKS reference oracle -- TEST INFRASTRUCTURE.

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this module.  The product path never does.

The C source (``cdugks_oracle.c``) follows Sec. 2 and Sec. 2.1 of the paper
step by step; :func:`build` compiles it with gcc and OpenMP.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cdugks_oracle.c")
LIB = os.path.join(HERE, "libcdugks_oracle.so")

BC = {"periodic": 0, "outflow": 1, "dirichlet": 2}
QUAD = {"trapezoid": 0, "boole": 1}
RECON = {"slopes_of_slopes": 0, "single_slope": 1}


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/libcdugks_oracle.so``."""
    stale = not os.path.exists(LIB) or os.path.getmtime(LIB) < max(
        os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "cdugks_oracle.h")))
    if force or stale:
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
               "-o", tmp, SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("n", ctypes.c_long * 3),
        ("lo", ctypes.c_double * 3),
        ("hi", ctypes.c_double * 3),
        ("bc", ctypes.c_int * 3),
        ("dirichlet", ctypes.c_double * 30),
        ("nv", ctypes.c_long * 3),
        ("vmin", ctypes.c_double * 3),
        ("vmax", ctypes.c_double * 3),
        ("quad", ctypes.c_int),
        ("gamma", ctypes.c_double),
        ("Pr", ctypes.c_double),
        ("R", ctypes.c_double),
        ("relax_mode", ctypes.c_int),
        ("mu_ref", ctypes.c_double),
        ("T_ref", ctypes.c_double),
        ("omega", ctypes.c_double),
        ("tau", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("accel", ctypes.c_double * 3),
        ("reconstruction", ctypes.c_int),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_create.restype = ctypes.c_void_p
        lib.oracle_create.argtypes = [ctypes.POINTER(_Params)]
        lib.oracle_destroy.argtypes = [ctypes.c_void_p]
        lib.oracle_init.argtypes = [ctypes.c_void_p, dp, dp, dp]
        lib.oracle_init.restype = ctypes.c_int
        lib.oracle_step.argtypes = [ctypes.c_void_p, ctypes.c_long]
        lib.oracle_step.restype = ctypes.c_int
        lib.oracle_moments.argtypes = [ctypes.c_void_p, dp, dp, dp]
        lib.oracle_get_state.argtypes = [ctypes.c_void_p, dp, dp, dp]
        lib.oracle_set_state.argtypes = [ctypes.c_void_p, dp, dp, dp]
        lib.oracle_van_leer.restype = ctypes.c_double
        lib.oracle_van_leer.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.oracle_velocity_axis.argtypes = [ctypes.c_long, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_int, dp, dp]
        lib.oracle_equilibrium_moments.argtypes = [ctypes.c_void_p, ctypes.c_double, dp,
                                                   ctypes.c_double, dp]
        lib.oracle_regrid.restype = ctypes.c_int
        lib.oracle_regrid.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_time.restype = ctypes.c_double
        lib.oracle_time.argtypes = [ctypes.c_void_p]
        lib.oracle_num_steps.restype = ctypes.c_long
        lib.oracle_num_steps.argtypes = [ctypes.c_void_p]
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_num_threads.argtypes = []
        _lib = lib
    return _lib


def num_threads() -> int:
    return _load().oracle_num_threads()


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def van_leer(s1: float, s2: float) -> float:
    return _load().oracle_van_leer(float(s1), float(s2))


def velocity_axis(nv: int, vmin: float, vmax: float, quad: str = "trapezoid"):
    nodes = np.zeros(nv)
    w = np.zeros(nv)
    _load().oracle_velocity_axis(nv, vmin, vmax, QUAD[quad], _ptr(nodes), _ptr(w))
    return nodes, w


def mu_ref_from_kn(Kn: float, L: float, rho_mean: float, R: float = 0.5, T_ref: float = 1.0) -> float:
    """Hard-sphere reading of the Knudsen number: lambda = 16 mu/(5 rho sqrt(2 pi R T)),
    Kn = lambda/L at the reference state (reproduces mu_r = 1 <-> Kn ~ 3.2 for the
    Sod problem of Sec. 3.1)."""
    return 5.0 / 16.0 * Kn * L * rho_mean * math.sqrt(2.0 * math.pi * R * T_ref)


def cfl_dt(cfl: float, dx_min: float, xi_max: float) -> float:
    """Sec. 4: dt = alpha dx_min / (2 |xi_max|)."""
    return cfl * dx_min / (2.0 * xi_max)


def fit_velocity(rho, u, T, R: float, tol: float, quad: str = "trapezoid"):
    """Velocity grid fitted to moments rho[N], u[D][N], T[N] by the paper's
    criterion for its fixed grid (Sec. 5: resolve the mass and hold all of
    it, to an integration error tol), written out: per axis the box holds
    u_d +- k s of every cell, s = sqrt(R T), k = sqrt(2 ln(1/tol)) (one-sided
    normal tail at most exp(-k^2/2)/2 = tol/2); the spacing is at most
    pi sqrt(2) s_min / sqrt(ln(2/tol)), where the trapezoid rule's first
    aliasing error on a Gaussian, 2 exp(-2 pi^2 s^2/h^2), equals tol;
    nv = ceil(width/spacing) + 1, rounded up to 4n + 1 for Boole.  Returns
    (nv, vmin, vmax) lists."""
    u = np.asarray(u, dtype=np.float64)
    s = np.sqrt(R * np.asarray(T, dtype=np.float64))
    k = math.sqrt(2.0 * math.log(1.0 / tol))
    h = math.pi * float(s.min()) * math.sqrt(2.0) / math.sqrt(math.log(2.0 / tol))
    nv, vmin, vmax = [], [], []
    for d in range(u.shape[0]):
        lo, hi = float(np.min(u[d] - k * s)), float(np.max(u[d] + k * s))
        n = max(int(math.ceil((hi - lo) / h)) + 1, 2)
        if quad == "boole":
            n = (n - 1 + 3) // 4 * 4 + 1
        nv.append(n)
        vmin.append(lo)
        vmax.append(hi)
    return nv, vmin, vmax


class Oracle:
    """One CDUGKS problem on the CPU.

    ``prob`` is a dict with keys dim, n, lo, hi, bc (list of
    'periodic'/'outflow'/'dirichlet'), nv, vmin, vmax, quad, gamma, Pr, R,
    relax ('mu' or 'tau'), mu_ref, T_ref, omega, tau, dt, reconstruction
    ('slopes_of_slopes', the paper's, or 'single_slope'), and for Dirichlet
    dimensions ``dirichlet[d] = [[rho, u_1..u_D, T] low side, [..] high side]``,
    and optionally ``accel`` (the external acceleration a, D components).
    """

    def __init__(self, prob: dict):
        lib = _load()
        p = _Params()
        D = int(prob["dim"])
        p.dim = D
        for d in range(3):
            if d < D:
                p.n[d] = int(prob["n"][d])
                p.lo[d] = float(prob["lo"][d])
                p.hi[d] = float(prob["hi"][d])
                p.bc[d] = BC[prob["bc"][d]]
                if prob["bc"][d] == "dirichlet":
                    for side in range(2):
                        st = [float(x) for x in prob["dirichlet"][d][side]]
                        rho, u, T = st[0], st[1:1 + D], st[1 + D]
                        row = [rho] + u + [0.0] * (3 - D) + [T]
                        for k in range(5):
                            p.dirichlet[(d * 2 + side) * 5 + k] = row[k]
                p.nv[d] = int(prob["nv"][d])
                p.vmin[d] = float(prob["vmin"][d])
                p.vmax[d] = float(prob["vmax"][d])
            else:
                p.n[d] = 1
                p.nv[d] = 1
                p.lo[d], p.hi[d] = 0.0, 1.0
        p.quad = QUAD[prob.get("quad", "trapezoid")]
        p.gamma = float(prob.get("gamma", 5.0 / 3.0))
        p.Pr = float(prob.get("Pr", 2.0 / 3.0))
        p.R = float(prob.get("R", 0.5))
        relax = prob.get("relax", "mu")
        p.relax_mode = 0 if relax == "mu" else 1
        p.mu_ref = float(prob.get("mu_ref") or 1e-3)
        p.T_ref = float(prob.get("T_ref") or 1.0)
        p.omega = float(prob.get("omega", 0.5))
        tau = prob.get("tau")
        p.tau = math.inf if tau is None else float(tau)
        p.dt = float(prob["dt"])
        p.reconstruction = RECON[prob.get("reconstruction", "slopes_of_slopes")]
        acc = prob.get("accel") or [0.0] * D
        for d in range(D):
            p.accel[d] = float(acc[d])
        self._p = p
        self.D = D
        self.N = int(np.prod([prob["n"][d] for d in range(D)]))
        self.V = int(np.prod([prob["nv"][d] for d in range(D)]))
        h = lib.oracle_create(ctypes.byref(p))
        if not h:
            raise ValueError("oracle_create rejected the problem")
        self._h = ctypes.c_void_p(h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.oracle_destroy(h)
            self._h = None

    def init(self, rho, u, T):
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(self.N)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.D * self.N)
        T = np.ascontiguousarray(T, dtype=np.float64).reshape(self.N)
        rc = _load().oracle_init(self._h, _ptr(rho), _ptr(u), _ptr(T))
        if rc:
            raise ValueError(f"oracle_init failed ({rc})")

    def step(self, n: int = 1) -> int:
        return _load().oracle_step(self._h, int(n))

    def moments(self):
        rho = np.zeros(self.N)
        u = np.zeros(self.D * self.N)
        T = np.zeros(self.N)
        _load().oracle_moments(self._h, _ptr(rho), _ptr(u), _ptr(T))
        return rho, u.reshape(self.D, self.N), T

    def state(self):
        g = np.zeros(self.N * self.V)
        b = np.zeros(self.N * self.V)
        W = np.zeros(self.N * (self.D + 2))
        _load().oracle_get_state(self._h, _ptr(g), _ptr(b), _ptr(W))
        return g.reshape(self.N, self.V), b.reshape(self.N, self.V), W.reshape(self.N, self.D + 2)

    def set_state(self, g, b, W):
        g = np.ascontiguousarray(g, dtype=np.float64).reshape(-1)
        b = np.ascontiguousarray(b, dtype=np.float64).reshape(-1)
        W = np.ascontiguousarray(W, dtype=np.float64).reshape(-1)
        _load().oracle_set_state(self._h, _ptr(g), _ptr(b), _ptr(W))

    def equilibrium_moments(self, rho, u, T):
        uu = np.ascontiguousarray(u, dtype=np.float64).reshape(self.D)
        out = np.zeros(self.D + 2)
        _load().oracle_equilibrium_moments(self._h, float(rho), _ptr(uu), float(T), _ptr(out))
        return out

    def regrid_from(self, src: "Oracle") -> None:
        """Take src's state on this problem's velocity grid (an adaptive
        velocity grid, Sec. 5): W unchanged; phi = the equilibrium of W here
        plus src's phi - phi_eq interpolated multilinearly in velocity (zero
        outside src's velocity box)."""
        if _load().oracle_regrid(src._h, self._h) != 0:
            raise ValueError("oracle_regrid: the problems differ in cells or dimension")

    @property
    def time(self) -> float:
        return _load().oracle_time(self._h)

    @property
    def steps(self) -> int:
        return _load().oracle_num_steps(self._h)
