"""Seeded synthetic workloads for the CDUGKS step.

This module holds only problem definitions and initial moment fields
(rho, u, T) plus the random draws that make them; it contains none of the
scheme's arithmetic, so both the GPU path and the CPU oracle take their inputs
from here.

A problem is a plain dict:

    dim, n[D], lo[D], hi[D], bc[D] ('periodic' | 'outflow' | 'dirichlet'),
    dirichlet[D] (Dirichlet dims: [[rho, u_1..u_D, T] low, [..] high], else None),
    nv[D], vmin[D], vmax[D], quad ('trapezoid' | 'boole'),
    gamma, Pr, R, omega, relax ('kn' | 'mu' | 'tau'), Kn, L_ref, rho_ref, T_ref,
    mu_ref, tau, cfl, dt (None -> from cfl), storage ('f64' | 'f32'),
    steps (number of steps the workload runs),
    rho[N], u[D][N], T[N]  (cells row-major, x fastest).

The initial conditions follow Sec. 3 of the paper (Sod, Kelvin-Helmholtz,
shear, Gresho vortex) with the sizes of the benchmark configurations; random
fields use SplitMix64 so that every consumer sees the same numbers.
"""
from __future__ import annotations

import math

import numpy as np

MASK64 = (1 << 64) - 1


class SplitMix64:
    """Counter-based generator (Steele, Lea & Flood 2014): state += golden gamma,
    then two xor-shift-multiply rounds."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self, a: float = 0.0, b: float = 1.0) -> float:
        return a + (b - a) * ((self.next_u64() >> 11) * (1.0 / 9007199254740992.0))

    def integer(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi] (inclusive)."""
        span = hi - lo + 1
        return lo + int(self.uniform() * span) % span

    def uniform_array(self, n: int, a: float, b: float) -> np.ndarray:
        return np.array([self.uniform(a, b) for _ in range(n)])


def cell_centres(dim, n, lo, hi):
    """Cell-centre coordinates as a list of D arrays of shape (N,), x fastest."""
    axes = [lo[d] + (np.arange(n[d]) + 0.5) * (hi[d] - lo[d]) / n[d] for d in range(dim)]
    grids = np.meshgrid(*axes[::-1], indexing="ij")  # slowest first
    return [g.reshape(-1) for g in grids[::-1]]


def _base(dim, n, lo, hi, bc, nv, vmin, vmax, **kw):
    p = dict(dim=dim, n=list(n), lo=list(lo), hi=list(hi), bc=list(bc), nv=list(nv),
             vmin=list(vmin), vmax=list(vmax), quad="trapezoid", gamma=5.0 / 3.0,
             Pr=2.0 / 3.0, R=0.5, omega=0.5, relax="kn", Kn=1e-3, L_ref=None,
             rho_ref=None, T_ref=1.0, mu_ref=None, tau=math.inf, cfl=0.5, dt=None,
             storage="f64", steps=1)
    p.update(kw)
    return p


def sod(n: int = 128, nv: int = 64, Kn: float = 1e-3, steps: int = 1024, boundary: str = "outflow", **kw):
    """1D Sod tube (Sec. 3.1 set-up, benchmark sizes): [0,1], left (1, 0, p=1),
    right (1/8, 0, p=1/10), gamma = 5/3, velocities on [-10, 10]; outflow
    ends, or Dirichlet ends holding the two initial states (the paper's)."""
    p = _base(1, [n], [0.0], [1.0], [boundary], [nv], [-10.0], [10.0], Kn=Kn,
              steps=steps, **kw)
    (x,) = cell_centres(1, p["n"], p["lo"], p["hi"])
    left = x <= 0.5
    rho = np.where(left, 1.0, 0.125)
    pres = np.where(left, 1.0, 0.1)
    p["rho"] = rho
    p["u"] = np.zeros((1, n))
    p["T"] = pres / (rho * p["R"])
    if boundary == "dirichlet":
        p["dirichlet"] = [[[1.0, 0.0, 1.0 / p["R"]], [0.125, 0.0, 0.1 / (0.125 * p["R"])]]]
    return p


def sod_validation(n: int = 1024, nv: int = 1025, mu_r: float = 1e-6, Pr: float = 2.0 / 3.0,
                   t_end: float = 0.15, **kw):
    """The Sec. 3.1 validation set-up: the Sod states on [0,1] with Dirichlet
    ends, K = 2 internal degrees of freedom (gamma = 7/5), hard-sphere
    viscosity exponent 1/2 with reference viscosity mu_r at T_r = 1, velocities
    on [-10, 10] with nv = 4k+1 points and the fourth-order Newton-Cotes
    (Boole) weights, CFL factor 0.75, run to t_end.  The step count is
    t_end / dt for the CFL step alpha dx / (2 max|xi|)."""
    if (nv - 1) % 4:
        raise ValueError("the Boole rule needs 4k+1 velocities")
    cfl = kw.pop("cfl", 0.75)
    steps = int(round(t_end * 2.0 * 10.0 * n / cfl))
    return sod(n=n, nv=nv, boundary="dirichlet", quad="boole", gamma=1.4, Pr=Pr, relax="mu",
               mu_ref=mu_r, T_ref=1.0, omega=0.5, cfl=cfl, steps=steps, **kw)


def thermoacoustic(n: int = 512, nv: int = 513, Pr: float = 2.0 / 3.0, delta: float = 0.05,
                   mu_r: float = 1e-3, t_end: float = 4.0, **kw):
    """Sec. 3 thermoacoustic wave: periodic [0,1] at pressure equilibrium,
    rho = 1 - delta sin 4 pi x, R T = P0 / rho with P0 = 1, u = 0; K = 2
    (gamma = 7/5), viscosity exponent 1/2 with mu_r at T_r = 1, velocities on
    [-10, 10] with nv = 4k+1 points (Boole weights), CFL factor 0.8."""
    cfl = kw.pop("cfl", 0.8)
    steps = int(round(t_end * 2.0 * 10.0 * n / cfl))
    p = _base(1, [n], [0.0], [1.0], ["periodic"], [nv], [-10.0], [10.0], quad="boole", gamma=1.4,
              Pr=Pr, relax="mu", mu_ref=mu_r, T_ref=1.0, omega=0.5, cfl=cfl, steps=steps, **kw)
    (x,) = cell_centres(1, p["n"], p["lo"], p["hi"])
    p["rho"] = 1.0 - delta * np.sin(4.0 * math.pi * x)
    p["u"] = np.zeros((1, n))
    p["T"] = 1.0 / (p["rho"] * p["R"])
    return p


def sine_wave(n: int = 128, nv: int = 16385, T0: float = 0.1, mu_r: float = 1e-5, v0: float = 1.0,
              t_end: float = 0.5, **kw):
    """Sec. 3 sine-wave perturbation: periodic [0,1], rho = 1, v = v0 sin 2 pi x,
    T = T0 (the energy per mass is C_v T0 + v^2/2); K = 2 (gamma = 7/5),
    viscosity exponent 1/2 with mu_r at T_r = 1, velocities on [-6, 6] with
    nv = 4k+1 points (Boole weights), CFL factor 0.5.  T0 = 1 with t_end = 0.1
    is the convergence study's variant."""
    cfl = kw.pop("cfl", 0.5)
    quad = kw.pop("quad", "boole")
    steps = int(round(t_end * 2.0 * 6.0 * n / cfl))
    p = _base(1, [n], [0.0], [1.0], ["periodic"], [nv], [-6.0], [6.0], quad=quad, gamma=1.4,
              relax="mu", mu_ref=mu_r, T_ref=1.0, omega=0.5, cfl=cfl, steps=steps, **kw)
    (x,) = cell_centres(1, p["n"], p["lo"], p["hi"])
    p["rho"] = np.ones(n)
    p["u"] = (v0 * np.sin(2.0 * math.pi * x))[None, :]
    p["T"] = np.full(n, T0)
    return p


def kelvin_helmholtz(n: int = 256, nv: int = 28, Kn: float = 1e-4, steps: int = 2000,
                     seed: int = 2208, storage: str = "f64", **kw):
    """2D sharp-interface Kelvin-Helmholtz layer (Sec. 3.3 family): periodic
    [-1/2, 1/2]^2, rho = 2 in |y| < 1/4 else 1, u_x = +-1/2, P = 2,
    v_y = 0.01 sin(4 pi x) + U(-1e-3, 1e-3) (one draw per cell, x fastest)."""
    p = _base(2, [n, n], [-0.5, -0.5], [0.5, 0.5], ["periodic", "periodic"], [nv, nv],
              [-8.0, -8.0], [8.0, 8.0], Kn=Kn, steps=steps, storage=storage, **kw)
    x, y = cell_centres(2, p["n"], p["lo"], p["hi"])
    inside = np.abs(y) < 0.25
    rho = np.where(inside, 2.0, 1.0)
    ux = np.where(inside, 0.5, -0.5)
    rng = SplitMix64(seed)
    noise = rng.uniform_array(n * n, -1e-3, 1e-3)
    uy = 0.01 * np.sin(4.0 * math.pi * x) + noise
    p["rho"] = rho
    p["u"] = np.stack([ux, uy])
    p["T"] = 2.0 / (rho * p["R"])
    return p


def shear3d(n: int = 64, nv: int = 16, Kn: float = 1e-3, steps: int = 500,
            storage: str = "f32", **kw):
    """3D sine-wave shear: periodic [0,1]^3, rho = 1, T = 1, u_x = 0.1 sin(2 pi y)."""
    p = _base(3, [n, n, n], [0.0] * 3, [1.0] * 3, ["periodic"] * 3, [nv] * 3,
              [-6.0] * 3, [6.0] * 3, Kn=Kn, steps=steps, storage=storage, **kw)
    x, y, z = cell_centres(3, p["n"], p["lo"], p["hi"])
    N = n ** 3
    p["rho"] = np.ones(N)
    p["u"] = np.stack([0.1 * np.sin(2.0 * math.pi * y), np.zeros(N), np.zeros(N)])
    p["T"] = np.ones(N)
    return p


def random_fourier_field(rng: SplitMix64, dim: int, coords, modes: int = 5):
    """S(x) = sum_m c_m cos(2 pi k_m.x + theta_m) / sum_m |c_m| with integer wave
    vectors k_m in {-4..4}^D \\ {0}, c_m ~ U(-1, 1), theta_m ~ U(0, 2 pi)."""
    acc = np.zeros_like(coords[0])
    norm = 0.0
    for _ in range(modes):
        while True:
            k = [rng.integer(-4, 4) for _ in range(dim)]
            if any(k):
                break
        c = rng.uniform(-1.0, 1.0)
        th = rng.uniform(0.0, 2.0 * math.pi)
        phase = sum(2.0 * math.pi * k[d] * coords[d] for d in range(dim))
        acc = acc + c * np.cos(phase + th)
        norm += abs(c)
    return acc / max(norm, 1e-300)


def random_fourier(dim: int, n, nv, rng: SplitMix64, amp: float = 0.1, **kw):
    """Smooth periodic state on [0,1]^D: rho, T = 1 + amp S, u_d = amp S."""
    p = _base(dim, list(n), [0.0] * dim, [1.0] * dim, ["periodic"] * dim, list(nv),
              [-6.0] * dim, [6.0] * dim, **kw)
    coords = cell_centres(dim, p["n"], p["lo"], p["hi"])
    p["rho"] = 1.0 + amp * random_fourier_field(rng, dim, coords)
    p["T"] = 1.0 + amp * random_fourier_field(rng, dim, coords)
    p["u"] = np.stack([amp * random_fourier_field(rng, dim, coords) for _ in range(dim)])
    return p


def gresho_profile(r):
    """Triangular Gresho vortex (Sec. 3.6): azimuthal speed (peak 1 at r = 0.2)
    and the balancing pressure with P0 = 5."""
    r = np.asarray(r, dtype=np.float64)
    P0 = 5.0
    uphi = np.where(r <= 0.2, 5.0 * r, np.where(r <= 0.4, 2.0 - 5.0 * r, 0.0))
    rs = np.maximum(r, 1e-300)
    P = np.where(
        r <= 0.2, P0 + 12.5 * r * r,
        np.where(r <= 0.4, P0 + 12.5 * r * r + 4.0 * (1.0 - 5.0 * r - math.log(0.2) + np.log(rs)),
                 P0 - 2.0 + 4.0 * math.log(2.0)))
    return uphi, P


def vortex(n: int, nv: int, **kw):
    """Gresho vortex centred at (1/2, 1/2) on periodic [0,1]^2, rho = 1,
    velocities on [-10, 10]^2."""
    p = _base(2, [n, n], [0.0, 0.0], [1.0, 1.0], ["periodic", "periodic"], [nv, nv],
              [-10.0, -10.0], [10.0, 10.0], **kw)
    x, y = cell_centres(2, p["n"], p["lo"], p["hi"])
    dx, dy = x - 0.5, y - 0.5
    r = np.hypot(dx, dy)
    uphi, P = gresho_profile(r)
    rs = np.maximum(r, 1e-300)
    p["rho"] = np.ones(n * n)
    p["u"] = np.stack([-uphi * dy / rs, uphi * dx / rs])
    p["T"] = P / (1.0 * p["R"])
    return p


def batched(count: int = 256, seed: int = 9132, storage: str = "f32"):
    """Uneven batch: 1D (Nx 64..1024, Nv 32..128) or 2D (n^2 with n 32..256,
    m^2 velocities with m 16..32) with probability 1/2 each; Kn log-uniform in
    [1e-4, 10]; Pr in {1/2, 2/3, 1, 2}; random-Fourier states (5 modes,
    amplitude 0.1); periodic; velocity box [-6, 6]^D."""
    rng = SplitMix64(seed)
    probs = []
    for _ in range(count):
        if rng.uniform() < 0.5:
            dim, n, nv = 1, [rng.integer(64, 1024)], [rng.integer(32, 128)]
        else:
            k, m = rng.integer(32, 256), rng.integer(16, 32)
            dim, n, nv = 2, [k, k], [m, m]
        Kn = 10.0 ** rng.uniform(-4.0, 1.0)
        Pr = [0.5, 2.0 / 3.0, 1.0, 2.0][rng.integer(0, 3)]
        probs.append(random_fourier(dim, n, nv, rng, Kn=Kn, Pr=Pr, storage=storage))
    return probs


def served_stream(count: int = 512, rate: float = 50.0, seed: int = 913, storage: str = "f32"):
    """Poisson arrivals of 2D solves: n^2 cells with n 64..512, m^2 velocities
    with m 16..32, half Gresho vortex and half random-Fourier states, Kn
    log-uniform in [1e-4, 1], 200..2000 steps each.  Returns a list of
    (arrival_time_s, problem)."""
    rng = SplitMix64(seed)
    t = 0.0
    out = []
    for _ in range(count):
        t += -math.log(max(1.0 - rng.uniform(), 1e-300)) / rate
        n, m = rng.integer(64, 512), rng.integer(16, 32)
        Kn = 10.0 ** rng.uniform(-4.0, 0.0)
        steps = rng.integer(200, 2000)
        if rng.uniform() < 0.5:
            p = vortex(n, m, Kn=Kn, steps=steps, storage=storage)
        else:
            p = random_fourier(2, [n, n], [m, m], rng, Kn=Kn, steps=steps, storage=storage)
        out.append((t, p))
    return out


def scaled(p: dict, **changes) -> dict:
    """Copy of a problem with some scalar fields replaced (initial fields kept)."""
    q = dict(p)
    q.update(changes)
    return q
