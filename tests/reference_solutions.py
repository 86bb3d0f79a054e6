"""Closed-form and textbook solutions used to pin the oracle.

* Exact Riemann solver for the 1D Euler equations of an ideal gas (the
  two-rarefaction / shock pressure function solved by Newton iteration and
  sampled along x/t, as in Toro, "Riemann Solvers and Numerical Methods for
  Fluid Dynamics", ch. 4), written here from the mathematics.
* Navier-Stokes decay of a transverse shear wave (Sec. 3.4, eq. NSshear) and
  isobaric decay of an entropy (temperature) wave by conduction.
* One Fourier mode of the 1D Navier-Stokes-Fourier equations linearised about
  a uniform gas at rest (the thermoacoustic wave of Sec. 3), with the
  transport coefficients of a BGK gas whose translational and internal
  energy relax together: longitudinal viscosity (3 - gamma) mu, that is
  4/3 mu plus a bulk viscosity (2/3 - (gamma - 1)) mu, and conductivity
  c_p mu / Pr.
"""
import math

import numpy as np


def _pressure_function(p, rho, pK, a, gamma):
    if p > pK:  # shock
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pK
        f = (p - pK) * math.sqrt(A / (p + B))
        df = math.sqrt(A / (B + p)) * (1.0 - 0.5 * (p - pK) / (B + p))
    else:  # rarefaction
        f = 2.0 * a / (gamma - 1.0) * ((p / pK) ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)
        df = 1.0 / (rho * a) * (p / pK) ** (-(gamma + 1.0) / (2.0 * gamma))
    return f, df


def riemann_star(left, right, gamma):
    """Star-region pressure and velocity for states (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    al, ar = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    p = max(1e-8, 0.5 * (pl + pr))
    for _ in range(100):
        fl, dfl = _pressure_function(p, rl, pl, al, gamma)
        fr, dfr = _pressure_function(p, rr, pr, ar, gamma)
        dp = (fl + fr + ur - ul) / (dfl + dfr)
        pn = max(1e-10, p - dp)
        if abs(pn - p) <= 1e-14 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _pressure_function(p, rl, pl, al, gamma)
    fr, _ = _pressure_function(p, rr, pr, ar, gamma)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def riemann_sample(left, right, gamma, s):
    """(rho, u, p) at similarity coordinate s = (x - x0)/t."""
    rl, ul, pl = left
    rr, ur, pr = right
    al, ar = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    ps, us = riemann_star(left, right, gamma)
    g1 = (gamma - 1.0) / (gamma + 1.0)
    if s <= us:  # left of contact
        if ps > pl:  # left shock
            rs = rl * ((ps / pl + g1) / (g1 * ps / pl + 1.0))
            S = ul - al * math.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pl + (gamma - 1.0) / (2.0 * gamma))
            return (rl, ul, pl) if s < S else (rs, us, ps)
        shl = ul - al
        asl = al * (ps / pl) ** ((gamma - 1.0) / (2.0 * gamma))
        stl = us - asl
        if s < shl:
            return (rl, ul, pl)
        if s > stl:
            return (rl * (ps / pl) ** (1.0 / gamma), us, ps)
        u = 2.0 / (gamma + 1.0) * (al + (gamma - 1.0) / 2.0 * ul + s)
        c = 2.0 / (gamma + 1.0) * (al + (gamma - 1.0) / 2.0 * (ul - s))
        rho = rl * (c / al) ** (2.0 / (gamma - 1.0))
        return (rho, u, pl * (c / al) ** (2.0 * gamma / (gamma - 1.0)))
    if ps > pr:  # right shock
        rs = rr * ((ps / pr + g1) / (g1 * ps / pr + 1.0))
        S = ur + ar * math.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pr + (gamma - 1.0) / (2.0 * gamma))
        return (rs, us, ps) if s < S else (rr, ur, pr)
    shr = ur + ar
    asr = ar * (ps / pr) ** ((gamma - 1.0) / (2.0 * gamma))
    str_ = us + asr
    if s > shr:
        return (rr, ur, pr)
    if s < str_:
        return (rr * (ps / pr) ** (1.0 / gamma), us, ps)
    u = 2.0 / (gamma + 1.0) * (-ar + (gamma - 1.0) / 2.0 * ur + s)
    c = 2.0 / (gamma + 1.0) * (ar - (gamma - 1.0) / 2.0 * (ur - s))
    rho = rr * (c / ar) ** (2.0 / (gamma - 1.0))
    return (rho, u, pr * (c / ar) ** (2.0 * gamma / (gamma - 1.0)))


def riemann_profile(left, right, gamma, x, x0, t):
    out = np.array([riemann_sample(left, right, gamma, (xx - x0) / t) for xx in x])
    return out[:, 0], out[:, 1], out[:, 2]


def ns_shear_amplitude(u0, nu, k, t):
    """Sec. 3.4, eq. NSshear: u(x, t) = u0(x) exp(-nu k^2 t) for zero mean."""
    return u0 * math.exp(-nu * k * k * t)


def entropy_wave_amplitude(a0, mu, rho, Pr, k, t):
    """Isobaric temperature perturbation decaying by conduction:
    rho c_p dT/dt = kappa lap T with kappa = c_p mu / Pr, so the rate is
    mu k^2 / (rho Pr)."""
    return a0 * math.exp(-mu * k * k * t / (rho * Pr))


def linear_nsf_mode(a0, c0, rho0, T0, R, gamma, mu, Pr, k, t):
    """rho' = a sin kx, u' = b cos kx, T' = c sin kx under

        d rho'/dt = -rho0 du'/dx
        rho0 du'/dt = -dp'/dx + mu_L d2u'/dx2,        p' = R (rho0 T' + T0 rho')
        rho0 c_v dT'/dt = -p0 du'/dx + kappa d2T'/dx2

    with mu_L = (3 - gamma) mu and kappa = c_p mu / Pr, starting from (a0, 0,
    c0).  Returns (a, b, c) at each time in t (matrix exponential of the 3x3
    system)."""
    from scipy.linalg import expm
    cv = R / (gamma - 1.0)
    cp = gamma * cv
    p0 = rho0 * R * T0
    muL = (3.0 - gamma) * mu
    kappa = cp * mu / Pr
    A = np.array([[0.0, rho0 * k, 0.0],
                  [-R * T0 * k / rho0, -muL * k * k / rho0, -R * k],
                  [0.0, p0 * k / (rho0 * cv), -kappa * k * k / (rho0 * cv)]])
    x0 = np.array([a0, 0.0, c0])
    return np.array([expm(A * tt) @ x0 for tt in np.atleast_1d(t)])
