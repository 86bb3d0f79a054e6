"""Test helpers: turn a workload dict into an oracle problem (oracle-side
parameter resolution) and compare moment fields."""
import math

import numpy as np

from oracle import oracle as orc


def xi_max(prob):
    D = prob["dim"]
    return math.sqrt(sum(max(abs(prob["vmin"][d]), abs(prob["vmax"][d])) ** 2 for d in range(D)))


def oracle_dt(prob):
    if prob.get("dt"):
        return float(prob["dt"])
    D = prob["dim"]
    dx = min((prob["hi"][d] - prob["lo"][d]) / prob["n"][d] for d in range(D))
    return orc.cfl_dt(prob.get("cfl", 0.5), dx, xi_max(prob))


def dt_checked(prob, gpu_dt):
    """The oracle's own static CFL step (Sec. 4) for prob, after checking that
    the library resolved the same step (to rounding).  Parity runs step the
    oracle with this value, so a wrong step in the library fails them."""
    dt = oracle_dt(prob)
    assert abs(gpu_dt - dt) <= 1e-15 * dt, f"library dt {gpu_dt!r} != oracle dt {dt!r}"
    return dt


def oracle_problem(prob, dt=None):
    q = dict(prob)
    relax = prob.get("relax", "kn")
    if relax == "kn":
        L = prob.get("L_ref") or (prob["hi"][0] - prob["lo"][0])
        rho_ref = prob.get("rho_ref") or float(np.mean(prob["rho"]))
        q["mu_ref"] = orc.mu_ref_from_kn(prob["Kn"], L, rho_ref, prob.get("R", 0.5), prob.get("T_ref", 1.0))
        q["relax"] = "mu"
    elif relax == "mu":
        q["relax"] = "mu"
    else:
        q["relax"] = "tau"
    q["dt"] = dt if dt is not None else oracle_dt(prob)
    return q


def make_oracle(prob, dt=None):
    o = orc.Oracle(oracle_problem(prob, dt))
    o.init(prob["rho"], prob["u"], prob["T"])
    return o


def moment_errors(ref, got, gamma=5.0 / 3.0, R=0.5):
    """Per-cell relative errors on rho and T; normwise error on u scaled by
    max(max|u|, sound speed at T_ref = 1)."""
    rho0, u0, T0 = ref
    rho1, u1, T1 = got
    e_rho = float(np.max(np.abs(rho1 - rho0) / np.abs(rho0)))
    e_T = float(np.max(np.abs(T1 - T0) / np.abs(T0)))
    scale = max(float(np.max(np.abs(u0))), math.sqrt(gamma * R * 1.0))
    e_u = float(np.max(np.abs(u1 - u0))) / scale
    return e_rho, e_u, e_T


def patch_problem(prob, centre, radius, extra=0):
    """A one-step result at a cell depends only on the cells within 3 cells of
    it (max-norm): a face value reads the slopes of its upwind cell and their
    limited differences, i.e. cells up to two away from that cell (the
    transverse neighbours included), and a cell is updated from its two faces
    along each axis.  After k steps the reach is 3k.  This builds the
    (2 radius + 1 + extra)^D block of cells starting radius cells below
    `centre` (periodic wrap when gathering the initial fields) as a problem of
    its own, with outflow ends, the same cell size and the same relaxation
    constants (Kn resolved with the full problem's length and mean density).
    The cells at least `radius` from the block's ends then step exactly as in
    the full problem.  Returns (block problem, full-grid indices of those
    cells, their block indices)."""
    D = prob["dim"]
    n = prob["n"]
    S = 2 * radius + 1 + extra
    q = dict(prob)
    dx = [(prob["hi"][d] - prob["lo"][d]) / n[d] for d in range(D)]
    start = [centre[d] - radius for d in range(D)]
    q["n"] = [S] * D
    q["lo"] = [prob["lo"][d] + start[d] * dx[d] for d in range(D)]
    q["hi"] = [q["lo"][d] + S * dx[d] for d in range(D)]
    q["bc"] = ["outflow"] * D
    q["dirichlet"] = None
    if prob.get("relax", "kn") == "kn":
        q["L_ref"] = prob.get("L_ref") or (prob["hi"][0] - prob["lo"][0])
        q["rho_ref"] = prob.get("rho_ref") or float(np.mean(prob["rho"]))
    axes = [(start[d] + np.arange(S)) % n[d] for d in range(D)]
    grids = np.meshgrid(*axes[::-1], indexing="ij")  # slowest first
    idx = np.zeros(S ** D, dtype=np.int64)
    stride = 1
    for d, g in enumerate(grids[::-1]):
        idx += g.reshape(-1) * stride
        stride *= n[d]
    q["rho"] = np.asarray(prob["rho"])[idx]
    q["T"] = np.asarray(prob["T"])[idx]
    q["u"] = np.asarray(prob["u"])[:, idx]
    inner = np.arange(radius, radius + 1 + extra)
    ig = np.meshgrid(*([inner] * D), indexing="ij")  # slowest first
    local = np.zeros(ig[0].size, dtype=np.int64)
    stride = 1
    for d, g in enumerate(ig[::-1]):
        local += g.reshape(-1) * stride
        stride *= S
    return q, idx[local], local
