"""Brute-force pin of the oracle's indexing and arithmetic: one CDUGKS step on
a tiny 2-D grid recomputed in 50-digit arithmetic (mpmath), written directly
from the equations of Sec. 2 and the algorithm of Sec. 2.1, one phase-space
point at a time, with no arrays of ghosts, no fused stages and no shared code.

The state is deliberately off equilibrium (random positive g, b) and the
carried conserved variables W differ from the discrete moments of g, b, so a
step that recomputed W from the distributions, dropped the S_b source, mixed
up the upwind side, the ghost map, an axis, the cross terms of the slope
reconstruction or the sign of the flux would miss the 50-digit result.
The readings are those the oracle documents: Van Leer of the one-sided
derivatives, face value q(u) + delta s_d(u) - h xi.(s(u) + delta t_d(u))
(the single-slope option: q(u) + delta s_d(u) - h xi.s(u)),
mean of the two one-sided values for xi_d = 0, outward-flux sign, outflow
ghosts clamp the index; with an external acceleration a (the cases with
accel), the sources of eqs. gsource and bsource with the velocity derivative
taken on the local equilibrium, grad_xi g ~ -(xi - u)/(R T) g_eq and
grad_xi b ~ xi g_eq - (xi - u)/(R T) b_eq, the face moments of eqs. rhoubar
and rhoEbar, and the source integrals (0, rho a, rho u.a) at t_n in the W
update (without a, the zero source integral of the Z term).
"""
import itertools

import numpy as np
import pytest

from oracle import oracle as orc

mp = pytest.importorskip("mpmath")
mp.mp.dps = 50
M = mp.mpf


def _vl(s1, s2):
    """eq. VanLeer: (sgn s1 + sgn s2) |s1||s2| / (|s1| + |s2|)."""
    if s1 == 0 and s2 == 0:
        return M(0)
    return (mp.sign(s1) + mp.sign(s2)) * abs(s1) * abs(s2) / (abs(s1) + abs(s2))


class Brute:
    def __init__(self, P):
        self.P = P
        self.D = 2
        self.n = P["n"]
        self.bc = P["bc"]
        self.dx = [(M(P["hi"][d]) - M(P["lo"][d])) / self.n[d] for d in range(2)]
        axes = []
        for d in range(2):
            nv, a, b = P["nv"][d], M(P["vmin"][d]), M(P["vmax"][d])
            dv = (b - a) / (nv - 1)
            nodes = [a + m * dv for m in range(nv)]
            wts = [dv * (M(1) / 2 if m in (0, nv - 1) else M(1)) for m in range(nv)]  # trapezoid
            axes.append((nodes, wts))
        # velocity index x fastest
        self.xi, self.w = [], []
        for my in range(P["nv"][1]):
            for mx in range(P["nv"][0]):
                self.xi.append((axes[0][0][mx], axes[1][0][my]))
                self.w.append(axes[0][1][mx] * axes[1][1][my])
        self.V = len(self.w)
        self.gamma = M(P["gamma"])
        self.K = (5 - 3 * self.gamma) / (self.gamma - 1)
        self.R = M(P["R"])
        self.Pr = M(P["Pr"])
        self.dt = M(P["dt"])
        self.h = self.dt / 2
        self.single_slope = P.get("reconstruction") == "single_slope"
        self.a = [M(v) for v in P.get("accel", [0.0, 0.0])]

    # ---- Sec. 2: primitives, relaxation times, equilibria ----
    def prim(self, W):
        rho = W[0]
        u = (W[1] / rho, W[2] / rho)
        E = W[3] / rho
        u2 = u[0] ** 2 + u[1] ** 2
        T = (self.gamma - 1) / self.R * (E - u2 / 2)
        p = rho * self.R * T
        mu = M(self.P["mu_ref"]) * (T / M(self.P["T_ref"])) ** M(self.P["omega"])
        tau_g = mu / p
        tau_b = tau_g / self.Pr
        inv_tau_bg = 1 / tau_b - 1 / tau_g  # tau_bg = tau_b tau_g / (tau_g - tau_b)
        return dict(rho=rho, u=u, T=T, tau_g=tau_g, tau_b=tau_b, inv_tau_bg=inv_tau_bg)

    def geq(self, q, i):
        RT = self.R * q["T"]
        c2 = sum((self.xi[i][d] - q["u"][d]) ** 2 for d in range(2))
        return q["rho"] / (2 * mp.pi * RT) ** (M(self.D) / 2) * mp.exp(-c2 / (2 * RT))

    def beq(self, q, i):
        x2 = self.xi[i][0] ** 2 + self.xi[i][1] ** 2
        return (x2 + (3 - self.D + self.K) * self.R * q["T"]) / 2 * self.geq(q, i)

    def Z(self, q, i):
        return sum(self.xi[i][d] * q["u"][d] for d in range(2)) - (q["u"][0] ** 2 + q["u"][1] ** 2) / 2

    def S(self, q, i, g):
        """eqs. gsource, bsource at velocity i for the state q and the value g
        of the mass distribution: S_g = -a.grad_xi g, S_b = Z (g - g_eq)/tau_bg
        + a.xi g - a.grad_xi b, with grad_xi g = -(xi - u) g_eq/(R T) and
        grad_xi b = xi g_eq - (xi - u) b_eq/(R T) (derivatives of eqs. geq, beq)."""
        RT = self.R * q["T"]
        ge, be = self.geq(q, i), self.beq(q, i)
        grad_g = [-(self.xi[i][d] - q["u"][d]) * ge / RT for d in range(2)]
        grad_b = [self.xi[i][d] * ge - (self.xi[i][d] - q["u"][d]) * be / RT for d in range(2)]
        Sg = -sum(self.a[d] * grad_g[d] for d in range(2))
        Sb = (self.Z(q, i) * q["inv_tau_bg"] * (g - ge) + sum(self.a[d] * self.xi[i][d] for d in range(2)) * g
              - sum(self.a[d] * grad_b[d] for d in range(2)))
        return Sg, Sb

    # ---- cells, ghosts ----
    def cell(self, x, y):
        """Source cell of a (possibly ghost) position: periodic wrap or outflow
        clamp; ('dir', d, side) for a ghost outside along a Dirichlet dimension
        (the highest such dimension)."""
        c = [x, y]
        for d in (1, 0):
            if self.bc[d] == "dirichlet" and not 0 <= c[d] < self.n[d]:
                return ("dir", d, 0 if c[d] < 0 else 1)
        for d in range(2):
            if self.bc[d] == "periodic":
                c[d] %= self.n[d]
            else:
                c[d] = min(max(c[d], 0), self.n[d] - 1)
        return c[0] + self.n[0] * c[1]

    def ghost_state(self, d, side):
        """The primitives of a Dirichlet side's fixed state (rho, u_x, u_y, T)."""
        rho, ux, uy, T = [M(v) for v in self.P["dirichlet"][d][side]]
        E = (ux ** 2 + uy ** 2) / 2 + self.R * T / (self.gamma - 1)
        return self.prim([rho, rho * ux, rho * uy, rho * E])

    def step(self, g, b, W):
        D, V, h, dt = self.D, self.V, self.h, self.dt
        N = self.n[0] * self.n[1]
        qc = [self.prim(W[j]) for j in range(N)]

        # eq. phibarplus
        def qbar(f, j, i):
            if isinstance(j, tuple):  # Dirichlet ghost: the side state's equilibrium
                q = self.ghost_state(j[1], j[2])
                ge, be = self.geq(q, i), self.beq(q, i)
                Sg, Sb = self.S(q, i, ge)
                return ge + h / 2 * Sg if f == 0 else be + h / 2 * Sb
            q = qc[j]
            ge = self.geq(q, i)
            Sg, Sb = self.S(q, i, g[j][i])
            if f == 0:
                return g[j][i] + h / 2 * (ge - g[j][i]) / q["tau_g"] + h / 2 * Sg
            return b[j][i] + h / 2 * (self.beq(q, i) - b[j][i]) / q["tau_b"] + h / 2 * Sb

        QB = {}

        def Q(f, x, y, i):
            key = (f, self.cell(x, y), i)
            if key not in QB:
                QB[key] = qbar(f, self.cell(x, y), i)
            return QB[key]

        unit = [(1, 0), (0, 1)]

        def slope(f, x, y, i, e):
            ex, ey = unit[e]
            s1 = (Q(f, x, y, i) - Q(f, x - ex, y - ey, i)) / self.dx[e]
            s2 = (Q(f, x + ex, y + ey, i) - Q(f, x, y, i)) / self.dx[e]
            return _vl(s1, s2)

        def slope2(f, x, y, i, d, e):
            dx_, dy_ = unit[d]
            s1 = (slope(f, x, y, i, e) - slope(f, x - dx_, y - dy_, i, e)) / self.dx[d]
            s2 = (slope(f, x + dx_, y + dy_, i, e) - slope(f, x, y, i, e)) / self.dx[d]
            return _vl(s1, s2)

        def from_cell(f, ux, uy, i, d, side):
            """phi_bar at the face t_{n+1/2}: upwind cell (ux, uy), face on its
            side +1 (right) or -1 (left) along d."""
            delta = side * self.dx[d] / 2
            at_face = Q(f, ux, uy, i) + delta * slope(f, ux, uy, i, d)
            if self.single_slope:  # the upwind cell's slopes carried to the foot
                sig = [slope(f, ux, uy, i, e) for e in range(2)]
            else:  # face gradient reconstructed from the slopes of the slopes
                sig = [slope(f, ux, uy, i, e) + delta * slope2(f, ux, uy, i, d, e) for e in range(2)]
            return at_face - h * (self.xi[i][0] * sig[0] + self.xi[i][1] * sig[1])

        def face_bar(f, x, y, i, d):
            """Face between (x, y) - e_d and (x, y) (left face of (x, y))."""
            dx_, dy_ = unit[d]
            xd = self.xi[i][d]
            L = from_cell(f, x - dx_, y - dy_, i, d, +1)
            Rr = from_cell(f, x, y, i, d, -1)
            if xd > 0:
                return L
            if xd < 0:
                return Rr
            return (L + Rr) / 2

        # faces along d: left faces of cells x = 0..n_d (n_d + 1 faces for
        # outflow, n_d for periodic)
        def faces(d):
            nx = self.n[0] + (1 if d == 0 and self.bc[0] != "periodic" else 0)
            ny = self.n[1] + (1 if d == 1 and self.bc[1] != "periodic" else 0)
            return [(x, y) for y in range(ny) for x in range(nx)]

        phi_face = {}
        for d in range(2):
            for (x, y) in faces(d):
                gb = [face_bar(0, x, y, i, d) for i in range(V)]
                bb = [face_bar(1, x, y, i, d) for i in range(V)]
                # eqs. rhobar..rhoEbar
                rho_f = sum(self.w[i] * gb[i] for i in range(V))
                mom_f = [sum(self.w[i] * self.xi[i][d] * gb[i] for i in range(V)) + h / 2 * rho_f * self.a[d]
                         for d in range(2)]
                ene_f = sum(self.w[i] * bb[i] for i in range(V)) + h / 2 * sum(mom_f[d] * self.a[d] for d in range(2))
                Wf = [rho_f, mom_f[0], mom_f[1], ene_f]
                qf = self.prim(Wf)
                gf, bf = [], []
                for i in range(V):
                    ge, be = self.geq(qf, i), self.beq(qf, i)
                    # invert eq. phibar: g first (S_g does not depend on g),
                    # then S_b with the face g, then b
                    ag, ab = h / (2 * qf["tau_g"]), h / (2 * qf["tau_b"])
                    Sg, _ = self.S(qf, i, M(0))
                    gi = (gb[i] + ag * ge + h / 2 * Sg) / (1 + ag)
                    _, Sb = self.S(qf, i, gi)
                    bi = (bb[i] + ab * be + h / 2 * Sb) / (1 + ab)
                    gf.append(gi)
                    bf.append(bi)
                phi_face[(d, x, y)] = (gf, bf)

        def face_key(d, x, y):
            if self.bc[d] == "periodic":
                c = [x, y]
                c[d] %= self.n[d]
                return (d, c[0], c[1])
            return (d, x, y)

        g1, b1, W1 = [], [], []
        for y in range(self.n[1]):
            for x in range(self.n[0]):
                j = x + self.n[0] * y
                # microflux per unit volume: sum_d xi_d (phi_right - phi_left) / dx_d
                Fg, Fb = [M(0)] * V, [M(0)] * V
                for d in range(2):
                    dx_, dy_ = unit[d]
                    left = phi_face[face_key(d, x, y)]
                    right = phi_face[face_key(d, x + dx_, y + dy_)]
                    for i in range(V):
                        Fg[i] += self.xi[i][d] * (right[0][i] - left[0][i]) / self.dx[d]
                        Fb[i] += self.xi[i][d] * (right[1][i] - left[1][i]) / self.dx[d]
                # eqs. rhoupdate..rhoEupdate, outward flux (minus); the source
                # integrals at t_n are 0, rho a and rho u.a
                Wn = [W[j][0] - dt * sum(self.w[i] * Fg[i] for i in range(V)),
                      W[j][1] - dt * sum(self.w[i] * self.xi[i][0] * Fg[i] for i in range(V)) + dt * W[j][0] * self.a[0],
                      W[j][2] - dt * sum(self.w[i] * self.xi[i][1] * Fg[i] for i in range(V)) + dt * W[j][0] * self.a[1],
                      W[j][3] - dt * sum(self.w[i] * Fb[i] for i in range(V))
                      + dt * (W[j][1] * self.a[0] + W[j][2] * self.a[1])]
                q0, q1 = qc[j], self.prim(Wn)
                gr, br = [], []
                for i in range(V):
                    ge0, be0 = self.geq(q0, i), self.beq(q0, i)
                    ge1, be1 = self.geq(q1, i), self.beq(q1, i)
                    Sg, Sb = self.S(q0, i, g[j][i])
                    # eq. phiupdate
                    gn = (g[j][i] + dt / 2 * (ge1 / q1["tau_g"] + (ge0 - g[j][i]) / q0["tau_g"]) - dt * Fg[i]
                          + dt * Sg) / (1 + dt / (2 * q1["tau_g"]))
                    bn = (b[j][i] + dt / 2 * (be1 / q1["tau_b"] + (be0 - b[j][i]) / q0["tau_b"]) - dt * Fb[i]
                          + dt * Sb) / (1 + dt / (2 * q1["tau_b"]))
                    gr.append(gn)
                    br.append(bn)
                g1.append(gr)
                b1.append(br)
                W1.append(Wn)
        return g1, b1, W1


@pytest.mark.parametrize("bc_y,recon,accel", [("outflow", "slopes_of_slopes", None),
                                               ("periodic", "slopes_of_slopes", None),
                                               ("outflow", "single_slope", None),
                                               ("dirichlet", "slopes_of_slopes", None),
                                               ("outflow", "slopes_of_slopes", [0.7, -1.3]),
                                               ("periodic", "single_slope", [-0.4, 0.9]),
                                               ("dirichlet", "slopes_of_slopes", [0.3, -1.1])])
def test_one_step_matches_50_digit_brute_force(bc_y, recon, accel):
    orc.build(force=False)
    P = dict(dim=2, n=[4, 3], lo=[0.0, -0.5], hi=[1.0, 0.25], bc=["periodic", bc_y], nv=[3, 4],
             vmin=[-2.0, -1.5], vmax=[2.0, 2.5], quad="trapezoid", gamma=7.0 / 5.0, Pr=2.0 / 3.0, R=0.5,
             relax="mu", mu_ref=0.02, T_ref=1.0, omega=0.5, dt=0.01, reconstruction=recon)
    if accel is not None:
        P["accel"] = accel
    if bc_y == "dirichlet":
        P["dirichlet"] = [None, [[1.3, 0.2, -0.1, 1.2], [0.9, -0.1, 0.05, 0.8]]]
    N, V = 12, 12
    rng = np.random.default_rng(2208)
    # smooth-ish positive distributions with random perturbations, off
    # equilibrium; W not the moments of g, b
    xi0 = np.array([[-2.0, 0.0, 2.0][i % 3] for i in range(V)])
    xi1 = np.array([[-1.5, -0.1666666666666667, 1.1666666666666667, 2.5][i // 3] for i in range(V)])
    base = np.exp(-(xi0 ** 2 + xi1 ** 2) / 2.0)
    g = base[None, :] * rng.uniform(0.5, 1.5, size=(N, V))
    b = base[None, :] * (0.5 * (xi0 ** 2 + xi1 ** 2) + 1.0)[None, :] * rng.uniform(0.5, 1.5, size=(N, V))
    W = np.zeros((N, 4))
    W[:, 0] = rng.uniform(0.8, 1.2, N)
    W[:, 1] = W[:, 0] * rng.uniform(-0.2, 0.2, N)
    W[:, 2] = W[:, 0] * rng.uniform(-0.2, 0.2, N)
    T = rng.uniform(0.8, 1.2, N)
    W[:, 3] = W[:, 0] * (T * 0.5 / (7.0 / 5.0 - 1.0) + 0.5 * (W[:, 1] ** 2 + W[:, 2] ** 2) / W[:, 0] ** 2)

    o = orc.Oracle(P)
    o.init(np.ones(N), np.zeros((2, N)), np.ones(N))
    o.set_state(g, b, W)
    assert o.step(1) == 0
    go, bo, Wo = o.state()

    br = Brute(P)
    gm = [[M(float(v)) for v in row] for row in g]
    bm = [[M(float(v)) for v in row] for row in b]
    Wm = [[M(float(v)) for v in row] for row in W]
    g1, b1, W1 = br.step(gm, bm, Wm)
    g1 = np.array([[float(v) for v in row] for row in g1])
    b1 = np.array([[float(v) for v in row] for row in b1])
    W1 = np.array([[float(v) for v in row] for row in W1])

    # the step changed the state substantially (not a no-op comparison)
    assert np.max(np.abs(g1 - g)) > 1e-2 * np.max(np.abs(g))
    for got, ref in ((go, g1), (bo, b1), (Wo, W1)):
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        assert err <= 1e-13, err
