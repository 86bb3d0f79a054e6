/*
 * CDUGKS reference oracle -- TEST INFRASTRUCTURE ONLY (see cdugks_oracle.h).
 *
 * Plain FP64 loops that follow the paper's algorithm in the paper's order
 * (Sec. 2.1, "The Algorithm"), with no fusion, blocking or reordering:
 *
 *   1. cell primitives and relaxation times from the carried W^n       (Sec. 2)
 *   2. quarter-step field phi_bar_plus at every cell (incl. ghosts)     eq. phibarplus
 *   3. Van Leer limited slopes sigma of phi_bar_plus                     eq. VanLeer
 *   4. limited slopes of the slopes ("gradients of the gradients")       Sec. 2.1
 *   5. phi_bar at each face centre at t_{n+1/2}: value at the
 *      characteristic foot x_f - h xi, upwind by the sign of xi.A         eq. relation
 *   6. face conserved variables from sums of phi_bar                    eq. rhobar..rhoEbar
 *   7. face equilibrium, relaxation times, inversion of phi_bar -> phi  eq. phibar
 *   8. microflux moments and the W update (minus sign: outward flux)    eq. rhoupdate..rhoEupdate
 *   9. phi update with the trapezoid collision term                      eq. phiupdate
 *
 * Readings of passages the paper leaves open or prints garbled are listed in
 * the project's design notes; the ones that shape code here are:
 *   - face slope sigma_f = sigma(u) + delta * t_{d,.}(u) with t the limited
 *     derivative along the face normal d of the slope vector, and the foot
 *     value phi_bar_plus(x_f) - h xi . sigma_f (the printed formula is garbled);
 *     the single-slope option drops step 4 and takes sigma_f = sigma(u), the
 *     classic upwind reconstruction phi_bar_plus(x_u) + (x_f - h xi - x_u) . sigma(u);
 *   - W^{n+1} = W^n - dt/|V| * sum of outward flux moments (the sign printed
 *     in eq. rhoupdate is inconsistent with eqs. implicit and phiupdate);
 *   - the source integrals in the W update are the velocity moments of the
 *     sources themselves, 0 and rho a for g and rho u.a for b (the Z term
 *     integrates to zero), with the cell's state at t_n (rectangle rule);
 *   - with an external acceleration a, the velocity derivatives in S_g, S_b
 *     (eqs. gsource, bsource) are evaluated on the local equilibrium (see
 *     sources() below);
 *   - a velocity with xi_d = 0 takes the mean of both one-sided values;
 *   - ghost cells: periodic wraps, outflow copies the boundary cell,
 *     Dirichlet holds the discrete equilibrium of the side's fixed state; a
 *     ghost outside along several Dirichlet dimensions takes the state of the
 *     highest of them (ghost layers filled dimension by dimension).
 */
#include "cdugks_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GHOST 3

struct oracle_state {
    oracle_params p;
    int D;
    long N, V;
    long ne[3];     /* ghost-extended extents (1 for unused dims) */
    long NE;        /* number of extended cells */
    double dx[3];
    double K, c_int; /* internal dof K and 3 - D + K */
    double *xi;      /* [V][3] */
    double *w;       /* [V]    */
    double *g, *b;   /* [N][V] */
    double *W;       /* [N][D+2] */
    double t;
    long steps;
    /* primitives of the Dirichlet states [dim][side] (set when used) */
    struct prim_s* dprim;
};

/* ------------------------------------------------------------------ */
/* small helpers                                                        */
/* ------------------------------------------------------------------ */

static long map_index(long j, long n, int bc)
{
    if (bc == ORC_BC_PERIODIC) {
        long r = j % n;
        return r < 0 ? r + n : r;
    }
    if (j < 0) return 0;
    if (j >= n) return n - 1;
    return j;
}

static long real_cell(const oracle_state* s, const long c[3])
{
    long r[3] = {0, 0, 0};
    for (int d = 0; d < s->D; ++d) r[d] = map_index(c[d], s->p.n[d], s->p.bc[d]);
    return r[0] + s->p.n[0] * (r[1] + s->p.n[1] * r[2]);
}

static long ext_cell(const oracle_state* s, const long c[3])
{
    long e[3] = {0, 0, 0};
    for (int d = 0; d < s->D; ++d) e[d] = c[d] + GHOST;
    return e[0] + s->ne[0] * (e[1] + s->ne[1] * e[2]);
}

static void ext_coords(const oracle_state* s, long e, long c[3])
{
    c[0] = c[1] = c[2] = 0;
    long r = e;
    for (int d = 0; d < 3; ++d) {
        long q = r % s->ne[d];
        r /= s->ne[d];
        if (d < s->D) c[d] = q - GHOST;
    }
}

/* Dirichlet side (2 d + side) whose state fills the ghost cell c, or -1. */
static int dirichlet_side(const oracle_state* s, const long c[3])
{
    int k = -1;
    for (int d = 0; d < s->D; ++d) {
        if (s->p.bc[d] != ORC_BC_DIRICHLET) continue;
        if (c[d] < 0) k = 2 * d;
        else if (c[d] >= s->p.n[d]) k = 2 * d + 1;
    }
    return k;
}

/* eq. VanLeer: sigma = (sgn s1 + sgn s2) |s1||s2| / (|s1| + |s2|), and 0
 * when both one-sided derivatives vanish. */
double oracle_van_leer(double s1, double s2)
{
    double a1 = fabs(s1), a2 = fabs(s2);
    double den = a1 + a2;
    if (den == 0.0) return 0.0;
    double sg = (s1 > 0.0) - (s1 < 0.0) + (s2 > 0.0) - (s2 < 0.0);
    return sg * a1 * a2 / den;
}

/* Uniform nodes including both end points; composite trapezoid weights, or
 * composite fourth-order Newton-Cotes (Boole) weights, which need nv = 4n+1
 * nodes (Sec. 3.1). */
void oracle_velocity_axis(long nv, double vmin, double vmax, int quad,
                          double* nodes, double* weights)
{
    double h = (vmax - vmin) / (double)(nv - 1);
    for (long m = 0; m < nv; ++m) nodes[m] = vmin + (double)m * h;
    if (quad == ORC_QUAD_BOOLE) {
        for (long m = 0; m < nv; ++m) weights[m] = 0.0;
        for (long p0 = 0; p0 + 4 < nv; p0 += 4) {
            static const double c[5] = {7.0, 32.0, 12.0, 32.0, 7.0};
            for (int k = 0; k < 5; ++k) weights[p0 + k] += c[k] * 2.0 * h / 45.0;
        }
    } else {
        for (long m = 0; m < nv; ++m) weights[m] = h;
        weights[0] = 0.5 * h;
        weights[nv - 1] = 0.5 * h;
    }
}

typedef struct prim_s {
    double rho, u[3], T, RT;
    double inv_tau_g, inv_tau_b, inv_tau_bg;
    int bad;
} prim_t;

/* Sec. 2: u = (rho u)/rho, T = (gamma-1)/R (E - u^2/2), p = rho R T,
 * mu = mu_r (T/T_r)^w (eq. visc), tau_g = mu/p, tau_b = tau_g/Pr,
 * tau_bg = tau_b tau_g/(tau_g - tau_b).  Inverse times are kept so that an
 * infinite relaxation time (free streaming) and Pr = 1 are representable:
 * 1/tau_bg = 1/tau_b - 1/tau_g. */
static prim_t primitives(const oracle_state* s, const double* Wc)
{
    prim_t q;
    memset(&q, 0, sizeof q);
    int D = s->D;
    q.rho = Wc[0];
    double u2 = 0.0;
    for (int d = 0; d < D; ++d) {
        q.u[d] = Wc[1 + d] / q.rho;
        u2 += q.u[d] * q.u[d];
    }
    double E = Wc[D + 1] / q.rho;
    q.T = (s->p.gamma - 1.0) / s->p.R * (E - 0.5 * u2);
    q.RT = s->p.R * q.T;
    double p = q.rho * s->p.R * q.T;
    if (s->p.relax_mode == ORC_RELAX_TAU) {
        q.inv_tau_g = isinf(s->p.tau) ? 0.0 : 1.0 / s->p.tau;
    } else {
        double mu = s->p.mu_ref * pow(q.T / s->p.T_ref, s->p.omega);
        q.inv_tau_g = p / mu;
    }
    q.inv_tau_b = q.inv_tau_g * s->p.Pr;
    q.inv_tau_bg = q.inv_tau_b - q.inv_tau_g;
    q.bad = !(q.rho > 0.0) || !(q.T > 0.0) || !isfinite(q.rho) || !isfinite(q.T);
    for (int d = 0; d < D; ++d) q.bad |= !isfinite(q.u[d]);
    return q;
}

/* eq. geq and eq. beq. */
static double g_equilibrium(const oracle_state* s, const prim_t* q, const double* xi)
{
    double c2 = 0.0;
    for (int d = 0; d < s->D; ++d) c2 += (xi[d] - q->u[d]) * (xi[d] - q->u[d]);
    return q->rho * pow(2.0 * M_PI * q->RT, -0.5 * s->D) * exp(-c2 / (2.0 * q->RT));
}

static double b_equilibrium(const oracle_state* s, const prim_t* q, const double* xi, double geq)
{
    double x2 = 0.0;
    for (int d = 0; d < s->D; ++d) x2 += xi[d] * xi[d];
    return 0.5 * (x2 + s->c_int * q->RT) * geq;
}

/* Z = xi.u - u^2/2 (Sec. 2, below eq. bPDE). */
static double Zfun(const oracle_state* s, const prim_t* q, const double* xi)
{
    double xu = 0.0, u2 = 0.0;
    for (int d = 0; d < s->D; ++d) {
        xu += xi[d] * q->u[d];
        u2 += q->u[d] * q->u[d];
    }
    return xu - 0.5 * u2;
}

/* Source terms S_g, S_b of eqs. gsource and bsource at one velocity, for the
 * state q (primitives) with distributions g, b and equilibria geq, beq.
 *   S_g = -a . grad_xi g
 *   S_b = (Z/tau_bg)(g - g_eq) + a . xi g - a . grad_xi b
 * The paper leaves the discretisation of the velocity derivative open.  It is
 * taken on the local equilibrium, the usual force model of the DUGKS family:
 *   grad_xi g ~ grad_xi g_eq = -(xi - u)/(R T) g_eq,
 *   grad_xi b ~ grad_xi b_eq = xi g_eq - (xi - u)/(R T) b_eq   (eq. beq),
 * so that
 *   S_g = a.(xi - u)/(R T) g_eq,
 *   S_b = (Z/tau_bg)(g - g_eq) + a.xi (g - g_eq) + a.(xi - u)/(R T) b_eq.
 * The velocity integrals of these are those of the exact sources: 0 and
 * rho a for S_g, rho u.a for S_b.  S_g does not depend on g, and S_b is
 * affine in g, so eq. phibar can still be inverted velocity by velocity. */
static void sources(const oracle_state* s, const prim_t* q, const double* xi, double g, double geq,
                    double beq, double* Sg, double* Sb)
{
    double axu = 0.0, ax = 0.0;
    for (int d = 0; d < s->D; ++d) {
        axu += s->p.accel[d] * (xi[d] - q->u[d]);
        ax += s->p.accel[d] * xi[d];
    }
    *Sg = axu / q->RT * geq;
    *Sb = Zfun(s, q, xi) * q->inv_tau_bg * (g - geq) + ax * (g - geq) + axu / q->RT * beq;
}

void oracle_equilibrium_moments(const oracle_state* s, double rho, const double* u,
                                double T, double* out)
{
    prim_t q;
    memset(&q, 0, sizeof q);
    q.rho = rho;
    for (int d = 0; d < s->D; ++d) q.u[d] = u[d];
    q.T = T;
    q.RT = s->p.R * T;
    int D = s->D;
    for (int k = 0; k < D + 2; ++k) out[k] = 0.0;
    for (long i = 0; i < s->V; ++i) {
        const double* xi = s->xi + 3 * i;
        double ge = g_equilibrium(s, &q, xi);
        double be = b_equilibrium(s, &q, xi, ge);
        out[0] += s->w[i] * ge;
        for (int d = 0; d < D; ++d) out[1 + d] += s->w[i] * xi[d] * ge;
        out[D + 1] += s->w[i] * be;
    }
}

/* ------------------------------------------------------------------ */
/* life cycle                                                           */
/* ------------------------------------------------------------------ */

/* Conserved variables of (rho, u, T): rho E = rho u^2/2 + rho c_v T with
 * c_v = (3+K)R/2 = R/(gamma-1).  u has stride ustride between components. */
static void conserved_of(const oracle_state* s, double rho, const double* u, long ustride, double T, double* Wc)
{
    double u2 = 0.0;
    Wc[0] = rho;
    for (int d = 0; d < s->D; ++d) {
        Wc[1 + d] = rho * u[d * ustride];
        u2 += u[d * ustride] * u[d * ustride];
    }
    Wc[s->D + 1] = rho * (0.5 * u2 + s->p.R * T / (s->p.gamma - 1.0));
}

oracle_state* oracle_create(const oracle_params* p)
{
    if (p->dim < 1 || p->dim > 3) return NULL;
    if (!(p->gamma > 1.0) || p->gamma > 5.0 / 3.0 + 1e-12) return NULL;
    if (!(p->Pr > 0.0) || !(p->R > 0.0) || !(p->dt > 0.0)) return NULL;
    if (p->reconstruction != ORC_RECON_SLOPES_OF_SLOPES && p->reconstruction != ORC_RECON_SINGLE_SLOPE) return NULL;
    oracle_state* s = (oracle_state*)calloc(1, sizeof *s);
    if (!s) return NULL;
    s->p = *p;
    s->D = p->dim;
    s->N = 1;
    s->V = 1;
    s->NE = 1;
    for (int d = 0; d < 3; ++d) {
        if (d < s->D) {
            if (p->n[d] < 1 || p->nv[d] < 2) { free(s); return NULL; }
            if (p->quad == ORC_QUAD_BOOLE && (p->nv[d] - 1) % 4 != 0) { free(s); return NULL; }
            s->N *= p->n[d];
            s->V *= p->nv[d];
            s->ne[d] = p->n[d] + 2 * GHOST;
            s->dx[d] = (p->hi[d] - p->lo[d]) / (double)p->n[d];
        } else {
            s->ne[d] = 1;
            s->p.n[d] = 1;
            s->p.nv[d] = 1;
            s->dx[d] = 1.0;
        }
        s->NE *= s->ne[d];
    }
    s->K = (5.0 - 3.0 * p->gamma) / (p->gamma - 1.0);
    s->c_int = 3.0 - s->D + s->K;

    s->xi = (double*)calloc((size_t)s->V * 3, sizeof(double));
    s->w = (double*)calloc((size_t)s->V, sizeof(double));
    s->g = (double*)calloc((size_t)s->N * s->V, sizeof(double));
    s->b = (double*)calloc((size_t)s->N * s->V, sizeof(double));
    s->W = (double*)calloc((size_t)s->N * (s->D + 2), sizeof(double));
    if (!s->xi || !s->w || !s->g || !s->b || !s->W) { oracle_destroy(s); return NULL; }

    /* tensor-product velocity grid: w_i = prod_d omega_d(m_d) */
    double* nodes[3] = {NULL, NULL, NULL};
    double* wts[3] = {NULL, NULL, NULL};
    int axes_ok = 1;
    for (int d = 0; d < s->D; ++d) {
        nodes[d] = (double*)malloc((size_t)p->nv[d] * sizeof(double));
        wts[d] = (double*)malloc((size_t)p->nv[d] * sizeof(double));
        if (!nodes[d] || !wts[d]) { axes_ok = 0; break; }
        oracle_velocity_axis(p->nv[d], p->vmin[d], p->vmax[d], p->quad, nodes[d], wts[d]);
    }
    if (!axes_ok) {
        for (int d = 0; d < 3; ++d) { free(nodes[d]); free(wts[d]); }
        oracle_destroy(s);
        return NULL;
    }
    for (long i = 0; i < s->V; ++i) {
        long m[3];
        long r = i;
        for (int d = 0; d < 3; ++d) { m[d] = r % s->p.nv[d]; r /= s->p.nv[d]; }
        double wi = 1.0;
        for (int d = 0; d < 3; ++d) {
            if (d < s->D) {
                s->xi[3 * i + d] = nodes[d][m[d]];
                wi *= wts[d][m[d]];
            } else {
                s->xi[3 * i + d] = 0.0;
            }
        }
        s->w[i] = wi;
    }
    for (int d = 0; d < 3; ++d) { free(nodes[d]); free(wts[d]); }

    /* Dirichlet states: validated, kept as primitives */
    s->dprim = (prim_t*)calloc(6, sizeof(prim_t));
    if (!s->dprim) { oracle_destroy(s); return NULL; }
    for (int d = 0; d < s->D; ++d) {
        if (p->bc[d] != ORC_BC_DIRICHLET) continue;
        for (int side = 0; side < 2; ++side) {
            const double* st = p->dirichlet[d][side];
            double Wd[5];
            if (!(st[0] > 0.0) || !(st[4] > 0.0)) { oracle_destroy(s); return NULL; }
            conserved_of(s, st[0], st + 1, 1, st[4], Wd);
            s->dprim[2 * d + side] = primitives(s, Wd);
            if (s->dprim[2 * d + side].bad) { oracle_destroy(s); return NULL; }
        }
    }
    return s;
}

void oracle_destroy(oracle_state* s)
{
    if (!s) return;
    free(s->xi); free(s->w); free(s->g); free(s->b); free(s->W); free(s->dprim);
    free(s);
}

/* Every test problem starts from the Maxwellian of its moments (Sec. 3.4). */
int oracle_init(oracle_state* s, const double* rho, const double* u, const double* T)
{
    int D = s->D;
    long N = s->N, V = s->V;
    for (long c = 0; c < N; ++c) {
        if (!(rho[c] > 0.0) || !(T[c] > 0.0)) return -1;
        double* Wc = s->W + c * (D + 2);
        conserved_of(s, rho[c], u + c, N, T[c], Wc);
        prim_t q = primitives(s, Wc);
        for (long i = 0; i < V; ++i) {
            const double* xi = s->xi + 3 * i;
            double ge = g_equilibrium(s, &q, xi);
            s->g[c * V + i] = ge;
            s->b[c * V + i] = b_equilibrium(s, &q, xi, ge);
        }
    }
    s->t = 0.0;
    s->steps = 0;
    return 0;
}

/* ------------------------------------------------------------------ */
/* one time step                                                        */
/* ------------------------------------------------------------------ */

static int one_step(oracle_state* s)
{
    const int D = s->D;
    const int NW = D + 2;
    const long N = s->N, V = s->V, NE = s->NE;
    const double dt = s->p.dt;
    const double h = 0.5 * dt; /* the paper's h = dt/2 (Sec. 2, below eq. phibar) */
    int bad = 0;

    /* 1. cell primitives at t_n */
    prim_t* cp = (prim_t*)malloc(sizeof(prim_t) * N);
    for (long c = 0; c < N; ++c) {
        cp[c] = primitives(s, s->W + c * NW);
        bad |= cp[c].bad;
    }
    if (bad) { free(cp); return -4; }

    /* 2. phi_bar_plus = phi + (h/2) Omega + (h/2) S on the ghost-extended
     *    grid (eq. phibarplus), with the sources of eqs. gsource, bsource. */
    double* qg = (double*)malloc(sizeof(double) * NE * V);
    double* qb = (double*)malloc(sizeof(double) * NE * V);
#pragma omp parallel for schedule(static)
    for (long e = 0; e < NE; ++e) {
        long c[3];
        ext_coords(s, e, c);
        const int ds = dirichlet_side(s, c);
        if (ds >= 0) {
            /* the ghost holds the equilibrium of the fixed state: its
             * relaxation and Z terms vanish, the acceleration terms remain */
            const prim_t* q = &s->dprim[ds];
            for (long i = 0; i < V; ++i) {
                const double* xi = s->xi + 3 * i;
                double geq = g_equilibrium(s, q, xi);
                double beq = b_equilibrium(s, q, xi, geq);
                double Sg, Sb;
                sources(s, q, xi, geq, geq, beq, &Sg, &Sb);
                qg[e * V + i] = geq + 0.5 * h * Sg;
                qb[e * V + i] = beq + 0.5 * h * Sb;
            }
            continue;
        }
        long r = real_cell(s, c);
        const prim_t* q = &cp[r];
        for (long i = 0; i < V; ++i) {
            const double* xi = s->xi + 3 * i;
            double g = s->g[r * V + i], b = s->b[r * V + i];
            double geq = g_equilibrium(s, q, xi);
            double beq = b_equilibrium(s, q, xi, geq);
            double Sg, Sb;
            sources(s, q, xi, g, geq, beq, &Sg, &Sb);
            double Og = (geq - g) * q->inv_tau_g;
            double Ob = (beq - b) * q->inv_tau_b;
            qg[e * V + i] = g + 0.5 * h * Og + 0.5 * h * Sg;
            qb[e * V + i] = b + 0.5 * h * Ob + 0.5 * h * Sb;
        }
    }

    /* strides of the extended grid */
    long st[3] = {1, s->ne[0], s->ne[0] * s->ne[1]};

    /* 3. limited slopes sig[e][d][i] (eq. VanLeer): sigma_1, sigma_2 are the
     *    one-sided finite-difference derivatives on either side of the cell. */
    double* sgg = (double*)calloc((size_t)NE * D * V, sizeof(double));
    double* sgb = (double*)calloc((size_t)NE * D * V, sizeof(double));
#pragma omp parallel for schedule(static)
    for (long e = 0; e < NE; ++e) {
        long c[3];
        ext_coords(s, e, c);
        int inside = 1;
        for (int d = 0; d < D; ++d) inside &= (c[d] >= -GHOST + 1 && c[d] < s->p.n[d] + GHOST - 1);
        if (!inside) continue;
        for (int d = 0; d < D; ++d) {
            for (long i = 0; i < V; ++i) {
                double s1 = (qg[e * V + i] - qg[(e - st[d]) * V + i]) / s->dx[d];
                double s2 = (qg[(e + st[d]) * V + i] - qg[e * V + i]) / s->dx[d];
                sgg[(e * D + d) * V + i] = oracle_van_leer(s1, s2);
                s1 = (qb[e * V + i] - qb[(e - st[d]) * V + i]) / s->dx[d];
                s2 = (qb[(e + st[d]) * V + i] - qb[e * V + i]) / s->dx[d];
                sgb[(e * D + d) * V + i] = oracle_van_leer(s1, s2);
            }
        }
    }

    /* 4. limited derivatives of the slopes: tt[e][d][k][i] is the derivative
     *    along d of slope component k (Sec. 2.1: the gradients of each
     *    component of the gradients, computed like the gradients). */
    double* ttg = (double*)calloc((size_t)NE * D * D * V, sizeof(double));
    double* ttb = (double*)calloc((size_t)NE * D * D * V, sizeof(double));
    const int single_slope = s->p.reconstruction == ORC_RECON_SINGLE_SLOPE;
#pragma omp parallel for schedule(static)
    for (long e = 0; e < NE; ++e) {
        if (single_slope) continue;  /* not used */
        long c[3];
        ext_coords(s, e, c);
        int inside = 1;
        for (int d = 0; d < D; ++d) inside &= (c[d] >= -GHOST + 2 && c[d] < s->p.n[d] + GHOST - 2);
        if (!inside) continue;
        for (int d = 0; d < D; ++d) {
            for (int k = 0; k < D; ++k) {
                for (long i = 0; i < V; ++i) {
                    long ik = (e * D + k) * V + i;
                    long im = ((e - st[d]) * D + k) * V + i;
                    long ip = ((e + st[d]) * D + k) * V + i;
                    double s1 = (sgg[ik] - sgg[im]) / s->dx[d];
                    double s2 = (sgg[ip] - sgg[ik]) / s->dx[d];
                    ttg[((e * D + d) * D + k) * V + i] = oracle_van_leer(s1, s2);
                    s1 = (sgb[ik] - sgb[im]) / s->dx[d];
                    s2 = (sgb[ip] - sgb[ik]) / s->dx[d];
                    ttb[((e * D + d) * D + k) * V + i] = oracle_van_leer(s1, s2);
                }
            }
        }
    }

    /* 5.-7. faces.  Faces along d are indexed by the cell on their right
     *    (face f lies between cells f-e_d and f); along d there are n_d faces
     *    for periodic and n_d+1 for outflow boundaries. */
    long nf[3][3], NF[3];
    for (int d = 0; d < D; ++d) {
        NF[d] = 1;
        for (int e2 = 0; e2 < 3; ++e2) {
            nf[d][e2] = s->p.n[e2];
            if (e2 == d && s->p.bc[d] != ORC_BC_PERIODIC) nf[d][e2] += 1;
            NF[d] *= nf[d][e2];
        }
    }
    double* gf[3] = {NULL, NULL, NULL};
    double* bf[3] = {NULL, NULL, NULL};
    double* Gf[3] = {NULL, NULL, NULL}; /* flux moments [face][D+2] */
    for (int d = 0; d < D; ++d) {
        gf[d] = (double*)malloc(sizeof(double) * NF[d] * V);
        bf[d] = (double*)malloc(sizeof(double) * NF[d] * V);
        Gf[d] = (double*)malloc(sizeof(double) * NF[d] * NW);
    }

    for (int d = 0; d < D; ++d) {
        int bad_d = 0;
#pragma omp parallel for schedule(static) reduction(| : bad_d)
        for (long f = 0; f < NF[d]; ++f) {
            long fc[3] = {0, 0, 0};
            long r = f;
            for (int e2 = 0; e2 < 3; ++e2) { fc[e2] = r % nf[d][e2]; r /= nf[d][e2]; }
            long cl[3] = {fc[0], fc[1], fc[2]};
            cl[d] -= 1; /* cell on the left of the face */
            long el = ext_cell(s, cl), er = ext_cell(s, fc);
            double* gface = gf[d] + f * V;
            double* bface = bf[d] + f * V;

            /* 5. phi_bar(x_f, t_n + h) = phi_bar_plus(x_f - h xi, t_n)
             *    (eq. relation).  Upwind linear reconstruction about the cell
             *    centre x_u: value at the face phi_bar_plus(x_u) + delta sigma_d,
             *    face gradient sigma_f = sigma(u) + delta t_{d,.}(u), and the
             *    foot value phi_bar_plus(x_f) - h xi . sigma_f. */
            for (long i = 0; i < V; ++i) {
                const double* xi = s->xi + 3 * i;
                double vg = 0.0, vb = 0.0;
                int nside = 0;
                for (int side = 0; side < 2; ++side) {
                    /* side 0: upwind cell on the left (xi_d > 0), delta = +dx/2
                     * side 1: upwind cell on the right (xi_d < 0), delta = -dx/2 */
                    if (side == 0 && !(xi[d] >= 0.0)) continue;
                    if (side == 1 && !(xi[d] <= 0.0)) continue;
                    long eu = side == 0 ? el : er;
                    double delta = side == 0 ? 0.5 * s->dx[d] : -0.5 * s->dx[d];
                    double fg = qg[eu * V + i] + delta * sgg[(eu * D + d) * V + i];
                    double fb = qb[eu * V + i] + delta * sgb[(eu * D + d) * V + i];
                    for (int k = 0; k < D; ++k) {
                        double sfg = sgg[(eu * D + k) * V + i];
                        double sfb = sgb[(eu * D + k) * V + i];
                        if (single_slope == 0) {  /* face gradient reconstructed too */
                            sfg += delta * ttg[((eu * D + d) * D + k) * V + i];
                            sfb += delta * ttb[((eu * D + d) * D + k) * V + i];
                        }
                        fg -= h * xi[k] * sfg;
                        fb -= h * xi[k] * sfb;
                    }
                    vg += fg;
                    vb += fb;
                    nside += 1;
                }
                gface[i] = vg / nside;
                bface[i] = vb / nside;
            }

            /* 6. W at the face from sums of phi_bar (eqs. rhobar..rhoEbar):
             *    rho u gains (h/2) rho a, rho E gains (h/2) (rho u).a with the
             *    face momentum just formed */
            double Wf[5] = {0, 0, 0, 0, 0};
            for (long i = 0; i < V; ++i) {
                const double* xi = s->xi + 3 * i;
                Wf[0] += s->w[i] * gface[i];
                for (int k = 0; k < D; ++k) Wf[1 + k] += s->w[i] * xi[k] * gface[i];
                Wf[D + 1] += s->w[i] * bface[i];
            }
            for (int k = 0; k < D; ++k) Wf[1 + k] += 0.5 * h * Wf[0] * s->p.accel[k];
            for (int k = 0; k < D; ++k) Wf[D + 1] += 0.5 * h * Wf[1 + k] * s->p.accel[k];

            /* 7. face equilibrium and relaxation times from W_f, then invert
             *    eq. phibar: phi = (phi_bar + (h/2) phi_eq/tau + (h/2) S)/(1 + h/(2 tau)).
             *    g first; its face value enters S_b at the face. */
            prim_t q = primitives(s, Wf);
            bad_d |= q.bad;
            for (long i = 0; i < V; ++i) {
                const double* xi = s->xi + 3 * i;
                double geq = g_equilibrium(s, &q, xi);
                double beq = b_equilibrium(s, &q, xi, geq);
                double Sg, Sb;
                sources(s, &q, xi, 0.0, geq, beq, &Sg, &Sb);  /* S_g does not depend on g */
                double gval = (gface[i] + 0.5 * h * q.inv_tau_g * geq + 0.5 * h * Sg) /
                              (1.0 + 0.5 * h * q.inv_tau_g);
                sources(s, &q, xi, gval, geq, beq, &Sg, &Sb);
                double bval = (bface[i] + 0.5 * h * q.inv_tau_b * beq + 0.5 * h * Sb) /
                              (1.0 + 0.5 * h * q.inv_tau_b);
                gface[i] = gval;
                bface[i] = bval;
            }

            /* microflux moments through the face, per unit area (eq. flux):
             * sum_i w_i xi_d (g, xi g, b) */
            double* G = Gf[d] + f * NW;
            for (int k = 0; k < NW; ++k) G[k] = 0.0;
            for (long i = 0; i < V; ++i) {
                const double* xi = s->xi + 3 * i;
                double wx = s->w[i] * xi[d];
                G[0] += wx * gface[i];
                for (int k = 0; k < D; ++k) G[1 + k] += wx * xi[k] * gface[i];
                G[D + 1] += wx * bface[i];
            }
        }
        bad |= bad_d;
    }

    free(qg); free(qb); free(sgg); free(sgb); free(ttg); free(ttb);
    if (bad) {
        for (int d = 0; d < D; ++d) { free(gf[d]); free(bf[d]); free(Gf[d]); }
        free(cp);
        return -4;
    }

    /* face index of the left face (side 0) or right face (side 1) of cell c along d */
#define FACE_OF(cc, d, side, out)                                                     \
    do {                                                                              \
        long fc_[3] = {(cc)[0], (cc)[1], (cc)[2]};                                    \
        if ((side) == 1) {                                                            \
            fc_[d] += 1;                                                              \
            if (s->p.bc[d] == ORC_BC_PERIODIC && fc_[d] == s->p.n[d]) fc_[d] = 0;     \
        }                                                                             \
        (out) = fc_[0] + nf[d][0] * (fc_[1] + nf[d][1] * fc_[2]);                      \
    } while (0)

    /* 8. W^{n+1} = W^n - (dt/|V_j|) sum_faces (A . flux moments) + dt (source
     *    integrals at t_n): for a Cartesian cell, - dt sum_d (G_{right} -
     *    G_{left}) / dx_d, plus dt (0, rho a, (rho u).a). */
    double* Wn = (double*)malloc(sizeof(double) * N * NW);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < N; ++c) {
        long cc[3] = {0, 0, 0};
        long r = c;
        for (int d = 0; d < 3; ++d) { cc[d] = r % s->p.n[d]; r /= s->p.n[d]; }
        for (int k = 0; k < NW; ++k) {
            double div = 0.0;
            for (int d = 0; d < D; ++d) {
                long fl, fr;
                FACE_OF(cc, d, 0, fl);
                FACE_OF(cc, d, 1, fr);
                div += (Gf[d][fr * NW + k] - Gf[d][fl * NW + k]) / s->dx[d];
            }
            Wn[c * NW + k] = s->W[c * NW + k] - dt * div;
        }
        const double* W0 = s->W + c * NW;
        for (int k = 0; k < D; ++k) {
            Wn[c * NW + 1 + k] += dt * W0[0] * s->p.accel[k];
            Wn[c * NW + D + 1] += dt * W0[1 + k] * s->p.accel[k];
        }
    }

    /* 9. eq. phiupdate:
     *   phi^{n+1} = (1 + dt/(2 tau^{n+1}))^{-1} [ phi^n
     *       + dt/2 (phi_eq^{n+1}/tau^{n+1} + (phi_eq^n - phi^n)/tau^n)
     *       - dt/|V| F + dt S^n ],  F/|V| = sum_d xi_d (phi_right - phi_left)/dx_d. */
    int bad2 = 0;
#pragma omp parallel for schedule(static) reduction(| : bad2)
    for (long c = 0; c < N; ++c) {
        long cc[3] = {0, 0, 0};
        long r = c;
        for (int d = 0; d < 3; ++d) { cc[d] = r % s->p.n[d]; r /= s->p.n[d]; }
        prim_t q0 = cp[c];
        prim_t q1 = primitives(s, Wn + c * NW);
        bad2 |= q1.bad;
        long fl[3], fr[3];
        for (int d = 0; d < D; ++d) {
            FACE_OF(cc, d, 0, fl[d]);
            FACE_OF(cc, d, 1, fr[d]);
        }
        for (long i = 0; i < V; ++i) {
            const double* xi = s->xi + 3 * i;
            double g = s->g[c * V + i], b = s->b[c * V + i];
            double geq0 = g_equilibrium(s, &q0, xi);
            double beq0 = b_equilibrium(s, &q0, xi, geq0);
            double geq1 = g_equilibrium(s, &q1, xi);
            double beq1 = b_equilibrium(s, &q1, xi, geq1);
            double Fg = 0.0, Fb = 0.0;
            for (int d = 0; d < D; ++d) {
                Fg += xi[d] * (gf[d][fr[d] * V + i] - gf[d][fl[d] * V + i]) / s->dx[d];
                Fb += xi[d] * (bf[d][fr[d] * V + i] - bf[d][fl[d] * V + i]) / s->dx[d];
            }
            double Sg, Sb;
            sources(s, &q0, xi, g, geq0, beq0, &Sg, &Sb);
            double gn = (g + 0.5 * dt * (geq1 * q1.inv_tau_g + (geq0 - g) * q0.inv_tau_g) - dt * Fg + dt * Sg) /
                        (1.0 + 0.5 * dt * q1.inv_tau_g);
            double bn = (b + 0.5 * dt * (beq1 * q1.inv_tau_b + (beq0 - b) * q0.inv_tau_b) - dt * Fb + dt * Sb) /
                        (1.0 + 0.5 * dt * q1.inv_tau_b);
            s->g[c * V + i] = gn;
            s->b[c * V + i] = bn;
        }
    }
#undef FACE_OF
    memcpy(s->W, Wn, sizeof(double) * N * NW);
    free(Wn);
    for (int d = 0; d < D; ++d) { free(gf[d]); free(bf[d]); free(Gf[d]); }
    free(cp);
    if (bad2) return -4;
    s->t += dt;
    s->steps += 1;
    return 0;
}

int oracle_step(oracle_state* s, long nsteps)
{
    for (long k = 0; k < nsteps; ++k) {
        int rc = one_step(s);
        if (rc) return rc;
    }
    return 0;
}

void oracle_moments(const oracle_state* s, double* rho, double* u, double* T)
{
    int D = s->D;
    for (long c = 0; c < s->N; ++c) {
        prim_t q = primitives(s, s->W + c * (D + 2));
        if (rho) rho[c] = q.rho;
        if (u) for (int d = 0; d < D; ++d) u[d * s->N + c] = q.u[d];
        if (T) T[c] = q.T;
    }
}

void oracle_get_state(const oracle_state* s, double* g, double* b, double* W)
{
    if (g) memcpy(g, s->g, sizeof(double) * s->N * s->V);
    if (b) memcpy(b, s->b, sizeof(double) * s->N * s->V);
    if (W) memcpy(W, s->W, sizeof(double) * s->N * (s->D + 2));
}

void oracle_set_state(oracle_state* s, const double* g, const double* b, const double* W)
{
    if (g) memcpy(s->g, g, sizeof(double) * s->N * s->V);
    if (b) memcpy(s->b, b, sizeof(double) * s->N * s->V);
    if (W) memcpy(s->W, W, sizeof(double) * s->N * (s->D + 2));
}

/* ------------------------------------------------------------------ */
/* velocity-grid refit (an adaptive velocity grid, Sec. 5)              */
/* ------------------------------------------------------------------ */

/* The state of src carried to the velocity grid of dst (same cells, gas and
 * boundaries; dst's own velocity grid).  The paper names adaptive velocity
 * grids only as an extension (Sec. 5).  Reading taken here, at a step
 * boundary: the conserved variables W are carried unchanged (they are the
 * scheme's state, Sec. 2.1); on the new grid each distribution is the
 * equilibrium of the cell's W (eqs. geq, beq) plus the departure from
 * equilibrium phi - phi_eq of the old grid, interpolated multilinearly in
 * velocity between the old nodes and zero outside the old velocity box.
 * Time and step count carry over.  Returns 0, -1 when the problems differ
 * in their cells or dimension. */
int oracle_regrid(const oracle_state* src, oracle_state* dst)
{
    const int D = src->D;
    if (dst->D != D || dst->N != src->N) return -1;
    for (int d = 0; d < D; ++d)
        if (dst->p.n[d] != src->p.n[d]) return -1;
    /* old axes: nodes per dimension */
    double* ax[3] = {NULL, NULL, NULL};
    long nvo[3] = {1, 1, 1};
    for (int d = 0; d < D; ++d) {
        nvo[d] = src->p.nv[d];
        ax[d] = malloc(sizeof(double) * nvo[d]);
        double* wtmp = malloc(sizeof(double) * nvo[d]);
        if (!ax[d] || !wtmp) return -1;
        oracle_velocity_axis(nvo[d], src->p.vmin[d], src->p.vmax[d], src->p.quad, ax[d], wtmp);
        free(wtmp);
    }
    memcpy(dst->W, src->W, sizeof(double) * src->N * (D + 2));
    for (long c = 0; c < src->N; ++c) {
        prim_t q = primitives(src, src->W + c * (D + 2));
        const double* go = src->g + c * src->V;
        const double* bo = src->b + c * src->V;
        for (long i = 0; i < dst->V; ++i) {
            const double* xi = dst->xi + 3 * i;
            double geq = g_equilibrium(dst, &q, xi);
            double beq = b_equilibrium(dst, &q, xi, geq);
            /* cell of the old grid holding xi, and the weights along each axis */
            int inside = 1;
            long m[3] = {0, 0, 0};
            double t[3] = {0.0, 0.0, 0.0};
            for (int d = 0; d < D; ++d) {
                double lo = ax[d][0], hi = ax[d][nvo[d] - 1], h = ax[d][1] - ax[d][0];
                if (xi[d] < lo || xi[d] > hi) {
                    inside = 0;
                    break;
                }
                long k = (long)floor((xi[d] - lo) / h);
                if (k > nvo[d] - 2) k = nvo[d] - 2;
                if (k < 0) k = 0;
                m[d] = k;
                t[d] = (xi[d] - ax[d][k]) / h;
            }
            double dg = 0.0, db = 0.0;
            if (inside) {
                /* the 2^D corners of the old cell */
                for (int corner = 0; corner < (1 << D); ++corner) {
                    double wgt = 1.0;
                    long io = 0, stride = 1;
                    double xo[3] = {0.0, 0.0, 0.0};
                    for (int d = 0; d < D; ++d) {
                        int up = (corner >> d) & 1;
                        wgt *= up ? t[d] : 1.0 - t[d];
                        io += (m[d] + up) * stride;
                        stride *= nvo[d];
                        xo[d] = ax[d][m[d] + up];
                    }
                    double ge = g_equilibrium(src, &q, xo);
                    double be = b_equilibrium(src, &q, xo, ge);
                    dg += wgt * (go[io] - ge);
                    db += wgt * (bo[io] - be);
                }
            }
            dst->g[c * dst->V + i] = geq + dg;
            dst->b[c * dst->V + i] = beq + db;
        }
    }
    for (int d = 0; d < D; ++d) free(ax[d]);
    dst->t = src->t;
    dst->steps = src->steps;
    return 0;
}

double oracle_time(const oracle_state* s) { return s->t; }

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
long oracle_num_steps(const oracle_state* s) { return s->steps; }
