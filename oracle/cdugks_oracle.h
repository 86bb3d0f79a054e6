/*
 * CDUGKS reference oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow FP64 CPU implementation of one CDUGKS time step (Zamora,
 * Slaughter & Abel, "Computational Fluid Dynamics with the Coupled Discrete
 * Unified Gas Kinetic Scheme", Sec. 2 and Sec. 2.1).  It exists to check the
 * GPU library; only the test suite, the smoke check and the benchmark's CPU
 * baseline may call it.  It shares no code, header or table with the GPU path.
 *
 * Layout: distributions are [cell][velocity] (velocity index fastest),
 * cells row-major with x fastest, velocity index i = mx + nvx*(my + nvy*mz).
 */
#ifndef CDUGKS_ORACLE_H
#define CDUGKS_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Boundary conditions per dimension: periodic wraps, outflow copies the
 * boundary cell into the ghost layers, Dirichlet fills them with the
 * equilibrium of a fixed state per side (Sec. 2.1: boundary conditions enter
 * through the ghost cells). */
enum { ORC_BC_PERIODIC = 0, ORC_BC_OUTFLOW = 1, ORC_BC_DIRICHLET = 2 };
enum { ORC_QUAD_TRAPEZOID = 0, ORC_QUAD_BOOLE = 1 };
enum { ORC_RELAX_MU = 0, ORC_RELAX_TAU = 1 };
enum { ORC_RECON_SLOPES_OF_SLOPES = 0, ORC_RECON_SINGLE_SLOPE = 1 };

typedef struct {
    int dim;              /* D = 1, 2 or 3 */
    long n[3];            /* cells per dimension */
    double lo[3], hi[3];  /* domain box */
    int bc[3];            /* boundary condition per dimension (both sides) */
    double dirichlet[3][2][5]; /* Dirichlet dims: (rho, u_x, u_y, u_z, T) at the
                                  low [0] and high [1] side */
    long nv[3];           /* discrete velocities per dimension */
    double vmin[3], vmax[3];
    int quad;             /* velocity quadrature rule */
    double gamma;         /* adiabatic index, K = (5-3 gamma)/(gamma-1) */
    double Pr;            /* Prandtl number = tau_g / tau_b */
    double R;             /* gas constant */
    int relax_mode;       /* ORC_RELAX_MU: mu = mu_ref (T/T_ref)^omega, tau_g = mu/p
                             ORC_RELAX_TAU: tau_g = tau (may be +inf) */
    double mu_ref, T_ref, omega;
    double tau;
    double dt;            /* time step */
    double accel[3];      /* external acceleration a (eqs. gPDE, bPDE); zero
                             gives the scheme without it */
    int reconstruction;   /* ORC_RECON_SLOPES_OF_SLOPES (the paper's Sec. 2.1:
                             the face gradient is itself reconstructed from
                             limited derivatives of the slopes) or
                             ORC_RECON_SINGLE_SLOPE (the upwind cell's limited
                             slopes alone carried to the foot of the
                             characteristic) */
} oracle_params;

typedef struct oracle_state oracle_state;

/* Returns NULL on invalid parameters or allocation failure. */
oracle_state* oracle_create(const oracle_params* p);
void oracle_destroy(oracle_state* s);

/* Conserved variables from (rho, u[D][N], T); distributions set to the
 * discrete equilibria of those moments.  Returns 0 on success. */
int oracle_init(oracle_state* s, const double* rho, const double* u, const double* T);

/* Advance nsteps time steps.  Returns 0, or -4 if a non-physical state
 * (rho <= 0, T <= 0 or non-finite) appears in a cell or at a face. */
int oracle_step(oracle_state* s, long nsteps);

/* rho[N], u[D][N], T[N] from the carried conserved variables. */
void oracle_moments(const oracle_state* s, double* rho, double* u, double* T);

/* Raw state: g[N][V], b[N][V], W[N][D+2] (rho, rho u, rho E).  Any pointer
 * may be NULL. */
void oracle_get_state(const oracle_state* s, double* g, double* b, double* W);
void oracle_set_state(oracle_state* s, const double* g, const double* b, const double* W);

/* Velocity-grid refit (an adaptive velocity grid; Sec. 5 names the idea):
 * dst takes src's conserved variables unchanged and, on its own velocity
 * grid, the equilibrium of each cell's W plus src's departure from
 * equilibrium interpolated multilinearly in velocity (zero outside src's
 * velocity box); time and step count carry over.  The problems must share
 * dimension and cells.  Returns 0 or -1. */
int oracle_regrid(const oracle_state* src, oracle_state* dst);

/* Pieces exposed so tests can pin them individually. */
double oracle_van_leer(double s1, double s2);
void oracle_velocity_axis(long nv, double vmin, double vmax, int quad,
                          double* nodes, double* weights);
/* Discrete moments (sum_i w_i g_eq, sum_i w_i xi g_eq, sum_i w_i b_eq) of the
 * equilibria of one state on the oracle's velocity grid. */
void oracle_equilibrium_moments(const oracle_state* s, double rho, const double* u,
                                double T, double* out /* D+2 */);
double oracle_time(const oracle_state* s);
long oracle_num_steps(const oracle_state* s);
/* OpenMP threads the oracle runs on. */
int oracle_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
