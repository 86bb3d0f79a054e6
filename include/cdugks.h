/*
 * cdugks.h -- C ABI of the MI355X (gfx950) CDUGKS time-step library.
 *
 * The library advances the reduced distributions g (mass) and b (total
 * energy) of the Coupled Discrete Unified Gas Kinetic Scheme over the full
 * phase-space grid (spatial cells x discrete velocities) of Zamora, Slaughter
 * & Abel, "Computational Fluid Dynamics with the Coupled Discrete Unified Gas
 * Kinetic Scheme" (arXiv 2208.09132), Sec. 2 and Sec. 2.1.  Every stage of a
 * step runs in hand-written HIP kernels on one GPU.
 *
 * Conventions
 *  - All functions return an int status (CDUGKS_OK = 0, negative on error);
 *    no exception crosses the ABI.  cdugks_last_error() gives a thread-local
 *    message for the last failure on the calling thread.
 *  - Host arrays passed in are owned by the caller and only read during the
 *    call (cdugks_submit copies them).  Device state is owned by the library,
 *    or lives in a caller-supplied arena.
 *  - Moment arrays are structure-of-arrays: rho[N], u[dim][N], T[N], cells
 *    row-major with x fastest, N = n[0]*n[1]*n[2] over the used dimensions.
 *  - Streams are hipStream_t passed as void* (NULL = default stream).
 *  - An error raised while a step runs on the device (non-physical state:
 *    rho <= 0, T <= 0 or non-finite, in a cell or at a face) is sticky on the
 *    context and reported by cdugks_sync / cdugks_moments; the state after it
 *    is unspecified.
 */
#ifndef CDUGKS_H
#define CDUGKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CDUGKS_OK = 0,
    CDUGKS_PENDING = 1,
    CDUGKS_ERR_INVALID = -1,
    CDUGKS_ERR_NOMEM = -2,
    CDUGKS_ERR_DEVICE = -3,
    CDUGKS_ERR_NONPHYSICAL = -4,
    CDUGKS_ERR_TOO_LARGE = -5,
    CDUGKS_ERR_BUSY = -6,
    CDUGKS_ERR_UNKNOWN = -7
};

/* Boundary conditions per dimension.  Periodic wraps; outflow copies the
 * boundary cell into the ghost layers (zero gradient); Dirichlet holds, on
 * each side, the discrete equilibrium of a fixed state given in
 * cdugks_space.dirichlet (the paper's Sod runs, Sec. 3.1; boundary conditions
 * enter the scheme through the ghost cells, Sec. 2.1).  A ghost outside the
 * domain along several Dirichlet dimensions takes the state of the highest of
 * them. */
enum { CDUGKS_BC_PERIODIC = 0, CDUGKS_BC_OUTFLOW = 1, CDUGKS_BC_DIRICHLET = 2 };

/* How the relaxation time is given (Sec. 2, eq. visc and tau_g = mu/p):
 *  KN : Knudsen number; hard-sphere mean free path 16 mu/(5 rho sqrt(2 pi R T))
 *       at (rho_ref, T_ref) over the length L_ref gives mu_ref, then
 *       mu = mu_ref (T/T_ref)^omega.
 *  MU : mu_ref given directly.
 *  TAU: constant tau_g (may be +inf: free streaming). */
enum { CDUGKS_RELAX_KN = 0, CDUGKS_RELAX_MU = 1, CDUGKS_RELAX_TAU = 2 };

/* Velocity quadrature per axis (Sec. 2 conserved variables; Sec. 3.1):
 * composite trapezoid, or composite fourth-order Newton-Cotes, which needs
 * nv = 4k+1 nodes.  Nodes include both end points. */
enum { CDUGKS_QUAD_TRAPEZOID = 0, CDUGKS_QUAD_BOOLE = 1 };

/* Storage precision of g and b in device memory.  The conserved variables,
 * equilibria, velocity sums and relaxation coefficients are FP64 in every
 * mode; F32 only rounds the stored distributions (and the face values and
 * stencil arithmetic derived from them).  F32_BF16TAIL is F32 except that
 * the velocity rows of the far tails hold BF16 (round to nearest even from
 * the FP32 value): rows whose node lies more than 4 thermal speeds
 * sqrt(R T_max) from the box of initial bulk velocities (T_max the largest
 * initial temperature), so every initial Maxwellian is below exp(-8) of its
 * peak there.  The set is fixed at cdugks_init; cdugks_required_bytes
 * reserves FP32 rows for it. */
enum { CDUGKS_STORE_F64 = 0, CDUGKS_STORE_F32 = 1, CDUGKS_STORE_F32_BF16TAIL = 2 };

/* Face reconstruction of the quarter-step field at t_{n+1/2} (Sec. 2.1,
 * eq. relation).  SLOPES_OF_SLOPES is the paper's: the value at the face is
 * phi_bar_plus(x_u) + delta sigma_d(u) from the upwind cell u, and the face
 * gradient is itself reconstructed, sigma_f = sigma(u) + delta t_d(u) with t
 * the Van Leer limited derivatives of the slopes along the face normal; the
 * foot value is phi_bar_plus(x_f) - h xi . sigma_f.  SINGLE_SLOPE carries the
 * upwind cell's limited slopes alone to the foot, phi_bar_plus(x_u) +
 * (x_f - h xi - x_u) . sigma(u): the classic DUGKS form, D limited slopes
 * per field and update instead of D + D^2. */
enum { CDUGKS_RECON_SLOPES_OF_SLOPES = 0, CDUGKS_RECON_SINGLE_SLOPE = 1 };

typedef struct {
    int dim;                /* D = 1, 2 or 3 */
    int64_t n[3];           /* cells per dimension (entries >= dim ignored) */
    double lo[3], hi[3];    /* domain box; uniform Cartesian cells */
    int bc[3];              /* CDUGKS_BC_* per dimension */
    double dirichlet[3][2][5]; /* DIRICHLET dimensions: (rho, u_x, u_y, u_z, T) on
                                  the low [0] and high [1] side; rho, T > 0;
                                  velocity components >= dim are ignored */
} cdugks_space;

typedef struct {
    int64_t nv[3];          /* discrete velocities per axis (>= 2) */
    double vmin[3], vmax[3];/* velocity box per axis */
    int quadrature;         /* CDUGKS_QUAD_* */
} cdugks_velocity;

typedef struct {
    double gamma;           /* adiabatic index, 1 < gamma <= 5/3; K = (5-3 gamma)/(gamma-1) */
    double Pr;              /* Prandtl number = tau_g / tau_b, > 0 */
    double R;               /* gas constant (the paper uses 1/2) */
    double omega;           /* viscosity exponent w of eq. visc */
    int relax_mode;         /* CDUGKS_RELAX_* */
    double Kn, L_ref, rho_ref, T_ref;  /* KN mode; L_ref <= 0 -> x extent,
                                          rho_ref <= 0 -> mean initial density,
                                          T_ref <= 0 -> 1 */
    double mu_ref;          /* MU mode */
    double tau;             /* TAU mode, may be +inf */
    double cfl;             /* alpha of the static CFL step (Sec. 4) */
    double dt;              /* <= 0: dt = cfl dx_min / (2 max_i |xi_i|) */
    int storage;            /* CDUGKS_STORE_* */
    int velocity_slices;    /* velocity-loop split across workgroups; 0 = auto */
    int reconstruction;     /* CDUGKS_RECON_* */
    int face_tile;          /* face-sum tile shape: 0 = automatic (the autotuner's
                               choice for the problem's class, else the default:
                               the first shape in 1-D and 2-D, the 16x16 column
                               in 3-D); k >= 1 = the k-th shape of the
                               dimension's list, cells along (x, y, z) per
                               workgroup:
                                 dim 1: 256
                                 dim 2: 16x16, 32x8, 8x32, 32x24
                                 dim 3: 16x4x4, 32x4x2, 64x2x2, 32x6x4, 64x4x3, 16x8x6,
                                        16x16xZ, 32x8xZ, 32x16xZ
                               (xZ: a column that walks the whole z extent for
                               one velocity, storing the face values, followed by
                               a kernel that sums them over velocities).  The
                               first shape and the default take every problem;
                               the others need the paper's reconstruction, no
                               Dirichlet side and no acceleration, and all need
                               their staged planes or boxes to fit a CU's LDS in
                               the storage form (the 768-cell 64-wide 3-D box
                               does not in FP64); else CDUGKS_ERR_INVALID.
                               Every shape gives bitwise the same result. */
    double accel[3];        /* external acceleration a (e.g. gravity; Sec. 2,
                               eqs. gPDE, bPDE), components >= dim ignored; all
                               zero = none.  The sources of eqs. gsource and
                               bsource take the velocity derivative on the local
                               equilibrium, grad_xi g ~ -(xi - u)/(R T) g_eq and
                               grad_xi b ~ xi g_eq - (xi - u)/(R T) b_eq; the face
                               moments gain (h/2) rho a and (h/2) rho u.a (eqs.
                               rhoubar, rhoEbar) and the W update the source
                               integrals dt (0, rho a, rho u.a) at t_n.  Needs the
                               paper's reconstruction and the default face tile
                               (in batches, the batched tile of the storage form);
                               batches, the server and the autotuner take such
                               problems in classes of their own. */
} cdugks_params;

typedef struct cdugks_ctx cdugks_ctx;

/* Device bytes cdugks_init needs for this problem (for arenas and budgets). */
int cdugks_required_bytes(const cdugks_space* space, const cdugks_velocity* vel,
                          const cdugks_params* params, size_t* bytes);

/* Create a problem and set its state to the discrete equilibria of the given
 * moments (Sec. 3.4: every problem starts from the Maxwellian of its moments).
 * rho[N] > 0, u[dim][N], T[N] > 0 are host arrays.  hip_stream is the stream
 * all work of this context is enqueued on.  arena (device pointer, >= the
 * cdugks_required_bytes figure, 256-byte aligned) may be NULL, in which case
 * the library allocates.  Validation failures return CDUGKS_ERR_INVALID:
 * dim outside 1..3, n < 1, nv < 2, Boole with nv != 4k+1, gamma outside
 * (1, 5/3], Pr <= 0, R <= 0, rho <= 0, T <= 0 (in a cell or a Dirichlet
 * state), an unknown boundary condition, a requested dt above the CFL
 * bound, and sizes beyond the kernels' index ranges (faces >= 2^31,
 * velocities >= 2^24, cells x velocities > 2^40; cdugks_required_bytes
 * rejects these too).  Returns after enqueueing the initialisation. */
int cdugks_init(const cdugks_space* space, const cdugks_velocity* vel,
                const cdugks_params* params, const double* rho, const double* u,
                const double* T, void* hip_stream, void* arena, size_t arena_bytes,
                cdugks_ctx** out);

/* Enqueue nsteps time steps (Sec. 2.1) on the context's stream; returns
 * without waiting.  Steps are replayed from a captured HIP graph. */
int cdugks_step(cdugks_ctx* ctx, int64_t nsteps);

/* Wait for the context's stream; returns the sticky device error if any. */
int cdugks_sync(cdugks_ctx* ctx);

/* rho[N], u[dim][N], T[N] from the carried conserved variables (Sec. 2:
 * u = (rho u)/rho, T = (gamma-1)/R (E - u^2/2)).  If device_ptrs != 0 the
 * three pointers are device memory and the call only enqueues; otherwise
 * they are host memory and the call waits. */
int cdugks_moments(cdugks_ctx* ctx, double* rho, double* u, double* T, int device_ptrs);

/* Conserved variables W[N][dim+2] = (rho, rho u, rho E) copied to host. */
int cdugks_conserved(cdugks_ctx* ctx, double* W);

/* Distributions g[V][N], b[V][N] (velocity-major, cells fastest, FP64) copied
 * to host, V = nv[0]*nv[1]*nv[2] with the velocity index x fastest. */
int cdugks_distributions(cdugks_ctx* ctx, double* g, double* b);

/* ---------------- allocation-free read-out --------------------------------
 * For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): the same FP64 copies of g and b as
 * cdugks_distributions (bitwise), staged through a fixed device array of
 * CDUGKS_NOALLOC_SCRATCH_BYTES bytes that the library holds on every GPU it
 * runs on until the process ends, instead of a temporary allocation.  Calls
 * no hipMalloc, hipFree or other allocating routine.  Copies the velocity
 * rows in passes of as many rows as the array holds, on the context's stream
 * and device, and waits.  CDUGKS_ERR_TOO_LARGE (nothing copied) when one
 * velocity row of N FP64 values exceeds the array, i.e. N > 4194304 cells.
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents (nothing in it needs to start at zero); calls from threads of one
 * process are serialised by a lock, so they do not race on it. */
#define CDUGKS_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
int cdugks_distributions_noalloc(cdugks_ctx* ctx, double* g, double* b);

/* Velocity-grid refit: an adaptive velocity grid at a step boundary.  The
 * paper names adaptive velocity grids as an extension (Sec. 5) without an
 * algorithm; this is the reading taken.  Creates a new context (space and
 * params as for cdugks_init; same cells, dimension and storage form as src,
 * else CDUGKS_ERR_INVALID) on the velocity grid vel.  Its conserved
 * variables W are src's, bitwise (the scheme's state, Sec. 2.1); each
 * distribution is the equilibrium of the cell's W at the new node (eqs. geq,
 * beq) plus src's departure from equilibrium phi - phi_eq interpolated
 * multilinearly between src's nodes, zero outside src's velocity box.  The
 * new context has its own time step (the CFL bound of its grid unless
 * params->dt is set) and starts at src's simulated time and step count.
 * src is read, not changed; it must not belong to a batch and must live on
 * the current device.  hip_stream, arena and arena_bytes as for cdugks_init.
 * Waits for src's stream and for the refit. */
int cdugks_regrid(cdugks_ctx* src, const cdugks_space* space, const cdugks_velocity* vel,
                  const cdugks_params* params, void* hip_stream, void* arena, size_t arena_bytes,
                  cdugks_ctx** out);

/* Velocity grid fitted to a state (host only, no device work): the paper's
 * criterion for its fixed grid (Sec. 5: fine enough to resolve the mass and
 * wide enough to hold it, to an integration error tol) applied to the
 * moments rho[N], u[dim][N], T[N] (e.g. a context's current ones), for use
 * with cdugks_regrid.  Per axis d the box is [min_c (u_d - k s_c),
 * max_c (u_d + k s_c)] with s_c = sqrt(R T_c) and k = sqrt(2 ln(1/tol)) (the
 * normal tail beyond k s is at most tol/2 on each side); the node spacing is
 * at most pi sqrt(2) s_min / sqrt(ln(2/tol)) (the trapezoid rule's first
 * aliasing error on a Gaussian of deviation s_min, 2 exp(-2 pi^2 s^2/h^2),
 * is then at most tol); nv_d = ceil(width / spacing) + 1, rounded up to
 * 4n + 1 for CDUGKS_QUAD_BOOLE.  Uses space->dim and n, params->R (0: 1/2).
 * CDUGKS_ERR_INVALID for tol outside (0, 1), an unknown rule or
 * non-physical moments. */
int cdugks_fit_velocity(const cdugks_space* space, const cdugks_params* params, const double* rho,
                        const double* u, const double* T, double tol, int quadrature,
                        cdugks_velocity* out);

/* Storage of the context's distributions: the number of velocity rows held
 * in BF16 (0 unless CDUGKS_STORE_F32_BF16TAIL) and the bytes of one state
 * array (g or b) as laid out.  Either pointer may be NULL. */
int cdugks_storage_info(cdugks_ctx* ctx, int64_t* bf16_rows, size_t* state_array_bytes);

/* Launch shape of the context: its face-sum tile shape (1-based, as in
 * cdugks_params.face_tile), the velocity slices of the face-sum kernel (which
 * fix the summation order of the face sums) and of the update kernel.  Any
 * pointer may be NULL. */
int cdugks_launch_info(cdugks_ctx* ctx, int* face_tile, int* face_slices, int* update_slices);

/* Time step, simulated time and number of completed steps. */
int cdugks_info(cdugks_ctx* ctx, double* dt, double* t, int64_t* steps);

/* Timing helper: advance nsteps steps launching every phase on its own, with
 * HIP events recorded between the phases on the context's stream; ms[4]
 * receives the mean duration per step (milliseconds) of the four kernels of a
 * step: face sums, face closure, cell closure, update.  Waits for the stream. */
int cdugks_profile_phases(cdugks_ctx* ctx, int64_t nsteps, double* ms);

/* Release the context (waits for its stream).  NULL-safe.  A context that
 * belongs to a live batch is NOT released (the batch's graphs refer to its
 * memory): the call then only sets cdugks_last_error (CDUGKS_ERR_BUSY) and
 * the context stays valid; destroy the batch first. */
void cdugks_destroy(cdugks_ctx* ctx);

/* ---------------- batched form -------------------------------------------
 * Several independent problems advanced together: each kernel phase of a step
 * is ONE launch over a device work list that covers every tile of every
 * problem, and step sequences are captured as HIP graphs of chunk_steps
 * steps.  Every problem keeps its own context and gets bitwise the same
 * result as when stepped alone.  The batch runs on the first context's
 * stream; work already enqueued on the other members' streams is ordered
 * before each batch step call and their later work after it. */
typedef struct cdugks_batch cdugks_batch;

int cdugks_batch_create(cdugks_ctx* const* ctxs, int count, int chunk_steps,
                        cdugks_batch** out);
int cdugks_batch_step(cdugks_batch* batch, int64_t nsteps);
void cdugks_batch_destroy(cdugks_batch* batch);

/* ---------------- served form --------------------------------------------
 * Continuous batching: requests are admitted while slots and the device
 * memory budget allow, join the running batch at the next chunk boundary,
 * and leave it when their step count is reached; a host thread drives the
 * device that is current on the calling thread at cdugks_server_create (and
 * hip_stream, if given, must belong to it; NULL: the server makes its own).
 * Thread-safe. */
typedef struct cdugks_server cdugks_server;

/* chunk_steps: steps per admission round (rounded up to an even count, the
 * batch's graph chunk). */
int cdugks_server_create(size_t hbm_budget, int max_active, int chunk_steps,
                         void* hip_stream, cdugks_server** out);
/* Copies the request.  CDUGKS_ERR_TOO_LARGE if it can never fit the budget. */
int cdugks_submit(cdugks_server* srv, const cdugks_space* space, const cdugks_velocity* vel,
                  const cdugks_params* params, const double* rho, const double* u,
                  const double* T, int64_t nsteps, uint64_t* ticket);
/* CDUGKS_PENDING until done; then fills the moments (host arrays sized for
 * the request) and the queueing and service times, and forgets the ticket. */
int cdugks_poll(cdugks_server* srv, uint64_t ticket, double* rho, double* u, double* T,
                double* t_queue_s, double* t_service_s);
void cdugks_server_destroy(cdugks_server* srv);

/* ---------------- autotuner ----------------------------------------------
 * Times candidate launch shapes for the class of this problem (dimension,
 * storage, reconstruction, acceleration or none, velocity count, cell-count
 * bucket): the face-sum tile shape (cdugks_params.face_tile's list, the
 * shapes usable for the problem), the velocity split of the update kernel and the persistent grid
 * size of batched launches.  The fastest is kept in a process-wide table, and
 * written as text to the file named by $CDUGKS_TUNE_CACHE when that is set
 * (read back at first use); contexts created afterwards with face_tile = 0 use
 * it, and so does this context from its next step.  Every candidate computes
 * bitwise the same result, so tuning changes speed only.  The context is
 * advanced by the steps the update and grid trials time (the face-sum trials
 * rerun the first phase of a step without advancing it). */
int cdugks_autotune(cdugks_ctx* ctx, int steps_per_trial);

/* Thread-local message describing the last error on this thread. */
const char* cdugks_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CDUGKS_H */
