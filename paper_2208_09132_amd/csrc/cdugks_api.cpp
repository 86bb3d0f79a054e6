// Host side of the CDUGKS library: validation, device memory, step
// orchestration with HIP graphs, and the C ABI declared in include/cdugks.h.
#include "cdugks.h"
#include "cdugks_host.h"

#include <algorithm>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

namespace cdg {

static thread_local std::string g_last_error;

// ---------------------------------------------------------------------------
// Fixed device staging array of the allocation-free read-out
// (cdugks_distributions_noalloc).  Every GPU the library runs on holds its
// own copy until the process ends.  On the host the name is only a stand-in
// for the symbol, never a device address: host code passes the address that
// hipGetSymbolAddress returns for the current device (looked up once per
// device, on the entry point's first call there) to kernels and copies.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[CDUGKS_NOALLOC_SCRATCH_BYTES / sizeof(double)];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;               // serialises the calls that use the array
static double* g_scratch_dev[MAX_DEVICES];    // device address per device (null: not looked up)

// The array's device address on `dev`, which must be current; g_scratch_mu held.
static int scratch_on_device(int dev, double** out);

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(CDUGKS_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

static size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Bytes between consecutive velocity rows of a row of `bytes`: 256-byte
// aligned, plus ROW_PAD for rows of 64 KB or more (a multiple of 8 and of 4,
// so the pitch is a whole number of FP64 and FP32 elements).
constexpr size_t ROW_PAD = 4352;
constexpr size_t FV_ROW_PAD = 4352;
static size_t row_pitch_bytes(size_t bytes, size_t pad = ROW_PAD) {
    return align_up(bytes) + (bytes >= (size_t(1) << 16) ? pad : 0);
}

// ---------------------------------------------------------------------------
// problem set-up
// ---------------------------------------------------------------------------
int resolve(const cdugks_space* sp, const cdugks_velocity* ve, const cdugks_params* pa,
            const double* rho, Resolved* out) {
    if (!sp || !ve || !pa || !out) return fail(CDUGKS_ERR_INVALID, "null argument");
    Resolved r{};
    const int D = sp->dim;
    if (D < 1 || D > 3) return fail(CDUGKS_ERR_INVALID, "dim must be 1, 2 or 3 (got %d)", D);
    r.D = D;
    r.N = 1;
    r.NE = 1;
    r.V = 1;
    for (int d = 0; d < 3; ++d) {
        if (d < D) {
            if (sp->n[d] < 1 || sp->n[d] > (1 << 24)) return fail(CDUGKS_ERR_INVALID, "n[%d] out of range", d);
            if (!(sp->hi[d] > sp->lo[d])) return fail(CDUGKS_ERR_INVALID, "empty domain along %d", d);
            if (sp->bc[d] != CDUGKS_BC_PERIODIC && sp->bc[d] != CDUGKS_BC_OUTFLOW &&
                sp->bc[d] != CDUGKS_BC_DIRICHLET)
                return fail(CDUGKS_ERR_INVALID, "unsupported boundary condition %d along %d", sp->bc[d], d);
            if (sp->bc[d] == CDUGKS_BC_DIRICHLET) {
                for (int side = 0; side < 2; ++side) {
                    const double* st = sp->dirichlet[d][side];
                    bool ok = st[0] > 0.0 && st[4] > 0.0 && std::isfinite(st[0]) && std::isfinite(st[4]);
                    for (int e = 0; e < D; ++e) ok = ok && std::isfinite(st[1 + e]);
                    if (!ok)
                        return fail(CDUGKS_ERR_INVALID, "Dirichlet state along %d (side %d) needs rho > 0, T > 0",
                                    d, side);
                    for (int k = 0; k < 5; ++k) r.dir[d][side][k] = k >= 1 && k <= 3 && k - 1 >= D ? 0.0 : st[k];
                }
                r.any_dirichlet = true;
            }
            // the product of the counts is bounded below, with the cells
            if (ve->nv[d] < 2 || ve->nv[d] >= (1LL << 24))
                return fail(CDUGKS_ERR_INVALID, "nv[%d] must be in [2, 2^24)", d);
            if (!(ve->vmax[d] > ve->vmin[d])) return fail(CDUGKS_ERR_INVALID, "empty velocity box along %d", d);
            if (ve->quadrature == CDUGKS_QUAD_BOOLE && (ve->nv[d] - 1) % 4 != 0)
                return fail(CDUGKS_ERR_INVALID, "Boole quadrature needs nv = 4k+1 (nv[%d] = %lld)", d,
                            (long long)ve->nv[d]);
            r.n[d] = (int)sp->n[d];
            r.bc[d] = sp->bc[d];
            // outflow and Dirichlet dimensions carry both boundary faces
            r.ne[d] = r.n[d] + (r.bc[d] != CDUGKS_BC_PERIODIC ? 1 : 0);
            r.nv[d] = (int)ve->nv[d];
            r.dx[d] = (sp->hi[d] - sp->lo[d]) / r.n[d];
        } else {
            r.n[d] = r.ne[d] = r.nv[d] = 1;
            r.bc[d] = 0;
            r.dx[d] = 1.0;
        }
        r.N *= r.n[d];
        r.NE *= r.ne[d];
        r.V *= r.nv[d];
    }
    // index ranges the kernels assume: 32-bit cell and face indices, 32-bit
    // velocity indices, and at most 2^40 phase-space points per problem
    if (r.NE >= (1LL << 31) || r.V >= (1LL << 24) || r.N * r.V > (1LL << 40))
        return fail(CDUGKS_ERR_INVALID, "problem too large (%lld cells x %lld velocities)", (long long)r.N,
                    (long long)r.V);
    if (ve->quadrature != CDUGKS_QUAD_TRAPEZOID && ve->quadrature != CDUGKS_QUAD_BOOLE)
        return fail(CDUGKS_ERR_INVALID, "unknown quadrature %d", ve->quadrature);
    if (!(pa->gamma > 1.0) || pa->gamma > 5.0 / 3.0 + 1e-12)
        return fail(CDUGKS_ERR_INVALID, "gamma must lie in (1, 5/3] (got %g)", pa->gamma);
    if (!(pa->Pr > 0.0)) return fail(CDUGKS_ERR_INVALID, "Pr must be > 0");
    if (!(pa->R > 0.0)) return fail(CDUGKS_ERR_INVALID, "R must be > 0");
    if (pa->storage != CDUGKS_STORE_F64 && pa->storage != CDUGKS_STORE_F32 &&
        pa->storage != CDUGKS_STORE_F32_BF16TAIL)
        return fail(CDUGKS_ERR_INVALID, "unknown storage mode %d", pa->storage);
    r.storage = pa->storage;
    if (pa->reconstruction != CDUGKS_RECON_SLOPES_OF_SLOPES && pa->reconstruction != CDUGKS_RECON_SINGLE_SLOPE)
        return fail(CDUGKS_ERR_INVALID, "unknown reconstruction %d", pa->reconstruction);
    r.recon = pa->reconstruction;
    for (int d = 0; d < 3; ++d) {
        r.accel[d] = d < D ? pa->accel[d] : 0.0;
        if (!std::isfinite(r.accel[d])) return fail(CDUGKS_ERR_INVALID, "accel[%d] is not finite", d);
        r.has_accel = r.has_accel || r.accel[d] != 0.0;
    }
    if (r.has_accel && r.recon != CDUGKS_RECON_SLOPES_OF_SLOPES)
        return fail(CDUGKS_ERR_INVALID, "an external acceleration needs the paper's reconstruction");
    r.gamma = pa->gamma;
    r.Pr = pa->Pr;
    r.R = pa->R;
    r.omega = pa->omega;
    r.K = (5.0 - 3.0 * pa->gamma) / (pa->gamma - 1.0);
    r.c_int = 3.0 - D + r.K;

    // velocity axes: uniform nodes including both end points (Sec. 3.1)
    r.quad = ve->quadrature;
    for (int d = 0; d < D; ++d) {
        r.vmin[d] = ve->vmin[d];
        r.vmax[d] = ve->vmax[d];
    }
    double xi2 = 0.0;
    for (int d = 0; d < D; ++d) xi2 += std::max(ve->vmin[d] * ve->vmin[d], ve->vmax[d] * ve->vmax[d]);
    const double xi_max = std::sqrt(xi2);
    double dx_min = r.dx[0];
    for (int d = 1; d < D; ++d) dx_min = std::min(dx_min, r.dx[d]);
    // Sec. 4: dt = alpha dx_min / (2 |xi_max|), alpha in (0, 1]
    const double dt_bound = dx_min / (2.0 * xi_max);
    if (pa->dt > 0.0) {
        if (pa->dt > dt_bound * (1.0 + 1e-12))
            return fail(CDUGKS_ERR_INVALID, "dt %g above the CFL bound %g", pa->dt, dt_bound);
        r.dt = pa->dt;
    } else {
        if (!(pa->cfl > 0.0) || pa->cfl > 1.0) return fail(CDUGKS_ERR_INVALID, "cfl must lie in (0, 1]");
        r.dt = pa->cfl * dt_bound;
    }

    switch (pa->relax_mode) {
    case CDUGKS_RELAX_KN: {
        if (!(pa->Kn > 0.0)) return fail(CDUGKS_ERR_INVALID, "Kn must be > 0");
        double L = pa->L_ref > 0.0 ? pa->L_ref : (sp->hi[0] - sp->lo[0]);
        double rho_ref = pa->rho_ref;
        if (!(rho_ref > 0.0)) {
            if (!rho) return fail(CDUGKS_ERR_INVALID, "rho_ref needed");
            double s = 0.0;
            for (long long c = 0; c < r.N; ++c) s += rho[c];
            rho_ref = s / (double)r.N;
        }
        double T_ref = pa->T_ref > 0.0 ? pa->T_ref : 1.0;
        r.rho_ref = rho_ref;
        // hard-sphere mean free path lambda = 16 mu / (5 rho sqrt(2 pi R T))
        r.mu_ref = 5.0 / 16.0 * pa->Kn * L * rho_ref * std::sqrt(2.0 * M_PI * pa->R * T_ref);
        r.T_ref = T_ref;
        r.relax = 0;
        break;
    }
    case CDUGKS_RELAX_MU:
        if (!(pa->mu_ref > 0.0)) return fail(CDUGKS_ERR_INVALID, "mu_ref must be > 0");
        r.mu_ref = pa->mu_ref;
        r.T_ref = pa->T_ref > 0.0 ? pa->T_ref : 1.0;
        r.relax = 0;
        break;
    case CDUGKS_RELAX_TAU:
        if (!(pa->tau > 0.0)) return fail(CDUGKS_ERR_INVALID, "tau must be > 0 (or +inf)");
        r.tau_inv = std::isinf(pa->tau) ? 0.0 : 1.0 / pa->tau;
        r.relax = 1;
        r.mu_ref = 1.0;
        r.T_ref = 1.0;
        break;
    default:
        return fail(CDUGKS_ERR_INVALID, "unknown relax mode %d", pa->relax_mode);
    }

    // face-sum tiles: the default shape plans the velocity split (so the
    // shape a problem runs with never changes its result)
    const TileExt t0 = tile_shape(D, 0);
    const int td[3] = {t0.x, t0.y, t0.z};
    long long nt1 = 1;
    for (int d = 0; d < 3; ++d) {
        r.tiles1_def[d] = (r.ne[d] + td[d] - 1) / td[d];
        nt1 *= r.tiles1_def[d];
    }
    set_face_tile(r, 0);
    const long long nt2 = (r.N + WG - 1) / WG;  // update blocks of WG cells
    // Velocity slices: fill the chip's resident workgroup slots in whole
    // rounds.  The face-sum split fixes the summation order, so it depends only
    // on the problem and the device type, never on what else is running.
    long long R1, R2;
    resident_slots(D, r.storage, &R1, &R2);
    // at least 16 velocities per slice so the per-tile set-up stays amortised
    const long long smax = std::max(1LL, r.V / 16);
    // Workgroups of one launch run in rounds of R; a last round that is
    // mostly empty costs as much as a full one.  Take the smallest split whose
    // work items fill their rounds to 90%, else the best filling one.
    auto plan = [&](long long ntiles, long long R) {
        if (R <= 0) return 1LL;
        long long best = 1;
        double best_fill = -1.0;
        for (long long s = 1; s <= smax && s <= 64; ++s) {
            const long long items = ntiles * s;
            const long long rounds = (items + R - 1) / R;
            const double fill = (double)items / (double)(rounds * R);
            if (fill >= 0.9) return s;
            if (fill > best_fill + 1e-12) {
                best_fill = fill;
                best = s;
            }
        }
        return best;
    };
    int slices = pa->velocity_slices;
    long long s1 = slices > 0 ? std::min<long long>(slices, r.V) : plan(nt1, R1);
    r.nslices = (int)std::max(1LL, s1);
    r.nslices_upd = (int)std::max(1LL, plan(nt2, R2));
    // the autotuner may have picked another update split for this class
    // (speed only: the update's result does not depend on it)
    if (int tu = tuned_update_slices(r); tu > 0) r.nslices_upd = (int)std::min<long long>(tu, r.V);
    // face-sum tile shape: the caller's, else the autotuner's for this
    // class, else the default (speed only)
    if (pa->face_tile < 0 || pa->face_tile > tile_shape_count(D))
        return fail(CDUGKS_ERR_INVALID, "face_tile %d outside 0..%d for dim %d", pa->face_tile,
                    tile_shape_count(D), D);
    if (pa->face_tile > 0) {
        if (!face_tile_usable(r, pa->face_tile - 1))
            return fail(CDUGKS_ERR_INVALID,
                        "face_tile %d is not available for this problem (storage form, Dirichlet sides or "
                        "reconstruction option)",
                        pa->face_tile);
        set_face_tile(r, pa->face_tile - 1);
    } else if (int tt = tuned_face_tile(r); tt >= 0 && face_tile_usable(r, tt)) {
        set_face_tile(r, tt);
    } else if (face_tile_usable(r, default_face_tile(D))) {
        set_face_tile(r, default_face_tile(D));
    }

    // byte plan
    const size_t es = r.storage == CDUGKS_STORE_F64 ? 8 : 4;
    // a state array (g, b, quarter-step field): V rows of N values, r.pitch
    // elements apart; the BF16-tail form starts every row on a 256-byte
    // boundary and reserves an FP32 row for each (which rows hold BF16 is
    // decided at init).  Rows of 64 KB or more are padded by ROW_PAD bytes:
    // at power-of-two distances the same cells of consecutive velocity rows
    // contend for the same memory channels (3-D FP32 face sums 48 -> 33 ms).
    r.pitch = (long long)row_pitch_bytes((size_t)r.N * es) / (long long)es;
    // one spare element per face-value row: the face-sum kernels store the
    // values of faces outside the grid there, so their stores are
    // unconditional (no branch before the next velocity's loads are used)
    r.fv_pitch = (long long)row_pitch_bytes((size_t)(r.NE + 1) * es, FV_ROW_PAD) / (long long)es;
    const size_t state_bytes = r.storage == CDUGKS_STORE_F32_BF16TAIL
                                   ? (size_t)r.V * row_pitch_bytes((size_t)r.N * 4)
                                   : (size_t)r.V * (size_t)r.pitch * es;
    // Consecutive regions are staggered by 4.25 KB each: arrays read at the
    // same element index (g, b, the quarter-step fields, the face values)
    // would otherwise sit at offsets that are multiples of a large power of
    // two whenever their sizes are (the 3-D workload: 2^32 bytes each), and
    // contend for the same memory channels.
    constexpr size_t STAGGER = 4352;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align_up(bytes) + (bytes >= (1u << 20) ? STAGGER : 0);
        return o;
    };
    for (int k = 0; k < 2; ++k) {
        r.off_g[k] = take(state_bytes);
        r.off_b[k] = take(state_bytes);
        r.off_W[k] = take((size_t)(D + 2) * r.N * 8);
        r.off_P[k] = take((size_t)NPC * r.N * 8);
    }
    r.off_dir = r.any_dirichlet ? take((size_t)2 * D * r.V * 2 * 8) : 0;
    r.off_q[0] = quarter_stored(D) ? take(state_bytes) : 0;
    r.off_q[1] = quarter_stored(D) ? take(state_bytes) : 0;
    r.off_rows = r.storage == CDUGKS_STORE_F32_BF16TAIL ? take((size_t)r.V * 8) : 0;
    // face values: 2D blocks of V NE values, each block padded by the stagger
    r.fv_stride = (long long)r.V * r.fv_pitch + (long long)(STAGGER / es);
    r.off_FV = take((size_t)D * 2 * (size_t)r.fv_stride * es);
    r.off_FS = take((size_t)r.nslices * D * (2 * D + 3) * r.NE * 8);
    r.off_FP = take((size_t)D * NFP * r.NE * 8);
    r.off_G = take((size_t)D * (D + 2) * r.NE * 8);
    r.off_vel = take((size_t)r.V * NVEL * 8);
    r.off_axis = take((size_t)2 * (r.nv[0] + r.nv[1] + r.nv[2]) * 8);
    r.off_err = take(256);
    r.off_scratch = take((size_t)(D + 2) * r.N * 8);
    r.bytes = off;
    *out = r;
    return CDUGKS_OK;
}

void set_face_tile(Resolved& r, int tile) {
    const TileExt t = tile_shape(r.D, tile);
    // a z-marching column spans the face grid along z
    const int te[3] = {t.x, t.y, tile_zmarch(r.D, tile) ? r.ne[2] : t.z};
    r.tile = tile;
    for (int d = 0; d < 3; ++d) r.tiles1[d] = (r.ne[d] + te[d] - 1) / te[d];
}

bool face_tile_usable(const Resolved& r, int tile) {
    if (tile < 0 || tile >= tile_shape_count(r.D)) return false;
    if (tile == 0) return true;
    // shape 0 and the default shape take every problem, the others only those
    // without Dirichlet sides or acceleration that use the paper's
    // reconstruction
    if (tile != default_face_tile(r.D) &&
        (r.any_dirichlet || r.recon != CDUGKS_RECON_SLOPES_OF_SLOPES || r.has_accel))
        return false;
    if (!face_tile_fits(r.D, tile, r.storage == CDUGKS_STORE_F64 ? 8 : 4)) return false;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0) {
        (void)hipGetLastError();
        return true;  // no device to ask: the LDS check stands
    }
    return face_sum_blocks_per_cu(r.D, r.storage, tile) > 0;
}

void resident_slots(int D, int storage, long long* R1, long long* R2) {
    static std::mutex mu;
    std::lock_guard<std::mutex> lock(mu);
    static int cus = -1;
    static int cache[3][3][2];
    static bool have[3][3][2];
    if (cus < 0) {
        int dev = 0, n = 0;
        hipDeviceProp_t prop;
        if (hipGetDeviceCount(&n) == hipSuccess && n > 0 && hipGetDevice(&dev) == hipSuccess &&
            hipGetDeviceProperties(&prop, dev) == hipSuccess)
            cus = prop.multiProcessorCount;
        else
            cus = 0;
        (void)hipGetLastError();
    }
    int bp[2];
    for (int u = 0; u < 2; ++u) {
        if (!have[D - 1][storage][u]) {
            cache[D - 1][storage][u] = cus > 0 ? tile_blocks_per_cu(D, storage, u == 1) : 0;
            have[D - 1][storage][u] = true;
        }
        bp[u] = cache[D - 1][storage][u];
    }
    const long long c = cus > 0 ? cus : 256;
    *R1 = c * (bp[0] > 0 ? bp[0] : 4);
    *R2 = c * (bp[1] > 0 ? bp[1] : 4);
}

void velocity_tables(const Resolved& r, std::vector<double>& vel, std::vector<double>& axis) {
    const int D = r.D;
    std::vector<double> nodes[3], wts[3];
    for (int d = 0; d < 3; ++d) {
        int nv = r.nv[d];
        nodes[d].assign(nv, 0.0);
        wts[d].assign(nv, 1.0);
        if (d >= D) continue;
        double h = (r.vmax[d] - r.vmin[d]) / (nv - 1);
        for (int m = 0; m < nv; ++m) nodes[d][m] = r.vmin[d] + m * h;
        if (r.quad == CDUGKS_QUAD_BOOLE) {
            static const double c[5] = {7.0, 32.0, 12.0, 32.0, 7.0};
            std::fill(wts[d].begin(), wts[d].end(), 0.0);
            for (int p0 = 0; p0 + 4 < nv; p0 += 4)
                for (int k = 0; k < 5; ++k) wts[d][p0 + k] += c[k] * 2.0 * h / 45.0;
        } else {
            std::fill(wts[d].begin(), wts[d].end(), h);
            wts[d][0] = wts[d][nv - 1] = 0.5 * h;
        }
    }
    vel.assign((size_t)r.V * NVEL, 0.0);
    for (long long i = 0; i < r.V; ++i) {
        long long rem = i;
        int m[3];
        for (int d = 0; d < 3; ++d) {
            m[d] = (int)(rem % r.nv[d]);
            rem /= r.nv[d];
        }
        double* v = vel.data() + i * NVEL;
        double w = 1.0, x2 = 0.0;
        for (int d = 0; d < D; ++d) {
            double x = nodes[d][m[d]];
            v[VE_XI0 + d] = x;
            w *= wts[d][m[d]];
            x2 += x * x;
            v[VE_LAM0 + d] = r.dt * x / r.dx[d];  // twice (dt/2) xi_d / dx_d
        }
        v[VE_W] = w;
        v[VE_HX2] = 0.5 * x2;
        double ax = 0.0;
        for (int d = 0; d < D; ++d) ax += r.accel[d] * nodes[d][m[d]];
        v[VE_AX] = ax;
        for (int d = 0; d < D; ++d) {
            v[VE_WXI0 + d] = w * nodes[d][m[d]];
            for (int e = 0; e < D; ++e) v[VE_WXX + 3 * d + e] = w * nodes[d][m[d]] * nodes[e][m[e]];
        }
    }
    axis.clear();
    for (int d = 0; d < 3; ++d) axis.insert(axis.end(), nodes[d].begin(), nodes[d].end());
    for (int d = 0; d < 3; ++d) axis.insert(axis.end(), wts[d].begin(), wts[d].end());
}

// Quarter-step values of the Dirichlet ghosts, [2 d + side][V][g, b]: the
// ghost cells hold the discrete equilibria of the side states (eqs. geq,
// beq), so relaxation and the Z source vanish and the quarter-step value is
// the equilibrium itself, plus (h/2) S of an external acceleration,
// a.(xi - u)/(R T) times g_eq and b_eq (eqs. gsource, bsource with the
// velocity derivative on the equilibrium).  Sides of non-Dirichlet
// dimensions stay zero.
void dirichlet_tables(const Resolved& r, const std::vector<double>& vel, std::vector<double>& out) {
    const int D = r.D;
    out.assign((size_t)2 * D * r.V * 2, 0.0);
    for (int d = 0; d < D; ++d) {
        if (r.bc[d] != CDUGKS_BC_DIRICHLET) continue;
        for (int side = 0; side < 2; ++side) {
            const double* st = r.dir[d][side];
            const double rho = st[0], RT = r.R * st[4];
            const double two_pi_rt = 2.0 * M_PI * RT;
            const double A = rho * (D == 1 ? 1.0 / std::sqrt(two_pi_rt)
                                           : (D == 2 ? 1.0 / two_pi_rt : 1.0 / (two_pi_rt * std::sqrt(two_pi_rt))));
            const double inv2RT = 0.5 / RT, cRT2 = 0.5 * r.c_int * RT;
            double* o = out.data() + (size_t)(2 * d + side) * r.V * 2;
            for (long long i = 0; i < r.V; ++i) {
                const double* v = vel.data() + i * NVEL;
                double c2 = 0.0;
                for (int e = 0; e < D; ++e) {
                    const double x = v[VE_XI0 + e] - st[1 + e];
                    c2 += x * x;
                }
                const double geq = A * std::exp(-c2 * inv2RT);
                const double beq = (v[VE_HX2] + cRT2) * geq;
                double au = 0.0;
                for (int e = 0; e < D; ++e) au += r.accel[e] * st[1 + e];
                const double c = 0.5 * r.dt * inv2RT * (v[VE_AX] - au);  // (h/2) a.(xi - u)/(R T)
                o[2 * i] = geq + c * geq;
                o[2 * i + 1] = beq + c * beq;
            }
        }
    }
}

void fill_problem(const Resolved& r, char* base, Problem& P) {
    std::memset(&P, 0, sizeof P);
    P.D = r.D;
    P.storage = r.storage;
    P.nslices = r.nslices;
    P.nslices_upd = r.nslices_upd;
    P.relax = r.relax;
    for (int d = 0; d < 3; ++d) {
        P.n[d] = r.n[d];
        P.ne[d] = r.ne[d];
        P.bc[d] = r.bc[d];
        P.nv[d] = r.nv[d];
        P.tiles1[d] = r.tiles1[d];
        P.dx[d] = r.dx[d];
        P.inv_dx[d] = 1.0 / r.dx[d];
    }
    P.V = (int)r.V;
    P.N = r.N;
    P.NE = r.NE;
    P.dt = r.dt;
    P.gamma = r.gamma;
    P.Pr = r.Pr;
    P.R = r.R;
    P.c_int = r.c_int;
    P.omega = r.omega;
    P.mu_ref = r.mu_ref;
    P.T_ref = r.T_ref;
    P.tau_inv = r.tau_inv;
    P.hxi0 = (r.vmax[0] - r.vmin[0]) / (r.nv[0] - 1);
    P.vel = (const double*)(base + r.off_vel);
    P.axis_xi = (const double*)(base + r.off_axis);
    P.axis_w = P.axis_xi + (r.nv[0] + r.nv[1] + r.nv[2]);
    if (quarter_stored(r.D)) {
        P.qg = base + r.off_q[0];
        P.qb = base + r.off_q[1];
    }
    P.FV = base + r.off_FV;
    P.fv_stride = r.fv_stride;
    P.pitch = r.pitch;
    P.fv_pitch = r.fv_pitch;
    P.dir_eq = r.any_dirichlet ? (const double*)(base + r.off_dir) : nullptr;
    P.FS = (double*)(base + r.off_FS);
    P.FP = (double*)(base + r.off_FP);
    P.G = (double*)(base + r.off_G);
    P.err = (int*)(base + r.off_err);
    P.rows = r.storage == CDUGKS_STORE_F32_BF16TAIL ? (const long long*)(base + r.off_rows) : nullptr;
    P.recon = r.recon;
    P.tile = r.tile;
    P.has_accel = r.has_accel ? 1 : 0;
    for (int d = 0; d < 3; ++d) P.accel[d] = r.accel[d];
}

// Rows of the BF16-tail form: velocity i is a tail row when, for every
// initial cell state, |xi_i - u| exceeds TAIL_SIGMAS thermal speeds
// sqrt(R T), i.e. its equilibrium is below exp(-TAIL_SIGMAS^2 / 2) of the
// peak: the distance from xi_i to the box spanned by the initial velocities
// is compared with TAIL_SIGMAS sqrt(R T_max).  Row words: byte offset of the
// row in a state array, bit 0 set for a BF16 row; rows start on 256-byte
// boundaries.
long long tail_rows(const Resolved& r, const std::vector<double>& vel, const double* u, const double* T,
                    std::vector<long long>& rows) {
    constexpr double TAIL_SIGMAS = 4.0;
    const int D = r.D;
    double umin[3] = {0, 0, 0}, umax[3] = {0, 0, 0}, Tmax = 0.0;
    for (int d = 0; d < D; ++d) {
        umin[d] = umax[d] = u[(size_t)d * r.N];
        for (long long c = 0; c < r.N; ++c) {
            umin[d] = std::min(umin[d], u[(size_t)d * r.N + c]);
            umax[d] = std::max(umax[d], u[(size_t)d * r.N + c]);
        }
    }
    for (long long c = 0; c < r.N; ++c) Tmax = std::max(Tmax, T[c]);
    const double lim2 = TAIL_SIGMAS * TAIL_SIGMAS * r.R * Tmax;
    rows.assign((size_t)r.V, 0);
    long long off = 0, ntail = 0;
    for (long long i = 0; i < r.V; ++i) {
        double d2 = 0.0;
        for (int d = 0; d < D; ++d) {
            const double x = vel[(size_t)i * NVEL + VE_XI0 + d];
            const double g = x < umin[d] ? umin[d] - x : (x > umax[d] ? x - umax[d] : 0.0);
            d2 += g * g;
        }
        const bool tail = d2 > lim2;
        rows[i] = off | (tail ? 1 : 0);
        off += (long long)row_pitch_bytes((size_t)r.N * (tail ? 2 : 4));
        ntail += tail;
    }
    return ntail;
}

void set_pingpong(Problem& P, const Resolved& r, char* base, int cur) {
    int nxt = 1 - cur;
    P.g_in = base + r.off_g[cur];
    P.b_in = base + r.off_b[cur];
    P.g_out = base + r.off_g[nxt];
    P.b_out = base + r.off_b[nxt];
    P.W_in = (const double*)(base + r.off_W[cur]);
    P.W_out = (double*)(base + r.off_W[nxt]);
    P.P_in = (const double*)(base + r.off_P[cur]);
    P.P_out = (double*)(base + r.off_P[nxt]);
}

hipError_t enqueue_step(const Problem& P, hipStream_t s) {
    hipError_t e;
    if ((e = launch_face_sums(P, s)) != hipSuccess) return e;
    if ((e = launch_face_close(P, s)) != hipSuccess) return e;
    if ((e = launch_cell_close(P, s)) != hipSuccess) return e;
    return launch_update(P, s);
}

// Capture `steps` consecutive steps starting from buffer parity `cur` into a
// graph (kernel nodes only).
static hipError_t capture_steps(cdugks_ctx* c, int cur, int steps, hipGraphExec_t* exec) {
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    Problem P = c->P;
    int k = cur;
    hipError_t le = hipSuccess;
    for (int s = 0; s < steps && le == hipSuccess; ++s) {
        set_pingpong(P, c->r, c->base, k);
        le = enqueue_step(P, c->stream);
        k = 1 - k;
    }
    e = hipStreamEndCapture(c->stream, &g);
    if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return le;
    }
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    return e;
}

static int scratch_on_device(int dev, double** out) {
    if (dev < 0 || dev >= MAX_DEVICES) return fail(CDUGKS_ERR_DEVICE, "device %d outside the scratch table", dev);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch array address");
        g_scratch_dev[dev] = (double*)p;
    }
    *out = g_scratch_dev[dev];
    return CDUGKS_OK;
}

}  // namespace cdg

using namespace cdg;

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* cdugks_last_error(void) { return g_last_error.c_str(); }

int cdugks_required_bytes(const cdugks_space* space, const cdugks_velocity* vel,
                          const cdugks_params* params, size_t* bytes) {
    if (!bytes) return fail(CDUGKS_ERR_INVALID, "null bytes pointer");
    cdugks_params p = *params;
    if (p.relax_mode == CDUGKS_RELAX_KN && !(p.rho_ref > 0.0)) p.rho_ref = 1.0;  // size does not depend on it
    Resolved r;
    int rc = resolve(space, vel, &p, nullptr, &r);
    if (rc) return rc;
    *bytes = r.bytes;
    return CDUGKS_OK;
}

int cdugks_init(const cdugks_space* space, const cdugks_velocity* vel, const cdugks_params* params,
                const double* rho, const double* u, const double* T, void* hip_stream, void* arena,
                size_t arena_bytes, cdugks_ctx** out) {
    if (!out) return fail(CDUGKS_ERR_INVALID, "null output pointer");
    *out = nullptr;
    if (!rho || !u || !T) return fail(CDUGKS_ERR_INVALID, "null moment array");
    Resolved r;
    int rc = resolve(space, vel, params, rho, &r);
    if (rc) return rc;
    for (long long c = 0; c < r.N; ++c) {
        if (!(rho[c] > 0.0) || !std::isfinite(rho[c])) return fail(CDUGKS_ERR_INVALID, "rho[%lld] must be > 0", c);
        if (!(T[c] > 0.0) || !std::isfinite(T[c])) return fail(CDUGKS_ERR_INVALID, "T[%lld] must be > 0", c);
    }
    for (long long k = 0; k < (long long)r.D * r.N; ++k)
        if (!std::isfinite(u[k])) return fail(CDUGKS_ERR_INVALID, "u[%lld] is not finite", k);

    cdugks_ctx* c = new (std::nothrow) cdugks_ctx();
    if (!c) return fail(CDUGKS_ERR_NOMEM, "host allocation failed");
    c->r = r;
    c->stream = (hipStream_t)hip_stream;
    hipError_t e;
    if ((e = hipGetDevice(&c->device)) != hipSuccess) {
        delete c;
        return hip_fail(e, "get device");
    }
    if (!c->stream) {
        // a private stream (default priority): graphs cannot be captured on
        // the legacy null stream
        if ((e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking)) != hipSuccess) {
            delete c;
            return hip_fail(e, "stream create");
        }
        c->own_stream = true;
    }
    if (arena) {
        if (arena_bytes < r.bytes) {
            if (c->own_stream) (void)hipStreamDestroy(c->stream);
            delete c;
            return fail(CDUGKS_ERR_INVALID, "arena of %zu bytes is smaller than the %zu required", arena_bytes,
                        r.bytes);
        }
        if (((uintptr_t)arena & 255) != 0) {
            if (c->own_stream) (void)hipStreamDestroy(c->stream);
            delete c;
            return fail(CDUGKS_ERR_INVALID, "arena must be 256-byte aligned");
        }
        c->base = (char*)arena;
        c->own_memory = false;
    } else {
        void* p = nullptr;
        e = hipMalloc(&p, r.bytes);
        if (e != hipSuccess) {
            if (c->own_stream) (void)hipStreamDestroy(c->stream);
            delete c;
            (void)hipGetLastError();
            return fail(CDUGKS_ERR_NOMEM, "hipMalloc of %zu bytes failed", r.bytes);
        }
        c->base = (char*)p;
        c->own_memory = true;
    }
    fill_problem(r, c->base, c->P);

    std::vector<double> veltab, axis;
    velocity_tables(r, veltab, axis);
    std::vector<double> dirtab;
    if (r.any_dirichlet) dirichlet_tables(r, veltab, dirtab);
    std::vector<long long> rowtab;
    if (r.storage == CDUGKS_STORE_F32_BF16TAIL) c->bf16_rows = tail_rows(r, veltab, u, T, rowtab);
    // moments staged in the arena's staging region for the init kernel
    std::vector<double> stage((size_t)(r.D + 2) * r.N);
    std::memcpy(stage.data(), rho, sizeof(double) * r.N);
    std::memcpy(stage.data() + r.N, u, sizeof(double) * r.D * r.N);
    std::memcpy(stage.data() + (size_t)(r.D + 1) * r.N, T, sizeof(double) * r.N);
    double* stage_dev = (double*)(c->base + r.off_scratch);
    int zero[64] = {0};
    if ((e = hipMemcpyAsync(c->base + r.off_vel, veltab.data(), veltab.size() * 8, hipMemcpyHostToDevice,
                            c->stream)) != hipSuccess ||
        (e = hipMemcpyAsync(c->base + r.off_axis, axis.data(), axis.size() * 8, hipMemcpyHostToDevice,
                            c->stream)) != hipSuccess ||
        (r.any_dirichlet && (e = hipMemcpyAsync(c->base + r.off_dir, dirtab.data(), dirtab.size() * 8,
                                                 hipMemcpyHostToDevice, c->stream)) != hipSuccess) ||
        (!rowtab.empty() && (e = hipMemcpyAsync(c->base + r.off_rows, rowtab.data(), rowtab.size() * 8,
                                                 hipMemcpyHostToDevice, c->stream)) != hipSuccess) ||
        (e = hipMemcpyAsync(stage_dev, stage.data(), stage.size() * 8, hipMemcpyHostToDevice, c->stream)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(c->base + r.off_err, zero, sizeof zero, hipMemcpyHostToDevice, c->stream)) !=
            hipSuccess) {
        cdugks_destroy(c);
        return hip_fail(e, "upload");
    }
    c->cur = 0;
    Problem P = c->P;
    set_pingpong(P, r, c->base, 0);
    if ((e = launch_init(P, stage_dev, stage_dev + r.N, stage_dev + (size_t)(r.D + 1) * r.N, c->stream)) !=
        hipSuccess) {
        cdugks_destroy(c);
        return hip_fail(e, "init kernels");
    }
    // host staging buffers must outlive the async copies
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) {
        cdugks_destroy(c);
        return hip_fail(e, "init synchronize");
    }
    int flag = 0;
    if ((e = hipMemcpy(&flag, c->base + r.off_err, sizeof flag, hipMemcpyDeviceToHost)) != hipSuccess) {
        cdugks_destroy(c);
        return hip_fail(e, "error flag read");
    }
    if (flag) {
        cdugks_destroy(c);
        return fail(CDUGKS_ERR_NONPHYSICAL, "non-physical initial state");
    }
    *out = c;
    return CDUGKS_OK;
}

int cdugks_regrid(cdugks_ctx* src, const cdugks_space* space, const cdugks_velocity* vel,
                  const cdugks_params* params, void* hip_stream, void* arena, size_t arena_bytes,
                  cdugks_ctx** out) {
    if (!out) return fail(CDUGKS_ERR_INVALID, "null output pointer");
    *out = nullptr;
    if (!src || !space || !vel || !params) return fail(CDUGKS_ERR_INVALID, "null argument");
    if (src->in_batch) return fail(CDUGKS_ERR_BUSY, "context belongs to a batch");
    if (src->sticky) return fail(src->sticky, "context is in an error state");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != src->device) {
        (void)hipGetLastError();
        return fail(CDUGKS_ERR_INVALID, "the source context lives on another device than the current one");
    }
    const Resolved& ro = src->r;
    bool same = space->dim == ro.D;
    for (int d = 0; same && d < ro.D; ++d) same = space->n[d] == ro.n[d];
    if (!same) return fail(CDUGKS_ERR_INVALID, "a refit keeps the cells and dimension of its source");
    // a Knudsen number refers to the source's reference density, not to the
    // density the problem has reached
    cdugks_params pa = *params;
    if (pa.relax_mode == CDUGKS_RELAX_KN && !(pa.rho_ref > 0.0)) pa.rho_ref = ro.rho_ref;
    // the source's moments (waits for its stream) set up the new context; W
    // itself is then carried bitwise
    std::vector<double> rho(ro.N), u((size_t)ro.D * ro.N), T(ro.N);
    int rc = cdugks_moments(src, rho.data(), u.data(), T.data(), 0);
    if (rc) return rc;
    cdugks_ctx* c = nullptr;
    rc = cdugks_init(space, vel, &pa, rho.data(), u.data(), T.data(), hip_stream, arena, arena_bytes, &c);
    if (rc) return rc;
    const Resolved& rn = c->r;
    if (rn.N != ro.N || rn.storage != ro.storage) {
        cdugks_destroy(c);
        return fail(CDUGKS_ERR_INVALID, "a refit keeps the cells, dimension and storage form of its source");
    }
    Problem Pn = c->P, Po = src->P;
    set_pingpong(Pn, rn, c->base, 0);
    set_pingpong(Po, ro, src->base, src->cur);
    hipError_t e = hipMemcpyAsync(const_cast<double*>(Pn.W_in), Po.W_in, sizeof(double) * (ro.D + 2) * ro.N,
                                  hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = launch_regrid(Pn, Po, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    int flag = 0;
    if (e == hipSuccess) e = hipMemcpy(&flag, c->base + rn.off_err, sizeof flag, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        cdugks_destroy(c);
        return hip_fail(e, "velocity-grid refit");
    }
    if (flag) {
        cdugks_destroy(c);
        return fail(CDUGKS_ERR_NONPHYSICAL, "non-physical state in the refit");
    }
    c->t0 = src->t0 + ro.dt * (double)(src->steps - src->steps0);
    c->steps = c->steps0 = src->steps;
    *out = c;
    return CDUGKS_OK;
}

int cdugks_storage_info(cdugks_ctx* c, int64_t* bf16_rows, size_t* state_array_bytes) {
    if (!c) return fail(CDUGKS_ERR_INVALID, "null context");
    if (bf16_rows) *bf16_rows = c->bf16_rows;
    if (state_array_bytes) {
        const Resolved& r = c->r;
        if (r.storage == CDUGKS_STORE_F32_BF16TAIL)
            *state_array_bytes = (size_t)(r.V - c->bf16_rows) * row_pitch_bytes((size_t)r.N * 4) +
                                 (size_t)c->bf16_rows * row_pitch_bytes((size_t)r.N * 2);
        else
            *state_array_bytes = (size_t)r.V * (size_t)r.pitch * (r.storage == CDUGKS_STORE_F64 ? 8 : 4);
    }
    return CDUGKS_OK;
}

int cdugks_step(cdugks_ctx* c, int64_t nsteps) {
    if (!c) return fail(CDUGKS_ERR_INVALID, "null context");
    if (nsteps < 0) return fail(CDUGKS_ERR_INVALID, "negative step count");
    if (c->sticky) return fail(c->sticky, "context is in an error state");
    if (c->in_batch) return fail(CDUGKS_ERR_BUSY, "context belongs to a batch");
    hipError_t e;
    int64_t left = nsteps;
    // chunk graphs of CHUNK steps, built lazily per starting parity
    while (left >= ctx_chunk) {
        hipGraphExec_t& ge = c->graph[c->cur];
        if (!ge && (e = capture_steps(c, c->cur, ctx_chunk, &ge)) != hipSuccess) return hip_fail(e, "graph capture");
        if ((e = hipGraphLaunch(ge, c->stream)) != hipSuccess) return hip_fail(e, "graph launch");
        left -= ctx_chunk;
        if (ctx_chunk % 2) c->cur = 1 - c->cur;
        c->steps += ctx_chunk;
    }
    for (; left > 0; --left) {
        Problem P = c->P;
        set_pingpong(P, c->r, c->base, c->cur);
        if ((e = enqueue_step(P, c->stream)) != hipSuccess) return hip_fail(e, "step launch");
        c->cur = 1 - c->cur;
        c->steps += 1;
    }
    return CDUGKS_OK;
}

int cdugks_sync(cdugks_ctx* c) {
    if (!c) return fail(CDUGKS_ERR_INVALID, "null context");
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        c->sticky = CDUGKS_ERR_DEVICE;
        return hip_fail(e, "stream synchronize");
    }
    int flag = 0;
    e = hipMemcpy(&flag, c->base + c->r.off_err, sizeof flag, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        c->sticky = CDUGKS_ERR_DEVICE;
        return hip_fail(e, "error flag read");
    }
    if (flag) c->sticky = CDUGKS_ERR_NONPHYSICAL;
    if (c->sticky) return fail(c->sticky, "non-physical state reached (rho <= 0, T <= 0 or non-finite)");
    return CDUGKS_OK;
}

int cdugks_moments(cdugks_ctx* c, double* rho, double* u, double* T, int device_ptrs) {
    if (!c || !rho || !u || !T) return fail(CDUGKS_ERR_INVALID, "null argument");
    const Resolved& r = c->r;
    hipError_t e;
    const double* W = (const double*)(c->base + r.off_W[c->cur]);
    if (device_ptrs) {
        if ((e = launch_moments(c->P, W, rho, u, T, c->stream)) != hipSuccess) return hip_fail(e, "moments");
        return c->sticky ? fail(c->sticky, "context is in an error state") : CDUGKS_OK;
    }
    double* s = (double*)(c->base + r.off_scratch);
    if ((e = launch_moments(c->P, W, s, s + r.N, s + (size_t)(r.D + 1) * r.N, c->stream)) != hipSuccess)
        return hip_fail(e, "moments");
    int rc = cdugks_sync(c);
    if (rc) return rc;
    if ((e = hipMemcpy(rho, s, sizeof(double) * r.N, hipMemcpyDeviceToHost)) != hipSuccess ||
        (e = hipMemcpy(u, s + r.N, sizeof(double) * r.D * r.N, hipMemcpyDeviceToHost)) != hipSuccess ||
        (e = hipMemcpy(T, s + (size_t)(r.D + 1) * r.N, sizeof(double) * r.N, hipMemcpyDeviceToHost)) !=
            hipSuccess)
        return hip_fail(e, "moments copy");
    return CDUGKS_OK;
}

int cdugks_conserved(cdugks_ctx* c, double* W) {
    if (!c || !W) return fail(CDUGKS_ERR_INVALID, "null argument");
    int rc = cdugks_sync(c);
    if (rc) return rc;
    const Resolved& r = c->r;
    std::vector<double> tmp((size_t)(r.D + 2) * r.N);
    hipError_t e = hipMemcpy(tmp.data(), c->base + r.off_W[c->cur], tmp.size() * 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "W copy");
    for (long long cc = 0; cc < r.N; ++cc)
        for (int k = 0; k < r.D + 2; ++k) W[cc * (r.D + 2) + k] = tmp[(size_t)k * r.N + cc];
    return CDUGKS_OK;
}

int cdugks_distributions(cdugks_ctx* c, double* g, double* b) {
    if (!c || !g || !b) return fail(CDUGKS_ERR_INVALID, "null argument");
    int rc = cdugks_sync(c);
    if (rc) return rc;
    const Resolved& r = c->r;
    size_t n = (size_t)r.N * r.V;
    double* tmp = nullptr;
    hipError_t e = hipMalloc(&tmp, n * 8);
    if (e != hipSuccess) return hip_fail(e, "temporary allocation");
    double* outs[2] = {g, b};
    size_t offs[2] = {r.off_g[c->cur], r.off_b[c->cur]};
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
        e = launch_to_f64(c->P, c->base + offs[k], 0, (int)r.V, tmp, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e == hipSuccess) e = hipMemcpy(outs[k], tmp, n * 8, hipMemcpyDeviceToHost);
    }
    (void)hipFree(tmp);
    return e == hipSuccess ? CDUGKS_OK : hip_fail(e, "distribution copy");
}

int cdugks_distributions_noalloc(cdugks_ctx* c, double* g, double* b) {
    if (!c || !g || !b) return fail(CDUGKS_ERR_INVALID, "null argument");
    const Resolved& r = c->r;
    const size_t row_bytes = (size_t)r.N * sizeof(double);
    const long long per_pass = (long long)(CDUGKS_NOALLOC_SCRATCH_BYTES / row_bytes);
    if (per_pass < 1)
        return fail(CDUGKS_ERR_TOO_LARGE,
                    "a velocity row of %lld cells (%zu bytes as FP64) exceeds the %zu-byte scratch array",
                    (long long)r.N, row_bytes, (size_t)CDUGKS_NOALLOC_SCRATCH_BYTES);
    int rc = cdugks_sync(c);
    if (rc) return rc;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    int prev = -1;
    hipError_t e = hipGetDevice(&prev);
    if (e == hipSuccess && prev != c->device) e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(e, "select the context's device");
    double* buf = nullptr;
    rc = scratch_on_device(c->device, &buf);
    double* outs[2] = {g, b};
    const size_t offs[2] = {r.off_g[c->cur], r.off_b[c->cur]};
    for (int k = 0; k < 2 && rc == CDUGKS_OK; ++k) {
        for (long long i0 = 0; i0 < r.V && rc == CDUGKS_OK; i0 += per_pass) {
            const int nr = (int)std::min<long long>(per_pass, r.V - i0);
            e = launch_to_f64(c->P, c->base + offs[k], (int)i0, nr, buf, c->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(outs[k] + (size_t)i0 * r.N, buf, (size_t)nr * row_bytes, hipMemcpyDeviceToHost,
                                   c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            if (e != hipSuccess) rc = hip_fail(e, "distribution copy through the scratch array");
        }
    }
    if (prev >= 0 && prev != c->device) (void)hipSetDevice(prev);
    return rc;
}

int cdugks_launch_info(cdugks_ctx* c, int* face_tile, int* face_slices, int* update_slices) {
    if (!c) return fail(CDUGKS_ERR_INVALID, "null context");
    if (face_tile) *face_tile = c->r.tile + 1;
    if (face_slices) *face_slices = c->r.nslices;
    if (update_slices) *update_slices = c->r.nslices_upd;
    return CDUGKS_OK;
}

int cdugks_info(cdugks_ctx* c, double* dt, double* t, int64_t* steps) {
    if (!c) return fail(CDUGKS_ERR_INVALID, "null context");
    if (dt) *dt = c->r.dt;
    if (t) *t = c->t0 + c->r.dt * (double)(c->steps - c->steps0);
    if (steps) *steps = c->steps;
    return CDUGKS_OK;
}

int cdugks_profile_phases(cdugks_ctx* c, int64_t nsteps, double* ms) {
    if (!c || !ms || nsteps <= 0) return fail(CDUGKS_ERR_INVALID, "bad argument");
    if (c->sticky) return fail(c->sticky, "context is in an error state");
    hipEvent_t ev[5];
    for (int k = 0; k < 5; ++k)
        if (hipEventCreate(&ev[k]) != hipSuccess) return fail(CDUGKS_ERR_DEVICE, "event create");
    double acc[4] = {0, 0, 0, 0};
    hipError_t e = hipSuccess;
    for (int64_t s = 0; s < nsteps && e == hipSuccess; ++s) {
        Problem P = c->P;
        set_pingpong(P, c->r, c->base, c->cur);
        e = hipEventRecord(ev[0], c->stream);
        if (e == hipSuccess) e = launch_face_sums(P, c->stream);
        if (e == hipSuccess) e = hipEventRecord(ev[1], c->stream);
        if (e == hipSuccess) e = launch_face_close(P, c->stream);
        if (e == hipSuccess) e = hipEventRecord(ev[2], c->stream);
        if (e == hipSuccess) e = launch_cell_close(P, c->stream);
        if (e == hipSuccess) e = hipEventRecord(ev[3], c->stream);
        if (e == hipSuccess) e = launch_update(P, c->stream);
        if (e == hipSuccess) e = hipEventRecord(ev[4], c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(ev[4]);
        for (int k = 0; k < 4 && e == hipSuccess; ++k) {
            float t = 0.f;
            e = hipEventElapsedTime(&t, ev[k], ev[k + 1]);
            acc[k] += t;
        }
        c->cur = 1 - c->cur;
        c->steps += 1;
    }
    for (int k = 0; k < 5; ++k) (void)hipEventDestroy(ev[k]);
    if (e != hipSuccess) return hip_fail(e, "profiled step");
    for (int k = 0; k < 4; ++k) ms[k] = acc[k] / (double)nsteps;
    return cdugks_sync(c);
}

void cdugks_destroy(cdugks_ctx* c) {
    if (!c) return;
    if (c->in_batch) {
        // the batch's captured graphs and device problem table point into
        // this context's memory: refuse, and leave the context intact
        fail(CDUGKS_ERR_BUSY, "context belongs to a batch (destroy the batch first); not destroyed");
        return;
    }
    (void)hipStreamSynchronize(c->stream);
    for (int k = 0; k < 2; ++k)
        if (c->graph[k]) (void)hipGraphExecDestroy(c->graph[k]);
    if (c->own_memory && c->base) (void)hipFree(c->base);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

}  // extern "C"
