// HIP kernels of one CDUGKS time step for gfx950.
//
// Data layout (per problem):
//   g, b        [V][N]  velocity-major, cells fastest (x fastest); FP64 or FP32
//   W           [D+2][N] FP64 conserved variables (rho, rho u, rho E)
//   cell coefs  [NPC][N] FP64, derived from W (see cdugks_internal.h)
//   face sums   [slices][D][2D+3][NE], face coefs [D][NFP][NE], flux [D][D+2][NE]
// Faces along d are indexed by the cell on their right on the extended grid
// NE = prod_d (n_d + [outflow_d]).
//
// One step = four launches:
//   face_sums  (tile kernel) : quarter-step field phi_bar_plus (eq. phibarplus),
//                              Van Leer slopes (eq. VanLeer) and slopes of slopes,
//                              face value at the characteristic foot (eq. relation),
//                              and per-face velocity sums -> partial sums per slice
//   face_close (per face)    : face W (eqs. rhobar..rhoEbar), face equilibrium and
//                              relaxation, inversion coefficients (eq. phibar), and
//                              the flux moments in closed form
//   cell_close (per cell)    : W^{n+1} from the flux moments (eqs. rhoupdate..
//                              rhoEupdate, outward-flux sign), cell coefficients at n+1
//   update     (tile kernel) : face values again, inversion, microflux (eq. flux),
//                              and phi^{n+1} (eq. phiupdate)
//
// Tile kernels: one thread per cell of a 256-cell tile; the thread loops over
// its slice of discrete velocities, so the velocity sums of face_sums are
// serial per thread (no atomics, fixed order).  For each velocity the tile and
// its halo of phi_bar_plus and of the limited slopes are staged in LDS.
#include "cdugks_internal.h"

#include <math.h>

namespace cdg {

constexpr int WG = 256;

__device__ __forceinline__ int map_coord(int x, int n, int bc) {
    if (bc == 0) {
        int r = x % n;
        return r < 0 ? r + n : r;
    }
    return x < 0 ? 0 : (x >= n ? n - 1 : x);
}

// Van Leer limiter (eq. VanLeer) in the harmonic-mean form: identical to
// (sgn a + sgn b)|a||b|/(|a|+|b|); zero at extrema and for a flat side.
__device__ __forceinline__ double van_leer(double a, double b) {
    double p = a * b;
    return p > 0.0 ? (p + p) / (a + b) : 0.0;
}

template <typename ST>
__device__ __forceinline__ double ld(const void* base, long long idx) {
    return (double)reinterpret_cast<const ST*>(base)[idx];
}
template <typename ST>
__device__ __forceinline__ void st(void* base, long long idx, double v) {
    reinterpret_cast<ST*>(base)[idx] = (ST)v;
}

__device__ __forceinline__ void raise_error(int* err) { *err = 1; }

// ---------------------------------------------------------------------------
// primitives shared by the per-cell and per-face closures (Sec. 2)
// ---------------------------------------------------------------------------
struct Prim {
    double rho, u[3], RT, inv_tau_g;
    bool bad;
};

__device__ Prim primitives(const Problem& P, const double* Wv) {
    Prim q;
    const int D = P.D;
    q.rho = Wv[0];
    double u2 = 0.0;
    for (int d = 0; d < 3; ++d) {
        q.u[d] = d < D ? Wv[1 + d] / q.rho : 0.0;
        u2 += q.u[d] * q.u[d];
    }
    double E = Wv[D + 1] / q.rho;
    double T = (P.gamma - 1.0) / P.R * (E - 0.5 * u2);
    q.RT = P.R * T;
    if (P.relax == 0) {
        double mu = P.mu_ref * pow(T / P.T_ref, P.omega);
        q.inv_tau_g = q.rho * q.RT / mu;
    } else {
        q.inv_tau_g = P.tau_inv;
    }
    q.bad = !(q.rho > 0.0) || !(T > 0.0) || !isfinite(q.rho) || !isfinite(T) ||
            !isfinite(q.u[0]) || !isfinite(q.u[1]) || !isfinite(q.u[2]) || !isfinite(q.inv_tau_g);
    return q;
}

__device__ __forceinline__ double maxwell_prefactor(const Problem& P, double rho, double RT) {
    double two_pi_rt = 2.0 * M_PI * RT;
    double f = P.D == 1 ? 1.0 / sqrt(two_pi_rt)
                        : (P.D == 2 ? 1.0 / two_pi_rt : 1.0 / (two_pi_rt * sqrt(two_pi_rt)));
    return rho * f;
}

__device__ void write_cell_coefs(const Problem& P, double* Pc, long long N, long long c, const Prim& q) {
    double beta = 0.25 * P.dt * q.inv_tau_g;
    Pc[PC_A * N + c] = maxwell_prefactor(P, q.rho, q.RT);
    Pc[PC_INV2RT * N + c] = 0.5 / q.RT;
    Pc[PC_CRT2 * N + c] = 0.5 * P.c_int * q.RT;
    Pc[PC_BETA * N + c] = beta;
    Pc[PC_BETAB * N + c] = beta * P.Pr;
    Pc[PC_ETA * N + c] = beta * (P.Pr - 1.0);
    Pc[PC_HU2 * N + c] = 0.5 * (q.u[0] * q.u[0] + q.u[1] * q.u[1] + q.u[2] * q.u[2]);
    for (int d = 0; d < 3; ++d) Pc[(PC_U0 + d) * N + c] = q.u[d];
}

// ---------------------------------------------------------------------------
// init: W^0 from (rho, u, T) and the cell coefficients; then phi^0 = phi_eq
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(WG) void k_init_cells(Problem P, const double* rho, const double* u,
                                                   const double* T) {
    long long c = (long long)blockIdx.x * WG + threadIdx.x;
    if (c >= P.N) return;
    const int D = P.D;
    const long long N = P.N;
    double Wv[5];
    double u2 = 0.0;
    Wv[0] = rho[c];
    for (int d = 0; d < D; ++d) {
        double ud = u[d * N + c];
        Wv[1 + d] = rho[c] * ud;
        u2 += ud * ud;
    }
    // rho E = rho (u^2/2 + c_v T), c_v = (3+K)R/2 = R/(gamma-1)
    Wv[D + 1] = rho[c] * (0.5 * u2 + P.R * T[c] / (P.gamma - 1.0));
    for (int k = 0; k < D + 2; ++k) const_cast<double*>(P.W_in)[k * N + c] = Wv[k];
    Prim q = primitives(P, Wv);
    if (q.bad) raise_error(P.err);
    write_cell_coefs(P, const_cast<double*>(P.P_in), N, c, q);
}

template <typename ST>
__global__ __launch_bounds__(WG) void k_init_phi(Problem P) {
    long long idx = (long long)blockIdx.x * WG + threadIdx.x;
    const long long N = P.N;
    if (idx >= N * P.V) return;
    long long i = idx / N, c = idx - i * N;
    const double* ve = P.vel + i * NVEL;
    const double* Pc = P.P_in;
    double c2 = 0.0;
    for (int d = 0; d < P.D; ++d) {
        double x = ve[VE_XI0 + d] - Pc[(PC_U0 + d) * N + c];
        c2 += x * x;
    }
    double geq = Pc[PC_A * N + c] * exp(-c2 * Pc[PC_INV2RT * N + c]);
    double beq = (ve[VE_HX2] + Pc[PC_CRT2 * N + c]) * geq;
    st<ST>(const_cast<void*>(P.g_in), idx, geq);
    st<ST>(const_cast<void*>(P.b_in), idx, beq);
}

// ---------------------------------------------------------------------------
// tile kernels
// ---------------------------------------------------------------------------
template <int D> struct Tile;
template <> struct Tile<1> { static constexpr int X = 256, Y = 1, Z = 1; };
template <> struct Tile<2> { static constexpr int X = 16, Y = 16, Z = 1; };
template <> struct Tile<3> { static constexpr int X = 8, Y = 8, Z = 4; };

// XCD-aware order: consecutive workgroup ids are spread over the 8 XCDs, so
// give each XCD a contiguous block of the (tile, slice) space; neighbouring
// tiles then share halo lines in that XCD's L2.
__device__ __forceinline__ int xcd_remap(int lin, int total) {
    int per = total / 8;
    if (lin >= per * 8) return lin;
    return (lin % 8) * per + lin / 8;
}

// Box geometry of the staged halo for a tile: q box covers tile offsets
// [-3, T-1+QH], the limited-slope box [-2, T-1+AH].
template <int D, bool UPD>
struct Geo {
    static constexpr int TX = Tile<D>::X, TY = Tile<D>::Y, TZ = Tile<D>::Z;
    static constexpr int QH = UPD ? 3 : 2, AH = UPD ? 2 : 1;
    static constexpr int QX = TX + 3 + QH;
    static constexpr int QY = D >= 2 ? TY + 3 + QH : 1;
    static constexpr int QZ = D >= 3 ? TZ + 3 + QH : 1;
    static constexpr int AX = TX + 2 + AH;
    static constexpr int AY = D >= 2 ? TY + 2 + AH : 1;
    static constexpr int AZ = D >= 3 ? TZ + 2 + AH : 1;
    static constexpr int NQ = QX * QY * QZ;
    static constexpr int NA = AX * AY * AZ;
    static constexpr int NRQ = (NQ + WG - 1) / WG;   // q points per thread
    static constexpr int NRA = (NA + WG - 1) / WG;   // slope points per thread
    // face boxes of the update kernel: along d one more face than cells
    static constexpr int NF0 = (TX + 1) * TY * TZ;
    static constexpr int NF1 = D >= 2 ? TX * (TY + 1) * TZ : 0;
    static constexpr int NF2 = D >= 3 ? TX * TY * (TZ + 1) : 0;
    static constexpr int NFT = NF0 + NF1 + NF2;
    static constexpr int NRF = (NFT + WG - 1) / WG;
    static constexpr bool CACHE_COEF = (NQ - TX * TY * TZ + WG - 1) / WG + 1 <= 2;
    // offsets of tile coordinate 0 inside the boxes, and box strides
    static constexpr int OQX = 3, OQY = D >= 2 ? 3 : 0, OQZ = D >= 3 ? 3 : 0;
    static constexpr int OAX = 2, OAY = D >= 2 ? 2 : 0, OAZ = D >= 3 ? 2 : 0;
    __device__ static constexpr int SQ(int e) { return e == 0 ? 1 : (e == 1 ? QX : QX * QY); }
    __device__ static constexpr int SA(int e) { return e == 0 ? 1 : (e == 1 ? AX : AX * AY); }
    __device__ static int qidx(int x, int y, int z) { return (x + OQX) + QX * ((y + OQY) + QY * (z + OQZ)); }
    __device__ static int aidx(int x, int y, int z) { return (x + OAX) + AX * ((y + OAY) + AY * (z + OAZ)); }
};

struct CellCoef {
    double A, inv2RT, cRT2, beta, betab, eta, hu2, u[3];
};

__device__ __forceinline__ CellCoef load_coef(const double* Pc, long long N, long long c) {
    CellCoef k;
    k.A = Pc[PC_A * N + c];
    k.inv2RT = Pc[PC_INV2RT * N + c];
    k.cRT2 = Pc[PC_CRT2 * N + c];
    k.beta = Pc[PC_BETA * N + c];
    k.betab = Pc[PC_BETAB * N + c];
    k.eta = Pc[PC_ETA * N + c];
    k.hu2 = Pc[PC_HU2 * N + c];
    k.u[0] = Pc[PC_U0 * N + c];
    k.u[1] = Pc[(PC_U0 + 1) * N + c];
    k.u[2] = Pc[(PC_U0 + 2) * N + c];
    return k;
}

struct Vel {
    double xi[3], w, hx2, lam[3];
};

__device__ __forceinline__ Vel load_vel(const double* vel, int i) {
    const double* v = vel + (long long)i * NVEL;
    Vel r;
    r.xi[0] = v[0]; r.xi[1] = v[1]; r.xi[2] = v[2];
    r.w = v[VE_W]; r.hx2 = v[VE_HX2];
    r.lam[0] = v[VE_LAM0]; r.lam[1] = v[VE_LAM0 + 1]; r.lam[2] = v[VE_LAM0 + 2];
    return r;
}

// Equilibria, Z and the quarter-step fields at one (cell, velocity):
// phi_bar_plus = phi + (h/2)(phi_eq - phi)/tau + (h/2) S, S_b = Z (g - g_eq)/tau_bg.
// Returns g_eq.
template <int D>
__device__ __forceinline__ double quarter_step(const CellCoef& k, const Vel& v, double g, double b,
                                               double& qg, double& qb) {
    double c2 = 0.0, xu = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        double x = v.xi[d] - k.u[d];
        c2 += x * x;
        xu += v.xi[d] * k.u[d];
    }
    double geq = k.A * exp(-c2 * k.inv2RT);
    double beq = (v.hx2 + k.cRT2) * geq;
    double Z = xu - k.hu2;
    qg = g + k.beta * (geq - g);
    qb = b + k.betab * (beq - b) + k.eta * Z * (g - geq);
    return geq;
}

// Value of phi_bar at a face centre at t_{n+1/2}: upwind cell u (LDS indices
// qi, ai), side s = +1 when the face is u's right face, -1 when its left face.
//   v = q(u) + s a_d/2 - sum_e lambda_e (a_e + s b_de/2),
// a_e = VL of one-sided differences of q along e (slope times dx_e) and
// b_de = VL of differences of a_e along d (slope of the slope times dx_d dx_e).
template <int D, class GEO>
__device__ __forceinline__ double face_value(const double* sq, const double* sa, int d, int qi,
                                             int ai, double s, const Vel& v) {
    const int sd = GEO::SA(d);
    double val = sq[qi] + 0.5 * s * sa[d * GEO::NA + ai];
#pragma unroll
    for (int e = 0; e < D; ++e) {
        const double* ae = sa + e * GEO::NA;
        double a0 = ae[ai];
        double bde = van_leer(a0 - ae[ai - sd], ae[ai + sd] - a0);
        val -= v.lam[e] * (a0 + 0.5 * s * bde);
    }
    return val;
}

// Both one-sided candidates of a face: left upwind cell (qi_l, ai_l) used when
// xi_d > 0, right upwind cell (qi_r, ai_r) when xi_d < 0, their mean at xi_d = 0.
template <int D, class GEO>
__device__ __forceinline__ void face_pair(const double* const* sq, const double* const* sa, int d,
                                          int qi_l, int ai_l, int qi_r, int ai_r, const Vel& v,
                                          double& vg, double& vb) {
    const double xd = d == 0 ? v.xi[0] : (d == 1 ? v.xi[1] : v.xi[2]);
    if (xd > 0.0) {
        vg = face_value<D, GEO>(sq[0], sa[0], d, qi_l, ai_l, 1.0, v);
        vb = face_value<D, GEO>(sq[1], sa[1], d, qi_l, ai_l, 1.0, v);
    } else if (xd < 0.0) {
        vg = face_value<D, GEO>(sq[0], sa[0], d, qi_r, ai_r, -1.0, v);
        vb = face_value<D, GEO>(sq[1], sa[1], d, qi_r, ai_r, -1.0, v);
    } else {
        vg = 0.5 * (face_value<D, GEO>(sq[0], sa[0], d, qi_l, ai_l, 1.0, v) +
                    face_value<D, GEO>(sq[0], sa[0], d, qi_r, ai_r, -1.0, v));
        vb = 0.5 * (face_value<D, GEO>(sq[1], sa[1], d, qi_l, ai_l, 1.0, v) +
                    face_value<D, GEO>(sq[1], sa[1], d, qi_r, ai_r, -1.0, v));
    }
}

// Face coefficients used to invert eq. phibar at a face: NFC per face.
template <int D>
struct FaceCoef {
    static constexpr int NFC = 9 + D;
    double A, inv2RT, cRT2, ig, bg, ib, bb, eb, hu2, u[D];
    __device__ void load(const double* F, long long NE) {
        A = F[PF_A * NE];
        inv2RT = F[PF_INV2RT * NE];
        cRT2 = F[PF_CRT2 * NE];
        ig = F[PF_IG * NE];
        bg = F[PF_BG * NE];
        ib = F[PF_IB * NE];
        bb = F[PF_BB * NE];
        eb = F[PF_EB * NE];
        hu2 = F[PF_HU2 * NE];
#pragma unroll
        for (int e = 0; e < D; ++e) u[e] = F[(PF_U0 + e) * NE];
    }
    // LDS layout [NFC][stride]
    __device__ void store(double* s, int j, int stride) const {
        s[0 * stride + j] = A; s[1 * stride + j] = inv2RT; s[2 * stride + j] = cRT2;
        s[3 * stride + j] = ig; s[4 * stride + j] = bg; s[5 * stride + j] = ib;
        s[6 * stride + j] = bb; s[7 * stride + j] = eb; s[8 * stride + j] = hu2;
#pragma unroll
        for (int e = 0; e < D; ++e) s[(9 + e) * stride + j] = u[e];
    }
    __device__ void fetch(const double* s, int j, int stride) {
        A = s[0 * stride + j]; inv2RT = s[1 * stride + j]; cRT2 = s[2 * stride + j];
        ig = s[3 * stride + j]; bg = s[4 * stride + j]; ib = s[5 * stride + j];
        bb = s[6 * stride + j]; eb = s[7 * stride + j]; hu2 = s[8 * stride + j];
#pragma unroll
        for (int e = 0; e < D; ++e) u[e] = s[(9 + e) * stride + j];
    }
    // phi at the face from phi_bar: g = ig gbar + bg g_eq; b likewise with the
    // S_b source at the face evaluated with the face g.
    __device__ __forceinline__ void invert(const Vel& v, double vg, double vb, double& gF, double& bF) const {
        double c2 = 0.0, xu = 0.0;
#pragma unroll
        for (int e = 0; e < D; ++e) {
            double x = v.xi[e] - u[e];
            c2 += x * x;
            xu += v.xi[e] * u[e];
        }
        double geq = A * exp(-c2 * inv2RT);
        double beq = (v.hx2 + cRT2) * geq;
        double Z = xu - hu2;
        gF = ig * vg + bg * geq;
        bF = ib * vb + bb * beq + eb * Z * (gF - geq);
    }
};

template <int D, typename ST, bool UPD>
struct TileKernel {
    using G = Geo<D, UPD>;
    static constexpr int NT = G::TX * G::TY * G::TZ;
    // face coefficients staged in LDS once for the whole velocity loop (1-D
    // and 2-D); the 3-D kernel reads them from memory (LDS is full)
    static constexpr bool CACHE_FACE = D <= 2;
    static constexpr int NFC = FaceCoef<D>::NFC;
    // q-box points per thread: slot 0 is the thread's own cell, the other
    // slots cover the halo
    static constexpr int NHALO = G::NQ - NT;
    static constexpr int NSLOT = 1 + (NHALO + WG - 1) / WG;

    struct Smem {
        double q[2][G::NQ];              // phi_bar_plus for g, b
        double a[2][D * G::NA];          // limited differences for g, b
        double f[UPD ? 2 * G::NFT : 1];  // face phi (update kernel)
        double fc[UPD && CACHE_FACE ? NFC * G::NFT : 1];  // face coefficients
    };

    __device__ static void run(const Problem& P, int tile, int slice, int nslices, Smem& sm) {
        const int tid = threadIdx.x;
        const long long N = P.N;
        const int* tiles = UPD ? P.tiles2 : P.tiles1;
        int t = tile;
        const int ox = (t % tiles[0]) * G::TX;
        t /= tiles[0];
        const int oy = D >= 2 ? (t % tiles[1]) * G::TY : 0;
        t /= tiles[1];
        const int oz = D >= 3 ? t * G::TZ : 0;
        const int v0 = (int)((long long)P.V * slice / nslices);
        const int v1 = (int)((long long)P.V * (slice + 1) / nslices);
        const double* sqp[2] = {sm.q[0], sm.q[1]};
        const double* sap[2] = {sm.a[0], sm.a[1]};

        // q-box points of this thread: slot 0 its own cell, then halo points
        // (halo enumerated in box order, interior skipped); source cell after
        // periodic wrap / outflow clamp
        long long srcq[NSLOT];
        int lq[NSLOT];
        CellCoef kq[G::CACHE_COEF ? NSLOT : 1];
        {
            int want[NSLOT];
#pragma unroll
            for (int k = 0; k < NSLOT; ++k) {
                lq[k] = -1;
                want[k] = k == 0 ? -1 : tid + (k - 1) * WG;  // halo ordinal
            }
            {
                int lx = tid % G::TX, ly = (tid / G::TX) % G::TY, lz = tid / (G::TX * G::TY);
                lq[0] = G::qidx(lx, ly, lz);
            }
            int h = 0;
            for (int r = 0; r < G::NQ; ++r) {
                int rx = r % G::QX, ry = (r / G::QX) % G::QY, rz = r / (G::QX * G::QY);
                int lx = rx - G::OQX, ly = ry - G::OQY, lz = rz - G::OQZ;
                bool interior = lx >= 0 && lx < G::TX && ly >= 0 && ly < G::TY && lz >= 0 && lz < G::TZ;
                if (interior) continue;
#pragma unroll
                for (int k = 1; k < NSLOT; ++k)
                    if (want[k] == h) lq[k] = r;
                ++h;
            }
#pragma unroll
            for (int k = 0; k < NSLOT; ++k) {
                srcq[k] = -1;
                if (lq[k] < 0) continue;
                int r = lq[k];
                int rx = r % G::QX, ry = (r / G::QX) % G::QY, rz = r / (G::QX * G::QY);
                int cx = map_coord(ox + rx - G::OQX, P.n[0], P.bc[0]);
                int cy = D >= 2 ? map_coord(oy + ry - G::OQY, P.n[1], P.bc[1]) : 0;
                int cz = D >= 3 ? map_coord(oz + rz - G::OQZ, P.n[2], P.bc[2]) : 0;
                srcq[k] = cx + (long long)P.n[0] * (cy + (long long)P.n[1] * cz);
                if constexpr (G::CACHE_COEF) kq[k] = load_coef(P.P_in, N, srcq[k]);
            }
        }

        // own cell
        const int tx = tid % G::TX, ty = (tid / G::TX) % G::TY, tz = tid / (G::TX * G::TY);
        const int gx = ox + tx, gy = oy + ty, gz = oz + tz;

        // face-sum accumulators (face_sums)
        constexpr int NS = 2 * D + 3;
        double acc[UPD ? 1 : D][UPD ? 1 : NS];
        if constexpr (!UPD) {
#pragma unroll
            for (int d = 0; d < D; ++d)
#pragma unroll
                for (int j = 0; j < NS; ++j) acc[d][j] = 0.0;
        }
        const bool own_inside = gx < P.n[0] && (D < 2 || gy < P.n[1]) && (D < 3 || gz < P.n[2]);
        const long long own = own_inside ? gx + (long long)P.n[0] * (gy + (long long)P.n[1] * gz) : 0;

        // update kernel: own-cell coefficients at n and n+1, and the faces this
        // thread reconstructs (left faces of tile cells [0, T_d] along d)
        CellCoef k0, k1;
        int fd[UPD ? G::NRF : 1], fql[UPD ? G::NRF : 1], fal[UPD ? G::NRF : 1];
        int fqr[UPD ? G::NRF : 1], far_[UPD ? G::NRF : 1];
        long long fidx[UPD ? G::NRF : 1];
        double own_g = 0.0, own_b = 0.0, own_geq = 0.0;
        if constexpr (UPD) {
            if (own_inside) {
                k0 = load_coef(P.P_in, N, own);
                k1 = load_coef(P.P_out, N, own);
            }
#pragma unroll
            for (int k = 0; k < G::NRF; ++k) {
                int j = tid + k * WG;
                fidx[k] = -1;
                fd[k] = 0;
                fql[k] = fal[k] = fqr[k] = far_[k] = 0;
                if (j >= G::NFT) continue;
                int d, fx, fy, fz;
                int jj = j;
                if (jj < G::NF0) {
                    d = 0; fx = jj % (G::TX + 1); fy = (jj / (G::TX + 1)) % G::TY; fz = jj / ((G::TX + 1) * G::TY);
                } else if (D >= 2 && (jj -= G::NF0) < G::NF1) {
                    d = 1; fx = jj % G::TX; fy = (jj / G::TX) % (G::TY + 1); fz = jj / (G::TX * (G::TY + 1));
                } else {
                    if (D >= 2) jj -= G::NF1;
                    d = 2; fx = jj % G::TX; fy = (jj / G::TX) % G::TY; fz = jj / (G::TX * G::TY);
                }
                int dxo = d == 0, dyo = d == 1, dzo = d == 2;
                int cc[3] = {ox + fx, oy + fy, oz + fz};
                bool valid = true;
#pragma unroll
                for (int e = 0; e < D; ++e) {
                    if (e == d) {
                        if (cc[e] > P.n[e]) valid = false;
                        else if (cc[e] == P.n[e] && P.bc[e] == 0) cc[e] = 0;
                    } else if (cc[e] >= P.n[e]) {
                        valid = false;
                    }
                }
                fd[k] = d;
                fql[k] = G::qidx(fx - dxo, fy - dyo, fz - dzo);
                fal[k] = G::aidx(fx - dxo, fy - dyo, fz - dzo);
                fqr[k] = G::qidx(fx, fy, fz);
                far_[k] = G::aidx(fx, fy, fz);
                if (valid) fidx[k] = cc[0] + (long long)P.ne[0] * (cc[1] + (long long)P.ne[1] * cc[2]);
                if constexpr (CACHE_FACE) {
                    FaceCoef<D> fcv{};
                    if (valid) fcv.load(P.FP + (long long)d * NFP * P.NE + fidx[k], P.NE);
                    fcv.store(sm.fc, j, G::NFT);
                }
            }
            if constexpr (CACHE_FACE) __syncthreads();
        }

        for (int i = v0; i < v1; ++i) {
            const Vel v = load_vel(P.vel, i);
            const long long vb = (long long)i * N;

            // stage 1: quarter-step fields on the q box
#pragma unroll
            for (int k = 0; k < NSLOT; ++k) {
                const int r = lq[k];
                if (r >= 0) {
                    double g = ld<ST>(P.g_in, vb + srcq[k]);
                    double b = ld<ST>(P.b_in, vb + srcq[k]);
                    double qg, qb, geq;
                    if constexpr (G::CACHE_COEF) {
                        geq = quarter_step<D>(kq[k], v, g, b, qg, qb);
                    } else {
                        CellCoef kk = load_coef(P.P_in, N, srcq[k]);
                        geq = quarter_step<D>(kk, v, g, b, qg, qb);
                    }
                    sm.q[0][r] = qg;
                    sm.q[1][r] = qb;
                    if (k == 0) {
                        own_g = g;
                        own_b = b;
                        own_geq = geq;
                    }
                }
            }
            __syncthreads();

            // stage 2: limited differences on the slope box
#pragma unroll
            for (int k = 0; k < G::NRA; ++k) {
                int p = tid + k * WG;
                if (p < G::NA) {
                    int px = p % G::AX, py = (p / G::AX) % G::AY, pz = p / (G::AX * G::AY);
                    int qi = (px + 1) + G::QX * ((py + (D >= 2 ? 1 : 0)) + G::QY * (pz + (D >= 3 ? 1 : 0)));
#pragma unroll
                    for (int e = 0; e < D; ++e) {
                        int sq = G::SQ(e);
#pragma unroll
                        for (int f = 0; f < 2; ++f) {
                            const double* q = sm.q[f];
                            double c = q[qi];
                            sm.a[f][e * G::NA + p] = van_leer(c - q[qi - sq], q[qi + sq] - c);
                        }
                    }
                }
            }
            __syncthreads();

            if constexpr (!UPD) {
                // stage 3: left face of the own cell along each d
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    const double xd = v.xi[d];
                    int dxo = d == 0, dyo = d == 1, dzo = d == 2;
                    double vg, vb2;
                    face_pair<D, G>(sqp, sap, d, G::qidx(tx - dxo, ty - dyo, tz - dzo),
                                    G::aidx(tx - dxo, ty - dyo, tz - dzo), G::qidx(tx, ty, tz),
                                    G::aidx(tx, ty, tz), v, vg, vb2);
                    const double wg = v.w * vg, wb = v.w * vb2;
                    acc[d][0] += wg;
#pragma unroll
                    for (int e = 0; e < D; ++e) acc[d][1 + e] += v.xi[e] * wg;
                    acc[d][D + 1] += wb;
#pragma unroll
                    for (int e = 0; e < D; ++e) acc[d][D + 2 + e] += xd * v.xi[e] * wg;
                    acc[d][2 * D + 2] += xd * wb;
                }
                __syncthreads();
            } else {
                // stage 3: phi at every face of the tile, inverted with the face
                // coefficients (eq. phibar)
#pragma unroll
                for (int k = 0; k < G::NRF; ++k) {
                    int j = tid + k * WG;
                    if (j >= G::NFT) continue;
                    double gF = 0.0, bF = 0.0;
                    if (fidx[k] >= 0) {
                        double vg, vb2;
                        face_pair<D, G>(sqp, sap, fd[k], fql[k], fal[k], fqr[k], far_[k], v, vg, vb2);
                        if constexpr (CACHE_FACE) {
                            FaceCoef<D> f;
                            f.fetch(sm.fc, j, G::NFT);
                            f.invert(v, vg, vb2, gF, bF);
                        } else {
                            FaceCoef<D> f;
                            f.load(P.FP + (long long)fd[k] * NFP * P.NE + fidx[k], P.NE);
                            f.invert(v, vg, vb2, gF, bF);
                        }
                    }
                    sm.f[j] = gF;
                    sm.f[G::NFT + j] = bF;
                }
                __syncthreads();

                // stage 4: microflux and the phi update of the own cell
                if (own_inside) {
                    double Fg = 0.0, Fb = 0.0;
#pragma unroll
                    for (int d = 0; d < D; ++d) {
                        int jl, jr;
                        if (d == 0) {
                            jl = tx + (G::TX + 1) * (ty + G::TY * tz);
                            jr = jl + 1;
                        } else if (d == 1) {
                            jl = G::NF0 + tx + G::TX * (ty + (G::TY + 1) * tz);
                            jr = jl + G::TX;
                        } else {
                            jl = G::NF0 + G::NF1 + tx + G::TX * (ty + G::TY * tz);
                            jr = jl + G::TX * G::TY;
                        }
                        double sxd = v.xi[d] * P.inv_dx[d];
                        Fg += sxd * (sm.f[jr] - sm.f[jl]);
                        Fb += sxd * (sm.f[G::NFT + jr] - sm.f[G::NFT + jl]);
                    }
                    const double g = own_g, b = own_b, geq0 = own_geq;
                    double c21 = 0.0, xu0 = 0.0;
#pragma unroll
                    for (int d = 0; d < D; ++d) {
                        double x1 = v.xi[d] - k1.u[d];
                        c21 += x1 * x1;
                        xu0 += v.xi[d] * k0.u[d];
                    }
                    double beq0 = (v.hx2 + k0.cRT2) * geq0;
                    double geq1 = k1.A * exp(-c21 * k1.inv2RT);
                    double beq1 = (v.hx2 + k1.cRT2) * geq1;
                    double Z0 = xu0 - k0.hu2;
                    const double dt = P.dt;
                    // eq. phiupdate with dt/(2 tau) = 2 beta and dt S_b = 4 eta Z (g - g_eq)
                    double gn = (g + 2.0 * k1.beta * geq1 + 2.0 * k0.beta * (geq0 - g) - dt * Fg) /
                                (1.0 + 2.0 * k1.beta);
                    double bn = (b + 2.0 * k1.betab * beq1 + 2.0 * k0.betab * (beq0 - b) - dt * Fb +
                                 4.0 * k0.eta * Z0 * (g - geq0)) /
                                (1.0 + 2.0 * k1.betab);
                    st<ST>(P.g_out, vb + own, gn);
                    st<ST>(P.b_out, vb + own, bn);
                }
                // q and a are rewritten by the next velocity only after every
                // thread has passed this velocity's third barrier, the face buffer
                // after the next velocity's second
            }
        }

        if constexpr (!UPD) {
            // partial face sums of this velocity slice
            const long long NE = P.NE;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                int cc[3] = {gx, gy, gz};
                bool valid = true;
#pragma unroll
                for (int e = 0; e < D; ++e) {
                    if (e == d) valid &= cc[e] < P.ne[e];
                    else valid &= cc[e] < P.n[e];
                }
                if (!valid) continue;
                long long fe = cc[0] + (long long)P.ne[0] * (cc[1] + (long long)P.ne[1] * cc[2]);
                double* out = P.FS + ((long long)(slice * D + d) * NS) * NE + fe;
#pragma unroll
                for (int j = 0; j < NS; ++j) out[(long long)j * NE] = acc[d][j];
            }
        }
    }
};

template <int D, typename ST, bool UPD>
__global__ __launch_bounds__(WG) void k_tile(Problem P) {
    using TK = TileKernel<D, ST, UPD>;
    __shared__ typename TK::Smem sm;
    const int* tiles = UPD ? P.tiles2 : P.tiles1;
    int ntiles = tiles[0] * tiles[1] * tiles[2];
    int q = xcd_remap(blockIdx.x, gridDim.x);
    int tile = q % ntiles, slice = q / ntiles;
    TK::run(P, tile, slice, UPD ? P.nslices_upd : P.nslices, sm);
}

template <int D, typename ST, bool UPD>
__global__ __launch_bounds__(WG) void k_tile_batched(const Problem* probs, const WorkItem* items) {
    using TK = TileKernel<D, ST, UPD>;
    __shared__ typename TK::Smem sm;
    const WorkItem it = items[xcd_remap(blockIdx.x, gridDim.x)];
    const Problem P = probs[it.prob];
    TK::run(P, it.tile, it.slice, UPD ? P.nslices_upd : P.nslices, sm);
}

// ---------------------------------------------------------------------------
// face closure: W_f, coefficients, flux moments (one thread per (d, face))
// ---------------------------------------------------------------------------
__device__ void face_close_one(const Problem& P, long long idx) {
    const int D = P.D;
    const long long NE = P.NE;
    if (idx >= NE * D) return;
    const int d = (int)(idx / NE);
    const long long f = idx - (long long)d * NE;
    long long r = f;
    int cc[3];
    for (int e = 0; e < 3; ++e) {
        cc[e] = (int)(r % P.ne[e]);
        r /= P.ne[e];
    }
    for (int e = 0; e < D; ++e)
        if (e != d && cc[e] >= P.n[e]) return;
    if (P.bc[d] == 0 && cc[d] >= P.n[d]) return;

    const int NS = 2 * D + 3;
    double S[MAX_NSUM];
    for (int j = 0; j < NS; ++j) S[j] = 0.0;
    for (int s = 0; s < P.nslices; ++s) {
        const double* in = P.FS + ((long long)(s * D + d) * NS) * NE + f;
        for (int j = 0; j < NS; ++j) S[j] += in[(long long)j * NE];
    }
    double Wf[5] = {S[0], S[1], D >= 2 ? S[2] : 0.0, D >= 3 ? S[3] : 0.0, 0.0};
    Wf[D + 1] = S[D + 1];
    Prim q = primitives(P, Wf);
    if (q.bad) {
        raise_error(P.err);
        return;
    }
    const double beta = 0.25 * P.dt * q.inv_tau_g;
    const double betab = beta * P.Pr;
    const double eta = beta * (P.Pr - 1.0);
    const double A = maxwell_prefactor(P, q.rho, q.RT);
    const double inv2RT = 0.5 / q.RT;
    const double hu2 = 0.5 * (q.u[0] * q.u[0] + q.u[1] * q.u[1] + q.u[2] * q.u[2]);
    const double cRT2 = 0.5 * P.c_int * q.RT;

    // separable discrete moments of the face Maxwellian: M[k][p] = sum_m w_m xi_m^p E_k(m)
    double M[3][4];
    int off = 0;
    for (int k = 0; k < 3; ++k) {
        for (int p = 0; p < 4; ++p) M[k][p] = 0.0;
        if (k >= D) {
            M[k][0] = 1.0;
            continue;
        }
        for (int m = 0; m < P.nv[k]; ++m) {
            double x = P.axis_xi[off + m];
            double e = P.axis_w[off + m] * exp(-(x - q.u[k]) * (x - q.u[k]) * inv2RT);
            M[k][0] += e;
            M[k][1] += e * x;
            M[k][2] += e * x * x;
            M[k][3] += e * x * x * x;
        }
        off += P.nv[k];
    }
    auto prod0 = [&](int skip1, int skip2) {
        double p = 1.0;
        for (int k = 0; k < D; ++k)
            if (k != skip1 && k != skip2) p *= M[k][0];
        return p;
    };
    // equilibrium flux moments through a face with normal d
    double E1 = A * M[d][1] * prod0(d, -1);
    double E2[3];
    for (int e = 0; e < D; ++e)
        E2[e] = e == d ? A * M[d][2] * prod0(d, -1) : A * M[d][1] * M[e][1] * prod0(d, e);
    double X3 = M[d][3] * prod0(d, -1);
    for (int e = 0; e < D; ++e)
        if (e != d) X3 += M[d][1] * M[e][2] * prod0(d, e);
    X3 *= A;
    double E3 = 0.5 * X3 + cRT2 * E1;
    double EZ = -hu2 * E1;
    for (int e = 0; e < D; ++e) EZ += q.u[e] * E2[e];

    // phi at the face is affine in phi_bar (inversion of eq. phibar), so the
    // flux moments follow from the velocity sums of phi_bar and the
    // equilibrium moments above.
    const double ig = 1.0 / (1.0 + beta), ib = 1.0 / (1.0 + betab);
    double Gm = (S[1 + d] + beta * E1) * ig;
    double Gp[3];
    double ZG = -hu2 * Gm;
    for (int e = 0; e < D; ++e) {
        Gp[e] = (S[D + 2 + e] + beta * E2[e]) * ig;
        ZG += q.u[e] * Gp[e];
    }
    double Ge = (S[2 * D + 2] + betab * E3 + eta * (ZG - EZ)) * ib;

    double* Go = P.G + (long long)d * (D + 2) * NE + f;
    Go[0] = Gm;
    for (int e = 0; e < D; ++e) Go[(long long)(1 + e) * NE] = Gp[e];
    Go[(long long)(D + 1) * NE] = Ge;

    double* F = P.FP + (long long)d * NFP * NE + f;
    F[PF_A * NE] = A;
    F[PF_INV2RT * NE] = inv2RT;
    F[PF_CRT2 * NE] = cRT2;
    F[PF_IG * NE] = ig;
    F[PF_BG * NE] = beta * ig;
    F[PF_IB * NE] = ib;
    F[PF_BB * NE] = betab * ib;
    F[PF_EB * NE] = eta * ib;
    F[PF_HU2 * NE] = hu2;
    for (int e = 0; e < 3; ++e) F[(PF_U0 + e) * NE] = q.u[e];
}

__global__ __launch_bounds__(WG) void k_face_close(Problem P) {
    face_close_one(P, (long long)blockIdx.x * WG + threadIdx.x);
}

// ---------------------------------------------------------------------------
// cell closure: W^{n+1} = W^n - dt sum_d (G_right - G_left)/dx_d; coefs at n+1
// ---------------------------------------------------------------------------
__device__ void cell_close_one(const Problem& P, long long c) {
    if (c >= P.N) return;
    const int D = P.D;
    const long long N = P.N, NE = P.NE;
    long long r = c;
    int cc[3];
    for (int e = 0; e < 3; ++e) {
        cc[e] = (int)(r % P.n[e]);
        r /= P.n[e];
    }
    long long fl = cc[0] + (long long)P.ne[0] * (cc[1] + (long long)P.ne[1] * cc[2]);
    double Wn[5];
    for (int k = 0; k < D + 2; ++k) Wn[k] = P.W_in[k * N + c];
    for (int d = 0; d < D; ++d) {
        int rc[3] = {cc[0], cc[1], cc[2]};
        rc[d] += 1;
        if (P.bc[d] == 0 && rc[d] == P.n[d]) rc[d] = 0;
        long long fr = rc[0] + (long long)P.ne[0] * (rc[1] + (long long)P.ne[1] * rc[2]);
        const double* Gd = P.G + (long long)d * (D + 2) * NE;
        for (int k = 0; k < D + 2; ++k)
            Wn[k] -= P.dt * P.inv_dx[d] * (Gd[k * NE + fr] - Gd[k * NE + fl]);
    }
    for (int k = 0; k < D + 2; ++k) P.W_out[k * N + c] = Wn[k];
    Prim q = primitives(P, Wn);
    if (q.bad) raise_error(P.err);
    write_cell_coefs(P, P.P_out, N, c, q);
}

__global__ __launch_bounds__(WG) void k_cell_close(Problem P) {
    cell_close_one(P, (long long)blockIdx.x * WG + threadIdx.x);
}

// per-problem thread ranges for the batched per-face / per-cell launches
__device__ __forceinline__ int find_problem(const long long* offsets, int nprob, long long g) {
    int lo = 0, hi = nprob - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) / 2;
        if (offsets[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(WG) void k_face_close_batched(const Problem* probs, const long long* offsets,
                                                           int nprob, long long total) {
    long long g = (long long)blockIdx.x * WG + threadIdx.x;
    if (g >= total) return;
    int p = find_problem(offsets, nprob, g);
    const Problem P = probs[p];
    face_close_one(P, g - offsets[p]);
}

__global__ __launch_bounds__(WG) void k_cell_close_batched(const Problem* probs, const long long* offsets,
                                                           int nprob, long long total) {
    long long g = (long long)blockIdx.x * WG + threadIdx.x;
    if (g >= total) return;
    int p = find_problem(offsets, nprob, g);
    const Problem P = probs[p];
    cell_close_one(P, g - offsets[p]);
}

// ---------------------------------------------------------------------------
// moments out and FP64 copies
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(WG) void k_moments(Problem P, const double* W, double* rho, double* u,
                                                double* T) {
    long long c = (long long)blockIdx.x * WG + threadIdx.x;
    if (c >= P.N) return;
    const int D = P.D;
    const long long N = P.N;
    double Wv[5];
    for (int k = 0; k < D + 2; ++k) Wv[k] = W[k * N + c];
    double r = Wv[0], u2 = 0.0;
    for (int d = 0; d < D; ++d) {
        double ud = Wv[1 + d] / r;
        u[d * N + c] = ud;
        u2 += ud * ud;
    }
    rho[c] = r;
    T[c] = (P.gamma - 1.0) / P.R * (Wv[D + 1] / r - 0.5 * u2);
}

template <typename ST>
__global__ __launch_bounds__(WG) void k_to_f64(long long n, const void* src, double* dst) {
    long long i = (long long)blockIdx.x * WG + threadIdx.x;
    if (i < n) dst[i] = ld<ST>(src, i);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(long long n) { return (unsigned)((n + WG - 1) / WG); }

hipError_t launch_init(const Problem& P, const double* rho, const double* u, const double* T,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_init_cells, dim3(blocks_for(P.N)), dim3(WG), 0, s, P, rho, u, T);
    if (P.storage == 0)
        hipLaunchKernelGGL(k_init_phi<double>, dim3(blocks_for(P.N * P.V)), dim3(WG), 0, s, P);
    else
        hipLaunchKernelGGL(k_init_phi<float>, dim3(blocks_for(P.N * P.V)), dim3(WG), 0, s, P);
    return hipGetLastError();
}

template <bool UPD>
static hipError_t launch_tile(const Problem& P, hipStream_t s) {
    const int* tl = UPD ? P.tiles2 : P.tiles1;
    unsigned nb = (unsigned)(tl[0] * tl[1] * tl[2] * (UPD ? P.nslices_upd : P.nslices));
#define CDG_TILE(DD, TT) hipLaunchKernelGGL((k_tile<DD, TT, UPD>), dim3(nb), dim3(WG), 0, s, P)
    if (P.storage == 0) {
        if (P.D == 1) CDG_TILE(1, double);
        else if (P.D == 2) CDG_TILE(2, double);
        else CDG_TILE(3, double);
    } else {
        if (P.D == 1) CDG_TILE(1, float);
        else if (P.D == 2) CDG_TILE(2, float);
        else CDG_TILE(3, float);
    }
#undef CDG_TILE
    return hipGetLastError();
}

template <bool UPD>
static int blocks_per_cu(int D, int storage) {
    int n = 0;
    hipError_t e;
#define CDG_OCC(DD, TT) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (k_tile<DD, TT, UPD>), WG, 0)
    if (storage == 0) {
        if (D == 1) CDG_OCC(1, double);
        else if (D == 2) CDG_OCC(2, double);
        else CDG_OCC(3, double);
    } else {
        if (D == 1) CDG_OCC(1, float);
        else if (D == 2) CDG_OCC(2, float);
        else CDG_OCC(3, float);
    }
#undef CDG_OCC
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return n;
}

int tile_blocks_per_cu(int D, int storage, bool update) {
    return update ? blocks_per_cu<true>(D, storage) : blocks_per_cu<false>(D, storage);
}

hipError_t launch_face_sums(const Problem& P, hipStream_t s) { return launch_tile<false>(P, s); }
hipError_t launch_update(const Problem& P, hipStream_t s) { return launch_tile<true>(P, s); }

hipError_t launch_face_close(const Problem& P, hipStream_t s) {
    hipLaunchKernelGGL(k_face_close, dim3(blocks_for(P.NE * P.D)), dim3(WG), 0, s, P);
    return hipGetLastError();
}

hipError_t launch_cell_close(const Problem& P, hipStream_t s) {
    hipLaunchKernelGGL(k_cell_close, dim3(blocks_for(P.N)), dim3(WG), 0, s, P);
    return hipGetLastError();
}

hipError_t launch_moments(const Problem& P, const double* W, double* rho, double* u, double* T,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_moments, dim3(blocks_for(P.N)), dim3(WG), 0, s, P, W, rho, u, T);
    return hipGetLastError();
}

hipError_t launch_to_f64(const Problem& P, const void* src, double* dst, hipStream_t s) {
    long long n = P.N * P.V;
    if (P.storage == 0)
        hipLaunchKernelGGL(k_to_f64<double>, dim3(blocks_for(n)), dim3(WG), 0, s, n, src, dst);
    else
        hipLaunchKernelGGL(k_to_f64<float>, dim3(blocks_for(n)), dim3(WG), 0, s, n, src, dst);
    return hipGetLastError();
}

template <bool UPD>
static hipError_t launch_tile_batched(const Problem* probs, const WorkItem* items, int nitems, int dim,
                                      int storage, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
#define CDG_TILEB(DD, TT) hipLaunchKernelGGL((k_tile_batched<DD, TT, UPD>), dim3(nitems), dim3(WG), 0, s, probs, items)
    if (storage == 0) {
        if (dim == 1) CDG_TILEB(1, double);
        else if (dim == 2) CDG_TILEB(2, double);
        else CDG_TILEB(3, double);
    } else {
        if (dim == 1) CDG_TILEB(1, float);
        else if (dim == 2) CDG_TILEB(2, float);
        else CDG_TILEB(3, float);
    }
#undef CDG_TILEB
    return hipGetLastError();
}

hipError_t launch_face_sums_batched(const Problem* probs, const WorkItem* items, int nitems, int dim,
                                    int storage, hipStream_t s) {
    return launch_tile_batched<false>(probs, items, nitems, dim, storage, s);
}
hipError_t launch_update_batched(const Problem* probs, const WorkItem* items, int nitems, int dim,
                                 int storage, hipStream_t s) {
    return launch_tile_batched<true>(probs, items, nitems, dim, storage, s);
}
hipError_t launch_face_close_batched(const Problem* probs, const long long* offsets, int nprob,
                                     long long total, hipStream_t s) {
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_face_close_batched, dim3(blocks_for(total)), dim3(WG), 0, s, probs, offsets, nprob,
                       total);
    return hipGetLastError();
}
hipError_t launch_cell_close_batched(const Problem* probs, const long long* offsets, int nprob,
                                     long long total, hipStream_t s) {
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cell_close_batched, dim3(blocks_for(total)), dim3(WG), 0, s, probs, offsets, nprob,
                       total);
    return hipGetLastError();
}

}  // namespace cdg
