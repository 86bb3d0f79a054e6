// Device-side building blocks of the CDUGKS kernels (included by every
// kernel translation unit): storage access, primitives, the face-sum and
// update kernel bodies, and the per-face / per-cell closures.  The data
// layout and the structure of a step are described in cdugks_kernels.hip.
#pragma once

#include "cdugks_internal.h"

#include <math.h>

#include <type_traits>

namespace cdg {

__device__ __forceinline__ int map_coord(int x, int n, int bc) {
    if (bc == 0) {
        int r = x % n;
        return r < 0 ? r + n : r;
    }
    return x < 0 ? 0 : (x >= n ? n - 1 : x);
}

// Reciprocal from the hardware estimate (relative error below 1e-7) refined
// by one Newton-Raphson step, which squares the error to about 2e-15.  Used
// where the operand is a nonzero finite sum.
__device__ __forceinline__ double rcp_nr(double s) {
    const double r = __builtin_amdgcn_rcp(s);
    return fma(r, fma(-s, r, 1.0), r);
}

// Van Leer limiter (eq. VanLeer) at half scale: H(a, b) = ab/(a + b) when
// ab > 0, else 0, which is half the harmonic-mean form 2ab/(a+b) =
// (sgn a + sgn b)|a||b|/(|a|+|b|): zero at extrema and for a flat side.  The
// kernels carry every limited slope at half scale (and slopes of slopes at a
// quarter), folding the factors into the Courant numbers; all the scalings
// are powers of two, so the values are those of the full-scale form exactly
// (except where a product is subnormal, as in the far velocity tails of the
// FP32 form).
// When ab > 0 the sum a + b is nonzero, so the reciprocal is safe; otherwise
// its value is discarded by the select.
__device__ __forceinline__ double half_van_leer(double a, double b) {
    double p = a * b;
    double v = p * rcp_nr(a + b);
    return p > 0.0 ? v : 0.0;
}

// FP32 form for the FP32-storage stencil: the hardware reciprocal alone
// (within 1 ulp), so the limited slope is within about 2 ulp of the rounded
// quotient, below the rounding of the FP32 values it is built from and
// stored as.
__device__ __forceinline__ float half_van_leer(float a, float b) {
    float p = a * b;
    float v = p * __builtin_amdgcn_rcpf(a + b);
    return p > 0.0f ? v : 0.0f;
}

template <typename ST>
__device__ __forceinline__ double ld(const void* base, long long idx) {
    return (double)reinterpret_cast<const ST*>(base)[idx];
}
template <typename ST>
__device__ __forceinline__ void st(void* base, long long idx, double v) {
    reinterpret_cast<ST*>(base)[idx] = (ST)v;
}

// Streaming store for data the writing kernel never reads again (face values,
// the new distributions): marked non-temporal so it does not push the halo
// lines that neighbouring workgroups still need out of L2.
template <typename ST>
__device__ __forceinline__ void st_stream(void* base, long long idx, double v) {
    __builtin_nontemporal_store((ST)v, reinterpret_cast<ST*>(base) + idx);
}

__device__ __forceinline__ void raise_error(int* err) { *err = 1; }

// ---------------------------------------------------------------------------
// storage forms of the distributions g, b (and of the 3-D quarter-step fields)
// ---------------------------------------------------------------------------
// double, float: every velocity row [N] in that precision.
// Bf16Tail: the FP32 form, except that the rows of the far velocity tails
// (fixed at set-up) hold BF16.  P.rows[i] is the byte offset of row i inside
// each state array, with bit 0 set for a BF16 row.  The stencil arithmetic
// and the stored face values are FP32 as in the FP32 form.  Values are
// rounded to FP32 and then, in a BF16 row, to BF16 (round to nearest even).
struct Bf16Tail {};

template <typename ST>
struct StoreT {
    using C = ST;  // stencil arithmetic and stored face values
    using R = ST;  // a loaded state value, as held in registers until used
    static constexpr bool MIXED = false;
};
template <>
struct StoreT<Bf16Tail> {
    using C = float;
    using R = unsigned;  // raw bits: the FP32 word, or the BF16 half zero-extended
    static constexpr bool MIXED = true;
};

// row word of velocity i (uniform: a scalar load)
__device__ __forceinline__ long long row_word(const Problem& P, int i) {
    return ((const __attribute__((address_space(4))) long long*)(const void*)P.rows)[i];
}

// state value at (velocity i, cell c), raw until state_value converts it
template <typename ST>
__device__ __forceinline__ typename StoreT<ST>::R state_load(const Problem& P, const void* base, int i,
                                                            long long c) {
    if constexpr (StoreT<ST>::MIXED) {
        const long long o = row_word(P, i);
        const char* row = (const char*)base + (o & ~1LL);
        if (o & 1) return (unsigned)((const unsigned short*)row)[c];
        return ((const unsigned*)row)[c];
    } else {
        return ((const ST*)base)[(long long)i * P.pitch + c];
    }
}
template <typename ST>
__device__ __forceinline__ double state_value(const Problem& P, int i, typename StoreT<ST>::R r) {
    if constexpr (StoreT<ST>::MIXED) {
        return (double)__uint_as_float((row_word(P, i) & 1) ? r << 16 : r);
    } else {
        return (double)r;
    }
}
template <typename ST>
__device__ __forceinline__ double state_ld(const Problem& P, const void* base, int i, long long c) {
    return state_value<ST>(P, i, state_load<ST>(P, base, i, c));
}
template <typename ST, bool STREAM>
__device__ __forceinline__ void state_st(const Problem& P, void* base, int i, long long c, double v) {
    if constexpr (StoreT<ST>::MIXED) {
        const long long o = row_word(P, i);
        char* row = (char*)base + (o & ~1LL);
        const float f = (float)v;
        if (o & 1) {
            const unsigned short h = __builtin_bit_cast(unsigned short, (__bf16)f);
            if constexpr (STREAM) __builtin_nontemporal_store(h, (unsigned short*)row + c);
            else ((unsigned short*)row)[c] = h;
        } else {
            if constexpr (STREAM) __builtin_nontemporal_store(f, (float*)row + c);
            else ((float*)row)[c] = f;
        }
    } else {
        if constexpr (STREAM) st_stream<ST>(base, (long long)i * P.pitch + c, v);
        else st<ST>(base, (long long)i * P.pitch + c, v);
    }
}

// The fields of velocity i at NS source cells of one thread, raw until
// slot_value.  The BF16-tail form has two ways to read a row whose kind is
// uniform per velocity:
//  WORDS: one 32-bit load per slot whatever the row's kind (element c of a
//    BF16 row is a half of word c/2, which slot_value takes out), so no branch
//    on the row kind stands between these loads and the values that use them
//    (at a branch's join the compiler waits for every load in flight).  The
//    word of a BF16 row's last element reaches past the row's 2N bytes only
//    for an odd N, into the padding that rounds the row to 256 bytes.  For
//    loops over velocities.
//  !WORDS: 16-bit loads under a branch on the row kind (the value in the low
//    half, as for an even cell), for a velocity fixed over the loop.
template <typename ST, int NS, bool WORDS = true>
__device__ __forceinline__ void load_slots(const Problem& P, const void* sg, const void* sb, int i,
                                           const long long (&src)[NS], typename StoreT<ST>::R (&og)[NS],
                                           typename StoreT<ST>::R (&ob)[NS]) {
    if constexpr (StoreT<ST>::MIXED && WORDS) {
        const long long o = row_word(P, i);
        const int h = (int)(o & 1);
        const unsigned* rg = (const unsigned*)((const char*)sg + (o & ~1LL));
        const unsigned* rb = (const unsigned*)((const char*)sb + (o & ~1LL));
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            const long long w = src[k] >> h;
            og[k] = rg[w];
            ob[k] = rb[w];
        }
    } else if constexpr (StoreT<ST>::MIXED) {
        const long long o = row_word(P, i);
        const char* rg = (const char*)sg + (o & ~1LL);
        const char* rb = (const char*)sb + (o & ~1LL);
        if (o & 1) {
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                og[k] = ((const unsigned short*)rg)[src[k]];
                ob[k] = ((const unsigned short*)rb)[src[k]];
            }
        } else {
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                og[k] = ((const unsigned*)rg)[src[k]];
                ob[k] = ((const unsigned*)rb)[src[k]];
            }
        }
    } else {
        // the row's base address is uniform (scalar) and the cell offsets
        // are loop-invariant, so each load is a scalar base plus a fixed
        // vector offset
        const ST* const rg = (const ST*)sg + (long long)i * P.pitch;
        const ST* const rb = (const ST*)sb + (long long)i * P.pitch;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            og[k] = rg[src[k]];
            ob[k] = rb[src[k]];
        }
    }
}
// value of a raw slot of cell c: in a BF16 row (half, uniform) a word loaded
// by WORDS holds cells c and c ^ 1, the odd cell in the upper half; a 16-bit
// load is passed as an even cell
template <typename ST>
__device__ __forceinline__ double slot_value(typename StoreT<ST>::R r, bool half, long long c) {
    if constexpr (StoreT<ST>::MIXED) {
        const unsigned bits = half ? ((c & 1) ? (r & 0xFFFF0000u) : (r << 16)) : r;
        return (double)__uint_as_float(bits);
    } else {
        return (double)r;
    }
}

// Access within one velocity row of the update kernel, whose element kind is
// known at compile time: double or float rows, or the BF16 rows of the
// BF16-tail form (Bf16Row).  `off` is the row's byte offset in the array.
// Stores are non-temporal (the kernel never reads them back); round() gives
// the value as it will be stored.
struct Bf16Row {};
template <typename E>
struct RowIO {
    using Raw = E;  // a loaded element, as held until used
    __device__ static Raw raw(const void* base, long long off, long long c) {
        return ((const E*)((const char*)base + off))[c];
    }
    __device__ static double val(Raw r) { return (double)r; }
    __device__ static double ld(const void* base, long long off, long long c) {
        return (double)((const E*)((const char*)base + off))[c];
    }
    __device__ static void st(void* base, long long off, long long c, double v) {
        __builtin_nontemporal_store((E)v, (E*)((char*)base + off) + c);
    }
    __device__ static double round(double v) { return (double)(E)v; }
};
template <>
struct RowIO<Bf16Row> {
    using Raw = __bf16;
    __device__ static Raw raw(const void* base, long long off, long long c) {
        return ((const __bf16*)((const char*)base + off))[c];
    }
    __device__ static double val(Raw r) { return (double)(float)r; }
    __device__ static double ld(const void* base, long long off, long long c) {
        return (double)(float)((const __bf16*)((const char*)base + off))[c];
    }
    __device__ static void st(void* base, long long off, long long c, double v) {
        const unsigned short h = __builtin_bit_cast(unsigned short, (__bf16)(float)v);
        __builtin_nontemporal_store(h, (unsigned short*)((char*)base + off) + c);
    }
    __device__ static double round(double v) { return (double)(float)(__bf16)(float)v; }
};

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
// tile kernels
// ---------------------------------------------------------------------------
// XCD-aware order: consecutive workgroup ids are spread over the 8 XCDs, so
// give each XCD a contiguous block of the (tile, slice) space; neighbouring
// tiles then share halo lines in that XCD's L2.
__device__ __forceinline__ int xcd_remap(int lin, int total) {
    int per = total / 8;
    if (lin >= per * 8) return lin;
    return (lin % 8) * per + lin / 8;
}

// Box geometry of the staged halo for a face-sum tile: the q box covers tile
// offsets [-3, T+1], the limited-difference box [-2, T].  (The left face of
// cell c along d needs the upwind cell c-d or c, its slopes at the upwind
// cell +-1 along d, and those need q one further out.)
template <int D, int TID>
struct Geo {
    static constexpr TileExt T = tile_shape(D, TID);
    static constexpr int TX = T.x, TY = T.y, TZ = T.z;
    static constexpr int NT = TX * TY * TZ;  // threads of a workgroup, one per cell
    static constexpr int QX = TX + 5;
    static constexpr int QY = D >= 2 ? TY + 5 : 1;
    static constexpr int QZ = D >= 3 ? TZ + 5 : 1;
    static constexpr int AX = TX + 3;
    static constexpr int AY = D >= 2 ? TY + 3 : 1;
    static constexpr int AZ = D >= 3 ? TZ + 3 : 1;
    static constexpr int NQ = QX * QY * QZ;
    static constexpr int NA = AX * AY * AZ;
    static constexpr int NRA = (NA + NT - 1) / NT;   // slope points per thread
    static constexpr bool CACHE_COEF = (NQ - NT + NT - 1) / NT + 1 <= 2;
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
    double xi[3], w, hx2, lam2[3], ax;
};

// The velocity table is read-only for the whole launch: reading it through the
// constant address space makes the per-velocity loads scalar (SMEM), so they
// neither occupy vector-memory slots nor delay waits on the field loads.
typedef const __attribute__((address_space(4))) double* const_dptr;

__device__ __forceinline__ const_dptr vel_ptr(const double* vel, int i) {
    return (const_dptr)(const void*)(vel + (long long)i * NVEL);
}

__device__ __forceinline__ Vel load_vel(const double* vel, int i) {
    const_dptr v = vel_ptr(vel, i);
    Vel r;
    r.xi[0] = v[0]; r.xi[1] = v[1]; r.xi[2] = v[2];
    r.w = v[VE_W]; r.hx2 = v[VE_HX2]; r.ax = v[VE_AX];
    r.lam2[0] = v[VE_LAM0]; r.lam2[1] = v[VE_LAM0 + 1]; r.lam2[2] = v[VE_LAM0 + 2];
    return r;
}

// Z and the quarter-step fields at one (cell, velocity), given g_eq:
// phi_bar_plus = phi + (h/2)(phi_eq - phi)/tau + (h/2) S (eq. phibarplus),
// S_b = Z (g - g_eq)/tau_bg + ... .  ACC adds the external acceleration's
// terms of the sources (eqs. gsource, bsource) with the velocity derivative
// taken on the equilibrium: S_g = a.(xi - u)/(R T) g_eq and, in S_b,
// a.xi (g - g_eq) + a.(xi - u)/(R T) b_eq; (h/2)/(R T) = (dt/2)/(2 R T).
template <int D, bool ACC = false>
__device__ __forceinline__ void quarter_step_eq(const CellCoef& k, const Vel& v, double geq, double g, double b,
                                                double& qg, double& qb, const Problem* P = nullptr) {
    double xu = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) xu += v.xi[d] * k.u[d];
    double beq = (v.hx2 + k.cRT2) * geq;
    double Z = xu - k.hu2;
    qg = g + k.beta * (geq - g);
    qb = b + k.betab * (beq - b) + k.eta * Z * (g - geq);
    if constexpr (ACC) {
        double au = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) au += P->accel[d] * k.u[d];
        const double c = 0.5 * P->dt * k.inv2RT * (v.ax - au);
        qg += c * geq;
        qb += 0.25 * P->dt * v.ax * (g - geq) + c * beq;
    }
}

// Value of phi_bar at a face centre at t_{n+1/2} from the upwind cell u,
// side s = +1 when the face is u's right face, -1 when its left face:
//   v = q(u) + s a_d/2 - sum_e lambda_e (a_e + s b_de/2),
// a_e = VL of one-sided differences of q along e (slope times dx_e) and
// b_de = VL of differences of a_e along d (slope of the slope times dx_d dx_e).
// Arguments at the scales the kernels carry: ha = a/2 at u (haU) and at
// u - d (haL), u + d (haR); lam2 = 2 lambda.  Then
//   v = q(u) + s ha_d - sum_e lam2_e (ha_e + s hb_de),  hb_de = b_de/4 = H(ha differences).
template <int D, typename CT>
__device__ __forceinline__ CT face_value_at(CT qU, const CT* haU, const CT* haL, const CT* haR, int d, CT s,
                                            const Vel& v) {
    CT val = qU + s * haU[d];
#pragma unroll
    for (int e = 0; e < D; ++e) {
        CT hb = half_van_leer(haU[e] - haL[e], haR[e] - haU[e]);
        val -= CT(v.lam2[e]) * (haU[e] + s * hb);
    }
    return val;
}

// The single-slope option: the upwind cell's own slopes carried to the foot,
// v = q(u) + s ha_d - sum_e lam2_e ha_e (no slopes of slopes).
template <int D, typename CT>
__device__ __forceinline__ CT face_value_single(CT qU, const CT* haU, int d, CT s, const Vel& v) {
    CT val = qU + s * haU[d];
#pragma unroll
    for (int e = 0; e < D; ++e) val -= CT(v.lam2[e]) * haU[e];
    return val;
}

// Face coefficients used to invert eq. phibar at a face.  The inversion
// g = ig gbar + bg g_eq with bg = 1 - ig is evaluated as g_eq + ig (gbar -
// g_eq) (likewise b with ib), so bg and bb need no registers.
template <int D>
struct FaceCoef {
    double A, inv2RT, cRT2, ig, ib, eb, hu2, u[D];
    __device__ void load(const double* F, long long NE) {
        A = F[PF_A * NE];
        inv2RT = F[PF_INV2RT * NE];
        cRT2 = F[PF_CRT2 * NE];
        ig = F[PF_IG * NE];
        ib = F[PF_IB * NE];
        eb = F[PF_EB * NE];
        hu2 = F[PF_HU2 * NE];
#pragma unroll
        for (int e = 0; e < D; ++e) u[e] = F[(PF_U0 + e) * NE];
    }
    // Z = xi.u - |u|^2/2 at the face
    __device__ __forceinline__ double z(const Vel& v) const {
        double xu = 0.0;
#pragma unroll
        for (int e = 0; e < D; ++e) xu += v.xi[e] * u[e];
        return xu - hu2;
    }
    // phi at the face from phi_bar (eq. phibar inverted): g first, then b with
    // the S_b source at the face evaluated with the face g.
    __device__ __forceinline__ void invert(const Vel& v, double geq, double vg, double vb, double& gF,
                                           double& bF) const {
        invert_z(v, geq, z(v), vg, vb, gF, bF);
    }
    __device__ __forceinline__ void invert_z(const Vel& v, double geq, double Z, double vg, double vb, double& gF,
                                             double& bF) const {
        double beq = (v.hx2 + cRT2) * geq;
        gF = geq + ig * (vg - geq);
        bF = beq + ib * (vb - beq) + eb * Z * (gF - geq);
    }
    // The same with an external acceleration a: the face's (h/2) S terms
    // (eqs. gsource, bsource, velocity derivative on the equilibrium), with
    // au = a.u_f and c2 = (dt/2)/(2 R T_f) prepared once per face.
    double au, c2;
    __device__ void prepare_accel(const double* a, double dt) {
        au = 0.0;
#pragma unroll
        for (int e = 0; e < D; ++e) au += a[e] * u[e];
        c2 = 0.5 * dt * inv2RT;
    }
    __device__ __forceinline__ void invert_accel(const Vel& v, double dt, double geq, double vg, double vb,
                                                 double& gF, double& bF) const {
        invert_accel_z(v, dt, geq, z(v), vg, vb, gF, bF);
    }
    __device__ __forceinline__ void invert_accel_z(const Vel& v, double dt, double geq, double Z, double vg,
                                                   double vb, double& gF, double& bF) const {
        double beq = (v.hx2 + cRT2) * geq;
        const double c = c2 * (v.ax - au);
        gF = geq + ig * (vg - geq + c * geq);
        bF = beq + ib * (vb - beq + 0.25 * dt * v.ax * (gF - geq) + c * beq) + eb * Z * (gF - geq);
    }
};

// ---------------------------------------------------------------------------
// Maxwellian by recurrence along the fastest velocity axis.  The nodes of
// velocity axis 0 are uniform (spacing h); with x_k = xi_k - u_x, s = 1/(2RT)
// and everything else fixed,
//   g_eq(k+1) = g_eq(k) R_k,  R_k = exp(-(2 x_k + h) h s),  R_{k+1} = R_k C,
//   C = exp(-2 h^2 s).
// g_eq and R are set from direct exponentials at every WALK-th node of axis 0
// (anchors; a row of the velocity grid starts with one), which bounds the
// rounding drift of the products to about WALK^2 ulp.  A block whose
// exponents could leave the range where the products stay normal numbers
// uses direct exponentials throughout.  The value at a node depends only on
// the node, not on where a velocity slice starts: a slice starting inside a
// block walks from that block's anchor.
// ---------------------------------------------------------------------------
constexpr int WALK = 8;

template <int D>
__device__ __forceinline__ double maxwellian(double A, double s, const double* u, const Vel& v) {
    double c2 = 0.0;
#pragma unroll
    for (int e = 0; e < D; ++e) {
        const double x = v.xi[e] - u[e];
        c2 += x * x;
    }
    return A * exp(-c2 * s);
}

// The Maxwellian at FP32 accuracy, for the update kernel of the FP32 storage
// forms (whose stored values carry a relative rounding of 2^-24): the exponent
// is split in FP64 as -c2 s log2(e) = n + f with n an integer and |f| <= 1/2;
// 2^f is the hardware FP32 base-2 exponential (within 1 ulp) of f rounded to
// FP32 (an argument error below 2^-25), and 2^n is applied exactly.  The
// relative error is below 1e-7, against about 1e-16 for the FP64 exponential
// at a quarter of the instructions.  Exponents below -1500 give 0.
template <int D>
__device__ __forceinline__ double maxwellian_f32(double A, double s, const double* u, const Vel& v) {
    double c2 = 0.0;
#pragma unroll
    for (int e = 0; e < D; ++e) {
        const double x = v.xi[e] - u[e];
        c2 += x * x;
    }
    const double t = fmin(fmax(-c2 * s * M_LOG2E, -1500.0), 1500.0);
    const double n = rint(t);
    return A * ldexp((double)__builtin_amdgcn_exp2f((float)(t - n)), (int)n);
}
// The same from Z = xi.u - |u|^2/2, which the face inversion and the S_b
// source need anyway: |xi - u|^2 = 2 (|xi|^2/2 - Z), so the exponent takes one
// subtraction instead of D differences and squares.  The rounding of the
// expanded square (relative 1e-16 of |xi|^2 + |u|^2) stays far below the
// FP32 accuracy of the result.
__device__ __forceinline__ double maxwellian_f32z(double A, double s, double Z, double hx2) {
    const double t = fmin(fmax(2.0 * M_LOG2E * s * (Z - hx2), -1500.0), 1500.0);
    const double n = rint(t);
    return A * ldexp((double)__builtin_amdgcn_exp2f((float)(t - n)), (int)n);
}

struct GaussWalk {
    double E, R, C;
    bool ok;
    __device__ __forceinline__ void init(double s, double h) { C = exp(-2.0 * h * h * s); }
    // anchor at the current node (its axis-0 coordinate is v.xi[0])
    template <int D>
    __device__ __forceinline__ void anchor(double A, double s, const double* u, const Vel& v, double h) {
        const double x = v.xi[0] - u[0];
        E = maxwellian<D>(A, s, u, v);
        R = exp(-(x + x + h) * h * s);
        const double m = fmax(fabs(x), fabs(x + (WALK - 1) * h));
        ok = m * m * s < 600.0 && (m + m + h) * h * s < 600.0 && h * h * s < 300.0;
    }
    __device__ __forceinline__ void advance() {
        E *= R;
        R *= C;
    }
    template <int D>
    __device__ __forceinline__ double value(double A, double s, const double* u, const Vel& v) const {
        double geq = E;
        if (!ok) geq = maxwellian<D>(A, s, u, v);
        return geq;
    }
};

// ---------------------------------------------------------------------------
// face-sum kernel: for every velocity of the slice, phi_bar at the left face
// of each tile cell along each d (stored for the update kernel), and the
// velocity sums of the face (serial per thread, fixed order)
// ---------------------------------------------------------------------------
// DIR: the problem has Dirichlet sides; their ghost slots of the q box take
// the fixed states' equilibria (a separate instantiation keeps the register
// budget of the others unchanged).
// SS: the single-slope reconstruction option (stage 3 reads only the upwind
// cell's slopes).
// ACC: the problem has an external acceleration (stage 1 adds its source
// terms; the a = 0 instantiations keep their register budget).
template <int D, typename ST, bool DIR = false, bool SS = false, int TID = 0, bool ACC = false>
struct FaceSumKernel {
    using G = Geo<D, TID>;
    static constexpr int NT = G::NT;
    // every 2-D shape keeps the q-box slots and their Maxwellian recurrence
    // in registers (so the shape does not change a result)
    static_assert(D != 2 || G::CACHE_COEF, "2-D tile shapes must keep their q-box slots in registers");
    // stencil arithmetic (quarter-step values in LDS, limiters, face values) in
    // the storage precision; equilibria and the velocity sums stay FP64
    using CT = typename StoreT<ST>::C;
    using RT = typename StoreT<ST>::R;
    // q-box points per thread: slot 0 is the thread's own cell, the other
    // slots cover the halo
    static constexpr int NHALO = G::NQ - NT;
    static constexpr int NSLOT = 1 + (NHALO + NT - 1) / NT;

    // Box index of the h-th point of a box (extents BX, BY, BZ; the tile sits
    // at offsets OX, OY, OZ) that lies outside the tile, in box order: planes
    // below the tile in z are full, the tile's planes miss its TX x TY block,
    // and likewise rows within a plane.
    template <int BX, int BY, int OX, int OY, int OZ>
    __device__ static int ring_point(int h) {
        constexpr int PL = BX * BY;                 // points per full plane
        constexpr int PI = PL - G::TX * G::TY;      // ring points per tile plane
        constexpr int RI = BX - G::TX;              // ring points per tile row
        if (h < OZ * PL) return h;  // below the tile: box order equals ring order
        h -= OZ * PL;
        if (h >= G::TZ * PI) return (OZ + G::TZ) * PL + (h - G::TZ * PI);  // above
        const int z = OZ + h / PI;
        int rem = h % PI, y, x;
        if (rem < OY * BX) {
            y = rem / BX;
            x = rem % BX;
        } else {
            rem -= OY * BX;
            if (rem >= G::TY * RI) {
                rem -= G::TY * RI;
                y = OY + G::TY + rem / BX;
                x = rem % BX;
            } else {
                y = OY + rem / RI;
                const int c = rem % RI;
                x = c < OX ? c : c + G::TX;
            }
        }
        return x + BX * (y + BY * z);
    }
    __device__ static int halo_point(int h) { return ring_point<G::QX, G::QY, G::OQX, G::OQY, G::OQZ>(h); }
    __device__ static int slope_ring_point(int h) {
        return ring_point<G::AX, G::AY, G::OAX, G::OAY, G::OAZ>(h);
    }
    // slope-box points outside the tile, and passes over them
    static constexpr int NARING = G::NA - NT;
    static constexpr int NRING2 = (2 * NARING + NT - 1) / NT;  // (point, field) passes

    // With stored quarter-step fields (3-D) the q box is loaded; otherwise
    // it is computed from g, b and the cell coefficients of the q-box slots,
    // which every 1-D and 2-D shape keeps in registers.
    static constexpr bool QS = quarter_stored(D);
    static constexpr bool KQ = G::CACHE_COEF && !QS;
    static_assert(QS || KQ, "a tile shape must keep its q-box slot coefficients in registers");

    // 1-D and 2-D alternate two LDS buffers between consecutive velocities,
    // which removes the barrier that would otherwise end each velocity
    static constexpr int NBUF = D <= 2 ? 2 : 1;

    struct Smem {
        CT q[NBUF][2][G::NQ + 1];  // phi_bar_plus for g, b (entry NQ: unused slots)
        CT a[NBUF][2][D * G::NA];  // limited differences for g, b
    };

    __device__ static void run(const Problem& P, int tile, int slice, int nslices, Smem& sm) {
        const int tid = threadIdx.x;
        const long long N = P.N;
        int t = tile;
        const int ox = (t % P.tiles1[0]) * G::TX;
        t /= P.tiles1[0];
        const int oy = D >= 2 ? (t % P.tiles1[1]) * G::TY : 0;
        t /= P.tiles1[1];
        const int oz = D >= 3 ? t * G::TZ : 0;
        const int v0 = (int)((long long)P.V * slice / nslices);
        const int v1 = (int)((long long)P.V * (slice + 1) / nslices);

        // q-box points of this thread: slot 0 its own cell, then halo points
        // (halo enumerated in box order, interior skipped); source cell after
        // periodic wrap / outflow clamp
        // lq: box index in the low 20 bits; for a Dirichlet ghost, its side
        // 2 d + side plus one in the bits above (-1: unused slot)
        long long srcq[NSLOT];
        int lq[NSLOT];
        CellCoef kq[KQ ? NSLOT : 1];
        {
            int lx = tid % G::TX, ly = (tid / G::TX) % G::TY, lz = tid / (G::TX * G::TY);
            lq[0] = G::qidx(lx, ly, lz);
#pragma unroll
            for (int k = 1; k < NSLOT; ++k) {
                const int h = tid + (k - 1) * NT;  // halo ordinal
                lq[k] = h < NHALO ? halo_point(h) : -1;
            }
#pragma unroll
            for (int k = 0; k < NSLOT; ++k) {
                srcq[k] = 0;  // unused slots still load a valid address
                if (lq[k] < 0) continue;
                int r = lq[k];
                int rx = r % G::QX, ry = (r / G::QX) % G::QY, rz = r / (G::QX * G::QY);
                const int c3[3] = {ox + rx - G::OQX, oy + ry - G::OQY, oz + rz - G::OQZ};
                if constexpr (DIR) {
                    int side = 0;
#pragma unroll
                    for (int d = 0; d < D; ++d)
                        if (P.bc[d] == 2 && (c3[d] < 0 || c3[d] >= P.n[d])) side = 2 * d + (c3[d] >= P.n[d]) + 1;
                    lq[k] = r | (side << 20);
                }
                int cx = map_coord(c3[0], P.n[0], P.bc[0]);
                int cy = D >= 2 ? map_coord(c3[1], P.n[1], P.bc[1]) : 0;
                int cz = D >= 3 ? map_coord(c3[2], P.n[2], P.bc[2]) : 0;
                srcq[k] = cx + (long long)P.n[0] * (cy + (long long)P.n[1] * cz);
            }
            // every slot's coefficients, an unused slot's those of cell 0:
            // stage 1 evaluates each slot (its result unread for an unused one)
            if constexpr (KQ) {
#pragma unroll
                for (int k = 0; k < NSLOT; ++k) kq[k] = load_coef(P.P_in, N, srcq[k]);
            }
        }
        // own cell = the left faces this thread reconstructs
        const int tx = tid % G::TX, ty = (tid / G::TX) % G::TY, tz = tid / (G::TX * G::TY);
        const int gx = ox + tx, gy = oy + ty, gz = oz + tz;
        const long long NE = P.NE;
        long long fe = -1;  // extended-grid index of the own cell's left faces
        bool fvalid[D];
        {
            int cc[3] = {gx, gy, gz};
            bool any = false;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                bool ok = true;
#pragma unroll
                for (int e = 0; e < D; ++e) ok &= e == d ? cc[e] < P.ne[e] : cc[e] < P.n[e];
                fvalid[d] = ok;
                any |= ok;
            }
            if (any) fe = cc[0] + (long long)P.ne[0] * (cc[1] + (long long)P.ne[1] * cc[2]);
        }

        constexpr int NS = 2 * D + 3;
        double acc[D][NS];
#pragma unroll
        for (int d = 0; d < D; ++d)
#pragma unroll
            for (int j = 0; j < NS; ++j) acc[d][j] = 0.0;

        // Software pipelining: the next velocity's fields are loaded while the
        // current one is processed (when the q-box slots fit in registers).
        // The loop is unrolled by two over two named register sets, so a
        // register with a load in flight is never copied: a copy would make
        // the compiler wait for every outstanding memory operation, the face
        // value stores included.
        constexpr bool PREFETCH = NSLOT <= 2 || QS;
        const void* const src_g = QS ? P.qg : P.g_in;
        const void* const src_b = QS ? P.qb : P.b_in;
        RT pa_g[NSLOT], pa_b[NSLOT], pb_g[NSLOT], pb_b[NSLOT];
        if constexpr (PREFETCH) {
            load_slots<ST, NSLOT>(P, src_g, src_b, v0 < v1 ? v0 : 0, srcq, pa_g, pa_b);
        }
        const long long fstride = P.fv_stride;  // per (d, field) block of FV

        // Maxwellians of the q-box slots by recurrence along velocity axis 0
        // (when the slot coefficients live in registers)
        constexpr bool WALKER = KQ;
        const double h = P.hxi0;
        const int nvx = P.nv[0];
        GaussWalk wq[WALKER ? NSLOT : 1];
        if constexpr (WALKER) {
#pragma unroll
            for (int k = 0; k < NSLOT; ++k) wq[k].init(kq[k].inv2RT, h);
        }
        int ix = v0 % nvx;

        // one velocity: cur_* hold its prefetched fields, nxt_* receive the next
        auto velocity = [&](int i, int buf, RT(&cur_g)[NSLOT], RT(&cur_b)[NSLOT], RT(&nxt_g)[NSLOT],
                            RT(&nxt_b)[NSLOT]) __attribute__((always_inline)) {
            const Vel v = load_vel(P.vel, i);
            if constexpr (WALKER) {
                if (i == v0 || ix % WALK == 0) {
                    const int a0 = ix - ix % WALK;
                    const Vel va = a0 == ix ? v : load_vel(P.vel, i - (ix - a0));
#pragma unroll
                    for (int k = 0; k < NSLOT; ++k) wq[k].template anchor<D>(kq[k].A, kq[k].inv2RT, kq[k].u, va, h);
                    for (int j = a0; j < ix; ++j)
#pragma unroll
                        for (int k = 0; k < NSLOT; ++k) wq[k].advance();
                }
            }
            // BF16 rows: the raw halves move to the top of an FP32 word
            const bool half = StoreT<ST>::MIXED && (row_word(P, i) & 1);
            CT* const sq0 = sm.q[buf][0];
            CT* const sq1 = sm.q[buf][1];
            CT* const sa0 = sm.a[buf][0];
            CT* const sa1 = sm.a[buf][1];
            CT q_own[2], a_own[2][D];  // the own cell's q and slopes
            if constexpr (PREFETCH) {
                // unconditional loads (the last velocity re-reads itself) keep
                // the wait counts exact
                load_slots<ST, NSLOT>(P, src_g, src_b, i + 1 < v1 ? i + 1 : i, srcq, nxt_g, nxt_b);
            }

            // stage 1: quarter-step fields on the q box; a slot without a
            // point (the last ones of the halo) computes from cell 0 and
            // writes LDS entry NQ, which nothing reads, so the loop has no
            // branch between the loads of the previous velocity and their use
#pragma unroll
            for (int k = 0; k < NSLOT; ++k) {
                {
                    const int r = lq[k] >= 0 ? (lq[k] & 0xFFFFF) : G::NQ;
                    double g, b;
                    if constexpr (PREFETCH) {
                        g = slot_value<ST>(cur_g[k], half, srcq[k]);
                        b = slot_value<ST>(cur_b[k], half, srcq[k]);
                    } else {
                        g = state_ld<ST>(P, src_g, i, srcq[k]);
                        b = state_ld<ST>(P, src_b, i, srcq[k]);
                    }
                    double qg, qb;
                    if constexpr (QS) {
                        qg = g;
                        qb = b;
                    } else {
                        const double geq = wq[k].template value<D>(kq[k].A, kq[k].inv2RT, kq[k].u, v);
                        quarter_step_eq<D, ACC>(kq[k], v, geq, g, b, qg, qb, &P);
                    }
                    if constexpr (DIR) {
                        if (lq[k] > 0 && (lq[k] >> 20)) {  // Dirichlet ghost: the fixed state's equilibrium
                            const double* de = P.dir_eq + ((long long)((lq[k] >> 20) - 1) * P.V + i) * 2;
                            qg = de[0];
                            qb = de[1];
                        }
                    }
                    sq0[r] = CT(qg);
                    sq1[r] = CT(qb);
                    if (k == 0) {  // slot 0 is the own cell
                        q_own[0] = CT(qg);
                        q_own[1] = CT(qb);
                    }
                }
            }
            __syncthreads();

            // stage 2: limited differences on the slope box; the own cell first
            // (its values stay in registers for stage 3), then the ring
            {
                const int ai = G::aidx(tx, ty, tz), qi = G::qidx(tx, ty, tz);
#pragma unroll
                for (int e = 0; e < D; ++e) {
                    const int sq = G::SQ(e);
#pragma unroll
                    for (int f = 0; f < 2; ++f) {
                        const CT* q = f == 0 ? sq0 : sq1;
                        const CT c = q_own[f];
                        const CT a = half_van_leer(c - q[qi - sq], q[qi + sq] - c);
                        (f == 0 ? sa0 : sa1)[e * G::NA + ai] = a;
                        a_own[f][e] = a;
                    }
                }
            }
            // the ring: one (point, field) pair per thread and pass, so the
            // work spreads over all waves of the workgroup
#pragma unroll
            for (int k = 0; k < NRING2; ++k) {
                const int t = tid + k * NT;
                if (t < 2 * NARING) {
                    const int f = t >= NARING;
                    const int h = t - f * NARING;
                    const int p = slope_ring_point(h);
                    const int px = p % G::AX, py = (p / G::AX) % G::AY, pz = p / (G::AX * G::AY);
                    const int qi = (px + 1) + G::QX * ((py + (D >= 2 ? 1 : 0)) + G::QY * (pz + (D >= 3 ? 1 : 0)));
                    const CT* q = f == 0 ? sq0 : sq1;
                    CT* a = sa0 + f * (D * G::NA);
                    const CT c = q[qi];
#pragma unroll
                    for (int e = 0; e < D; ++e) {
                        const int sq = G::SQ(e);
                        a[e * G::NA + p] = half_van_leer(c - q[qi - sq], q[qi + sq] - c);
                    }
                }
            }
            __syncthreads();

            // stage 3: left face of the own cell along each d.  Upwind cell u
            // is c - d (xi_d > 0) or c (xi_d < 0); the own cell's q and slopes
            // come from registers, the others from LDS.
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const int dxo = d == 0, dyo = d == 1, dzo = d == 2;
                const double xd = d == 0 ? v.xi[0] : (d == 1 ? v.xi[1] : v.xi[2]);
                const int q_m = G::qidx(tx - dxo, ty - dyo, tz - dzo);
                const int a_m = G::aidx(tx - dxo, ty - dyo, tz - dzo);
                const int a_mm = G::aidx(tx - 2 * dxo, ty - 2 * dyo, tz - 2 * dzo);
                const int a_p = G::aidx(tx + dxo, ty + dyo, tz + dzo);
                // Upwind side by the sign of xi_d, which is uniform across the
                // workgroup: tested on its bits with scalar integer
                // instructions, so each velocity takes one branch (the mean
                // of both one-sided values only for xi_d = 0).
                const long long xbits = __builtin_bit_cast(long long, xd);
                const bool from_left = xbits > 0;                               // xi_d > 0
                const bool from_right = xbits < 0 && (xbits << 1) != 0;          // xi_d < 0
                // the face value from the upwind cell c - d (left) or c (right)
                auto left_value = [&](int f) __attribute__((always_inline)) {
                    const CT* sq = f == 0 ? sq0 : sq1;
                    const CT* sa = f == 0 ? sa0 : sa1;
                    CT aU[D], aL[D], aR[D];
#pragma unroll
                    for (int e = 0; e < D; ++e) aU[e] = sa[e * G::NA + a_m];
                    if constexpr (SS) return face_value_single<D, CT>(sq[q_m], aU, d, CT(1), v);
                    // upwind c - d: its left and right neighbours are c - 2d and c
#pragma unroll
                    for (int e = 0; e < D; ++e) {
                        aL[e] = sa[e * G::NA + a_mm];
                        aR[e] = a_own[f][e];
                    }
                    return face_value_at<D, CT>(sq[q_m], aU, aL, aR, d, CT(1), v);
                };
                auto right_value = [&](int f) __attribute__((always_inline)) {
                    const CT* sa = f == 0 ? sa0 : sa1;
                    if constexpr (SS) return face_value_single<D, CT>(q_own[f], a_own[f], d, CT(-1), v);
                    // upwind c: neighbours c - d and c + d
                    CT aL[D], aR[D];
#pragma unroll
                    for (int e = 0; e < D; ++e) {
                        aL[e] = sa[e * G::NA + a_m];
                        aR[e] = sa[e * G::NA + a_p];
                    }
                    return face_value_at<D, CT>(q_own[f], a_own[f], aL, aR, d, CT(-1), v);
                };
                CT fv[2];
                if (from_left) {
                    fv[0] = left_value(0);
                    fv[1] = left_value(1);
                } else if (from_right) {
                    fv[0] = right_value(0);
                    fv[1] = right_value(1);
                } else {
                    fv[0] = CT(0.5) * (left_value(0) + right_value(0));
                    fv[1] = CT(0.5) * (left_value(1) + right_value(1));
                }
                const double vg = fv[0], vb2 = fv[1];
                {
                    // a face outside the grid goes to the row's spare element
                    // NE: with the store unconditional the compiler need not
                    // wait for it before using the next velocity's loads
                    const long long o =
                        (long long)(2 * d) * fstride + (long long)i * P.fv_pitch + (fvalid[d] ? fe : NE);
                    st_stream<CT>(P.FV, o, vg);
                    st_stream<CT>(P.FV, o + fstride, vb2);
                }
                // weighted velocity products come from the table (uniform)
                const const_dptr vp = vel_ptr(P.vel, i);
                acc[d][0] += v.w * vg;
#pragma unroll
                for (int e = 0; e < D; ++e) acc[d][1 + e] += vp[VE_WXI0 + e] * vg;
                acc[d][D + 1] += v.w * vb2;
#pragma unroll
                for (int e = 0; e < D; ++e) acc[d][D + 2 + e] += vp[VE_WXX + 3 * d + e] * vg;
                acc[d][2 * D + 2] += vp[VE_WXI0 + d] * vb2;
            }
            if constexpr (WALKER) {
#pragma unroll
                for (int k = 0; k < NSLOT; ++k) wq[k].advance();
                if (++ix == nvx) ix = 0;
            }
            // single-buffered: the next velocity must not overwrite q and a
            // before every thread has read them; double-buffered: the next
            // velocity writes the other buffer, and the one after that comes
            // only after two more barriers
            if constexpr (NBUF == 1) __syncthreads();
        };

        if constexpr (D <= 2) {
            // The first velocity is peeled off, so the loop is entered, like
            // its back edge, with a velocity's face-value stores in flight:
            // the compiler's wait counts at the loop head then need not wait
            // for those stores before the fields loaded ahead are used.
            int i = v0;
            if (i < v1) velocity(i++, 0, pa_g, pa_b, pb_g, pb_b);
            for (; i + 1 < v1; i += 2) {
                velocity(i, NBUF - 1, pb_g, pb_b, pa_g, pa_b);
                velocity(i + 1, 0, pa_g, pa_b, pb_g, pb_b);
            }
            if (i < v1) velocity(i, NBUF - 1, pb_g, pb_b, pa_g, pa_b);
        } else {
            // 3-D: registers allow one set; the copy costs a wait per velocity
            for (int i = v0; i < v1; ++i) {
                RT cg[NSLOT], cb[NSLOT];
#pragma unroll
                for (int k = 0; k < NSLOT; ++k) {
                    cg[k] = pa_g[k];
                    cb[k] = pa_b[k];
                }
                velocity(i, 0, cg, cb, pa_g, pa_b);
            }
        }

        // partial face sums of this velocity slice
#pragma unroll
        for (int d = 0; d < D; ++d) {
            if (!fvalid[d]) continue;
            double* out = P.FS + ((long long)(slice * D + d) * NS) * NE + fe;
#pragma unroll
            for (int j = 0; j < NS; ++j) out[(long long)j * NE] = acc[d][j];
        }
    }
};

// ---------------------------------------------------------------------------
// update kernel: streaming, one thread per cell over a velocity slice.
// Reads phi^n and the stored phi_bar at the cell's 2D faces, inverts eq.
// phibar with the face coefficients, forms the microflux (eq. flux) and writes
// phi^{n+1} (eq. phiupdate).
// ---------------------------------------------------------------------------
// ACC: the problem has an external acceleration (face inversion, the cell
// source of eq. phiupdate and, in 3-D, the next quarter-step fields carry
// its terms).
// ROWS (BF16-tail form only): 0 updates every velocity row of the slice,
// 1 only its FP32 rows, 2 only its BF16 rows.  The 3-D single-problem step
// runs the two row kinds as two launches, so that each holds one loop body
// (see launch_update).
template <int D, typename ST, bool ACC = false, int ROWS = 0>
struct UpdateKernel {
    using CT = typename StoreT<ST>::C;  // stored face values
    __device__ static void run(const Problem& P, long long c, int slice, int nslices) {
        const long long N = P.N, NE = P.NE;
        const bool inside = c < N;
        const long long cc = inside ? c : 0;
        int co[3];
        {
            long long r = cc;
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                co[e] = (int)(r % P.n[e]);
                r /= P.n[e];
            }
        }
        // left and right faces along each d (periodic wrap at the right end);
        // face indices fit 32 bits (checked at set-up)
        unsigned fl[D], fr[D];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            int rc[3] = {co[0], co[1], co[2]};
            fl[d] = (unsigned)(rc[0] + (long long)P.ne[0] * (rc[1] + (long long)P.ne[1] * rc[2]));
            rc[d] += 1;
            if (P.bc[d] == 0 && rc[d] == P.n[d]) rc[d] = 0;
            fr[d] = (unsigned)(rc[0] + (long long)P.ne[0] * (rc[1] + (long long)P.ne[1] * rc[2]));
        }
        const CellCoef k0 = load_coef(P.P_in, N, cc);
        const CellCoef k1 = load_coef(P.P_out, N, cc);
        FaceCoef<D> fcl[D], fcr[D];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const double* F = P.FP + (long long)d * NFP * NE;
            fcl[d].load(F + fl[d], NE);
            fcr[d].load(F + fr[d], NE);
            if constexpr (ACC) {
                fcl[d].prepare_accel(P.accel, P.dt);
                fcr[d].prepare_accel(P.accel, P.dt);
            }
        }
        // the cell's source terms at t_n: dt S_g = c0 g_eq, dt S_b = dt a.xi (g - g_eq) + c0 b_eq
        // with c0 = dt a.(xi - u)/(R T) = 2 dt (a.xi - a.u)/(2 R T)
        double au0 = 0.0;
        if constexpr (ACC) {
#pragma unroll
            for (int d = 0; d < D; ++d) au0 += P.accel[d] * k0.u[d];
        }
        const int v0 = (int)((long long)P.V * slice / nslices);
        const int v1 = (int)((long long)P.V * (slice + 1) / nslices);
        const long long fstride = P.fv_stride;
        const double dt = P.dt;
        // constant parts of eq. phiupdate
        const double inv_g = 1.0 / (1.0 + 2.0 * k1.beta), inv_b = 1.0 / (1.0 + 2.0 * k1.betab);

        // Maxwellians by recurrence along velocity axis 0 for FP64 storage in
        // 1-D and 2-D.  The 3-D kernel has no registers to spare, and the FP32
        // kernel runs a third wave per SIMD without the recurrence state,
        // which outweighs the exponentials it saves.
        constexpr bool WALKER = D <= 2 && std::is_same<ST, double>::value;
        const double h = P.hxi0;
        const int nvx = P.nv[0];
        GaussWalk w0, w1, wl[D], wr[D];
        if constexpr (WALKER) {
            w0.init(k0.inv2RT, h);
            w1.init(k1.inv2RT, h);
#pragma unroll
            for (int d = 0; d < D; ++d) {
                wl[d].init(fcl[d].inv2RT, h);
                wr[d].init(fcr[d].inv2RT, h);
            }
        }
        int ix = v0 % nvx;
        // Maxwellians without the recurrence: the FP64 exponential for FP64
        // storage; FP32 accuracy for the FP32 forms, from Z = xi.u - |u|^2/2,
        // which the inversion and the S_b source use as well
        constexpr bool FZ = !std::is_same<ST, double>::value;
        auto equilibrium = [](double A, double s, const double* u, double Z, const Vel& v)
                               __attribute__((always_inline)) {
            if constexpr (FZ) return maxwellian_f32z(A, s, Z, v.hx2);
            else return maxwellian<D>(A, s, u, v);
        };

        // The loads of one velocity: g and b of the cell, and the stored face
        // values at its 2D faces ([d][left g, left b, right g, right b]).
        auto load = [&](int i, long long off, auto kind, typename RowIO<decltype(kind)>::Raw& rg,
                        typename RowIO<decltype(kind)>::Raw& rb, CT (&fv)[4 * D]) __attribute__((always_inline)) {
            using IO = RowIO<decltype(kind)>;
            rg = IO::raw(P.g_in, off, cc);
            rb = IO::raw(P.b_in, off, cc);
            const CT* const F = (const CT*)P.FV;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const long long o = (long long)(2 * d) * fstride + (long long)i * P.fv_pitch;
                fv[4 * d] = F[o + fl[d]];
                fv[4 * d + 1] = F[o + fstride + fl[d]];
                fv[4 * d + 2] = F[o + fr[d]];
                fv[4 * d + 3] = F[o + fstride + fr[d]];
            }
        };
        // One velocity of the slice from its loads; its rows (g, b in and
        // out, and the 3-D quarter-step fields) hold elements of kind E and
        // start `off` bytes into each state array.  Every storage form runs
        // this one body.
        auto velocity = [&](int i, long long off, auto kind, const typename RowIO<decltype(kind)>::Raw& rg,
                            const typename RowIO<decltype(kind)>::Raw& rb, const CT (&fv)[4 * D])
                            __attribute__((always_inline)) {
            using IO = RowIO<decltype(kind)>;
            const Vel v = load_vel(P.vel, i);
            if constexpr (WALKER) {
                if (i == v0 || ix % WALK == 0) {
                    const int a0 = ix - ix % WALK;
                    // a slice starting inside a block walks from its anchor
                    const Vel va = a0 == ix ? v : load_vel(P.vel, i - (ix - a0));
                    w0.anchor<D>(k0.A, k0.inv2RT, k0.u, va, h);
                    w1.anchor<D>(k1.A, k1.inv2RT, k1.u, va, h);
#pragma unroll
                    for (int d = 0; d < D; ++d) {
                        wl[d].template anchor<D>(fcl[d].A, fcl[d].inv2RT, fcl[d].u, va, h);
                        wr[d].template anchor<D>(fcr[d].A, fcr[d].inv2RT, fcr[d].u, va, h);
                    }
                    for (int j = a0; j < ix; ++j) {
                        w0.advance();
                        w1.advance();
#pragma unroll
                        for (int d = 0; d < D; ++d) {
                            wl[d].advance();
                            wr[d].advance();
                        }
                    }
                }
            }
            const double g = IO::val(rg);
            const double b = IO::val(rb);
            double Fg = 0.0, Fb = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const double Zl = fcl[d].z(v), Zr = fcr[d].z(v);
                const double eql = WALKER ? wl[d].template value<D>(fcl[d].A, fcl[d].inv2RT, fcl[d].u, v)
                                          : equilibrium(fcl[d].A, fcl[d].inv2RT, fcl[d].u, Zl, v);
                const double eqr = WALKER ? wr[d].template value<D>(fcr[d].A, fcr[d].inv2RT, fcr[d].u, v)
                                          : equilibrium(fcr[d].A, fcr[d].inv2RT, fcr[d].u, Zr, v);
                double gl, bl, gr, br;
                const double flg = fv[4 * d], flb = fv[4 * d + 1], frg = fv[4 * d + 2], frb = fv[4 * d + 3];
                if constexpr (ACC) {
                    fcl[d].invert_accel_z(v, dt, eql, Zl, flg, flb, gl, bl);
                    fcr[d].invert_accel_z(v, dt, eqr, Zr, frg, frb, gr, br);
                } else {
                    fcl[d].invert_z(v, eql, Zl, flg, flb, gl, bl);
                    fcr[d].invert_z(v, eqr, Zr, frg, frb, gr, br);
                }
                const double sxd = v.xi[d] * P.inv_dx[d];
                Fg += sxd * (gr - gl);
                Fb += sxd * (br - bl);
            }
            double xu0 = 0.0, xu1 = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                xu0 += v.xi[d] * k0.u[d];
                xu1 += v.xi[d] * k1.u[d];
            }
            const double Z0 = xu0 - k0.hu2;
            const double geq0 =
                WALKER ? w0.value<D>(k0.A, k0.inv2RT, k0.u, v) : equilibrium(k0.A, k0.inv2RT, k0.u, Z0, v);
            const double beq0 = (v.hx2 + k0.cRT2) * geq0;
            const double geq1 = WALKER ? w1.value<D>(k1.A, k1.inv2RT, k1.u, v)
                                       : equilibrium(k1.A, k1.inv2RT, k1.u, xu1 - k1.hu2, v);
            const double beq1 = (v.hx2 + k1.cRT2) * geq1;
            // eq. phiupdate with dt/(2 tau) = 2 beta and dt S_b = 4 eta Z (g - g_eq)
            double gn = g + 2.0 * k1.beta * geq1 + 2.0 * k0.beta * (geq0 - g) - dt * Fg;
            double bn = b + 2.0 * k1.betab * beq1 + 2.0 * k0.betab * (beq0 - b) - dt * Fb +
                        4.0 * k0.eta * Z0 * (g - geq0);
            if constexpr (ACC) {
                const double c0 = 2.0 * dt * k0.inv2RT * (v.ax - au0);
                gn += c0 * geq0;
                bn += dt * v.ax * (g - geq0) + c0 * beq0;
            }
            gn *= inv_g;
            bn *= inv_b;
            if (inside) {
                IO::st(P.g_out, off, cc, gn);
                IO::st(P.b_out, off, cc, bn);
                if constexpr (quarter_stored(D)) {
                    // next step's phi_bar_plus from the state as stored
                    double qg, qb;
                    quarter_step_eq<D, ACC>(k1, v, geq1, IO::round(gn), IO::round(bn), qg, qb, &P);
                    IO::st(P.qg, off, cc, qg);
                    IO::st(P.qb, off, cc, qb);
                }
            }
            if constexpr (WALKER) {
                w0.advance();
                w1.advance();
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    wl[d].advance();
                    wr[d].advance();
                }
                if (++ix == nvx) ix = 0;
            }
        };

        auto off_of = [&](int i) { return (long long)i * P.pitch * (long long)sizeof(ST); };
        // FP64 in 1-D and 2-D has the registers to load a velocity ahead; the
        // FP32 forms would lose a wave per SIMD (2-D) or spill (3-D)
        constexpr bool AHEAD = std::is_same<ST, double>::value && D <= 2;
        if constexpr (!StoreT<ST>::MIXED && !AHEAD) {
            for (int i = v0; i < v1; ++i) {
                typename RowIO<ST>::Raw rg, rb;
                CT fv[4 * D];
                load(i, off_of(i), ST{}, rg, rb, fv);
                velocity(i, off_of(i), ST{}, rg, rb, fv);
            }
        } else if constexpr (!StoreT<ST>::MIXED) {
            // The loads of velocity i+1 are issued before velocity i is
            // processed, into the other of two named register sets (the loop
            // is unrolled by two), so a register with a load in flight is
            // never copied; the last trip re-reads its own velocity.
            typename RowIO<ST>::Raw ga, ba, gb, bb;
            CT fa[4 * D], fb[4 * D];
            if (v0 < v1) load(v0, off_of(v0), ST{}, ga, ba, fa);
            int i = v0;
            for (; i + 1 < v1; i += 2) {
                load(i + 1, off_of(i + 1), ST{}, gb, bb, fb);
                velocity(i, off_of(i), ST{}, ga, ba, fa);
                const int n2 = i + 2 < v1 ? i + 2 : i + 1;
                load(n2, off_of(n2), ST{}, ga, ba, fa);
                velocity(i + 1, off_of(i + 1), ST{}, gb, bb, fb);
            }
            if (i < v1) velocity(i, off_of(i), ST{}, ga, ba, fa);
        } else {
            // BF16-tail form: the row kind is uniform, so each velocity runs
            // the body for FP32 or BF16 rows; the FP32 rows of the slice
            // first, then its BF16 rows (every (cell, velocity) is updated on
            // its own, so the order is free); no recurrence for the equilibria
            if constexpr (ROWS != 2) {
                for (int i = v0; i < v1; ++i) {
                    const long long o = row_word(P, i);
                    if (!(o & 1)) {
                        float rg, rb;
                        CT fv[4 * D];
                        load(i, o, float{}, rg, rb, fv);
                        velocity(i, o, float{}, rg, rb, fv);
                    }
                }
            }
            if constexpr (ROWS != 1) {
                for (int i = v0; i < v1; ++i) {
                    const long long o = row_word(P, i);
                    if (o & 1) {
                        __bf16 rg, rb;
                        CT fv[4 * D];
                        load(i, o & ~1LL, Bf16Row{}, rg, rb, fv);
                        velocity(i, o & ~1LL, Bf16Row{}, rg, rb, fv);
                    }
                }
            }
        }
    }
};

// waves per SIMD the face-sum kernel is compiled for (register budget; 3-D
// takes what it needs, within what a workgroup of its shape requires)
template <int D>
constexpr int face_sum_waves() { return D == 1 ? 4 : (D == 2 ? 3 : 1); }

// The single-problem face-sum kernel of tile shape TID.
template <int D, typename ST, bool DIR, bool SS, int TID, bool ACC>
__global__ __launch_bounds__(tile_threads(D, TID), face_sum_waves<D>()) void k_face_sums(Problem P) {
    using K = FaceSumKernel<D, ST, DIR, SS, TID, ACC>;
    static_assert(sizeof(typename K::Smem) == face_sum_lds_bytes(D, TID, sizeof(typename K::CT)),
                  "host and kernel LDS sizes differ");
    __shared__ typename K::Smem sm;
    int ntiles = P.tiles1[0] * P.tiles1[1] * P.tiles1[2];
    int q = xcd_remap(blockIdx.x, gridDim.x);
    K::run(P, q % ntiles, q / ntiles, P.nslices, sm);
}

// Launch the face sums of a problem of dimension D: the kernel of its tile
// shape, storage form, boundary kind and reconstruction.  Shapes whose boxes
// do not fit a CU's LDS for the storage form are refused (the host never
// selects them).
template <int D, typename ST, bool DIR, bool SS, int TID, bool ACC = false>
hipError_t launch_face_sums_shape(const Problem& P, hipStream_t s) {
    if constexpr (face_tile_fits(D, TID, sizeof(typename StoreT<ST>::C))) {
        const unsigned nb = (unsigned)(P.tiles1[0] * P.tiles1[1] * P.tiles1[2] * P.nslices);
        hipLaunchKernelGGL((k_face_sums<D, ST, DIR, SS, TID, ACC>), dim3(nb), dim3(tile_threads(D, TID)), 0, s, P);
        return hipGetLastError();
    } else {
        return hipErrorInvalidConfiguration;
    }
}

template <int D, typename ST, int TID>
int face_sum_occupancy_shape() {
    if constexpr (face_tile_fits(D, TID, sizeof(typename StoreT<ST>::C))) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (k_face_sums<D, ST, false, false, TID, false>),
                                                        tile_threads(D, TID), 0) != hipSuccess) {
            (void)hipGetLastError();
            return 0;
        }
        return n;
    } else {
        return 0;
    }
}

// ---------------------------------------------------------------------------
// 3-D face values by z-march (the tile shapes with z = 0).  A workgroup owns a
// TX x TY column of the face grid for one velocity i and walks it along z.
// Step z stages the quarter-step fields of plane z+2 (with the xy halo,
// offsets -3..T+1), forms the limited differences of plane z+1 (all three
// components, offsets -2..T) and reconstructs the three left faces of its
// cells in plane z with the box kernel's operands and operations, so the face
// values are bitwise those of the box kernel.  LDS holds the q planes
// z-1..z+2 in a ring of four and the differences of planes z and z+1 in a
// ring of two; the own column's differences of planes z-2 and z-1 and its q
// of plane z-1 stay in registers.  Each plane is staged once per column
// (plus the xy halo), where a box stages (T_z + 5) planes per T_z.
// Two barriers per step keep the rings safe: the q store of step z goes to
// the slot of plane z-2, whose last reader is step z-1's differences (before
// that step's second barrier); the differences of step z go to the slot of
// plane z-1, whose last reader is step z-1's faces (before step z's first
// barrier).
// NF threads per cell: with NF = 2 (FP64, whose LDS allows two workgroups per
// CU) one thread per cell takes g and another b, which doubles the waves that
// hide the LDS and memory latency; with NF = 1 a thread takes both fields.
// The kernel stores the face values only; k_face_reduce forms their velocity
// sums.
template <typename CT>
constexpr int zmarch_threads_per_cell() { return sizeof(CT) == 8 ? 2 : 1; }

template <typename ST, bool DIR, bool SS, int TX, int TY>
struct ZMarch {
    using CT = typename StoreT<ST>::C;
    using RT = typename StoreT<ST>::R;
    static constexpr int NT = TX * TY;                        // cells of the column
    static constexpr int NF = zmarch_threads_per_cell<CT>();  // threads per cell
    static constexpr int NTH = NF * NT;                       // threads of the workgroup
    static constexpr int FL = 2 / NF;                         // fields per thread
    static constexpr int QX = TX + 5, QY = TY + 5, NQ = QX * QY;  // q plane
    static constexpr int AX = TX + 3, AY = TY + 3, NA = AX * AY;  // difference plane
    static constexpr int NSLOT = (NQ + NT - 1) / NT;              // q points per thread
    static constexpr int NPASS = (2 * NA + NTH - 1) / NTH;        // (point, field) passes
    static_assert(NF == 1 || !StoreT<ST>::MIXED, "the BF16-tail form loads its rows through load_slots");
    struct Smem {
        CT q[4][2][NQ];
        CT a[2][2][3][NA];  // [ring][field][component][point]
    };
    __device__ static int qidx(int x, int y) { return (x + 3) + QX * (y + 3); }
    __device__ static int aidx(int x, int y) { return (x + 2) + AX * (y + 2); }

    __device__ static void run(const Problem& P, int tile, int i, Smem& sm) {
        const int tid = threadIdx.x;
        const int ct = tid % NT;           // cell of the column
        const int f0 = NF == 2 ? tid / NT : 0;  // first field of the thread (uniform per wave)
        const int ox = (tile % P.tiles1[0]) * TX, oy = (tile / P.tiles1[0]) * TY;
        const int n0 = P.n[0], n1 = P.n[1], n2 = P.n[2];
        const long long nplane = (long long)n0 * n1;
        // q-plane points of this thread: in-plane source offset after the
        // periodic wrap / outflow clamp, and for Dirichlet sides the side of
        // the point's x or y coordinate (2 d + side + 1, y over x, 0: none)
        long long off[NSLOT];
        int lq[NSLOT];
        int sxy[DIR ? NSLOT : 1];
#pragma unroll
        for (int k = 0; k < NSLOT; ++k) {
            const int p = ct + k * NT;
            lq[k] = p < NQ ? p : -1;
            const int pp = p < NQ ? p : 0;
            const int x = ox + pp % QX - 3, y = oy + pp / QX - 3;
            off[k] = map_coord(x, n0, P.bc[0]) + (long long)n0 * map_coord(y, n1, P.bc[1]);
            if constexpr (DIR) {
                int side = 0;
                if (P.bc[0] == 2 && (x < 0 || x >= n0)) side = (x >= n0) + 1;
                if (P.bc[1] == 2 && (y < 0 || y >= n1)) side = 2 + (y >= n1) + 1;
                sxy[k] = side;
            }
        }
        const Vel v = load_vel(P.vel, i);
        const bool half = StoreT<ST>::MIXED && (row_word(P, i) & 1);

        // raw fields of the next plane to stage: both, or the thread's one
        RT pg[NSLOT], pb[NSLOT];
        auto load_plane = [&](int z) __attribute__((always_inline)) {
            const long long base = (long long)map_coord(z, n2, P.bc[2]) * nplane;
            long long src[NSLOT];
#pragma unroll
            for (int k = 0; k < NSLOT; ++k) src[k] = base + off[k];
            if constexpr (NF == 1) {
                load_slots<ST, NSLOT, false>(P, P.qg, P.qb, i, src, pg, pb);
            } else {
                const void* const q = f0 ? P.qb : P.qg;
#pragma unroll
                for (int k = 0; k < NSLOT; ++k) pg[k] = state_load<ST>(P, q, i, src[k]);
            }
        };
        auto store_plane = [&](int z) __attribute__((always_inline)) {
            const int r = (z + 8) & 3;
            int zs = 0;  // Dirichlet side of the plane (z over x and y)
            if constexpr (DIR) {
                if (P.bc[2] == 2 && (z < 0 || z >= n2)) zs = 4 + (z >= n2) + 1;
            }
#pragma unroll
            for (int k = 0; k < NSLOT; ++k) {
                if (lq[k] < 0) continue;
#pragma unroll
                for (int j = 0; j < FL; ++j) {
                    const int f = f0 + j;
                    double val = slot_value<ST>(j == 0 ? pg[k] : pb[k], half, 0);
                    if constexpr (DIR) {
                        const int side = zs ? zs : sxy[k];
                        if (side) val = P.dir_eq[((long long)(side - 1) * P.V + i) * 2 + f];
                    }
                    sm.q[r][f][lq[k]] = CT(val);
                }
            }
        };
        // limited differences of plane z on the difference plane
        auto differences = [&](int z) __attribute__((always_inline)) {
            const int rm = (z + 7) & 3, r0 = (z + 8) & 3, rp = (z + 9) & 3, ra = (z + 8) & 1;
#pragma unroll
            for (int k = 0; k < NPASS; ++k) {
                const int t = tid + k * NTH;
                if (t < 2 * NA) {
                    const int f = t >= NA;
                    const int pt = t - f * NA;
                    const int qi = (pt % AX + 1) + QX * (pt / AX + 1);
                    const CT* q = sm.q[r0][f];
                    const CT c = q[qi];
                    sm.a[ra][f][0][pt] = half_van_leer(c - q[qi - 1], q[qi + 1] - c);
                    sm.a[ra][f][1][pt] = half_van_leer(c - q[qi - QX], q[qi + QX] - c);
                    sm.a[ra][f][2][pt] = half_van_leer(c - sm.q[rm][f][qi], sm.q[rp][f][qi] - c);
                }
            }
        };

        // own cell, the validity of its left faces and their face-grid index
        const int tx = ct % TX, ty = ct / TX;
        const int gx = ox + tx, gy = oy + ty;
        const bool vx = gx < P.ne[0] && gy < n1, vy = gx < n0 && gy < P.ne[1], vz = gx < n0 && gy < n1;
        const long long fplane = (long long)P.ne[0] * P.ne[1];
        const long long fe0 = gx + (long long)P.ne[0] * gy;
        const long long fstride = P.fv_stride;
        const int qo_i = qidx(tx, ty), ao_i = aidx(tx, ty);

        // own column, per field of the thread: differences of planes z-2 and
        // z-1, q of plane z-1
        CT am2[FL][3], am1[FL][3], qm1[FL];
        auto faces = [&](int z, bool emit) __attribute__((always_inline)) {
            const int rq = (z + 8) & 3, ra = (z + 8) & 1, ra1 = (z + 9) & 1;
            CT qo[FL], ao[FL][3];
#pragma unroll
            for (int j = 0; j < FL; ++j) {
                qo[j] = sm.q[rq][f0 + j][qo_i];
#pragma unroll
                for (int e = 0; e < 3; ++e) ao[j][e] = sm.a[ra][f0 + j][e][ao_i];
            }
            if (emit) {
                const long long fe = fe0 + fplane * z;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const bool valid = d == 0 ? (vx && z < n2) : (d == 1 ? (vy && z < n2) : vz);
                    const int dx = d == 0, dy = d == 1;
                    const int a_m = aidx(tx - dx, ty - dy), a_mm = aidx(tx - 2 * dx, ty - 2 * dy);
                    const int a_p = aidx(tx + dx, ty + dy), q_m = qidx(tx - dx, ty - dy);
                    // the face value from the upwind cell c - d (left) or c
                    // (right), for field slot j of the thread
                    auto left_value = [&](int j) __attribute__((always_inline)) {
                        const int f = f0 + j;
                        CT qU, aU[3], aL[3];
                        if (d == 2) {
                            qU = qm1[j];
#pragma unroll
                            for (int e = 0; e < 3; ++e) {
                                aU[e] = am1[j][e];
                                aL[e] = am2[j][e];
                            }
                        } else {
                            qU = sm.q[rq][f][q_m];
#pragma unroll
                            for (int e = 0; e < 3; ++e) {
                                aU[e] = sm.a[ra][f][e][a_m];
                                aL[e] = sm.a[ra][f][e][a_mm];
                            }
                        }
                        if constexpr (SS) return face_value_single<3, CT>(qU, aU, d, CT(1), v);
                        return face_value_at<3, CT>(qU, aU, aL, ao[j], d, CT(1), v);
                    };
                    auto right_value = [&](int j) __attribute__((always_inline)) {
                        const int f = f0 + j;
                        if constexpr (SS) return face_value_single<3, CT>(qo[j], ao[j], d, CT(-1), v);
                        CT aL[3], aR[3];
#pragma unroll
                        for (int e = 0; e < 3; ++e) {
                            aL[e] = d == 2 ? am1[j][e] : sm.a[ra][f][e][a_m];
                            aR[e] = d == 2 ? sm.a[ra1][f][e][ao_i] : sm.a[ra][f][e][a_p];
                        }
                        return face_value_at<3, CT>(qo[j], ao[j], aL, aR, d, CT(-1), v);
                    };
                    // upwind side by the bits of the uniform xi_d, as in the
                    // box kernel
                    const long long xbits = __builtin_bit_cast(long long, v.xi[d]);
                    const bool from_left = xbits > 0;
                    const bool from_right = xbits < 0 && (xbits << 1) != 0;
                    CT fv[FL];
                    if (from_left) {
#pragma unroll
                        for (int j = 0; j < FL; ++j) fv[j] = left_value(j);
                    } else if (from_right) {
#pragma unroll
                        for (int j = 0; j < FL; ++j) fv[j] = right_value(j);
                    } else {
#pragma unroll
                        for (int j = 0; j < FL; ++j) fv[j] = CT(0.5) * (left_value(j) + right_value(j));
                    }
                    {
                        // a face outside the grid goes to the row's spare
                        // element NE (the store stays unconditional)
                        const long long o = (long long)(2 * d + f0) * fstride + (long long)i * P.fv_pitch +
                                            (valid ? fe : P.NE);
#pragma unroll
                        for (int j = 0; j < FL; ++j) st_stream<CT>(P.FV, o + j * fstride, fv[j]);
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < FL; ++j) {
                qm1[j] = qo[j];
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    am2[j][e] = am1[j][e];
                    am1[j][e] = ao[j][e];
                }
            }
        };

        // Planes z0-3 and z0-2 first; then step z stages plane z+2 (loaded
        // during the previous step), loads plane z+3, forms the differences of
        // plane z+1 and, from z0 on, the faces of plane z.  The steps before
        // z0 only fill the rings and the column registers (the differences of
        // plane z0-3 they shift through are never used).  The last step's
        // load of a plane past the column reads a mapped, valid address.
        const int z0 = 0, z1 = P.ne[2];
        load_plane(z0 - 3);
        store_plane(z0 - 3);
        load_plane(z0 - 2);
        store_plane(z0 - 2);
        load_plane(z0 - 1);
        for (int z = z0 - 3; z < z1; ++z) {
            store_plane(z + 2);
            load_plane(z + 3);
            __syncthreads();
            differences(z + 1);
            __syncthreads();
            faces(z, z >= z0);
        }
    }
};

template <typename ST, bool DIR, bool SS, int TX, int TY>
__global__ __launch_bounds__((ZMarch<ST, DIR, SS, TX, TY>::NTH)) void k_face_values_z(Problem P) {
    using K = ZMarch<ST, DIR, SS, TX, TY>;
    __shared__ typename K::Smem sm;
    const int ntiles = P.tiles1[0] * P.tiles1[1];
    const int q = xcd_remap(blockIdx.x, gridDim.x);
    K::run(P, q % ntiles, q / ntiles, sm);
}

// Velocity sums of the stored face values of one velocity slice: per face
// along d, the 2D+3 sums of the box kernel with the same products in the same
// ascending-velocity order, so the partial sums are bitwise those the box
// kernel accumulates in registers.  One thread per face-grid point takes its
// D faces.
template <int D, typename CT>
__global__ __launch_bounds__(WG) void k_face_reduce(Problem P) {
    const long long fe = (long long)blockIdx.x * WG + threadIdx.x;
    const int slice = blockIdx.y;
    if (fe >= P.NE) return;
    const int c[3] = {(int)(fe % P.ne[0]), (int)((fe / P.ne[0]) % P.ne[1]),
                      (int)(fe / ((long long)P.ne[0] * P.ne[1]))};
    bool valid[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        bool ok = true;
#pragma unroll
        for (int e = 0; e < D; ++e) ok &= e == d ? c[e] < P.ne[e] : c[e] < P.n[e];
        valid[d] = ok;
    }
    const int v0 = (int)((long long)P.V * slice / P.nslices);
    const int v1 = (int)((long long)P.V * (slice + 1) / P.nslices);
    constexpr int NS = 2 * D + 3;
    double acc[D][NS];
#pragma unroll
    for (int d = 0; d < D; ++d)
#pragma unroll
        for (int j = 0; j < NS; ++j) acc[d][j] = 0.0;
    const CT* const fv = (const CT*)P.FV + fe;
#pragma unroll 4
    for (int i = v0; i < v1; ++i) {
        const Vel v = load_vel(P.vel, i);
        const const_dptr vp = vel_ptr(P.vel, i);
        const long long row = (long long)i * P.fv_pitch;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            // invalid faces read a stored slot of the block and discard it
            const double vg = fv[(long long)(2 * d) * P.fv_stride + row];
            const double vb2 = fv[(long long)(2 * d + 1) * P.fv_stride + row];
            acc[d][0] += v.w * vg;
#pragma unroll
            for (int e = 0; e < D; ++e) acc[d][1 + e] += vp[VE_WXI0 + e] * vg;
            acc[d][D + 1] += v.w * vb2;
#pragma unroll
            for (int e = 0; e < D; ++e) acc[d][D + 2 + e] += vp[VE_WXX + 3 * d + e] * vg;
            acc[d][2 * D + 2] += vp[VE_WXI0 + d] * vb2;
        }
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
        if (!valid[d]) continue;
        double* out = P.FS + ((long long)(slice * D + d) * NS) * P.NE + fe;
#pragma unroll
        for (int j = 0; j < NS; ++j) out[(long long)j * P.NE] = acc[d][j];
    }
}

// Face values by z-march, then their velocity sums (tile shape TID with z = 0).
template <typename ST, bool DIR, bool SS, int TID>
hipError_t launch_face_sums_zmarch(const Problem& P, hipStream_t s) {
    constexpr TileExt T = tile_shape(3, TID);
    static_assert(tile_zmarch(3, TID), "not a z-marching shape");
    using K = ZMarch<ST, DIR, SS, T.x, T.y>;
    static_assert(sizeof(typename K::Smem) == face_sum_lds_bytes(3, TID, sizeof(typename K::CT)),
                  "host and kernel LDS sizes differ");
    if constexpr (face_tile_fits(3, TID, sizeof(typename K::CT))) {
        const unsigned nb = (unsigned)((long long)P.tiles1[0] * P.tiles1[1] * P.V);
        hipLaunchKernelGGL((k_face_values_z<ST, DIR, SS, T.x, T.y>), dim3(nb), dim3(K::NTH), 0, s, P);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_face_reduce<3, typename K::CT>), dim3((unsigned)((P.NE + WG - 1) / WG), P.nslices),
                           dim3(WG), 0, s, P);
        return hipGetLastError();
    } else {
        return hipErrorInvalidConfiguration;
    }
}

template <typename ST, int TID>
int face_values_z_occupancy() {
    constexpr TileExt T = tile_shape(3, TID);
    if constexpr (face_tile_fits(3, TID, sizeof(typename StoreT<ST>::C))) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (k_face_values_z<ST, false, false, T.x, T.y>),
                                                        ZMarch<ST, false, false, T.x, T.y>::NTH, 0) != hipSuccess) {
            (void)hipGetLastError();
            return 0;
        }
        return n;
    } else {
        return 0;
    }
}

// Batched face sums: one launch for every tile of every problem of a storage
// class.  Persistent: the grid covers the resident slots and the workgroups
// take (cost-sorted, largest first) items from a device queue: an atomic
// counter, so a workgroup that finishes early takes the next item.  Which
// workgroup computes an item does not change its result.  The launch resets
// the other kernel's counter (that kernel's previous launch has finished and
// its next one starts after this one), so no memset enters a graph.
// Problems of different dimension share the launch; LDS is the union of their
// needs.
// The item index is uniform across the workgroup; readfirstlane tells the
// compiler so, and the item and its problem descriptor are then read through
// the constant address space: scalar loads into SGPRs instead of a copy of
// the descriptor in vector registers (the FP32 1-D/2-D face-sum class then
// runs 3 waves per SIMD, like the single-problem kernel).  Forcing the update
// class to 3 waves as well spills registers and is slower.
__device__ __forceinline__ int next_item(int* queue, int* slot) {
    if (threadIdx.x == 0) *slot = atomicAdd(queue, 1);
    __syncthreads();
    const int w = __builtin_amdgcn_readfirstlane(*slot);
    __syncthreads();  // every thread has read the slot before it is refilled
    return w;
}

// word-wise copy of a uniform descriptor through the constant address space
template <typename T>
__device__ __forceinline__ T load_uniform(const T* p) {
    static_assert(sizeof(T) % 4 == 0, "descriptor size");
    typedef const __attribute__((address_space(4))) unsigned* const_uptr;
    const const_uptr s = (const_uptr)(const void*)p;
    unsigned words[sizeof(T) / 4];
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / 4); ++k) words[k] = s[k];
    T r;
    __builtin_memcpy(&r, words, sizeof(T));
    return r;
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
    if (P.has_accel) {
        // eqs. rhoubar, rhoEbar: (h/2) rho a and (h/2) (rho u).a, h/2 = dt/4,
        // with the face momentum just formed
        for (int e = 0; e < D; ++e) Wf[1 + e] += 0.25 * P.dt * Wf[0] * P.accel[e];
        for (int e = 0; e < D; ++e) Wf[D + 1] += 0.25 * P.dt * Wf[1 + e] * P.accel[e];
    }
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
    double M[3][5];
    int off = 0;
    for (int k = 0; k < 3; ++k) {
        for (int p = 0; p < 5; ++p) M[k][p] = 0.0;
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
            M[k][4] += e * x * x * x * x;
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
    for (int e = 0; e < D; ++e) Gp[e] = (S[D + 2 + e] + beta * E2[e]) * ig;
    double accE = 0.0;
    if (P.has_accel) {
        // The acceleration's (h/2) S terms at the face (eqs. gsource,
        // bsource with the velocity derivative on the equilibrium) enter g_f
        // as ig c (a.xi - a.u) g_eq and b_f as ib [(dt/4) a.xi (g_f - g_eq)
        // + c (a.xi - a.u) b_eq], c = (h/2)/(R T); their flux moments need
        // third and fourth separable moments of the face Maxwellian.
        auto mom = [&](const int* p) { return A * M[0][p[0]] * M[1][p[1]] * M[2][p[2]]; };
        const double c = 0.5 * P.dt * inv2RT;
        double au = 0.0, aE2 = 0.0;
        for (int k = 0; k < D; ++k) {
            au += P.accel[k] * q.u[k];
            aE2 += P.accel[k] * E2[k];
        }
        Gm += ig * c * (aE2 - au * E1);
        for (int e = 0; e < D; ++e) {
            double t3 = 0.0;  // sum_k a_k sum_i w_i xi_d xi_e xi_k g_eq
            for (int k = 0; k < D; ++k) {
                int p[3] = {0, 0, 0};
                p[d] += 1;
                p[e] += 1;
                p[k] += 1;
                t3 += P.accel[k] * mom(p);
            }
            Gp[e] += ig * c * (t3 - au * E2[e]);
        }
        double aB2 = 0.0, aG = 0.0;  // sum_k a_k sum_i w_i xi_d xi_k b_eq; sum_k a_k (G_k - E2_k)
        for (int k = 0; k < D; ++k) {
            double q4 = 0.0;
            for (int m = 0; m < D; ++m) {
                int p[3] = {0, 0, 0};
                p[d] += 1;
                p[k] += 1;
                p[m] += 2;
                q4 += mom(p);
            }
            aB2 += P.accel[k] * (0.5 * q4 + cRT2 * E2[k]);
            aG += P.accel[k] * (Gp[k] - E2[k]);
        }
        accE = 0.25 * P.dt * aG + c * (aB2 - au * E3);
    }
    double ZG = -hu2 * Gm;
    for (int e = 0; e < D; ++e) ZG += q.u[e] * Gp[e];
    double Ge = (S[2 * D + 2] + betab * E3 + eta * (ZG - EZ) + accE) * ib;

    double* Go = P.G + (long long)d * (D + 2) * NE + f;
    Go[0] = Gm;
    for (int e = 0; e < D; ++e) Go[(long long)(1 + e) * NE] = Gp[e];
    Go[(long long)(D + 1) * NE] = Ge;

    double* F = P.FP + (long long)d * NFP * NE + f;
    F[PF_A * NE] = A;
    F[PF_INV2RT * NE] = inv2RT;
    F[PF_CRT2 * NE] = cRT2;
    F[PF_IG * NE] = ig;
    F[PF_IB * NE] = ib;
    F[PF_EB * NE] = eta * ib;
    F[PF_HU2 * NE] = hu2;
    for (int e = 0; e < 3; ++e) F[(PF_U0 + e) * NE] = q.u[e];
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
    double Wn[5], W0[5];
    for (int k = 0; k < D + 2; ++k) W0[k] = Wn[k] = P.W_in[k * N + c];
    for (int d = 0; d < D; ++d) {
        int rc[3] = {cc[0], cc[1], cc[2]};
        rc[d] += 1;
        if (P.bc[d] == 0 && rc[d] == P.n[d]) rc[d] = 0;
        long long fr = rc[0] + (long long)P.ne[0] * (rc[1] + (long long)P.ne[1] * rc[2]);
        const double* Gd = P.G + (long long)d * (D + 2) * NE;
        for (int k = 0; k < D + 2; ++k)
            Wn[k] -= P.dt * P.inv_dx[d] * (Gd[k * NE + fr] - Gd[k * NE + fl]);
    }
    if (P.has_accel) {
        // source integrals at t_n (eqs. rhouupdate, rhoEupdate): rho a, (rho u).a
        for (int e = 0; e < D; ++e) {
            Wn[1 + e] += P.dt * W0[0] * P.accel[e];
            Wn[D + 1] += P.dt * W0[1 + e] * P.accel[e];
        }
    }
    for (int k = 0; k < D + 2; ++k) P.W_out[k * N + c] = Wn[k];
    Prim q = primitives(P, Wn);
    if (q.bad) raise_error(P.err);
    write_cell_coefs(P, P.P_out, N, c, q);
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

}  // namespace cdg
