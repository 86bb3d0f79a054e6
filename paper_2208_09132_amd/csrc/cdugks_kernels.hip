// HIP kernels of one CDUGKS time step for gfx950.
//
// Data layout (per problem):
//   g, b        [V][pitch]  velocity-major, cells fastest (x fastest); FP64 or
//               FP32; rows of pitch >= N elements (padded so that large rows
//               do not sit at power-of-two distances)
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
//                              stored per (face, velocity), and per-face velocity
//                              sums -> partial sums per slice
//   face_close (per face)    : face W (eqs. rhobar..rhoEbar), face equilibrium and
//                              relaxation, inversion coefficients (eq. phibar), and
//                              the flux moments in closed form
//   cell_close (per cell)    : W^{n+1} from the flux moments (eqs. rhoupdate..
//                              rhoEupdate, outward-flux sign), cell coefficients at n+1
//   update     (streaming)   : stored face values, inversion (eq. phibar),
//                              microflux (eq. flux) and phi^{n+1} (eq. phiupdate)
//
// Face sums: one thread per cell of a 256-cell tile; the thread loops over
// its slice of discrete velocities, so the velocity sums are serial per
// thread (no atomics, fixed order).  For each velocity the tile and its halo
// of phi_bar_plus and of the limited slopes are staged in LDS.  The face
// values phi_bar (velocity-major [d][g|b][V][NE]) are written once and read
// by the update, which therefore needs no stencil and no halo.
#include "cdugks_device.h"

namespace cdg {

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
    state_st<ST, false>(P, const_cast<void*>(P.g_in), (int)i, c, geq);
    state_st<ST, false>(P, const_cast<void*>(P.b_in), (int)i, c, beq);
}



// Quarter-step fields of the initial state (when they are stored): the same
// arithmetic the update kernel applies to each new state.
template <int D, typename ST>
__global__ __launch_bounds__(256) void k_init_quarter(Problem P) {
    long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long N = P.N;
    if (idx >= N * P.V) return;
    const long long i = idx / N, c = idx - i * N;
    const CellCoef k = load_coef(P.P_in, N, c);
    const Vel v = load_vel(P.vel, (int)i);
    double c2 = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const double x = v.xi[d] - k.u[d];
        c2 += x * x;
    }
    const double geq = k.A * exp(-c2 * k.inv2RT);
    double qg, qb;
    const double g = state_ld<ST>(P, P.g_in, (int)i, c), b = state_ld<ST>(P, P.b_in, (int)i, c);
    if (P.has_accel) quarter_step_eq<D, true>(k, v, geq, g, b, qg, qb, &P);
    else quarter_step_eq<D>(k, v, geq, g, b, qg, qb);
    state_st<ST, false>(P, P.qg, (int)i, c, qg);
    state_st<ST, false>(P, P.qb, (int)i, c, qb);
}



// ---------------------------------------------------------------------------
// Velocity-grid refit (an adaptive velocity grid; Sec. 5 names the idea).
// The new problem Pn already holds the carried W.  k_cell_coefs sets its cell
// coefficient sets from that W (with the new problem's dt); k_regrid writes,
// per (new velocity, cell), phi_eq of the cell's W at the new node plus the
// old problem's (Po) phi - phi_eq interpolated multilinearly between the old
// nodes, zero outside the old velocity box.  Threads run velocity-major over
// the cells, so the loads of one old node and the stores of one new node are
// coalesced rows.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(WG) void k_cell_coefs(Problem P) {
    const long long c = (long long)blockIdx.x * WG + threadIdx.x;
    if (c >= P.N) return;
    double Wv[5];
    for (int k = 0; k < P.D + 2; ++k) Wv[k] = P.W_in[k * P.N + c];
    const Prim q = primitives(P, Wv);
    if (q.bad) raise_error(P.err);
    write_cell_coefs(P, const_cast<double*>(P.P_in), P.N, c, q);
}

template <int D, typename ST>
__global__ __launch_bounds__(WG) void k_regrid(Problem Pn, Problem Po) {
    const long long idx = (long long)blockIdx.x * WG + threadIdx.x;
    const long long N = Pn.N;
    if (idx >= N * Pn.V) return;
    const long long i = idx / N, c = idx - i * N;
    const CellCoef k = load_coef(Pn.P_in, N, c);
    const double* ve = Pn.vel + i * NVEL;
    double xi[3] = {0.0, 0.0, 0.0};
    double c2 = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        xi[d] = ve[VE_XI0 + d];
        const double x = xi[d] - k.u[d];
        c2 += x * x;
    }
    const double geq = k.A * exp(-c2 * k.inv2RT);
    const double beq = (ve[VE_HX2] + k.cRT2) * geq;
    // the old grid's cell holding xi, and the weights along each axis
    bool inside = true;
    int m[3] = {0, 0, 0}, off[3] = {0, 0, 0};
    double t[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int d = 0; d < D; ++d) {
        off[d] = d == 0 ? 0 : off[d - 1] + Po.nv[d - 1];
        const double* ax = Po.axis_xi + off[d];
        const int nvo = Po.nv[d];
        const double lo = ax[0], hi = ax[nvo - 1], h = ax[1] - ax[0];
        if (!(xi[d] >= lo && xi[d] <= hi)) {
            inside = false;
        } else {
            int kk = (int)floor((xi[d] - lo) / h);
            kk = kk > nvo - 2 ? nvo - 2 : (kk < 0 ? 0 : kk);
            m[d] = kk;
            t[d] = (xi[d] - ax[kk]) / h;
        }
    }
    double dg = 0.0, db = 0.0;
    if (inside) {
        for (int corner = 0; corner < (1 << D); ++corner) {
            double wgt = 1.0, co2 = 0.0, xo2 = 0.0;
            long long io = 0, stride = 1;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const int up = (corner >> d) & 1;
                wgt *= up ? t[d] : 1.0 - t[d];
                const int mo = m[d] + up;
                io += mo * stride;
                stride *= Po.nv[d];
                const double xo = Po.axis_xi[off[d] + mo];
                const double x = xo - k.u[d];
                co2 += x * x;
                xo2 += xo * xo;
            }
            const double ge = k.A * exp(-co2 * k.inv2RT);
            const double be = (0.5 * xo2 + k.cRT2) * ge;
            dg += wgt * (state_ld<ST>(Po, Po.g_in, (int)io, c) - ge);
            db += wgt * (state_ld<ST>(Po, Po.b_in, (int)io, c) - be);
        }
    }
    state_st<ST, false>(Pn, const_cast<void*>(Pn.g_in), (int)i, c, geq + dg);
    state_st<ST, false>(Pn, const_cast<void*>(Pn.b_in), (int)i, c, beq + db);
}

// update grid: blocks of 256 consecutive cells x velocity slices
template <int D, typename ST, bool ACC = false, int ROWS = 0>
__global__ __launch_bounds__(WG, 2) void k_update(Problem P) {
    const int nblk = (int)((P.N + WG - 1) / WG);
    int q = xcd_remap(blockIdx.x, gridDim.x);
    int blk = q % nblk, slice = q / nblk;
    UpdateKernel<D, ST, ACC, ROWS>::run(P, (long long)blk * WG + threadIdx.x, slice, P.nslices_upd);
}

// ACC: the class's problems have an external acceleration
template <typename ST, int MAXD, bool ACC>
__global__ __launch_bounds__(WG) void k_update_batched(const Problem* probs, const WorkItem* items, int nitems,
                                                       int* queue, int* other) {
    __shared__ int slot;
    if (blockIdx.x == 0 && threadIdx.x == 0) *other = 0;
    for (int w = next_item(queue, &slot); w < nitems; w = next_item(queue, &slot)) {
        const WorkItem it = load_uniform(items + w);
        const Problem P = load_uniform(probs + it.prob);
        const long long c = (long long)it.tile * WG + threadIdx.x;
        if (P.D == 1) UpdateKernel<1, ST, ACC>::run(P, c, it.slice, it.nslices);
        else if (MAXD >= 2 && P.D == 2) UpdateKernel<MAXD >= 2 ? 2 : 1, ST, ACC>::run(P, c, it.slice, it.nslices);
        else if (MAXD >= 3) UpdateKernel<MAXD >= 3 ? 3 : 1, ST, ACC>::run(P, c, it.slice, it.nslices);
    }
}

__global__ __launch_bounds__(WG) void k_face_close(Problem P) {
    face_close_one(P, (long long)blockIdx.x * WG + threadIdx.x);
}

__global__ __launch_bounds__(WG) void k_cell_close(Problem P) {
    cell_close_one(P, (long long)blockIdx.x * WG + threadIdx.x);
}


// Batched closures: every problem's range of threads starts on a workgroup
// boundary (offsets in threads, multiples of WG), so a workgroup serves one
// problem, found once per workgroup (its descriptor then read at one address
// by every lane); threads past the problem's faces (cells) return.
__global__ __launch_bounds__(WG) void k_face_close_batched(const Problem* probs, const long long* offsets,
                                                           int nprob, long long total) {
    const long long g0 = (long long)blockIdx.x * WG;
    if (g0 >= total) return;
    const int p = __builtin_amdgcn_readfirstlane(find_problem(offsets, nprob, g0));
    face_close_one(probs[p], g0 - offsets[p] + threadIdx.x);  // by reference: no private copy
}

__global__ __launch_bounds__(WG) void k_cell_close_batched(const Problem* probs, const long long* offsets,
                                                           int nprob, long long total) {
    const long long g0 = (long long)blockIdx.x * WG;
    if (g0 >= total) return;
    const int p = __builtin_amdgcn_readfirstlane(find_problem(offsets, nprob, g0));
    cell_close_one(probs[p], g0 - offsets[p] + threadIdx.x);
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

// velocity rows [row0, row0 + nrows) of a state array ([V][N] in the
// problem's storage form) as FP64, dst[nrows][N]
template <typename ST>
__global__ __launch_bounds__(WG) void k_to_f64(Problem P, const void* src, int row0, int nrows, double* dst) {
    const long long idx = (long long)blockIdx.x * WG + threadIdx.x;
    if (idx >= P.N * nrows) return;
    const long long i = idx / P.N;
    dst[idx] = state_ld<ST>(P, src, row0 + (int)i, idx - i * P.N);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(long long n) { return (unsigned)((n + WG - 1) / WG); }



#define CDG_DISPATCH(STORAGE, DIM, MACRO)                            \
    do {                                                             \
        if ((STORAGE) == 0) {                                        \
            if ((DIM) == 1) MACRO(1, double);                        \
            else if ((DIM) == 2) MACRO(2, double);                   \
            else MACRO(3, double);                                   \
        } else if ((STORAGE) == 1) {                                 \
            if ((DIM) == 1) MACRO(1, float);                         \
            else if ((DIM) == 2) MACRO(2, float);                    \
            else MACRO(3, float);                                    \
        } else {                                                     \
            if ((DIM) == 1) MACRO(1, Bf16Tail);                      \
            else if ((DIM) == 2) MACRO(2, Bf16Tail);                 \
            else MACRO(3, Bf16Tail);                                 \
        }                                                            \
    } while (0)

hipError_t launch_init(const Problem& P, const double* rho, const double* u, const double* T,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_init_cells, dim3(blocks_for(P.N)), dim3(WG), 0, s, P, rho, u, T);
    const dim3 gphi(blocks_for(P.N * P.V));
    if (P.storage == 0) hipLaunchKernelGGL(k_init_phi<double>, gphi, dim3(WG), 0, s, P);
    else if (P.storage == 1) hipLaunchKernelGGL(k_init_phi<float>, gphi, dim3(WG), 0, s, P);
    else hipLaunchKernelGGL(k_init_phi<Bf16Tail>, gphi, dim3(WG), 0, s, P);
    if (quarter_stored(P.D)) {
        const dim3 grid(blocks_for(P.N * P.V));
#define CDG_L(D, ST) hipLaunchKernelGGL((k_init_quarter<D, ST>), grid, dim3(256), 0, s, P)
        CDG_DISPATCH(P.storage, P.D, CDG_L);
#undef CDG_L
    }
    return hipGetLastError();
}

hipError_t launch_regrid(const Problem& Pn, const Problem& Po, hipStream_t s) {
    hipLaunchKernelGGL(k_cell_coefs, dim3(blocks_for(Pn.N)), dim3(WG), 0, s, Pn);
    const dim3 grid(blocks_for(Pn.N * Pn.V));
#define CDG_L(D, ST) hipLaunchKernelGGL((k_regrid<D, ST>), grid, dim3(WG), 0, s, Pn, Po)
    CDG_DISPATCH(Pn.storage, Pn.D, CDG_L);
#undef CDG_L
    if (quarter_stored(Pn.D)) {
#define CDG_L(D, ST) hipLaunchKernelGGL((k_init_quarter<D, ST>), grid, dim3(256), 0, s, Pn)
        CDG_DISPATCH(Pn.storage, Pn.D, CDG_L);
#undef CDG_L
    }
    return hipGetLastError();
}

hipError_t launch_face_sums(const Problem& P, hipStream_t s) {
    if (P.D == 1) return launch_face_sums_d1(P, s);
    if (P.D == 2) return launch_face_sums_d2(P, s);
    return launch_face_sums_d3(P, s);
}

int face_sum_blocks_per_cu(int D, int storage, int tile) {
    if (D == 1) return face_sum_blocks_per_cu_d1(storage, tile);
    if (D == 2) return face_sum_blocks_per_cu_d2(storage, tile);
    return face_sum_blocks_per_cu_d3(storage, tile);
}

hipError_t launch_update(const Problem& P, hipStream_t s) {
    unsigned nb = (unsigned)(((P.N + WG - 1) / WG) * P.nslices_upd);
    if (P.storage == 2 && P.D == 3) {
        // 3-D BF16-tail form: the FP32 rows, then the BF16 rows, as two
        // launches (each (cell, velocity) is updated on its own, so the split
        // is free).  With both in one kernel the 3-D update sat at the
        // register limit and its face-value loads were serialised (37.8 ->
        // 17.4 ms per launch with the split); in 1-D and 2-D one kernel is
        // faster (KH: 0.57 ms against 0.73 ms for the two launches).
#define CDG_L2(DD, AC)                                                                       \
    do {                                                                                     \
        hipLaunchKernelGGL((k_update<DD, Bf16Tail, AC, 1>), dim3(nb), dim3(WG), 0, s, P);    \
        hipLaunchKernelGGL((k_update<DD, Bf16Tail, AC, 2>), dim3(nb), dim3(WG), 0, s, P);    \
    } while (0)
        if (P.has_accel) CDG_L2(3, true);
        else CDG_L2(3, false);
#undef CDG_L2
        return hipGetLastError();
    }
    if (P.has_accel) {
#define CDG_L(DD, TT) hipLaunchKernelGGL((k_update<DD, TT, true>), dim3(nb), dim3(WG), 0, s, P)
        CDG_DISPATCH(P.storage, P.D, CDG_L);
#undef CDG_L
    } else {
#define CDG_L(DD, TT) hipLaunchKernelGGL((k_update<DD, TT>), dim3(nb), dim3(WG), 0, s, P)
        CDG_DISPATCH(P.storage, P.D, CDG_L);
#undef CDG_L
    }
    return hipGetLastError();
}

int tile_blocks_per_cu(int D, int storage, bool update) {
    if (!update) return face_sum_blocks_per_cu(D, storage, 0);
    int n = 0;
    hipError_t e = hipSuccess;
#define CDG_L(DD, TT) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (k_update<DD, TT>), WG, 0)
    CDG_DISPATCH(storage, D, CDG_L);
#undef CDG_L
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return n;
}

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

hipError_t launch_to_f64(const Problem& P, const void* src, int row0, int nrows, double* dst, hipStream_t s) {
    if (row0 < 0 || nrows <= 0 || row0 + nrows > P.V) return hipErrorInvalidValue;
    const dim3 grid(blocks_for(P.N * nrows));
    if (P.storage == 0) hipLaunchKernelGGL(k_to_f64<double>, grid, dim3(WG), 0, s, P, src, row0, nrows, dst);
    else if (P.storage == 1) hipLaunchKernelGGL(k_to_f64<float>, grid, dim3(WG), 0, s, P, src, row0, nrows, dst);
    else hipLaunchKernelGGL(k_to_f64<Bf16Tail>, grid, dim3(WG), 0, s, P, src, row0, nrows, dst);
    return hipGetLastError();
}

#define CDG_DISPATCH_MAXD(STORAGE, MAXD, MACRO)                      \
    do {                                                             \
        if ((STORAGE) == 0) {                                        \
            if ((MAXD) == 1) MACRO(double, 1);                       \
            else if ((MAXD) == 2) MACRO(double, 2);                  \
            else MACRO(double, 3);                                   \
        } else if ((STORAGE) == 1) {                                 \
            if ((MAXD) == 1) MACRO(float, 1);                        \
            else if ((MAXD) == 2) MACRO(float, 2);                   \
            else MACRO(float, 3);                                    \
        } else {                                                     \
            if ((MAXD) == 1) MACRO(Bf16Tail, 1);                     \
            else if ((MAXD) == 2) MACRO(Bf16Tail, 2);                \
            else MACRO(Bf16Tail, 3);                                 \
        }                                                            \
    } while (0)

hipError_t launch_update_batched(const Problem* probs, const WorkItem* items, int nitems, int grid, int maxd,
                                 int storage, bool accel, int* queue, int* other, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    if (accel) {
#define CDG_L(TT, MD)                                                                                          \
    hipLaunchKernelGGL((k_update_batched<TT, MD, true>), dim3(grid), dim3(WG), 0, s, probs, items, nitems, queue, \
                       other)
        CDG_DISPATCH_MAXD(storage, maxd, CDG_L);
#undef CDG_L
    } else {
#define CDG_L(TT, MD)                                                                                           \
    hipLaunchKernelGGL((k_update_batched<TT, MD, false>), dim3(grid), dim3(WG), 0, s, probs, items, nitems, queue, \
                       other)
        CDG_DISPATCH_MAXD(storage, maxd, CDG_L);
#undef CDG_L
    }
    return hipGetLastError();
}

int batched_blocks_per_cu(int maxd, int storage, bool accel, bool update) {
    if (!update) return batched_face_blocks_per_cu(maxd, storage, accel);
    int n = 0;
    hipError_t e = hipSuccess;
    if (accel) {
#define CDG_L(TT, MD) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (k_update_batched<TT, MD, true>), WG, 0)
        CDG_DISPATCH_MAXD(storage, maxd, CDG_L);
#undef CDG_L
    } else {
#define CDG_L(TT, MD) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (k_update_batched<TT, MD, false>), WG, 0)
        CDG_DISPATCH_MAXD(storage, maxd, CDG_L);
#undef CDG_L
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return n;
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