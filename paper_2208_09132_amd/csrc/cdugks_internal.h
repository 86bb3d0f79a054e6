// Internal declarations shared by the kernels and the host side of the
// CDUGKS library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cdg {

// Per-cell coefficient set (structure of arrays, [NPC][N]), computed from W:
//   A      = rho (2 pi R T)^(-D/2)        Maxwellian prefactor (eq. geq)
//   INV2RT = 1 / (2 R T)
//   CRT2   = (3 - D + K) R T / 2           so b_eq = (|xi|^2/2 + CRT2) g_eq (eq. beq)
//   BETA   = (dt/4) / tau_g               = (h/2)/tau_g, h = dt/2
//   BETAB  = (dt/4) / tau_b
//   ETA    = (dt/4) / tau_bg              = (dt/4)(Pr - 1)/tau_g
//   HU2    = |u|^2 / 2
//   U0..U2 = bulk velocity
enum { PC_A = 0, PC_INV2RT, PC_CRT2, PC_BETA, PC_BETAB, PC_ETA, PC_HU2, PC_U0, NPC = PC_U0 + 3 };

// Per-face coefficient set ([D][NFP][NE]), computed from the face W:
//   A, INV2RT, CRT2, HU2, U0..U2 as above at the face, plus the inversion of
//   eq. phibar:  g = g_eq + IG (gbar - g_eq),
//                b = b_eq + IB (bbar - b_eq) + EB * Z * (g - g_eq)
enum { PF_A = 0, PF_INV2RT, PF_CRT2, PF_IG, PF_IB, PF_EB, PF_HU2, PF_U0, NFP = PF_U0 + 3 };

// Per-velocity constants ([V][NVEL]): xi, weight, |xi|^2/2, twice the
// Courant-like numbers, 2 lambda_d = dt xi_d / dx_d (the face value is
// assembled from half-scale slopes), the weighted products used by the
// face sums, w xi_e and w xi_d xi_e ([d][e], 3 x 3), and a . xi for the
// external acceleration a.
enum { VE_XI0 = 0, VE_W = 3, VE_HX2 = 4, VE_LAM0 = 5, VE_WXI0 = 8, VE_WXX = 11, VE_AX = 20, NVEL = 21 };

constexpr int MAX_NSUM = 9;  // 2D+3 face sums for D = 3
// threads per workgroup of the update and closure kernels (the per-problem
// thread ranges of batched closures start on multiples of it)
constexpr int WG = 256;

// Whether the update kernel also stores the next step's quarter-step fields
// phi_bar_plus (eq. phibarplus, from the new state and the new equilibrium it
// has at hand), so that the face-sum kernel loads them instead of evaluating
// the equilibrium on its whole halo box.  Done in 3-D, where that box is 5.9
// times the tile; in 1-D and 2-D (1.7 times) the extra 2 stores per update
// cost the update kernel about what the face-sum kernel saves.
constexpr bool quarter_stored(int D) { return D == 3; }

// Device-side description of one problem.  Pointers are device addresses.
struct Problem {
    int D;
    int storage;       // 0 = f64, 1 = f32, 2 = f32 with BF16 tail rows
    int nslices;       // velocity slices of the face-sum kernel (fixes the summation order)
    int nslices_upd;   // velocity slices of the update kernel (throughput only)
    int relax;         // 0: mu law, 1: constant tau
    int n[3];          // cells per dimension (1 when unused)
    int ne[3];         // extended (face) grid: n + 1 for outflow dims
    int bc[3];         // 0 periodic, 1 outflow, 2 Dirichlet
    int nv[3];
    int V;
    int tiles1[3];     // tiles per dimension over the face grid (face-sum kernel)
    long long N, NE;
    double dx[3], inv_dx[3];
    double dt, gamma, Pr, R, c_int, omega, mu_ref, T_ref, tau_inv;
    double hxi0;          // node spacing of velocity axis 0 (the fastest velocity index)
    const double* vel;    // [V][NVEL]
    const double* axis_xi;  // concatenated 1-D nodes, offsets 0, nv0, nv0+nv1
    const double* axis_w;   // concatenated 1-D weights
    // ping-pong state: *_in read, *_out written
    const void* g_in; const void* b_in; void* g_out; void* b_out;
    const double* W_in; double* W_out;
    const double* P_in; double* P_out;
    void* qg;     // quarter-step fields [V][pitch] for g and b, storage precision
    void* qb;     // (null unless quarter_stored(D))
    void* FV;     // face values phi_bar [D][2][fv_stride], block (d, field) holds [V][fv_pitch]
    long long fv_stride;  // >= V fv_pitch (padded so the blocks do not alias)
    long long pitch;      // elements between velocity rows of g, b and the quarter-step fields (>= N)
    long long fv_pitch;   // elements between velocity rows of a face-value block (>= NE)
    double* FS;   // face partial sums [nslices][D][2D+3][NE]
    double* FP;   // face coefficients [D][NFP][NE]
    double* G;    // flux moments [D][D+2][NE]
    int* err;     // sticky non-physical flag
    const double* dir_eq;  // Dirichlet ghosts: [2 d + side][V][g_eq, b_eq], or null
    // storage 2 (FP32 with BF16 tail rows): byte offset of each velocity row
    // inside the state arrays g, b and the quarter-step fields, bit 0 set for
    // a BF16 row; null otherwise
    const long long* rows;
    int recon;    // 0: slopes of slopes (Sec. 2.1), 1: single slope
    int tile;     // face-sum tile shape (index into tile_shape(D, .))
    int has_accel;     // external acceleration present (a != 0)
    double accel[3];   // external acceleration a (eqs. gPDE, bPDE)
};

// One workgroup's assignment in a batched launch.
struct WorkItem {
    int prob;     // index into the problem table
    int tile;     // face sums: linear tile index; update: block of 256 cells
    int slice;    // velocity slice
    int nslices;  // update items: the problem's velocity slices in this batch (face items: unused)
};

// Launchers (stream-ordered).  Single-problem forms take the descriptor by
// value; batched forms read descriptors and items from device memory.
hipError_t launch_init(const Problem& P, const double* rho, const double* u, const double* T,
                       hipStream_t s);
hipError_t launch_face_sums(const Problem& P, hipStream_t s);
// per dimension (one translation unit each)
hipError_t launch_face_sums_d1(const Problem& P, hipStream_t s);
hipError_t launch_face_sums_d2(const Problem& P, hipStream_t s);
hipError_t launch_face_sums_d3(const Problem& P, hipStream_t s);
// Resident workgroups per CU of the single-problem face-sum kernel of shape
// `tile` (0 when that shape does not exist for the storage form or no device
// answers).
int face_sum_blocks_per_cu(int D, int storage, int tile);
int face_sum_blocks_per_cu_d1(int storage, int tile);
int face_sum_blocks_per_cu_d2(int storage, int tile);
int face_sum_blocks_per_cu_d3(int storage, int tile);
// Resident workgroups per CU of the batched face-sum kernel of a class.
int batched_face_blocks_per_cu(int maxd, int storage, bool accel);
// Velocity-grid refit: Pn (holding the carried W) takes Po's distributions
// on its own velocity grid; same cells and storage form.
hipError_t launch_regrid(const Problem& Pn, const Problem& Po, hipStream_t s);
hipError_t launch_face_close(const Problem& P, hipStream_t s);
hipError_t launch_cell_close(const Problem& P, hipStream_t s);
hipError_t launch_update(const Problem& P, hipStream_t s);
hipError_t launch_moments(const Problem& P, const double* W, double* rho, double* u, double* T,
                          hipStream_t s);
// velocity rows [row0, row0 + nrows) of a state array as FP64 into dst[nrows][N]
hipError_t launch_to_f64(const Problem& P, const void* src, int row0, int nrows, double* dst, hipStream_t s);

// Batched: one launch per phase across problems of one class (storage,
// whether they have Dirichlet sides, the reconstruction option and whether
// they have an external acceleration, which select the kernel variants).  The
// tile-kernel launches are persistent (grid = resident slots; workgroups take
// items from the device counter `queue`, which must be 0 at launch, and reset
// the counter `other` of the other kernel of the pair); maxd is the largest
// dimension in the class.  The per-face and per-cell closures take
// per-problem prefix offsets (in threads).
hipError_t launch_face_sums_batched(const Problem* probs, const WorkItem* items, int nitems, int grid,
                                    int maxd, int storage, bool dirichlet, bool single_slope, bool accel,
                                    int* queue, int* other, hipStream_t s);
hipError_t launch_update_batched(const Problem* probs, const WorkItem* items, int nitems, int grid, int maxd,
                                 int storage, bool accel, int* queue, int* other, hipStream_t s);
int batched_blocks_per_cu(int maxd, int storage, bool accel, bool update);
hipError_t launch_face_close_batched(const Problem* probs, const long long* offsets, int nprob,
                                     long long total, hipStream_t s);
hipError_t launch_cell_close_batched(const Problem* probs, const long long* offsets, int nprob,
                                     long long total, hipStream_t s);

// Resident workgroups per CU of the face-sum (update = false) or update kernel
// (0 when no device answers).
int tile_blocks_per_cu(int D, int storage, bool update);

// Face-sum tile shapes: cells per workgroup along x, y, z, one thread per
// cell.  Shape 0 of each dimension plans the velocity split;
// batched_face_tile(D, storage) is the shape of batched launches and
// default_face_tile(D) the one a single problem runs
// unless the caller (cdugks_params.face_tile) or the autotuner chooses
// another.  A cell's arithmetic does not depend on the tile it sits in (in
// 2-D every shape keeps its q-box slots in registers, see Geo), and the
// velocity split is planned with shape 0, so every shape gives bitwise the
// same result.  Shapes wider along x use more of each 128-byte line of a halo
// row; shapes of 768 cells stage larger boxes per workgroup (less halo per
// cell).
// 3-D shapes with z = 0 are z-marching columns: a workgroup of x * y threads
// owns an x * y column of the face grid for one velocity and walks it along
// z (ZMarch in cdugks_device.h), so each staged plane serves the three planes
// of faces that need it instead of being staged again by the tile above.
struct TileExt {
    int x, y, z;
};
constexpr int MAX_TILE_SHAPES = 9;
constexpr int tile_shape_count(int D) { return D == 1 ? 1 : (D == 2 ? 4 : 9); }
constexpr TileExt tile_shape(int D, int id) {
    if (D == 1) return TileExt{256, 1, 1};
    if (D == 2) {
        switch (id) {
        case 1: return TileExt{32, 8, 1};
        case 2: return TileExt{8, 32, 1};
        case 3: return TileExt{32, 24, 1};
        default: return TileExt{16, 16, 1};
        }
    }
    switch (id) {
    case 1: return TileExt{32, 4, 2};
    case 2: return TileExt{64, 2, 2};
    case 3: return TileExt{32, 6, 4};
    case 4: return TileExt{64, 4, 3};
    case 5: return TileExt{16, 8, 6};
    case 6: return TileExt{16, 16, 0};
    case 7: return TileExt{32, 8, 0};
    case 8: return TileExt{32, 16, 0};
    default: return TileExt{16, 4, 4};
    }
}
constexpr bool tile_zmarch(int D, int id) { return D == 3 && tile_shape(D, id).z == 0; }
// Tile shape of batched face-sum launches.  The FP32 forms of 2-D problems
// take 32 x 8: a 16-wide tile row of FP32 face values or fields is half a
// 128-byte line, whose other half belongs to a tile that in a batch seldom
// runs beside it on the same XCD, so half of each line fetched would be
// wasted.  Every shape gives the same results.
constexpr int batched_face_tile(int D, int storage) { return D == 2 && storage != 0 ? 1 : 0; }
constexpr int default_face_tile(int D) { return D == 3 ? 6 : 0; }
constexpr int tile_threads(int D, int id) {
    return tile_shape(D, id).x * tile_shape(D, id).y * (tile_zmarch(D, id) ? 1 : tile_shape(D, id).z);
}
// Static LDS of a face-sum workgroup (element size es of the stencil
// arithmetic).  Box shapes: q box (plus one entry for unused slots) and
// limited-difference box for g and b, double-buffered in 1-D and 2-D.  z-marching columns: a ring of four q
// planes and a ring of two planes of the three limited differences.  Shapes
// whose LDS exceeds the 160 KB of a CU do not exist for that storage form.
constexpr long long face_sum_lds_bytes(int D, int id, int es) {
    const TileExt t = tile_shape(D, id);
    const long long qx = t.x + 5, qy = D >= 2 ? t.y + 5 : 1, qz = D >= 3 ? t.z + 5 : 1;
    const long long ax = t.x + 3, ay = D >= 2 ? t.y + 3 : 1, az = D >= 3 ? t.z + 3 : 1;
    if (tile_zmarch(D, id)) return 2LL * es * (4 * qx * qy + 2 * 3 * ax * ay);
    const long long nbuf = D <= 2 ? 2 : 1;
    return nbuf * 2 * es * (qx * qy * qz + 1 + D * ax * ay * az);
}
constexpr long long LDS_PER_CU = 160 * 1024;
constexpr bool face_tile_fits(int D, int id, int es) { return face_sum_lds_bytes(D, id, es) <= LDS_PER_CU; }

}  // namespace cdg
