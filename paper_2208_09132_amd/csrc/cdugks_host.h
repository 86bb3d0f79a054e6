// Host-side internals of the CDUGKS library (contexts, byte plans).
#pragma once

#include <cstdarg>
#include <cstddef>
#include <vector>

#include "cdugks.h"
#include "cdugks_internal.h"

namespace cdg {

// Everything derived from the user's description of a problem.
struct Resolved {
    int D;
    int n[3], ne[3], bc[3], nv[3];
    int tiles1[3];      // face-sum tiles per dimension for the chosen shape
    int tiles1_def[3];  // ... and for shape 0 (the velocity-slice plan)
    int tile;           // face-sum tile shape (index into tile_shape(D, .))
    long long N, NE, V;
    double dx[3];
    double vmin[3], vmax[3];
    int quad;
    int storage;
    int recon;  // CDUGKS_RECON_*
    int nslices, nslices_upd;
    int relax;
    double dt, gamma, Pr, R, omega, K, c_int, mu_ref, T_ref, tau_inv;
    double rho_ref;     // reference density of a Knudsen-number relaxation (0 otherwise)
    // byte offsets inside the problem's device block
    size_t off_g[2], off_b[2], off_W[2], off_P[2];
    size_t off_q[2], off_dir, off_FV, off_FS, off_FP, off_G, off_vel, off_axis, off_err, off_scratch;
    size_t off_rows;      // BF16-tail form: row words [V]
    size_t bytes;
    long long fv_stride;  // elements between the (d, field) blocks of the face values
    long long pitch, fv_pitch;  // elements between velocity rows (state arrays, face values)
    double dir[3][2][5];  // Dirichlet states (rho, u_x, u_y, u_z, T) per dimension and side
    bool any_dirichlet;
    double accel[3];      // external acceleration (zero beyond D)
    bool has_accel;
};

// Steps per captured graph of a single context.
constexpr int ctx_chunk = 50;

int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
int resolve(const cdugks_space* sp, const cdugks_velocity* ve, const cdugks_params* pa,
            const double* rho, Resolved* out);
void resident_slots(int D, int storage, long long* R1, long long* R2);
void velocity_tables(const Resolved& r, std::vector<double>& vel, std::vector<double>& axis);
void dirichlet_tables(const Resolved& r, const std::vector<double>& vel, std::vector<double>& out);
void fill_problem(const Resolved& r, char* base, Problem& P);
long long tail_rows(const Resolved& r, const std::vector<double>& vel, const double* u, const double* T,
                    std::vector<long long>& rows);
void set_pingpong(Problem& P, const Resolved& r, char* base, int cur);
hipError_t enqueue_step(const Problem& P, hipStream_t s);
int tuned_update_slices(const Resolved& r);
int tuned_face_tile(const Resolved& r);
// Whether face-sum shape `tile` can serve this problem (exists for its
// dimension, fits the LDS for its storage form, default shape for problems
// with Dirichlet sides or the single-slope option, and launches on the
// current device when one is present).
bool face_tile_usable(const Resolved& r, int tile);
void set_face_tile(Resolved& r, int tile);

}  // namespace cdg

struct cdugks_ctx {
    cdg::Resolved r;
    cdg::Problem P;       // descriptor without the ping-pong pointers
    hipStream_t stream = nullptr;
    bool own_stream = false;  // created here when the caller passes NULL
    int device = 0;           // the device current at cdugks_init
    char* base = nullptr;
    bool own_memory = false;
    int cur = 0;          // buffer parity holding the current state
    int64_t steps = 0;
    double t0 = 0.0;      // simulated time at steps0 (a refit context starts at its source's)
    int64_t steps0 = 0;
    int sticky = 0;
    bool in_batch = false;
    long long bf16_rows = 0;  // BF16-tail form: velocity rows held in BF16
    hipGraphExec_t graph[2] = {nullptr, nullptr};
};
