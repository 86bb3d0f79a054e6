// Single-problem face-sum kernels of one dimension, every tile shape and
// storage form.  The build compiles this file once per dimension
// (CDG_FACE_DIM = 1, 2, 3), in parallel with the other translation units.
// Shape 0 and the dimension's default shape take every problem (Dirichlet
// sides, the single-slope option and an external acceleration select the
// kernel); the other shapes exist for problems without Dirichlet sides or
// external acceleration that use the paper's reconstruction, and the host
// selects them only for those.  In 3-D the quarter-step fields are loaded,
// already holding an acceleration's source terms, so the face-sum kernels
// take no acceleration variant there.
#include "cdugks_device.h"

#ifndef CDG_FACE_DIM
#error "compile with CDG_FACE_DIM = 1, 2 or 3"
#endif

#define CDG_CAT2(a, b) a##b
#define CDG_CAT(a, b) CDG_CAT2(a, b)

namespace cdg {
namespace {

constexpr int FD = CDG_FACE_DIM;

template <typename ST, int TID>
hipError_t by_shape(const Problem& P, hipStream_t s) {
    if constexpr (TID < tile_shape_count(FD)) {
        if (P.tile == TID) {
            if constexpr (tile_zmarch(FD, TID)) return launch_face_sums_zmarch<ST, false, false, TID>(P, s);
            else return launch_face_sums_shape<FD, ST, false, false, TID>(P, s);
        }
        return by_shape<ST, TID + 1>(P, s);
    } else {
        return hipErrorInvalidValue;
    }
}

// Dirichlet sides (DIR) and the single-slope option (SS) on shape 0 or on the
// dimension's default shape.
template <typename ST, bool DIR, bool SS>
hipError_t variant(const Problem& P, hipStream_t s) {
    constexpr int TD = default_face_tile(FD);
    if (P.tile == 0) return launch_face_sums_shape<FD, ST, DIR, SS, 0>(P, s);
    if constexpr (tile_zmarch(FD, TD)) {
        if (P.tile == TD) return launch_face_sums_zmarch<ST, DIR, SS, TD>(P, s);
    }
    return hipErrorInvalidValue;
}

template <typename ST>
hipError_t launch_storage(const Problem& P, hipStream_t s) {
    if (P.has_accel && FD <= 2) {
        // external acceleration (1-D, 2-D): shape 0, the paper's reconstruction
        if (P.tile != 0 || P.recon) return hipErrorInvalidValue;
        return P.dir_eq ? launch_face_sums_shape<FD, ST, true, false, 0, true>(P, s)
                        : launch_face_sums_shape<FD, ST, false, false, 0, true>(P, s);
    }
    if (P.dir_eq) return P.recon ? variant<ST, true, true>(P, s) : variant<ST, true, false>(P, s);
    if (P.recon) return variant<ST, false, true>(P, s);
    if (P.has_accel && P.tile != 0 && P.tile != default_face_tile(FD)) return hipErrorInvalidValue;
    return by_shape<ST, 0>(P, s);
}

template <typename ST, int TID>
int occupancy_by_shape(int tile) {
    if constexpr (TID < tile_shape_count(FD)) {
        if (tile == TID) {
            if constexpr (tile_zmarch(FD, TID)) return face_values_z_occupancy<ST, TID>();
            else return face_sum_occupancy_shape<FD, ST, TID>();
        }
        return occupancy_by_shape<ST, TID + 1>(tile);
    } else {
        return 0;
    }
}

}  // namespace

hipError_t CDG_CAT(launch_face_sums_d, CDG_FACE_DIM)(const Problem& P, hipStream_t s) {
    if (P.storage == 0) return launch_storage<double>(P, s);
    if (P.storage == 1) return launch_storage<float>(P, s);
    return launch_storage<Bf16Tail>(P, s);
}

int CDG_CAT(face_sum_blocks_per_cu_d, CDG_FACE_DIM)(int storage, int tile) {
    if (storage == 0) return occupancy_by_shape<double, 0>(tile);
    if (storage == 1) return occupancy_by_shape<float, 0>(tile);
    return occupancy_by_shape<Bf16Tail, 0>(tile);
}

}  // namespace cdg
