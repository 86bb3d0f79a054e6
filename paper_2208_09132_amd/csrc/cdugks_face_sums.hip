// Single-problem face-sum kernels of one dimension, every tile shape and
// storage form.  The build compiles this file once per dimension
// (CDG_FACE_DIM = 1, 2, 3), in parallel with the other translation units.
// Shapes other than the default exist for problems without Dirichlet sides
// or external acceleration that use the paper's reconstruction; the host
// selects only those.  Problems with an external acceleration run the
// paper's reconstruction only.
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
        if (P.tile == TID) return launch_face_sums_shape<FD, ST, false, false, TID>(P, s);
        return by_shape<ST, TID + 1>(P, s);
    } else {
        return hipErrorInvalidValue;
    }
}

template <typename ST>
hipError_t launch_storage(const Problem& P, hipStream_t s) {
    if (P.has_accel) {
        // external acceleration: default shape, the paper's reconstruction
        if (P.tile != 0 || P.recon) return hipErrorInvalidValue;
        return P.dir_eq ? launch_face_sums_shape<FD, ST, true, false, 0, true>(P, s)
                        : launch_face_sums_shape<FD, ST, false, false, 0, true>(P, s);
    }
    if (P.dir_eq || P.recon) {
        if (P.tile != 0) return hipErrorInvalidValue;
        if (P.dir_eq)
            return P.recon ? launch_face_sums_shape<FD, ST, true, true, 0>(P, s)
                           : launch_face_sums_shape<FD, ST, true, false, 0>(P, s);
        return launch_face_sums_shape<FD, ST, false, true, 0>(P, s);
    }
    return by_shape<ST, 0>(P, s);
}

template <typename ST, int TID>
int occupancy_by_shape(int tile) {
    if constexpr (TID < tile_shape_count(FD)) {
        if (tile == TID) return face_sum_occupancy_shape<FD, ST, TID>();
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
