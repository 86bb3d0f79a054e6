// Batched face-sum kernels: one persistent launch per class over a device
// work list that covers every tile of every problem of the class.
#include "cdugks_device.h"

namespace cdg {

// waves per SIMD the batched face sums are compiled for: 3 for the FP32
// forms of 1-D and 2-D classes, like the single-problem 2-D kernel
template <typename ST, int MAXD>
constexpr int batched_face_waves() { return MAXD <= 2 && !std::is_same<ST, double>::value ? 3 : 1; }

// ACC: the class's problems have an external acceleration (stage 1 of the
// 1-D and 2-D face sums adds its source; 3-D problems load quarter-step
// fields that already carry it)
template <typename ST, int MAXD, bool DIR, bool SS, bool ACC>
__global__ __launch_bounds__(WG, (batched_face_waves<ST, MAXD>())) void k_face_sums_batched(const Problem* probs, const WorkItem* items, int nitems,
                                                          int* queue, int* other) {
    // 2-D problems in the batched tile shape of the storage form
    constexpr int T2 = MAXD >= 2 ? batched_face_tile(2, std::is_same<ST, double>::value ? 0 : 1) : 0;
    using K1 = FaceSumKernel<1, ST, DIR, SS, 0, ACC>;
    using K2 = FaceSumKernel<MAXD >= 2 ? 2 : 1, ST, DIR, SS, T2, ACC>;
    using K3 = FaceSumKernel<MAXD >= 3 ? 3 : 1, ST, DIR, SS>;
    __shared__ union U {
        typename K1::Smem s1;
        typename K2::Smem s2;
        typename K3::Smem s3;
    } sm;
    __shared__ int slot;
    if (blockIdx.x == 0 && threadIdx.x == 0) *other = 0;
    for (int w = next_item(queue, &slot); w < nitems; w = next_item(queue, &slot)) {
        const WorkItem it = load_uniform(items + w);
        const Problem P = load_uniform(probs + it.prob);
        if (P.D == 1) K1::run(P, it.tile, it.slice, P.nslices, sm.s1);
        else if (MAXD >= 2 && P.D == 2) K2::run(P, it.tile, it.slice, P.nslices, sm.s2);
        else if (MAXD >= 3) K3::run(P, it.tile, it.slice, P.nslices, sm.s3);
    }
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

hipError_t launch_face_sums_batched(const Problem* probs, const WorkItem* items, int nitems, int grid,
                                    int maxd, int storage, bool dirichlet, bool single_slope, bool accel,
                                    int* queue, int* other, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
#define CDG_B(DIRV, SSV, ACCV)                                                                               \
    do {                                                                                                     \
        if ((STORAGE_) == 0) {                                                                               \
            if (maxd == 1) CDG_LB(double, 1, DIRV, SSV, ACCV);                                                     \
            else if (maxd == 2) CDG_LB(double, 2, DIRV, SSV, ACCV);                                                \
            else CDG_LB(double, 3, DIRV, SSV, ACCV);                                                               \
        } else if ((STORAGE_) == 1) {                                                                        \
            if (maxd == 1) CDG_LB(float, 1, DIRV, SSV, ACCV);                                                      \
            else if (maxd == 2) CDG_LB(float, 2, DIRV, SSV, ACCV);                                                 \
            else CDG_LB(float, 3, DIRV, SSV, ACCV);                                                                \
        } else {                                                                                             \
            if (maxd == 1) CDG_LB(Bf16Tail, 1, DIRV, SSV, ACCV);                                                   \
            else if (maxd == 2) CDG_LB(Bf16Tail, 2, DIRV, SSV, ACCV);                                              \
            else CDG_LB(Bf16Tail, 3, DIRV, SSV, ACCV);                                                             \
        }                                                                                                    \
    } while (0)
#define CDG_LB(TT, MD, DIRV, SSV, ACCV)                                                                      \
    hipLaunchKernelGGL((k_face_sums_batched<TT, MD, DIRV, SSV, ACCV>), dim3(grid), dim3(WG), 0, s, probs,   \
                       items, nitems, queue, other)
#define STORAGE_ storage
    // the acceleration never comes with the single-slope option (refused at
    // problem set-up)
    if (dirichlet) {
        if (single_slope) CDG_B(true, true, false);
        else if (accel) CDG_B(true, false, true);
        else CDG_B(true, false, false);
    } else {
        if (single_slope) CDG_B(false, true, false);
        else if (accel) CDG_B(false, false, true);
        else CDG_B(false, false, false);
    }
#undef STORAGE_
#undef CDG_LB
#undef CDG_B
    return hipGetLastError();
}

int batched_face_blocks_per_cu(int maxd, int storage, bool accel) {
    int n = 0;
    hipError_t e = hipSuccess;
    if (accel) {
#define CDG_L(TT, MD) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (k_face_sums_batched<TT, MD, false, false, true>), WG, 0)
        CDG_DISPATCH_MAXD(storage, maxd, CDG_L);
#undef CDG_L
    } else {
#define CDG_L(TT, MD) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (k_face_sums_batched<TT, MD, false, false, false>), WG, 0)
        CDG_DISPATCH_MAXD(storage, maxd, CDG_L);
#undef CDG_L
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return n;
}

}  // namespace cdg
