// Fitness kernel instances: exact shapes of the three standard workloads.
#include "fit_kernel.h"

namespace mgfwa {
namespace fit {

namespace {
const KernelEntry kEntries[] = {
    // 8-16-1 tanh: weights in LDS; FP32 with 2 wavefronts x 2 slabs, so that a
    // 256-sample launch spreads over 4 blocks per spark (measured 0.042 -> 0.040
    // ms per generation against 4 x 4; 1 x 2, 2 x 1 and 4 x 1 within noise of it)
    FIT_ENTRY_ACT(false, true, 2, 2, 2, 1, 1, 0, 0),
    FIT_ENTRY_ACT(false, true, 4, 4, 2, 1, 1, 0, 0),
    FIT_ENTRY_ACT(true, true, 4, 4, 2, 2, 1, 0, 0),
    // 64-128-128-10 ReLU: weights in LDS.  Measured best: FP32 with 16
    // wavefronts x 1 slab (four per SIMD: one wavefront's waits are covered by
    // the others' multiplies), each fragment fetched one row block ahead
    // (SCHED 1): 0.794 -> 0.824 of the FP32 peak against the next entry, 8 x 2
    // with fragments fetched right before use and zero-addend first K blocks
    // (SCHED 2), which the tuner still tries.  (BF16 takes the LDS-staged
    // 4 x 2 instance of the batched-job table: 0.60 ms per explosion-fitness
    // launch, against 0.84 ms for 4 x 4 and 0.87 ms for 16 x 1.)
    FIT_ENTRY_SCHED(false, true, 16, 1, 1, 1, 8, 8, 1, 0),
    FIT_ENTRY_SCHED(false, true, 8, 2, 1, 2, 8, 8, 1, 0),
    // 784-256-10 ReLU: the first layer does not fit in LDS
    FIT_ENTRY_ACT(false, false, 4, 2, 1, 16, 1, 0, 0),
    FIT_ENTRY_ACT(true, false, 4, 2, 1, 16, 1, 0, 0),
};
}  // namespace

const KernelEntry *table_std(int *n)
{
    *n = (int)(sizeof kEntries / sizeof kEntries[0]);
    return kEntries;
}

}  // namespace fit
}  // namespace mgfwa
