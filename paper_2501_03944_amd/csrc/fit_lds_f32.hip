// Fitness kernel instances: FP32, ReLU, weights staged in LDS, two layers with
// hidden widths up to 256 and three with hidden widths up to 160, up to 16
// outputs (batched jobs of uneven width in FP32, and the FP32 re-check of BF16
// selection winners).  P = 4 slabs for narrow nets, 2 for wide ones; wide nets
// also with 16 wavefronts x 1 slab and each fragment fetched one row block ahead
// (SCHED 1), listed first: their weights fill the LDS, so a CU holds one block,
// and four wavefronts per SIMD cover each other's waits (1.15-1.26x over 4 x 2
// at 64-192-10, 64-256-10 and 32-160-160-10).
#include "fit_kernel.h"

namespace mgfwa {
namespace fit {

namespace {
const KernelEntry kEntries[] = {
    FIT_ENTRY_ACT(false, true, 4, 4, 1, 2, 1, 0, 0),
    FIT_ENTRY_ACT(false, true, 4, 4, 1, 4, 1, 0, 0),
    FIT_ENTRY_ACT(false, true, 4, 4, 1, 6, 1, 0, 0),
    FIT_ENTRY_SCHED(false, true, 16, 1, 1, 1, 8, 1, 0, 0),
    FIT_ENTRY_ACT(false, true, 4, 2, 1, 8, 1, 0, 0),
    FIT_ENTRY_SCHED(false, true, 16, 1, 1, 1, 10, 1, 0, 0),
    FIT_ENTRY_ACT(false, true, 4, 2, 1, 10, 1, 0, 0),
    FIT_ENTRY_SCHED(false, true, 16, 1, 1, 1, 12, 1, 0, 0),
    FIT_ENTRY_ACT(false, true, 4, 2, 1, 12, 1, 0, 0),
    FIT_ENTRY_SCHED(false, true, 16, 1, 1, 1, 14, 1, 0, 0),
    FIT_ENTRY_ACT(false, true, 4, 2, 1, 14, 1, 0, 0),
    FIT_ENTRY_SCHED(false, true, 16, 1, 1, 1, 16, 1, 0, 0),
    FIT_ENTRY_ACT(false, true, 4, 2, 1, 16, 1, 0, 0),
    FIT_ENTRY_ACT(false, true, 4, 4, 1, 2, 2, 1, 0),
    FIT_ENTRY_ACT(false, true, 4, 4, 1, 4, 4, 1, 0),
    FIT_ENTRY_SCHED(false, true, 16, 1, 1, 1, 6, 6, 1, 0),
    FIT_ENTRY_ACT(false, true, 4, 2, 1, 6, 6, 1, 0),
    FIT_ENTRY_SCHED(false, true, 16, 1, 1, 1, 8, 8, 1, 0),
    FIT_ENTRY_ACT(false, true, 4, 2, 1, 8, 8, 1, 0),
    FIT_ENTRY_SCHED(false, true, 16, 1, 1, 1, 10, 10, 1, 0),
    FIT_ENTRY_ACT(false, true, 4, 2, 1, 10, 10, 1, 0),
};
}  // namespace

const KernelEntry *table_lds_f32(int *n)
{
    *n = (int)(sizeof kEntries / sizeof kEntries[0]);
    return kEntries;
}

}  // namespace fit
}  // namespace mgfwa
