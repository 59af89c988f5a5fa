// Fitness kernel instances: BF16, ReLU, weights staged in LDS, two and three
// layers with hidden widths up to 256 / 224 and up to 16 outputs (the shapes of
// batched jobs of uneven width; every such network's BF16 weights fit in LDS).
// Bias folded into the first K block and ReLU applied on the BF16 conversion
// (SCHED 3); P = 4 slabs for narrow nets, 2 for wide ones.  Wide nets also get
// 8 wavefronts per block: their weights fill the LDS, so a CU holds one block,
// and with 4 wavefronts each SIMD would run a single instruction stream (8 x 2
// measured 1.45x faster than 4 x 2 at 64-256-10 and 64-174-174-10; at 128-wide
// layers 4 x 2 stays ahead).  An instance listed first is the shape's default
// before tuning.
#include "fit_kernel.h"

namespace mgfwa {
namespace fit {

namespace {
const KernelEntry kEntries[] = {
    FIT_ENTRY_SCHED(true, true, 4, 4, 1, 3, 2, 1, 0, 0),
    FIT_ENTRY_SCHED(true, true, 4, 4, 1, 3, 4, 1, 0, 0),
    FIT_ENTRY_SCHED(true, true, 4, 4, 1, 3, 6, 1, 0, 0),
    FIT_ENTRY_SCHED(true, true, 4, 2, 1, 3, 8, 1, 0, 0),
    FIT_ENTRY_SCHED(true, true, 8, 2, 1, 3, 8, 1, 0, 0),
    FIT_ENTRY_SCHED(true, true, 8, 2, 1, 3, 10, 1, 0, 0),
    FIT_ENTRY_SCHED(true, true, 4, 2, 1, 3, 10, 1, 0, 0),
    FIT_ENTRY_SCHED(true, true, 8, 2, 1, 3, 12, 1, 0, 0),
    FIT_ENTRY_SCHED(true, true, 4, 2, 1, 3, 12, 1, 0, 0),
    FIT_ENTRY_SCHED(true, true, 8, 2, 1, 3, 14, 1, 0, 0),
    FIT_ENTRY_SCHED(true, true, 4, 2, 1, 3, 14, 1, 0, 0),
    FIT_ENTRY_SCHED(true, true, 8, 2, 1, 3, 16, 1, 0, 0),
    FIT_ENTRY_SCHED(true, true, 4, 2, 1, 3, 16, 1, 0, 0),
    FIT_ENTRY_SCHED(true, true, 4, 4, 1, 3, 2, 2, 1, 0),
    FIT_ENTRY_SCHED(true, true, 4, 4, 1, 3, 4, 4, 1, 0),
    FIT_ENTRY_SCHED(true, true, 4, 2, 1, 3, 6, 6, 1, 0),
    FIT_ENTRY_SCHED(true, true, 8, 2, 1, 3, 6, 6, 1, 0),
    FIT_ENTRY_SCHED(true, true, 4, 2, 1, 3, 8, 8, 1, 0),
    FIT_ENTRY_SCHED(true, true, 8, 2, 1, 3, 8, 8, 1, 0),
    FIT_ENTRY_SCHED(true, true, 8, 2, 1, 3, 10, 10, 1, 0),
    FIT_ENTRY_SCHED(true, true, 4, 2, 1, 3, 10, 10, 1, 0),
    FIT_ENTRY_SCHED(true, true, 8, 2, 1, 3, 12, 12, 1, 0),
    FIT_ENTRY_SCHED(true, true, 4, 2, 1, 3, 12, 12, 1, 0),
    // two slabs of 14 + 14 row blocks would spill with 8 wavefronts
    FIT_ENTRY_SCHED(true, true, 8, 1, 1, 3, 14, 14, 1, 0),
    FIT_ENTRY_SCHED(true, true, 4, 2, 1, 3, 14, 14, 1, 0),
};
}  // namespace

const KernelEntry *table_lds_bf16(int *n)
{
    *n = (int)(sizeof kEntries / sizeof kEntries[0]);
    return kEntries;
}

}  // namespace fit
}  // namespace mgfwa
