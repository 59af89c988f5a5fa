// Fitness kernel instances: BF16, ReLU, weights staged in LDS, two and three
// layers with hidden widths up to 256 / 224 and up to 16 outputs (the shapes of
// batched jobs of uneven width; every such network's BF16 weights fit in LDS).
// Bias folded into the first K block and ReLU applied on the BF16 conversion
// (SCHED 3); P = 4 slabs for narrow nets, 2 for wide ones.
#include "fit_kernel.h"

namespace mgfwa {
namespace fit {

namespace {
const KernelEntry kEntries[] = {
    FIT_ENTRY_SCHED(true, true, 4, 4, 1, 3, 2, 1, 0, 0),
    FIT_ENTRY_SCHED(true, true, 4, 4, 1, 3, 4, 1, 0, 0),
    FIT_ENTRY_SCHED(true, true, 4, 4, 1, 3, 6, 1, 0, 0),
    FIT_ENTRY_SCHED(true, true, 4, 2, 1, 3, 8, 1, 0, 0),
    FIT_ENTRY_SCHED(true, true, 4, 2, 1, 3, 10, 1, 0, 0),
    FIT_ENTRY_SCHED(true, true, 4, 2, 1, 3, 12, 1, 0, 0),
    FIT_ENTRY_SCHED(true, true, 4, 2, 1, 3, 14, 1, 0, 0),
    FIT_ENTRY_SCHED(true, true, 4, 2, 1, 3, 16, 1, 0, 0),
    FIT_ENTRY_SCHED(true, true, 4, 4, 1, 3, 2, 2, 1, 0),
    FIT_ENTRY_SCHED(true, true, 4, 4, 1, 3, 4, 4, 1, 0),
    FIT_ENTRY_SCHED(true, true, 4, 2, 1, 3, 6, 6, 1, 0),
    FIT_ENTRY_SCHED(true, true, 4, 2, 1, 3, 8, 8, 1, 0),
    FIT_ENTRY_SCHED(true, true, 4, 2, 1, 3, 10, 10, 1, 0),
    FIT_ENTRY_SCHED(true, true, 4, 2, 1, 3, 12, 12, 1, 0),
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
