// Fitness kernel instances: FP32, ReLU, weights staged in LDS, two layers with
// hidden widths up to 256 and three with hidden widths up to 160, up to 16
// outputs (batched jobs of uneven width in FP32, and the FP32 re-check of BF16
// selection winners).  P = 4 slabs for narrow nets, 2 for wide ones.
#include "fit_kernel.h"

namespace mgfwa {
namespace fit {

namespace {
const KernelEntry kEntries[] = {
    FIT_ENTRY_ACT(false, true, 4, 4, 1, 2, 1, 0, 0),
    FIT_ENTRY_ACT(false, true, 4, 4, 1, 4, 1, 0, 0),
    FIT_ENTRY_ACT(false, true, 4, 4, 1, 6, 1, 0, 0),
    FIT_ENTRY_ACT(false, true, 4, 2, 1, 8, 1, 0, 0),
    FIT_ENTRY_ACT(false, true, 4, 2, 1, 10, 1, 0, 0),
    FIT_ENTRY_ACT(false, true, 4, 2, 1, 12, 1, 0, 0),
    FIT_ENTRY_ACT(false, true, 4, 2, 1, 14, 1, 0, 0),
    FIT_ENTRY_ACT(false, true, 4, 2, 1, 16, 1, 0, 0),
    FIT_ENTRY_ACT(false, true, 4, 4, 1, 2, 2, 1, 0),
    FIT_ENTRY_ACT(false, true, 4, 4, 1, 4, 4, 1, 0),
    FIT_ENTRY_ACT(false, true, 4, 2, 1, 6, 6, 1, 0),
    FIT_ENTRY_ACT(false, true, 4, 2, 1, 8, 8, 1, 0),
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
