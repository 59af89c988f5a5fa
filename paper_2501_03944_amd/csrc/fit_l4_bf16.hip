// Fitness kernel instances: four layers, hidden width up to 128, BF16.
#include "fit_kernel.h"

namespace mgfwa {
namespace fit {

namespace {
const KernelEntry kEntries[] = {
    FIT_ENTRY(true, false, 4, 4, 2, 2, 2, 1),
    FIT_ENTRY(true, false, 4, 4, 4, 4, 4, 1),
    FIT_ENTRY(true, false, 4, 4, 4, 4, 4, 4),
    FIT_ENTRY(true, false, 4, 4, 8, 8, 8, 1),
    FIT_ENTRY(true, false, 4, 4, 8, 8, 8, 4),
};
}  // namespace

const KernelEntry *table_l4_bf16(int *n)
{
    *n = (int)(sizeof kEntries / sizeof kEntries[0]);
    return kEntries;
}

}  // namespace fit
}  // namespace mgfwa
