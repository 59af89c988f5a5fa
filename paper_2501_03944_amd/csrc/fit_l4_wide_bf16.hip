// Fitness kernel instances: four layers, hidden width up to 256, BF16.
#include "fit_kernel.h"

namespace mgfwa {
namespace fit {

namespace {
const KernelEntry kEntries[] = {
    FIT_ENTRY(true, false, 4, 2, 16, 16, 16, 1),
};
}  // namespace

const KernelEntry *table_l4_wide_bf16(int *n)
{
    *n = (int)(sizeof kEntries / sizeof kEntries[0]);
    return kEntries;
}

}  // namespace fit
}  // namespace mgfwa
