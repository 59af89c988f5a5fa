// Fitness kernel instances: four layers, hidden width up to 256, FP32.
#include "fit_kernel.h"

namespace mgfwa {
namespace fit {

namespace {
const KernelEntry kEntries[] = {
    FIT_ENTRY(false, false, 4, 2, 16, 16, 16, 1),
};
}  // namespace

const KernelEntry *table_l4_wide_f32(int *n)
{
    *n = (int)(sizeof kEntries / sizeof kEntries[0]);
    return kEntries;
}

}  // namespace fit
}  // namespace mgfwa
