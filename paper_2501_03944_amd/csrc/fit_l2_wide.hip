// Fitness kernel instances: two layers, hidden width up to 256.
#include "fit_kernel.h"

namespace mgfwa {
namespace fit {

namespace {
const KernelEntry kEntries[] = {
    FIT_BOTH(2, 16, 4, 0, 0),
    FIT_BOTH(2, 16, 16, 0, 0),
};
}  // namespace

const KernelEntry *table_l2_wide(int *n)
{
    *n = (int)(sizeof kEntries / sizeof kEntries[0]);
    return kEntries;
}

}  // namespace fit
}  // namespace mgfwa
