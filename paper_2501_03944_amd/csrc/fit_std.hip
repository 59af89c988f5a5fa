// Fitness kernel instances: exact shapes of the three standard workloads.
#include "fit_kernel.h"

namespace mgfwa {
namespace fit {

namespace {
const KernelEntry kEntries[] = {
    FIT_ENTRY(false, 4, 1, 1, 0, 0),
    FIT_ENTRY(true, 4, 2, 1, 0, 0),
    FIT_BOTH(4, 8, 8, 1, 0),
    FIT_BOTH(2, 16, 1, 0, 0),
};
}  // namespace

const KernelEntry *table_std(int *n)
{
    *n = (int)(sizeof kEntries / sizeof kEntries[0]);
    return kEntries;
}

}  // namespace fit
}  // namespace mgfwa
