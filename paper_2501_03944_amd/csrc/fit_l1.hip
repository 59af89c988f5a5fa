// Fitness kernel instances: single-layer networks.
#include "fit_kernel.h"

namespace mgfwa {
namespace fit {

namespace {
const KernelEntry kEntries[] = {
    FIT_BOTH(4, 1, 0, 0, 0),
    FIT_BOTH(4, 4, 0, 0, 0),
    FIT_BOTH(2, 16, 0, 0, 0),
};
}  // namespace

const KernelEntry *table_l1(int *n)
{
    *n = (int)(sizeof kEntries / sizeof kEntries[0]);
    return kEntries;
}

}  // namespace fit
}  // namespace mgfwa
