// Fitness kernel instances: three layers, hidden width up to 128.
#include "fit_kernel.h"

namespace mgfwa {
namespace fit {

namespace {
const KernelEntry kEntries[] = {
    FIT_BOTH(4, 2, 2, 1, 0),
    FIT_BOTH(4, 4, 4, 1, 0),
    FIT_BOTH(4, 4, 4, 4, 0),
    FIT_BOTH(4, 8, 8, 4, 0),
};
}  // namespace

const KernelEntry *table_l3(int *n)
{
    *n = (int)(sizeof kEntries / sizeof kEntries[0]);
    return kEntries;
}

}  // namespace fit
}  // namespace mgfwa
