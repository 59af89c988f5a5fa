// Fitness kernel instances: three layers, hidden width up to 256, FP32, weights
// read from global memory.
#include "fit_kernel.h"

namespace mgfwa {
namespace fit {

namespace {
const KernelEntry kEntries[] = {
    FIT_ENTRY(false, false, 4, 2, 16, 16, 1, 0),
    FIT_ENTRY(false, false, 4, 2, 16, 16, 4, 0),
    // one slab per wavefront: narrower layers leave the registers for the
    // activation tiles of both layers (192- and 224-wide hidden layers; the
    // 256-wide instances above keep two slabs and spill a few tiles, which
    // measured faster than one slab there)
    FIT_ENTRY(false, false, 4, 1, 12, 12, 1, 0),
    FIT_ENTRY(false, false, 4, 1, 14, 14, 1, 0),
};
}  // namespace

const KernelEntry *table_l3_wide_f32(int *n)
{
    *n = (int)(sizeof kEntries / sizeof kEntries[0]);
    return kEntries;
}

}  // namespace fit
}  // namespace mgfwa
