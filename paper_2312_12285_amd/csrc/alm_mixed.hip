// Mixed-precision transform (FP32 recurrence and products): not yet built.
#include "ptalm_internal.h"

namespace ptalm {

bool mixed_variant_exists(int, int, int) { return false; }

hipError_t launch_alm_mixed(const AlmArgs &, int, int, int, hipStream_t, bool *supported) {
    *supported = false;
    return hipSuccess;
}

}  // namespace ptalm
