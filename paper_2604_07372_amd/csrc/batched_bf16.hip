// Batched kernels for format NSRGS_A_BF16 (grouped and persistent, every d class).
#include "batched_impl.h"

namespace nsrgs {
template hipError_t launch_group_fmt<NSRGS_A_BF16>(int, const GroupArgs &, int, int, hipStream_t);
template hipError_t launch_persistent_fmt<NSRGS_A_BF16>(int, const PersistArgs &, int, hipStream_t);
}  // namespace nsrgs
