// Instantiations of the symmetric half-stream step kernels: format NSRGS_A_BF16_SPLIT, d in [1, 16].
#include "symmetric_impl.h"

namespace nsrgs {
hipError_t launch_sym_split(int d, int rows, int unroll, const SymArgs &a, const StreamArgs &sa, int waves, int mode,
                          hipStream_t s) {
  return sym_launch_fmt<NSRGS_A_BF16_SPLIT>(d, rows, unroll, a, sa, waves, mode, s);
}
}  // namespace nsrgs
