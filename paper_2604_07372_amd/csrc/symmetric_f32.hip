// Instantiations of the symmetric half-stream step kernels: format NSRGS_A_F32, d in [1, 16].
#include "symmetric_impl.h"

namespace nsrgs {
hipError_t launch_sym_f32(int d, int rows, int unroll, const SymArgs &a, const StreamArgs &sa, int waves, int mode,
                          hipStream_t s) {
  return sym_launch_fmt<NSRGS_A_F32>(d, rows, unroll, a, sa, waves, mode, s);
}
}  // namespace nsrgs
