// Instantiations of the streaming kernel: format NSRGS_A_F64, mode 0, d in [5, 8].
#include "stream_impl.h"

namespace nsrgs {
hipError_t launch_stream_f64_m0b(const StreamConfig &cfg, const StreamArgs &args, hipStream_t s) {
  return launch_fmt_impl<0, NSRGS_A_F64, 5, 8>(cfg, args, s);
}
}  // namespace nsrgs
