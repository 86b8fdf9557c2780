// Instantiations of the streaming kernel: format NSRGS_A_BF16, mode 0, d in [9, 16].
#include "stream_impl.h"

namespace nsrgs {
hipError_t launch_stream_bf16_m0c(const StreamConfig &cfg, const StreamArgs &args, hipStream_t s) {
  return launch_fmt_impl<0, NSRGS_A_BF16, 9, 16>(cfg, args, s);
}
}  // namespace nsrgs
