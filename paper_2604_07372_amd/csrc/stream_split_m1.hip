// Instantiations of the streaming kernel: format NSRGS_A_BF16_SPLIT, mode 1.
#include "stream_impl.h"

namespace nsrgs {
hipError_t launch_stream_split_m1(const StreamConfig &cfg, const StreamArgs &args, hipStream_t s) {
  return launch_fmt_impl<1, NSRGS_A_BF16_SPLIT>(cfg, args, s);
}
}  // namespace nsrgs
