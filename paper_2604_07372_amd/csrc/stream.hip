// Dispatch of the streaming kernel over (mode, format).  The kernel itself
// is in stream_impl.h; each (format, mode) pair is instantiated in its own
// translation unit so the library builds in parallel.
#include "stream_impl.h"

namespace nsrgs {

hipError_t launch_stream_f64_m0a(const StreamConfig &, const StreamArgs &, hipStream_t);
hipError_t launch_stream_f64_m0b(const StreamConfig &, const StreamArgs &, hipStream_t);
hipError_t launch_stream_f64_m0c(const StreamConfig &, const StreamArgs &, hipStream_t);
hipError_t launch_stream_f64_m1(const StreamConfig &, const StreamArgs &, hipStream_t);
hipError_t launch_stream_f32_m0a(const StreamConfig &, const StreamArgs &, hipStream_t);
hipError_t launch_stream_f32_m0b(const StreamConfig &, const StreamArgs &, hipStream_t);
hipError_t launch_stream_f32_m0c(const StreamConfig &, const StreamArgs &, hipStream_t);
hipError_t launch_stream_f32_m1(const StreamConfig &, const StreamArgs &, hipStream_t);
hipError_t launch_stream_bf16_m0a(const StreamConfig &, const StreamArgs &, hipStream_t);
hipError_t launch_stream_bf16_m0b(const StreamConfig &, const StreamArgs &, hipStream_t);
hipError_t launch_stream_bf16_m0c(const StreamConfig &, const StreamArgs &, hipStream_t);
hipError_t launch_stream_bf16_m1(const StreamConfig &, const StreamArgs &, hipStream_t);
hipError_t launch_stream_split_m0a(const StreamConfig &, const StreamArgs &, hipStream_t);
hipError_t launch_stream_split_m0b(const StreamConfig &, const StreamArgs &, hipStream_t);
hipError_t launch_stream_split_m0c(const StreamConfig &, const StreamArgs &, hipStream_t);
hipError_t launch_stream_split_m1(const StreamConfig &, const StreamArgs &, hipStream_t);
hipError_t launch_stream_fp8_m0a(const StreamConfig &, const StreamArgs &, hipStream_t);
hipError_t launch_stream_fp8_m0b(const StreamConfig &, const StreamArgs &, hipStream_t);
hipError_t launch_stream_fp8_m0c(const StreamConfig &, const StreamArgs &, hipStream_t);
hipError_t launch_stream_fp8_m1(const StreamConfig &, const StreamArgs &, hipStream_t);

int stream_variants(int d, StreamConfig *opts, int max_opts) {
  int cnt = 0;
#define NSRGS_OPT(DD, BB, UU) \
  if (d == DD && cnt < max_opts) opts[cnt++] = StreamConfig{BB, 1, UU};
  NSRGS_BOPTS(NSRGS_OPT)
#undef NSRGS_OPT
  return cnt;
}

int stream_block_init(int d) {
#define NSRGS_OPT(DD, BB, UU) \
  if (d == DD) return BB;
  NSRGS_BOPTS_INIT(NSRGS_OPT)
#undef NSRGS_OPT
  return 0;
}

hipError_t launch_stream(int mode, int fmt, const StreamConfig &cfg, const StreamArgs &args,
                         hipStream_t s) {
  if (cfg.waves < 1 || cfg.waves > kMaxWaves) return hipErrorInvalidValue;
  switch (fmt * 2 + mode) {
    case NSRGS_A_F64 * 2 + 0:
      return args.d <= 4 ? launch_stream_f64_m0a(cfg, args, s)
           : args.d <= 8 ? launch_stream_f64_m0b(cfg, args, s) : launch_stream_f64_m0c(cfg, args, s);
    case NSRGS_A_F64 * 2 + 1: return launch_stream_f64_m1(cfg, args, s);
    case NSRGS_A_F32 * 2 + 0:
      return args.d <= 4 ? launch_stream_f32_m0a(cfg, args, s)
           : args.d <= 8 ? launch_stream_f32_m0b(cfg, args, s) : launch_stream_f32_m0c(cfg, args, s);
    case NSRGS_A_F32 * 2 + 1: return launch_stream_f32_m1(cfg, args, s);
    case NSRGS_A_BF16 * 2 + 0:
      return args.d <= 4 ? launch_stream_bf16_m0a(cfg, args, s)
           : args.d <= 8 ? launch_stream_bf16_m0b(cfg, args, s) : launch_stream_bf16_m0c(cfg, args, s);
    case NSRGS_A_BF16 * 2 + 1: return launch_stream_bf16_m1(cfg, args, s);
    case NSRGS_A_BF16_SPLIT * 2 + 0:
      return args.d <= 4 ? launch_stream_split_m0a(cfg, args, s)
           : args.d <= 8 ? launch_stream_split_m0b(cfg, args, s) : launch_stream_split_m0c(cfg, args, s);
    case NSRGS_A_BF16_SPLIT * 2 + 1: return launch_stream_split_m1(cfg, args, s);
    case NSRGS_A_FP8_E4M3 * 2 + 0:
      return args.d <= 4 ? launch_stream_fp8_m0a(cfg, args, s)
           : args.d <= 8 ? launch_stream_fp8_m0b(cfg, args, s) : launch_stream_fp8_m0c(cfg, args, s);
    case NSRGS_A_FP8_E4M3 * 2 + 1: return launch_stream_fp8_m1(cfg, args, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace nsrgs
