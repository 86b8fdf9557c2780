// Launch interface between the C-ABI runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nsrgs.h"

namespace nsrgs {

struct DevCtl;

// Arguments of the streaming kernel.  mode 0: one NS-RGS step (Alg. 2);
// mode 1: the bare product W = A Y of the spectral initialization with
// per-panel partial Grams Y^T W and W^T W.
struct StreamArgs {
  const void *A;          // format-specific storage, nd rows of ld elements
  const void *A_lo;       // BF16_SPLIT low part
  const float *scale;     // FP8 row scales
  int64_t ld;             // elements
  const void *X_in;       // X^t (mode 0) or Y (mode 1), nd x d
  void *X_out;            // X^{t+1} (mode 0) or W = A Y (mode 1), nd x d
  int n, d, nd;
  int num_panels;
  double mu;              // step size
  int ns_steps;           // Newton-Schulz steps
  void *partials;         // mode 0: PanelStat per panel; mode 1: 2 d^2 values per panel
  DevCtl *ctl;
  int iter;               // iteration index t (mode 0) / subspace iteration (mode 1)
  double tol;             // mode 0: relative-change tolerance (<= 0: none)
  const int *stop_flag;   // non-NULL: return at once when *stop_flag != 0
};

// Waves per workgroup of the software-pipelined (U = 0) step shapes: two
// register buffers of a column group need more than the 256 VGPRs of two
// waves per SIMD, so these are built for one wave per SIMD (512 VGPRs) and
// each wave hides its own load latency; launches cap W at this.
constexpr int kPipeMaxWaves = 4;

struct StreamConfig {
  int blocks_per_panel;   // B: rows per panel R = B d
  int waves;              // W: waves per workgroup splitting the columns
  int unroll;             // U: 16-byte column vectors per lane per row per iteration;
                          //    0: one, software-pipelined
};

// Compiled (B, U) variants for a given d (waves = 1); returns the count.
int stream_variants(int d, StreamConfig *opts, int max_opts);

// The one B used by the spectral-initialization product for a given d.
int stream_block_init(int d);

// Heuristic / tuned configuration for (fmt, d, nd).
StreamConfig choose_stream_config(int fmt, int d, int nd, int mode);

hipError_t launch_stream(int mode, int fmt, const StreamConfig &cfg,
                         const StreamArgs &args, hipStream_t stream);

// Spectral-initialization helpers (init.hip).
struct InitArgs {
  const void *W;          // A Y, nd x d
  const void *Y;          // current basis, nd x d
  void *Y_next;           // W R^{-1}, nd x d
  int nd, d;
  void *partials;         // per-workgroup residual partials (double)
  int num_groups;
  DevCtl *ctl;
  int iter;
  double tol;
};
hipError_t launch_init_random(int fmt, void *Y, int nd, int d, uint64_t seed,
                              hipStream_t stream);
hipError_t launch_init_apply(int fmt, const InitArgs &args, hipStream_t stream);
hipError_t launch_init_polar(int fmt, const void *Y, void *X0, int n, int d,
                             DevCtl *ctl, hipStream_t stream);
hipError_t launch_init_finish(DevCtl *ctl, int d, hipStream_t stream);
hipError_t launch_ctl_reset(DevCtl *ctl, int what, hipStream_t stream);

// Inputs (gen.hip).
hipError_t launch_generate(const double *Z, int n, int d, double sigma,
                           uint64_t seed, int zero_diag, double p, int fmt,
                           void *A, int64_t ld, hipStream_t stream);
hipError_t launch_convert(const float *A32, int nd, int64_t ld,
                          const nsrgs_matrix &out, hipStream_t stream);
// Row-chunk variants: rows [row0, row0 + nrows) of A; A_rows / A32_rows point
// at row row0 of a buffer holding those rows with leading dimension ld.
hipError_t launch_generate_rows(const double *Z, int n, int d, double sigma, uint64_t seed,
                                int zero_diag, double p, int fmt, void *A_rows, int64_t ld,
                                int row0, int nrows, hipStream_t stream);
hipError_t launch_convert_rows(const float *A32_rows, int nd, int64_t ld, const nsrgs_matrix &out,
                               int row0, int nrows, hipStream_t stream);
// Elementwise BF16 / BF16_SPLIT conversion of `count` contiguous values (the
// packed layout).
hipError_t launch_convert_flat(const float *A32, int64_t count, const nsrgs_matrix &out, hipStream_t stream);

}  // namespace nsrgs
