// Host-side helpers shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "nsrgs.h"

namespace nsrgs {

// Record an error message for nsrgs_last_error() and return `status`.
int fail(int status, const char *fmt, ...);
int dev_fail(hipError_t e, const char *what);
bool valid_fmt(int fmt);
size_t xbytes(int fmt);
size_t align256(size_t v);
int check_common(int n, int d);
bool aligned16(const void *p);
// packed_ok: the call reads the packed symmetric layout (NSRGS_LD_PACKED).
int check_matrix(const nsrgs_matrix *A, int n, int d, bool packed_ok = false);
int env_int(const char *name, int dflt);

#define NSRGS_HIP(call, what)                          \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return dev_fail(e_, what);   \
  } while (0)

// Results of one problem of a batched launch (host copy of device fields).
struct BatchResult {
  int iters, converged, nonfinite, panels, active;
  double rel_change, max_defect;
};

// Grouped launches: one iteration of many problems per launch (batched.hip).
struct GroupSpec {
  nsrgs_matrix A;
  int n, d, iters;        // iters: total budget (t counts from the first iteration)
  int t0;                 // iterations already done; X^t0 is in (t0 even ? X0 : X1)
  void *X0, *X1;          // X^t lives in X0 for even t, X1 for odd t
  void *stats;            // batch_panels(n, d) PanelStat entries
  double mu, tol;
};
int batch_rows_per_panel(int d);
int batch_panels(int n, int d);
size_t group_control_bytes(int count, size_t units);
int run_grouped(int fmt, const std::vector<GroupSpec> &specs, void *ctl, int launches, int ns_steps,
                int waves, int order, int check_every, hipStream_t s, std::vector<BatchResult> &out);

// One persistent launch for the remaining budget of every problem (batched.hip).
int run_persistent(int fmt, const std::vector<GroupSpec> &specs, void *ctl, int ns_steps, int waves,
                   int order, unsigned wait_polls, size_t min_ticket_bytes, hipStream_t s,
                   std::vector<BatchResult> &out);
size_t elem_size(int fmt);   // bytes per stored A element (hi + lo for the split format)

// Single-problem step with a given launch shape, and sync_step's argument
// checks (runtime.hip); used by the autotuner.
struct StreamConfig;
int step_with_config(const nsrgs_matrix *A, int n, int d, double mu, int ns_steps, const void *X_in,
                     void *X_out, void *ws, hipStream_t s, const StreamConfig &cfg);
int check_step_args(const nsrgs_matrix *A, int n, int d, int ns_steps, const void *X_in, void *X_out,
                    void *ws, size_t ws_bytes, bool packed_ok = false);

// sync_step with its argument checks, the control block at `ctl` and room
// for stats_bytes of panel monitors at `stats` (runtime.hip).
struct DevCtl;
int check_step_inputs(const nsrgs_matrix *A, int n, int d, double mu, int ns_steps, const void *X_in,
                      const void *X_out);
int step_checked_into(const nsrgs_matrix *A, int n, int d, double mu, int ns_steps, const void *X_in,
                      void *X_out, DevCtl *ctl, void *stats, size_t stats_bytes, hipStream_t s);

// Bytes of the single-problem workspace (control block, panel monitors,
// iterate and initialization buffers) and the offset of its panel monitors
// (runtime.hip).
size_t step_ws_bytes(int n, int d, int fmt);
// The part of it the streaming-kernel calls use (d <= 16, NS-RGS).
size_t narrow_ws_bytes(int n, int d, int fmt);
size_t step_ws_stats_offset(int n, int d, int fmt);

// Symmetric half-stream step (symmetric.hip): its own argument checks and
// one launch with the solve's iteration index, tolerance and stop flag.
int sym_check(const nsrgs_matrix *A, int n, int d, size_t ws_bytes);
int sym_step_launch(const nsrgs_matrix *A, int n, int d, double mu, int ns_steps, const void *X_in,
                    void *X_out, void *ws, hipStream_t s, int iter, double tol, bool check_done);
int sym_init_product(const nsrgs_matrix *A, int n, int d, const void *Y, void *W, void *parts, void *ws,
                     hipStream_t s, int iter);

// Block-sparse A (bsr.hip): the product for the matrix-core epilogue, and
// (runtime.hip) one step through that epilogue for d up to 32.
hipError_t launch_bsr_wide_product(const nsrgs_bsr_matrix &A, int n, int d, const float *X, float *P,
                                   double *sumsq, const int *stop_flag, hipStream_t s);
// The sliced block-sparse product (d <= 6) for solves: usable when ws holds
// sync_step_bsr_workspace_bytes; the bounds table is written once per matrix
// and then serves every product on it.
bool bsr_sliced(int n, int d, size_t ws_bytes);
hipError_t launch_bsr_slice_bounds(const nsrgs_bsr_matrix &A, int n, int d, void *ws, hipStream_t s);
hipError_t launch_bsr_slice_wide_product(const nsrgs_bsr_matrix &A, int n, int d, const float *X, float *P,
                                         void *ws, const int *stop_flag, hipStream_t s);
// One iteration of a solve on the sliced step (NS-RGS, relative-change rule):
// product on the bounds found before, the per-block epilogue of sync_step_bsr,
// the monitor finish with the stop rule (control block at ws).
int bsr_sliced_iterate(const nsrgs_bsr_matrix &A, int n, int d, double mu, int ns_steps, const void *X_in,
                       void *X_out, void *ws, hipStream_t s, int iter, double tol);
int bsr_wide_step(const nsrgs_bsr_matrix *A, int n, int d, double mu, int ns_steps, const void *X_in,
                  void *X_out, void *ws, size_t ws_bytes, hipStream_t s);

// Tuning table (runtime.hip): waves per workgroup of the grouped launch.
int tuned_batch_waves(int fmt, int dmax);

}  // namespace nsrgs
