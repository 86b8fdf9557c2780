// The matrix-core path: one iteration of the method for block sizes up to
// d = 32, with any of the three retractions the paper compares (Sec. 4.1):
//   NS-RGS       X_i <- Newton-Schulz^{Ts}(F_i)             (Algorithms 1, 2)
//   exact polar  X_i <- sgn(F_i)                             (the exact
//                retraction, the sequence with a tilde in Sec. 3)
//   GPM          X_i <- sgn((A X)_i)                         (the generalized
//                power method of the Sec. 4.1 comparison)
// and the objective F(X) of eq. (def:f) for the paper's stop rule
// R^t = (F(X^t) - F(X^{t+1})) / F(X^{t+1}) (Sec. 4.1).
//
// At d = 25 the product A X costs 2d = 50 flops per element of A, above what
// the vector units sustain against HBM, so it runs on MFMA: a workgroup owns
// 64 mt rows of A and one chunk of its columns, each wave 16 mt rows (mt
// 16-row tiles), and accumulates A_tile X_chunk with v_mfma_*_16x16x4 over columns
// padded to 16 or 32, reading X from a copy arranged in operand order.  The
// partial products of the column chunks go to the workspace; a per-block
// epilogue kernel sums them and runs the d x d part.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nsrgs.h"

namespace nsrgs {

struct DevCtl;

constexpr int kWideMaxD = 32;       // largest block size of this path
constexpr int kWideGramGroups = 64; // workgroups of the X^T X reduction

enum WideMethod { WIDE_NS = 0, WIDE_POLAR = 1, WIDE_GPM = 2 };
enum WideMode { WIDE_STEP = 0, WIDE_INIT = 1 };

// Per-block record of the epilogue (FP64 for every format).
struct WideStat {
  double dx2, x2, dmax, nonfinite;
  double xc;      // tr(X_i^T C_i), C_i = sum_{j != i} A_ij X_j     (objective)
  double hh;      // ||X_i^T X_i||_F^2                               (objective)
  double aii2;    // ||A_ii||_F^2                                    (objective constant)
  double polar_bad;   // exact polar did not converge (singular input)
};

// Control fields of the wide path that do not fit DevCtl (d up to 32).
struct alignas(256) WideCtl {
  double T[kWideMaxD * kWideMaxD];     // init: Rayleigh quotient Y^T A Y
  double Rinv[kWideMaxD * kWideMaxD];  // init: inverse Cholesky factor of W^T W
  double ritz[kWideMaxD];              // init: Ritz values, descending
  double obj_const;                    // (1/2) sum_{i != j} ||A_ij||_F^2
  double obj_prev;                     // F(X^{t-1})
  double obj;                          // F(X^t) of the last step's input
  double obj_ratio;                    // R^{t-1} of the last step (NaN before)
  int have_const, pad[7];
};

// Launch geometry of the product for a problem (n, d, storage format).
struct WideGeom {
  int nt;          // 16-column tiles (1: d <= 16, 2: d <= 32)
  int mt;          // 16-row tiles per wave (rows per workgroup = 64 mt)
  int rows;        // rows of A per workgroup
  int xcd_remap;   // deal column-chunk-major tile ranges to the XCDs
  int ku;          // 16-byte vectors per lane per tile row per step (8 / mt)
  int kstep;       // columns per step: 4 ku V (V = 2 for F64, 4 for F32)
  int steps;       // ceil(nd / kstep)
  int row_tiles;   // ceil(nd / rows)
  int rows_pad;    // row_tiles * rows
  int ks;          // column chunks
  int ks_max;      // bound on ks for every step width (sizes the workspace)
  int kchunk;      // columns per chunk (multiple of kstep)
};
WideGeom wide_geom(int n, int d, int fmt);

// Workspace areas of the wide path (offsets relative to its region).
struct WideLayout {
  size_t ctl, stats, part, xs, gram, sumsq, igram, total;
};
WideLayout wide_layout(int n, int d, int fmt);

struct WideArgs {
  const void *A;
  int64_t ld;
  int n, d, nd;
  const void *X_in;    // X^t, or Y (init)
  void *X_out;         // X^{t+1}, or W = A Y (init)
  void *part;          // ks x rows_pad x 32 partial products
  void *xs;            // X in the product's B-operand order (wide_xs_kernel)
  WideStat *stats;     // n per-block records (step)
  double *igram;       // n x 2 d^2 per-block Grams Y^T W, W^T W (init)
  double *gram;        // kWideGramGroups x d^2 partial X^T X (objective)
  double *sumsq;       // row_tiles x ks partial sums of squares of A, or NULL
  DevCtl *ctl;
  WideCtl *wctl;
  double mu;
  int ns_steps, method, mode;
  int iter;            // iteration index t
  double tol;          // stop tolerance (<= 0: none)
  int stop_rule;       // 0 relative change, 1 objective ratio R^t
  int objective;       // 1: evaluate F(X^t) this step
  const int *stop_flag;
  int no_diag;         // 1: the partials already exclude A_ii and A is not read
                       //    (block-sparse storage); A_ii counts as zero
  int p;               // columns of X (d, or the Stiefel width p >= d)
  int xs_ready;        // 1: xs already holds X_in (written by the previous
                       //    step's epilogue), so the product skips wide_xs_kernel
  int xs_write;        // 1: the step epilogue also writes X_out into xs
  WideGeom g;
};

// The arguments of a matrix-core launch bound to the single-problem
// workspace ws (its matrix-core region; sync_workspace_bytes layout) with
// p = d (runtime.hip).
WideArgs wide_args(const nsrgs_matrix *A, int n, int d, void *ws);

int wide_supported_fmt(int fmt);
hipError_t launch_wide_step(int fmt, const WideArgs &a, hipStream_t s);
hipError_t launch_wide_init_product(int fmt, const WideArgs &a, hipStream_t s);
// The parts around the product, for products computed elsewhere (block-sparse
// storage): X^T X partials; epilogue + finish; init epilogue + Gram reduction.
hipError_t launch_wide_gram(int fmt, const WideArgs &a, hipStream_t s);
hipError_t launch_wide_post(int fmt, const WideArgs &a, hipStream_t s);
hipError_t launch_wide_init_post(int fmt, const WideArgs &a, hipStream_t s);
hipError_t launch_wide_init_apply(int fmt, const void *W, const void *Y, void *Y_next, int nd, int d,
                                  double *partials, int num_groups, DevCtl *ctl, WideCtl *wctl,
                                  int iter, double tol, hipStream_t s);
hipError_t launch_wide_init_polar(int fmt, const void *Y, void *X0, int n, int d, DevCtl *ctl,
                                  hipStream_t s);
hipError_t launch_wide_init_finish(DevCtl *ctl, WideCtl *wctl, int d, hipStream_t s);
hipError_t launch_wide_ctl_reset(WideCtl *wctl, hipStream_t s);

// NS-RGS on St(p, d)^n (d x p blocks with orthonormal rows, p <= 32): the
// product A S (p columns), the per-block Stiefel step and the monitors.
hipError_t launch_wide_stiefel_step(int fmt, const WideArgs &a, hipStream_t s);
// Rounding of S to O(d)^n: X_i = sgn(S_i V), V the top-d eigenvectors of
// S^T S (p x p, FP64 Jacobi).  gram: kWideGramGroups p^2 doubles; basis:
// p d doubles; ctl->init_bad is set if a polar factor fails.
hipError_t launch_stiefel_round(int fmt, const void *S, int n, int d, int p, double *gram, double *basis,
                                void *X, DevCtl *ctl, hipStream_t s);

}  // namespace nsrgs
