// C ABI of the symmetric half-stream step (sync_step_symmetric): argument
// checks, tile shape, workspace carve-up and dispatch by format.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>

#include "host.h"
#include "kernels.h"
#include "nsrgs.h"
#include "symmetric_impl.h"

namespace nsrgs {

hipError_t launch_sym_f64(int, int, int, const SymArgs &, const StreamArgs &, int, int, hipStream_t);
hipError_t launch_sym_f32(int, int, int, const SymArgs &, const StreamArgs &, int, int, hipStream_t);
hipError_t launch_sym_bf16(int, int, int, const SymArgs &, const StreamArgs &, int, int, hipStream_t);
hipError_t launch_sym_split(int, int, int, const SymArgs &, const StreamArgs &, int, int, hipStream_t);

namespace {

struct SymConfig {
  int waves, rows, unroll, H, CW, nchunks, nstrips;
  size_t prow_bytes, pcol_bytes;
};

bool sym_format(int fmt) {
  return fmt == NSRGS_A_F64 || fmt == NSRGS_A_F32 || fmt == NSRGS_A_BF16 || fmt == NSRGS_A_BF16_SPLIT;
}

bool sym_shape_compiled(int d, int rows, int unroll) {
#define NSRGS_SYM_OK(DD, RR, UU) \
  if (d == DD && rows == RR && unroll == UU) return true;
  NSRGS_SYM_SHAPES(NSRGS_SYM_OK)
#undef NSRGS_SYM_OK
  return false;
}

void sym_default_shape(int d, int *rows, int *unroll) {
#define NSRGS_SYM_FIRST(DD, RR, UU) \
  if (d == DD && *rows == 0) {     \
    *rows = RR;                    \
    *unroll = UU;                  \
  }
  *rows = 0;
  NSRGS_SYM_SHAPES(NSRGS_SYM_FIRST)
#undef NSRGS_SYM_FIRST
}

// Tile shape: the first compiled (R, U) for d (or NSRGS_SYM_R / NSRGS_SYM_U
// when compiled), W waves (NSRGS_SYM_W) of U 16-byte vectors per lane per row
// (chunk width CW = 64 W V U), strips of about 384 rows (NSRGS_SYM_H) that
// are a multiple of the panel rows and of the epilogue panel, and at most
// 64 KiB of LDS.
SymConfig sym_config(int fmt, int d, int nd) {
  SymConfig c{};
  const int V = fmt == NSRGS_A_F64 ? 2 : fmt == NSRGS_A_F32 ? 4 : 8;
  const size_t tb = fmt == NSRGS_A_F64 ? 8 : 4;
  int W = env_int("NSRGS_SYM_W", 4);
  if (W != 1 && W != 2 && W != 4 && W != 8) W = 4;
  c.waves = W;
  sym_default_shape(d, &c.rows, &c.unroll);
  const int fr = env_int("NSRGS_SYM_R", 0), fu = env_int("NSRGS_SYM_U", 0);
  if (fr > 0 || fu > 0) {
    const int r = fr > 0 ? fr : c.rows, u = fu > 0 ? fu : c.unroll;
    if (sym_shape_compiled(d, r, u)) {
      c.rows = r;
      c.unroll = u;
    }
  }
  c.CW = W * kWave * V * c.unroll;
  const int R = c.rows, BE = sym_epi_blocks(d);
  const int unit = std::lcm(R, BE * d);
  const int maxH = (int)(65536 / ((size_t)W * d * tb));
  // measured at n d = 60000: FP32 is fastest with the tallest strips the LDS
  // allows, the 2-byte formats at 768 rows
  const int h_default = (fmt == NSRGS_A_F32 || fmt == NSRGS_A_F64) ? 1344 : 768;
  int H = unit * std::max(1, env_int("NSRGS_SYM_H", h_default) / unit);
  while (H > maxH && H > unit) H -= unit;
  c.H = H;
  c.nchunks = (nd + c.CW - 1) / c.CW;
  c.nstrips = (nd + H - 1) / H;
  c.prow_bytes = (size_t)c.nchunks * nd * d * tb;
  c.pcol_bytes = (size_t)c.nstrips * nd * d * tb;
  return c;
}

// The partial sums are sized for every format with the same accumulation
// type (F32, BF16 and BF16_SPLIT share one; F64 has its own), so one
// workspace serves a solve that refines on another format.  Row sums come
// first, then column sums, after the sync_step workspace.
void sym_partial_room(int n, int d, int fmt, size_t *prow, size_t *pcol) {
  const int fam32[] = {NSRGS_A_F32, NSRGS_A_BF16, NSRGS_A_BF16_SPLIT};
  const int fam64[] = {NSRGS_A_F64};
  const int *fam = fmt == NSRGS_A_F64 ? fam64 : fam32;
  const int count = fmt == NSRGS_A_F64 ? 1 : 3;
  *prow = *pcol = 0;
  for (int i = 0; i < count; ++i) {
    const SymConfig c = sym_config(fam[i], d, n * d);
    *prow = std::max(*prow, align256(c.prow_bytes));
    *pcol = std::max(*pcol, align256(c.pcol_bytes));
  }
}

size_t sym_ws_bytes(int n, int d, int fmt) {
  size_t prow, pcol;
  sym_partial_room(n, d, fmt, &prow, &pcol);
  return step_ws_bytes(n, d, fmt) + prow + pcol;
}

}  // namespace
}  // namespace nsrgs

namespace nsrgs {

// The symmetric step's own checks (after the common ones): format, d and
// workspace size for the tile shape in use.
int sym_check(const nsrgs_matrix *A, int n, int d, size_t ws_bytes) {
  if (!sym_format(A->fmt))
    return fail(NSRGS_ERR_UNSUPPORTED, "sync_step_symmetric: format %d is not stored symmetrically "
                "(FP8 row scales differ between A_ij and A_ji)", (int)A->fmt);
  if (d > kSymMaxD) return fail(NSRGS_ERR_UNSUPPORTED, "sync_step_symmetric supports d <= %d", kSymMaxD);
  if (d > kSymMaxD2 && (A->fmt == NSRGS_A_BF16 || A->fmt == NSRGS_A_BF16_SPLIT))
    return fail(NSRGS_ERR_UNSUPPORTED, "sync_step_symmetric on 2-byte formats supports d <= %d (larger d spill "
                "registers and run slower than sync_step)", kSymMaxD2);
  const size_t need = sym_ws_bytes(n, d, A->fmt);
  if (ws_bytes < need)
    return fail(NSRGS_ERR_OUT_OF_MEMORY, "workspace too small for sync_step_symmetric: %zu < %zu bytes", ws_bytes,
                need);
  return NSRGS_OK;
}

// One launch of the symmetric tiles and their epilogue.  mode 0: a step
// (X_in = X^t, X_out = X^{t+1}, monitors into the stats area); mode 1: the
// initialization's product (X_in = Y, X_out = W = A Y, partial Grams at
// `parts`, reduced and factored into the control block).
static int sym_launch(const nsrgs_matrix *A, int n, int d, double mu, int ns_steps, const void *X_in,
                      void *X_out, void *ws, hipStream_t s, int iter, double tol, const int *stop_flag,
                      int mode, void *parts) {
  const int nd = n * d;
  const SymConfig c = sym_config(A->fmt, d, nd);
  char *base = static_cast<char *>(ws);
  const size_t off = step_ws_bytes(n, d, A->fmt);
  SymArgs a{};
  a.A = A->data;
  a.A_lo = A->fmt == NSRGS_A_BF16_SPLIT ? A->data_lo : nullptr;
  a.ld = A->ld;
  a.ndp = packed_ndp(n, d);
  a.X_in = X_in;
  a.nd = nd;
  a.H = c.H;
  a.CW = c.CW;
  a.nchunks = c.nchunks;
  a.nstrips = c.nstrips;
  size_t prow_room, pcol_room;
  sym_partial_room(n, d, A->fmt, &prow_room, &pcol_room);
  a.prow = base + off;
  a.pcol = base + off + prow_room;
  a.stop_flag = stop_flag;
  StreamArgs sa{};
  sa.A = A->data;
  sa.ld = A->ld;
  sa.X_in = X_in;
  sa.X_out = X_out;
  sa.n = n;
  sa.d = d;
  sa.nd = nd;
  const int rows_e = sym_epi_blocks(d) * d;
  sa.num_panels = (nd + rows_e - 1) / rows_e;
  sa.mu = mu > 0.0 ? mu : 1.0 / n;
  sa.ns_steps = ns_steps;
  sa.partials = mode == 0 ? base + step_ws_stats_offset(n, d, A->fmt) : parts;
  sa.ctl = static_cast<DevCtl *>(ws);
  sa.iter = iter;
  sa.tol = tol;
  sa.stop_flag = stop_flag;
  hipError_t e;
  switch (A->fmt) {
    case NSRGS_A_F64: e = launch_sym_f64(d, c.rows, c.unroll, a, sa, c.waves, mode, s); break;
    case NSRGS_A_F32: e = launch_sym_f32(d, c.rows, c.unroll, a, sa, c.waves, mode, s); break;
    case NSRGS_A_BF16: e = launch_sym_bf16(d, c.rows, c.unroll, a, sa, c.waves, mode, s); break;
    default: e = launch_sym_split(d, c.rows, c.unroll, a, sa, c.waves, mode, s); break;
  }
  NSRGS_HIP(e, mode == 0 ? "symmetric step launch" : "symmetric init product launch");
  return NSRGS_OK;
}

// One symmetric step launch (tile, epilogue and monitor kernels); the
// arguments have passed the checks.  iter / tol / stop_flag as in sync_solve.
int sym_step_launch(const nsrgs_matrix *A, int n, int d, double mu, int ns_steps, const void *X_in,
                    void *X_out, void *ws, hipStream_t s, int iter, double tol, bool check_done) {
  DevCtl *ctl = static_cast<DevCtl *>(ws);
  return sym_launch(A, n, d, mu, ns_steps, X_in, X_out, ws, s, iter, tol, check_done ? &ctl->done : nullptr, 0,
                    nullptr);
}

// The initialization's product W = A Y from the symmetric tiles (blocks
// above the diagonal, each used twice) plus A_ii Y_i; partial Grams at
// `parts` (one 2 d^2 record per epilogue panel, at most n).  Launches after
// the residual test has passed return at once (they watch init_done).
int sym_init_product(const nsrgs_matrix *A, int n, int d, const void *Y, void *W, void *parts, void *ws,
                     hipStream_t s, int iter) {
  DevCtl *ctl = static_cast<DevCtl *>(ws);
  return sym_launch(A, n, d, 0.0, 0, Y, W, ws, s, iter, 0.0, &ctl->init_done, 1, parts);
}

}  // namespace nsrgs

using namespace nsrgs;

extern "C" {

size_t sync_step_symmetric_workspace_bytes(int n, int d, int fmt) {
  if (n < 2 || d < 1 || d > kSymMaxD || !sym_format(fmt)) return 0;
  if (d > kSymMaxD2 && (fmt == NSRGS_A_BF16 || fmt == NSRGS_A_BF16_SPLIT)) return 0;
  if ((int64_t)n * d >= (int64_t)1 << 31) return 0;
  return sym_ws_bytes(n, d, fmt);
}

int sync_step_symmetric(const nsrgs_matrix *A, int n, int d, double mu, int ns_steps, const void *X_in,
                        void *X_out, void *ws, size_t ws_bytes, void *stream) {
  int st;
  if ((st = check_step_args(A, n, d, ns_steps, X_in, X_out, ws, ws_bytes, true))) return st;
  if (!std::isfinite(mu)) return fail(NSRGS_ERR_INVALID_ARG, "mu must be finite");
  if ((st = sym_check(A, n, d, ws_bytes))) return st;
  return sym_step_launch(A, n, d, mu, ns_steps, X_in, X_out, ws, (hipStream_t)stream, 0, 0.0, false);
}

}  // extern "C"
