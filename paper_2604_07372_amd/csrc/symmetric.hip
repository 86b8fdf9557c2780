// C ABI of the symmetric half-stream step (sync_step_symmetric): argument
// checks, tile shape, workspace carve-up and dispatch by format.
#include <hip/hip_runtime.h>

#include <cmath>
#include <numeric>

#include "host.h"
#include "kernels.h"
#include "nsrgs.h"
#include "symmetric_impl.h"

namespace nsrgs {

hipError_t launch_sym_f64(int, int, const SymArgs &, const StreamArgs &, int, hipStream_t);
hipError_t launch_sym_f32(int, int, const SymArgs &, const StreamArgs &, int, hipStream_t);
hipError_t launch_sym_bf16(int, int, const SymArgs &, const StreamArgs &, int, hipStream_t);
hipError_t launch_sym_split(int, int, const SymArgs &, const StreamArgs &, int, hipStream_t);

namespace {

struct SymConfig {
  int waves, unroll, H, CW, nchunks, nstrips;
  size_t prow_bytes, pcol_bytes;
};

bool sym_format(int fmt) {
  return fmt == NSRGS_A_F64 || fmt == NSRGS_A_F32 || fmt == NSRGS_A_BF16 || fmt == NSRGS_A_BF16_SPLIT;
}

// Tile shape: W waves of one 16-byte vector per lane per row (chunk width
// CW = 64 W V), strips of about 384 rows (NSRGS_SYM_H) that are a multiple of
// the panel rows and of the epilogue panel, and at most 64 KiB of LDS.
SymConfig sym_config(int fmt, int d, int nd) {
  SymConfig c{};
  const int V = fmt == NSRGS_A_F64 ? 2 : fmt == NSRGS_A_F32 ? 4 : 8;
  const size_t tb = fmt == NSRGS_A_F64 ? 8 : 4;
  int W = env_int("NSRGS_SYM_W", 4);
  if (W != 1 && W != 2 && W != 4 && W != 8) W = 4;
  c.waves = W;
  c.unroll = 1;
  c.CW = W * kWave * V * c.unroll;
  const int R = sym_rows(d), BE = sym_epi_blocks(d);
  const int unit = std::lcm(R, BE * d);
  const int maxH = (int)(65536 / ((size_t)W * d * tb));
  int H = unit * std::max(1, env_int("NSRGS_SYM_H", 384) / unit);
  while (H > maxH && H > unit) H -= unit;
  c.H = H;
  c.nchunks = (nd + c.CW - 1) / c.CW;
  c.nstrips = (nd + H - 1) / H;
  c.prow_bytes = (size_t)c.nchunks * nd * d * tb;
  c.pcol_bytes = (size_t)c.nstrips * nd * d * tb;
  return c;
}

size_t sym_ws_bytes(int n, int d, int fmt, const SymConfig &c) {
  return step_ws_bytes(n, d, fmt) + align256(c.prow_bytes) + align256(c.pcol_bytes);
}

}  // namespace
}  // namespace nsrgs

using namespace nsrgs;

extern "C" {

size_t sync_step_symmetric_workspace_bytes(int n, int d, int fmt) {
  if (n < 2 || d < 1 || d > kSymMaxD || !sym_format(fmt)) return 0;
  if ((int64_t)n * d >= (int64_t)1 << 31) return 0;
  return sym_ws_bytes(n, d, fmt, sym_config(fmt, d, n * d));
}

int sync_step_symmetric(const nsrgs_matrix *A, int n, int d, double mu, int ns_steps, const void *X_in,
                        void *X_out, void *ws, size_t ws_bytes, void *stream) {
  int st;
  if ((st = check_step_args(A, n, d, ns_steps, X_in, X_out, ws, ws_bytes))) return st;
  if (!std::isfinite(mu)) return fail(NSRGS_ERR_INVALID_ARG, "mu must be finite");
  if (!sym_format(A->fmt))
    return fail(NSRGS_ERR_UNSUPPORTED, "sync_step_symmetric: format %d is not stored symmetrically "
                "(FP8 row scales differ between A_ij and A_ji)", (int)A->fmt);
  if (d > kSymMaxD) return fail(NSRGS_ERR_UNSUPPORTED, "sync_step_symmetric supports d <= %d", kSymMaxD);
  const int nd = n * d;
  const SymConfig c = sym_config(A->fmt, d, nd);
  const size_t need = sym_ws_bytes(n, d, A->fmt, c);
  if (ws_bytes < need)
    return fail(NSRGS_ERR_OUT_OF_MEMORY, "workspace too small for sync_step_symmetric: %zu < %zu bytes", ws_bytes,
                need);
  char *base = static_cast<char *>(ws);
  const size_t off = step_ws_bytes(n, d, A->fmt);
  SymArgs a{};
  a.A = A->data;
  a.A_lo = A->fmt == NSRGS_A_BF16_SPLIT ? A->data_lo : nullptr;
  a.ld = A->ld;
  a.X_in = X_in;
  a.nd = nd;
  a.H = c.H;
  a.CW = c.CW;
  a.nchunks = c.nchunks;
  a.nstrips = c.nstrips;
  a.prow = base + off;
  a.pcol = base + off + align256(c.prow_bytes);
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
  sa.partials = base + step_ws_stats_offset(n, d, A->fmt);
  sa.ctl = static_cast<DevCtl *>(ws);
  sa.iter = 0;
  sa.tol = 0.0;
  sa.stop_flag = nullptr;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  switch (A->fmt) {
    case NSRGS_A_F64: e = launch_sym_f64(d, c.unroll, a, sa, c.waves, s); break;
    case NSRGS_A_F32: e = launch_sym_f32(d, c.unroll, a, sa, c.waves, s); break;
    case NSRGS_A_BF16: e = launch_sym_bf16(d, c.unroll, a, sa, c.waves, s); break;
    default: e = launch_sym_split(d, c.unroll, a, sa, c.waves, s); break;
  }
  NSRGS_HIP(e, "symmetric step launch");
  return NSRGS_OK;
}

}  // extern "C"
