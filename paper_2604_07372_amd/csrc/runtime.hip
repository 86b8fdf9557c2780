// C ABI of the NS-RGS library: argument checks, workspace layout, launch
// configuration and the host side of the solve loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "device.h"
#include "host.h"
#include "kernels.h"
#include "nsrgs.h"
#include "wide.h"

namespace nsrgs {

static thread_local std::string g_last_error;

int fail(int status, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return status;
}

int dev_fail(hipError_t e, const char *what) {
  return fail(NSRGS_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}


bool valid_fmt(int fmt) { return fmt >= NSRGS_A_F64 && fmt <= NSRGS_A_FP8_E4M3; }
size_t xbytes(int fmt) { return fmt == NSRGS_A_F64 ? 8 : 4; }

size_t elem_size(int fmt) {
  switch (fmt) {
    case NSRGS_A_F64: return 8;
    case NSRGS_A_F32: return 4;
    case NSRGS_A_BF16: return 2;
    case NSRGS_A_BF16_SPLIT: return 4;
    default: return 1;
  }
}
size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// ---- workspace layout ------------------------------------------------------
struct WsLayout {
  size_t ctl, stats, xalt, y0, y1, w, parts, wide, total;
};

// The workspace of one problem.  It ends with the matrix-core path's region
// (partial products, per-block records, objective pieces), sized by the
// iterate precision only, so one workspace serves every retraction, every
// d <= 32, and every storage format with the same iterate precision.
static WsLayout layout(int n, int d, int fmt) {
  const size_t nd = (size_t)n * d;
  const size_t xb = xbytes(fmt);
  WsLayout L{};
  size_t off = 0;
  L.ctl = off;   off += align256(sizeof(DevCtl));
  L.stats = off; off += align256((size_t)n * sizeof(PanelStat));  // <= n panels
  L.xalt = off;  off += align256(nd * d * xb);                    // ping-pong iterate
  L.y0 = off;    off += align256(nd * d * xb);                    // init basis
  L.y1 = off;    off += align256(nd * d * xb);
  L.w = off;     off += align256(nd * d * xb);                    // A Y
  const size_t gram = (size_t)n * 2 * d * d * xb;                 // <= n panels
  const size_t apply = ((nd + 255) / 256) * 2 * sizeof(double);
  L.parts = off; off += align256(std::max(gram, apply));
  L.wide = off;
  off += align256(wide_layout(n, d, fmt).total);
  L.total = off;
  return L;
}

int check_common(int n, int d) {
  if (n < 2) return fail(NSRGS_ERR_INVALID_ARG, "n must be >= 2 (got %d)", n);
  if (d < 1 || d > kMaxD) return fail(NSRGS_ERR_INVALID_ARG, "d must be in [1, %d] (got %d)", kMaxD, d);
  if ((int64_t)n * d >= (int64_t)1 << 31) return fail(NSRGS_ERR_INVALID_ARG, "n*d too large");
  return NSRGS_OK;
}

// The single-problem calls also take 16 < d <= 32 (matrix-core path, F64 and
// F32 storage).
static int check_common_wide(int n, int d, int fmt) {
  if (d > kMaxD && d <= kWideMaxD) {
    if (n < 2) return fail(NSRGS_ERR_INVALID_ARG, "n must be >= 2 (got %d)", n);
    if ((int64_t)n * d >= (int64_t)1 << 31) return fail(NSRGS_ERR_INVALID_ARG, "n*d too large");
    if (!wide_supported_fmt(fmt))
      return fail(NSRGS_ERR_UNSUPPORTED, "d = %d (> %d) needs F64 or F32 storage", d, kMaxD);
    return NSRGS_OK;
  }
  if (d > kWideMaxD || d < 1) return fail(NSRGS_ERR_INVALID_ARG, "d must be in [1, %d] (got %d)", kWideMaxD, d);
  return check_common(n, d);
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

int check_matrix(const nsrgs_matrix *A, int n, int d, bool packed_ok) {
  if (!A) return fail(NSRGS_ERR_INVALID_ARG, "A is NULL");
  if (!valid_fmt(A->fmt)) return fail(NSRGS_ERR_INVALID_ARG, "unknown A format %d", (int)A->fmt);
  if (!A->data) return fail(NSRGS_ERR_INVALID_ARG, "A->data is NULL");
  const int64_t nd = (int64_t)n * d;
  if (A->ld == NSRGS_LD_PACKED) {
    if (!packed_ok)
      return fail(NSRGS_ERR_UNSUPPORTED, "packed storage is read by sync_step_symmetric, symmetric solves and "
                  "sync_init_spectral only");
  } else {
    if (A->ld < nd) return fail(NSRGS_ERR_INVALID_ARG, "ld (%lld) < n*d (%lld)", (long long)A->ld, (long long)nd);
    if (A->ld % 16) return fail(NSRGS_ERR_INVALID_ARG, "ld (%lld) must be a multiple of 16", (long long)A->ld);
  }
  if (!aligned16(A->data)) return fail(NSRGS_ERR_INVALID_ARG, "A->data must be 16-byte aligned");
  if (A->fmt == NSRGS_A_BF16_SPLIT) {
    if (!A->data_lo) return fail(NSRGS_ERR_INVALID_ARG, "BF16_SPLIT needs data_lo");
    if (!aligned16(A->data_lo)) return fail(NSRGS_ERR_INVALID_ARG, "A->data_lo must be 16-byte aligned");
  }
  if (A->fmt == NSRGS_A_FP8_E4M3 && !A->row_scale)
    return fail(NSRGS_ERR_INVALID_ARG, "FP8_E4M3 needs row_scale");
  return NSRGS_OK;
}

// A workspace of sync_workspace_bytes() serves every call; the calls that
// stay on the streaming kernels (d <= 16, NS-RGS, relative-change stop) only
// touch the part before the matrix-core region and accept that much.
static int check_ws(const void *ws, size_t ws_bytes, int n, int d, int fmt, bool wide = false) {
  if (!ws) return fail(NSRGS_ERR_INVALID_ARG, "workspace is NULL");
  if (((uintptr_t)ws & 255u) != 0) return fail(NSRGS_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  const WsLayout L = layout(n, d, fmt);
  const size_t need = wide ? L.total : L.wide;
  if (ws_bytes < need)
    return fail(NSRGS_ERR_OUT_OF_MEMORY, "workspace too small: %zu < %zu bytes", ws_bytes, need);
  return NSRGS_OK;
}

static bool overlap(const void *a, const void *b, size_t bytes) {
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + bytes && y < x + bytes;
}

// ---- launch configuration --------------------------------------------------
int env_int(const char *name, int dflt) {
  const char *v = getenv(name);
  return (v && *v) ? atoi(v) : dflt;
}

// ---- tuning table (written by the autotuner, read at every launch) --------
static std::mutex g_tune_mu;
static std::vector<nsrgs_tune_entry> g_tune;

static bool tuned_step(int fmt, int d, int nd, StreamConfig *cfg) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  StreamConfig v[16];
  const int nv = stream_variants(d, v, 16);
  for (const nsrgs_tune_entry &e : g_tune) {
    if (e.kind != 0 || e.fmt != fmt || e.d != d || nd < e.nd_min || nd > e.nd_max) continue;
    for (int i = 0; i < nv; ++i)
      if (v[i].blocks_per_panel == e.blocks_per_panel && v[i].unroll == e.unroll &&
          e.waves >= 1 && e.waves <= kMaxWaves) {
        *cfg = StreamConfig{e.blocks_per_panel, e.waves, e.unroll};
        return true;
      }
  }
  return false;
}

int tuned_batch_waves(int fmt, int dmax) {
  const int forced = env_int("NSRGS_BATCH_W", 0);
  if (forced >= 1 && forced <= kMaxWaves) return forced;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const nsrgs_tune_entry &e : g_tune)
    if (e.kind == 1 && e.fmt == fmt && dmax <= e.d && e.waves >= 1 && e.waves <= kMaxWaves) return e.waves;
  return 1;
}

StreamConfig choose_stream_config(int fmt, int d, int nd, int mode) {
  StreamConfig cfg{stream_block_init(d), 1, 1};
  const int fb = env_int("NSRGS_STEP_B", 0), fu = env_int("NSRGS_STEP_U", -1);
  const bool forced = fb > 0 || fu >= 0 || env_int("NSRGS_STEP_W", 0) > 0;
  if (mode == 0 && !forced && tuned_step(fmt, d, nd, &cfg)) return cfg;
  if (mode == 0) {
    StreamConfig v[16];
    const int nv = stream_variants(d, v, 16);
    // Default: one vector per row per iteration (U = 1) with the largest
    // panel of at most 12 rows (every d has a B = 1, U = 1 shape).  The
    // autotuner's table, or the environment (NSRGS_STEP_B/U/W), selects any
    // compiled shape.
    cfg.blocks_per_panel = 1;
    cfg.unroll = 1;
    for (int i = 0; i < nv; ++i)
      if (v[i].unroll == 1 && v[i].blocks_per_panel * d <= 12 && v[i].blocks_per_panel > cfg.blocks_per_panel)
        cfg.blocks_per_panel = v[i].blocks_per_panel;
    if (fb > 0 || fu >= 0) {
      const int wb = fb > 0 ? fb : cfg.blocks_per_panel, wu = fu >= 0 ? fu : cfg.unroll;
      for (int i = 0; i < nv; ++i)
        if (v[i].blocks_per_panel == wb && v[i].unroll == wu) {
          cfg.blocks_per_panel = wb;
          cfg.unroll = wu;
        }
    }
  }
  const int R = cfg.blocks_per_panel * d;
  const int panels = (nd + R - 1) / R;
  // Enough waves to cover 256 CUs several times over, while every wave keeps
  // a few column groups of work.
  const int V = fmt == NSRGS_A_F64 ? 2 : fmt == NSRGS_A_F32 ? 4 : fmt == NSRGS_A_FP8_E4M3 ? 16 : 8;
  const int group = 64 * V * (cfg.unroll > 0 ? cfg.unroll : 1);
  const int groups = (nd + group - 1) / group;
  int W = 1;
  while (W < kMaxWaves && (int64_t)panels * W < 8192 && groups / (2 * W) >= 4) W *= 2;
  const int forced_w = env_int("NSRGS_STEP_W", 0);
  if (forced_w >= 1 && forced_w <= kMaxWaves) W = forced_w;
  cfg.waves = W;
  return cfg;
}

static StreamArgs make_args(const nsrgs_matrix *A, int n, int d, const StreamConfig &cfg) {
  StreamArgs a{};
  a.A = A->data;
  a.A_lo = A->fmt == NSRGS_A_BF16_SPLIT ? A->data_lo : nullptr;
  a.scale = A->fmt == NSRGS_A_FP8_E4M3 ? A->row_scale : nullptr;
  a.ld = A->ld;
  a.n = n;
  a.d = d;
  a.nd = n * d;
  const int R = cfg.blocks_per_panel * d;
  a.num_panels = (a.nd + R - 1) / R;
  return a;
}

}  // namespace nsrgs

using namespace nsrgs;

extern "C" {

const char *nsrgs_status_string(int status) {
  switch (status) {
    case NSRGS_OK: return "ok";
    case NSRGS_ERR_INVALID_ARG: return "invalid argument";
    case NSRGS_ERR_UNSUPPORTED: return "unsupported";
    case NSRGS_ERR_OUT_OF_MEMORY: return "out of memory";
    case NSRGS_ERR_DEVICE: return "device error";
    case NSRGS_ERR_NOT_CONVERGED: return "not converged";
    case NSRGS_ERR_NONFINITE: return "non-finite iterate";
    default: return "unknown status";
  }
}

const char *nsrgs_last_error(void) { return g_last_error.c_str(); }

int nsrgs_version(void) { return NSRGS_VERSION; }

size_t sync_workspace_bytes(int n, int d, int fmt) {
  if (n < 2 || d < 1 || d > kWideMaxD || !valid_fmt(fmt)) return 0;
  if (d > kMaxD && !wide_supported_fmt(fmt)) return 0;
  return layout(n, d, fmt).total;
}

int sync_workspace_init(void *ws, size_t ws_bytes, void *stream) {
  if (!ws || ((uintptr_t)ws & 255u)) return fail(NSRGS_ERR_INVALID_ARG, "workspace must be non-NULL and 256-byte aligned");
  if (ws_bytes < sizeof(DevCtl)) return fail(NSRGS_ERR_OUT_OF_MEMORY, "workspace too small");
  NSRGS_HIP(launch_ctl_reset(static_cast<DevCtl *>(ws), 0, (hipStream_t)stream), "ctl reset");
  return NSRGS_OK;
}

// One step launch with the control block and panel monitors at given
// addresses; `force` (nullable) replaces the chosen launch shape.
static int step_into(const nsrgs_matrix *A, int n, int d, double mu, int ns_steps,
                     const void *X_in, void *X_out, DevCtl *ctl, void *stats, hipStream_t s,
                     int iter, double tol, bool check_done, const StreamConfig *force = nullptr) {
  const StreamConfig cfg = force ? *force : choose_stream_config(A->fmt, d, n * d, 0);
  StreamArgs a = make_args(A, n, d, cfg);
  a.X_in = X_in;
  a.X_out = X_out;
  a.mu = mu > 0.0 ? mu : 1.0 / n;
  a.ns_steps = ns_steps;
  a.partials = stats;
  a.ctl = ctl;
  a.iter = iter;
  a.tol = tol;
  a.stop_flag = check_done ? &a.ctl->done : nullptr;
  NSRGS_HIP(launch_stream(0, A->fmt, cfg, a, s), "step launch");
  return NSRGS_OK;
}

static int step_impl(const nsrgs_matrix *A, int n, int d, double mu, int ns_steps,
                     const void *X_in, void *X_out, void *ws, hipStream_t s, int iter,
                     double tol, bool check_done, const StreamConfig *force = nullptr) {
  const WsLayout L = layout(n, d, A->fmt);
  return step_into(A, n, d, mu, ns_steps, X_in, X_out, static_cast<DevCtl *>(ws),
                   static_cast<char *>(ws) + L.stats, s, iter, tol, check_done, force);
}

// sync_step's checks of everything but the workspace (wide: 16 < d <= 32
// allowed for F64 / F32 storage).
static int check_step_io(const nsrgs_matrix *A, int n, int d, double mu, int ns_steps,
                         const void *X_in, const void *X_out, bool wide = false) {
  int st;
  if (wide && A && valid_fmt(A->fmt)) {
    if ((st = check_common_wide(n, d, A->fmt))) return st;
  } else if ((st = check_common(n, d))) {
    return st;
  }
  if ((st = check_matrix(A, n, d))) return st;
  if (!X_in || !X_out) return fail(NSRGS_ERR_INVALID_ARG, "X_in / X_out is NULL");
  if (!aligned16(X_in) || !aligned16(X_out)) return fail(NSRGS_ERR_INVALID_ARG, "X buffers must be 16-byte aligned");
  if (ns_steps < 0 || ns_steps > 64) return fail(NSRGS_ERR_INVALID_ARG, "ns_steps must be in [0, 64]");
  if (!std::isfinite(mu)) return fail(NSRGS_ERR_INVALID_ARG, "mu must be finite");
  const size_t xb = (size_t)n * d * d * xbytes(A->fmt);
  if (overlap(X_in, X_out, xb)) return fail(NSRGS_ERR_INVALID_ARG, "X_in and X_out overlap");
  return NSRGS_OK;
}

// ---- matrix-core path (wide.h): d up to 32 and the three retractions ------
}  // extern "C"

namespace nsrgs {
WideArgs wide_args(const nsrgs_matrix *A, int n, int d, void *ws) {
  const WsLayout L = layout(n, d, A->fmt);
  const WideLayout W = wide_layout(n, d, A->fmt);
  char *base = static_cast<char *>(ws) + L.wide;
  WideArgs a{};
  a.A = A->data;
  a.ld = A->ld;
  a.n = n;
  a.d = d;
  a.p = d;
  a.nd = n * d;
  a.part = base + W.part;
  a.xs = base + W.xs;
  a.stats = reinterpret_cast<WideStat *>(base + W.stats);
  a.igram = reinterpret_cast<double *>(base + W.igram);
  a.gram = reinterpret_cast<double *>(base + W.gram);
  a.sumsq = nullptr;
  a.ctl = static_cast<DevCtl *>(ws);
  a.wctl = reinterpret_cast<WideCtl *>(base + W.ctl);
  a.g = wide_geom(n, d, A->fmt);
  return a;
}
}  // namespace nsrgs

extern "C" {

static WideCtl *wide_ctl(void *ws, int n, int d, int fmt) {
  return reinterpret_cast<WideCtl *>(static_cast<char *>(ws) + layout(n, d, fmt).wide + wide_layout(n, d, fmt).ctl);
}

// One iteration on the matrix-core path.  objective: evaluate F(X^t) (the
// constant part of F is computed from A on the solve's first iteration).
// chain: a step of a solve's run of steps on the same workspace; its
// epilogue writes X^{t+1} in the product's operand order as well, and
// xs_ready says that the previous step of the run did so for X_in.
static int wide_step_impl(const nsrgs_matrix *A, int n, int d, double mu, int ns_steps, int method,
                          const void *X_in, void *X_out, void *ws, hipStream_t s, int iter, double tol,
                          int stop_rule, bool objective, bool check_done, bool chain = false,
                          bool xs_ready = false) {
  WideArgs a = wide_args(A, n, d, ws);
  a.xs_write = chain ? 1 : 0;
  a.xs_ready = chain && xs_ready ? 1 : 0;
  a.X_in = X_in;
  a.X_out = X_out;
  a.mu = mu > 0.0 ? mu : 1.0 / n;
  a.ns_steps = ns_steps;
  a.method = method;
  a.mode = WIDE_STEP;
  a.iter = iter;
  a.tol = tol;
  a.stop_rule = stop_rule;
  a.objective = objective ? 1 : 0;
  if (objective && iter == 0) {
    const WsLayout L = layout(n, d, A->fmt);
    a.sumsq = reinterpret_cast<double *>(static_cast<char *>(ws) + L.wide + wide_layout(n, d, A->fmt).sumsq);
  }
  a.stop_flag = check_done ? &a.ctl->done : nullptr;
  NSRGS_HIP(launch_wide_step(A->fmt, a, s), "matrix-core step launch");
  return NSRGS_OK;
}

// NS-RGS with d <= 16 on F64 / F32 storage also runs on the matrix-core
// product when the workspace holds its region: from d = 10 (F64) and d = 13
// (F32) on, where it measured faster than the streaming kernel, whose 2d
// FMAs per element of A outgrow the vector units (n d = 30000: F64 d = 10
// 2.42 -> 1.72 ms, d = 16 49.7 -> 1.59 ms; F32 d = 13 1.14 -> 0.93 ms, d = 16
// 3.32 -> 0.92 ms).  NSRGS_WIDE_FROM_D overrides the threshold.
static bool ns_on_matrix_cores(int fmt, int d, size_t ws_bytes, int n) {
  if (d > kMaxD) return true;
  if (!wide_supported_fmt(fmt)) return false;
  const int from = env_int("NSRGS_WIDE_FROM_D", fmt == NSRGS_A_F64 ? 10 : 13);
  return d >= from && ws_bytes >= layout(n, d, fmt).total;
}

static int step_method_entry(const nsrgs_matrix *A, int n, int d, double mu, int ns_steps, int method,
                             const void *X_in, void *X_out, void *ws, size_t ws_bytes, void *stream) {
  int st;
  if ((st = check_step_io(A, n, d, mu, ns_steps, X_in, X_out, true))) return st;
  if ((st = check_ws(ws, ws_bytes, n, d, A->fmt, method != WIDE_NS || d > kMaxD))) return st;
  if (method == WIDE_NS && !ns_on_matrix_cores(A->fmt, d, ws_bytes, n))
    return step_impl(A, n, d, mu, ns_steps, X_in, X_out, ws, (hipStream_t)stream, 0, 0.0, false);
  if (!wide_supported_fmt(A->fmt))
    return fail(NSRGS_ERR_UNSUPPORTED, "this retraction / block size needs F64 or F32 storage");
  return wide_step_impl(A, n, d, mu, ns_steps, method, X_in, X_out, ws, (hipStream_t)stream, 0, 0.0, 0,
                        false, false);
}

int sync_step(const nsrgs_matrix *A, int n, int d, double mu, int ns_steps, const void *X_in,
              void *X_out, void *ws, size_t ws_bytes, void *stream) {
  return step_method_entry(A, n, d, mu, ns_steps, WIDE_NS, X_in, X_out, ws, ws_bytes, stream);
}

int sync_step_polar(const nsrgs_matrix *A, int n, int d, double mu, const void *X_in, void *X_out,
                    void *ws, size_t ws_bytes, void *stream) {
  return step_method_entry(A, n, d, mu, 0, WIDE_POLAR, X_in, X_out, ws, ws_bytes, stream);
}

int sync_step_gpm(const nsrgs_matrix *A, int n, int d, const void *X_in, void *X_out, void *ws,
                  size_t ws_bytes, void *stream) {
  return step_method_entry(A, n, d, 0.0, 0, WIDE_GPM, X_in, X_out, ws, ws_bytes, stream);
}

}  // extern "C"

namespace nsrgs {
int check_step_inputs(const nsrgs_matrix *A, int n, int d, double mu, int ns_steps, const void *X_in,
                      const void *X_out) {
  return check_step_io(A, n, d, mu, ns_steps, X_in, X_out);
}

// sync_step with caller-placed control block and panel monitors: the
// no-allocation entry point's path.  The arguments are checked here.
int step_checked_into(const nsrgs_matrix *A, int n, int d, double mu, int ns_steps, const void *X_in,
                      void *X_out, DevCtl *ctl, void *stats, size_t stats_bytes, hipStream_t s) {
  int st;
  if ((st = check_step_io(A, n, d, mu, ns_steps, X_in, X_out))) return st;
  const StreamConfig cfg = choose_stream_config(A->fmt, d, n * d, 0);
  const int R = cfg.blocks_per_panel * d;
  const size_t panels = (size_t)(n * d + R - 1) / R;
  if (panels * sizeof(PanelStat) > stats_bytes)
    return fail(NSRGS_ERR_OUT_OF_MEMORY,
                "problem too large for the fixed scratch: %zu panel monitors need %zu bytes, %zu available",
                panels, panels * sizeof(PanelStat), stats_bytes);
  return step_into(A, n, d, mu, ns_steps, X_in, X_out, ctl, stats, s, 0, 0.0, false, &cfg);
}

size_t step_ws_bytes(int n, int d, int fmt) { return layout(n, d, fmt).total; }
size_t narrow_ws_bytes(int n, int d, int fmt) { return layout(n, d, fmt).wide; }
size_t step_ws_stats_offset(int n, int d, int fmt) { return layout(n, d, fmt).stats; }

// sync_step with a given launch shape (the autotuner's timing loop); the
// arguments must already have passed sync_step's checks.
int step_with_config(const nsrgs_matrix *A, int n, int d, double mu, int ns_steps, const void *X_in,
                     void *X_out, void *ws, hipStream_t s, const StreamConfig &cfg) {
  return step_impl(A, n, d, mu, ns_steps, X_in, X_out, ws, s, 0, 0.0, false, &cfg);
}

int check_step_args(const nsrgs_matrix *A, int n, int d, int ns_steps, const void *X_in, void *X_out,
                    void *ws, size_t ws_bytes, bool packed_ok) {
  int st;
  if ((st = check_common(n, d))) return st;
  if ((st = check_matrix(A, n, d, packed_ok))) return st;
  if ((st = check_ws(ws, ws_bytes, n, d, A->fmt))) return st;
  if (!X_in || !X_out) return fail(NSRGS_ERR_INVALID_ARG, "X_in / X_out is NULL");
  if (!aligned16(X_in) || !aligned16(X_out)) return fail(NSRGS_ERR_INVALID_ARG, "X buffers must be 16-byte aligned");
  if (ns_steps < 0 || ns_steps > 64) return fail(NSRGS_ERR_INVALID_ARG, "ns_steps must be in [0, 64]");
  if (overlap(X_in, X_out, (size_t)n * d * d * xbytes(A->fmt)))
    return fail(NSRGS_ERR_INVALID_ARG, "X_in and X_out overlap");
  return NSRGS_OK;
}
}  // namespace nsrgs

extern "C" {

static void fill_info(const DevCtl &c, int d, nsrgs_info *info, int status) {
  if (!info) return;
  memset(info, 0, sizeof(*info));
  info->objective = NAN;
  info->objective_ratio = NAN;
  info->iters = c.iters;
  info->nonfinite = c.nonfinite;
  info->converged = c.converged;
  info->status = status;
  info->rel_change = c.rel_change;
  info->max_orth_defect = c.max_defect;
  info->init_residual = c.init_res;
  for (int i = 0; i < d && i < 16; ++i) info->ritz[i] = c.ritz[i];
  info->ritz_next = NAN;
}

static int read_ctl(const void *ws, DevCtl *host, hipStream_t s) {
  NSRGS_HIP(hipMemcpyAsync(host, ws, sizeof(DevCtl), hipMemcpyDeviceToHost, s), "ctl readback");
  NSRGS_HIP(hipStreamSynchronize(s), "stream sync");
  return NSRGS_OK;
}

// The objective and Ritz values the matrix-core path keeps in its own control block.
static int read_wide_info(const void *ws, int n, int d, int fmt, nsrgs_info *info, hipStream_t s) {
  if (!info || !wide_supported_fmt(fmt)) return NSRGS_OK;
  WideCtl w;
  NSRGS_HIP(hipMemcpyAsync(&w, wide_ctl(const_cast<void *>(ws), n, d, fmt), sizeof(WideCtl),
                           hipMemcpyDeviceToHost, s), "wide ctl readback");
  NSRGS_HIP(hipStreamSynchronize(s), "stream sync");
  info->objective = w.obj;
  info->objective_ratio = w.obj_ratio;
  if (d > kMaxD)
    for (int i = kMaxD; i < d; ++i) info->ritz_more[i - kMaxD] = w.ritz[i];
  return NSRGS_OK;
}

int sync_read_info(const void *ws, size_t ws_bytes, int n, int d, int fmt, nsrgs_info *info,
                   void *stream) {
  int st;
  if (!valid_fmt(fmt)) return fail(NSRGS_ERR_INVALID_ARG, "unknown format");
  if ((st = check_common_wide(n, d, fmt))) return st;
  if ((st = check_ws(ws, ws_bytes, n, d, fmt))) return st;
  if (!info) return fail(NSRGS_ERR_INVALID_ARG, "info is NULL");
  DevCtl c;
  if ((st = read_ctl(ws, &c, (hipStream_t)stream))) return st;
  fill_info(c, d, info, NSRGS_OK);
  info->iters = c.iters ? c.iters : c.init_iters;
  if (ws_bytes < layout(n, d, fmt).total) return NSRGS_OK;   // no matrix-core region
  return read_wide_info(ws, n, d, fmt, info, (hipStream_t)stream);
}

// Spectral initialization for 16 < d <= 32 on the matrix-core product (the
// same subspace iteration, Cholesky-QR and polar as init_impl).
// The subspace iteration of the initialization for the matrix-core epilogue,
// with the product launched by `product` (dense MFMA or block-sparse): it
// must write W = A Y's partials and run the init epilogue (launch_wide_init_post).
extern "C++" {
template <typename Product>
static int wide_init_loop(int fmt, int n, int d, void *X0, int max_iters, double tol, void *ws, hipStream_t s,
                          DevCtl *out_ctl, WideArgs a, Product product) {
  const int nd = n * d;
  const WsLayout L = layout(n, d, fmt);
  char *base = static_cast<char *>(ws);
  DevCtl *ctl = static_cast<DevCtl *>(ws);
  void *Y[2] = {base + L.y0, base + L.y1};
  void *W = base + L.w;
  if (max_iters <= 0) max_iters = 60;
  if (!(tol > 0.0)) tol = fmt == NSRGS_A_F64 ? 1e-13 : 1e-5;
  NSRGS_HIP(launch_ctl_reset(ctl, 2, s), "ctl reset");
  NSRGS_HIP(launch_init_random(fmt, Y[0], nd, d, 0x5eed5eedULL, s), "init random");
  a.mode = WIDE_INIT;
  a.X_out = W;
  a.stop_flag = &ctl->init_done;
  const int groups = (int)(((int64_t)nd * d + 255) / 256);
  // 2 doubles per 256 entries; the per-block Grams are consumed (reduced)
  // before the apply kernel runs, so their area holds the apply partials
  double *apply_part = a.igram;
  DevCtl host{};
  int k = 0;
  const int chunk = 4;
  while (k < max_iters) {
    const int kend = std::min(max_iters, k + chunk);
    for (; k < kend; ++k) {
      a.X_in = Y[k & 1];
      a.iter = k;
      NSRGS_HIP(product(a), "init product");
      NSRGS_HIP(launch_wide_init_apply(fmt, W, Y[k & 1], Y[(k + 1) & 1], nd, d, apply_part, groups, ctl,
                                       a.wctl, k, tol, s), "init apply");
    }
    int st;
    if ((st = read_ctl(ws, &host, s))) return st;
    if (host.init_done) break;
  }
  const int done_iters = host.init_iters;
  NSRGS_HIP(launch_wide_init_polar(fmt, Y[done_iters & 1], X0, n, d, ctl, s), "init polar");
  NSRGS_HIP(launch_wide_init_finish(ctl, a.wctl, d, s), "init finish");
  int st;
  if ((st = read_ctl(ws, &host, s))) return st;
  if (out_ctl) *out_ctl = host;
  if (host.init_bad) return fail(NSRGS_ERR_NONFINITE, "spectral init broke down (Cholesky/polar)");
  if (!host.init_done) return NSRGS_ERR_NOT_CONVERGED;
  return NSRGS_OK;
}
}  // extern "C++"

static int wide_init_impl(const nsrgs_matrix *A, int n, int d, void *X0, int max_iters, double tol,
                          void *ws, hipStream_t s, DevCtl *out_ctl) {
  const int fmt = A->fmt;
  return wide_init_loop(fmt, n, d, X0, max_iters, tol, ws, s, out_ctl, wide_args(A, n, d, ws),
                        [&](const WideArgs &a) { return launch_wide_init_product(fmt, a, s); });
}

// sym: the product runs on the symmetric half-stream tiles (A full or packed,
// ws sized for sync_step_symmetric).
static int init_impl(const nsrgs_matrix *A, int n, int d, void *X0, int max_iters, double tol,
                     void *ws, hipStream_t s, DevCtl *out_ctl, bool sym = false) {
  const int nd = n * d;
  const WsLayout L = layout(n, d, A->fmt);
  char *base = static_cast<char *>(ws);
  DevCtl *ctl = static_cast<DevCtl *>(ws);
  void *Y[2] = {base + L.y0, base + L.y1};
  void *W = base + L.w;
  if (max_iters <= 0) max_iters = 60;
  if (!(tol > 0.0)) tol = A->fmt == NSRGS_A_F64 ? 1e-13 : 1e-5;
  NSRGS_HIP(launch_ctl_reset(ctl, 2, s), "ctl reset");
  NSRGS_HIP(launch_init_random(A->fmt, Y[0], nd, d, 0x5eed5eedULL, s), "init random");
  const StreamConfig cfg = choose_stream_config(A->fmt, d, nd, 1);
  StreamArgs a = make_args(A, n, d, cfg);
  a.mu = 0.0;
  a.ns_steps = 0;
  a.partials = base + L.parts;
  a.ctl = ctl;
  a.tol = 0.0;
  a.stop_flag = &ctl->init_done;
  InitArgs ia{};
  ia.W = W;
  ia.nd = nd;
  ia.d = d;
  ia.partials = base + L.stats;
  ia.num_groups = (nd + 255) / 256;
  ia.ctl = ctl;
  ia.tol = tol;
  // The stats area holds the apply partials: 2 doubles per 256 rows <= n * 32 bytes.
  DevCtl host{};
  int k = 0;
  const int chunk = 4;
  while (k < max_iters) {
    const int kend = std::min(max_iters, k + chunk);
    for (; k < kend; ++k) {
      a.X_in = Y[k & 1];
      a.X_out = W;
      a.iter = k;
      // Launches enqueued after the residual test has passed return at once
      // (they watch init_done), so W, T and Y keep the converged iteration.
      if (sym) {
        const int st = sym_init_product(A, n, d, Y[k & 1], W, base + L.parts, ws, s, k);
        if (st) return st;
      } else {
        NSRGS_HIP(launch_stream(1, A->fmt, cfg, a, s), "init product");
      }
      ia.Y = Y[k & 1];
      ia.Y_next = Y[(k + 1) & 1];
      ia.iter = k;
      NSRGS_HIP(launch_init_apply(A->fmt, ia, s), "init apply");
    }
    int st;
    if ((st = read_ctl(ws, &host, s))) return st;
    if (host.init_done) break;
  }
  // The basis of the last completed apply is in Y[init_iters & 1].
  const int done_iters = host.init_iters;
  NSRGS_HIP(launch_init_polar(A->fmt, Y[done_iters & 1], X0, n, d, ctl, s), "init polar");
  NSRGS_HIP(launch_init_finish(ctl, d, s), "init finish");
  int st;
  if ((st = read_ctl(ws, &host, s))) return st;
  if (out_ctl) *out_ctl = host;
  if (host.init_bad) return fail(NSRGS_ERR_NONFINITE, "spectral init broke down (Cholesky/polar)");
  if (!host.init_done) return NSRGS_ERR_NOT_CONVERGED;
  return NSRGS_OK;
}

int sync_init_spectral(const nsrgs_matrix *A, int n, int d, void *X0, int max_iters, double tol,
                       void *ws, size_t ws_bytes, void *stream, nsrgs_info *info) {
  int st;
  if (!A) return fail(NSRGS_ERR_INVALID_ARG, "A is NULL");
  if ((st = check_common_wide(n, d, A->fmt))) return st;
  if ((st = check_matrix(A, n, d, true))) return st;
  const bool packed = A->ld == NSRGS_LD_PACKED;
  if (packed && d > kMaxD)
    return fail(NSRGS_ERR_UNSUPPORTED, "packed storage is read by the symmetric tiles, d <= %d", kMaxD);
  if ((st = check_ws(ws, ws_bytes, n, d, A->fmt, d > kMaxD))) return st;
  if (packed && (st = sym_check(A, n, d, ws_bytes))) return st;
  if (!X0 || !aligned16(X0)) return fail(NSRGS_ERR_INVALID_ARG, "X0 must be non-NULL and 16-byte aligned");
  DevCtl c{};
  st = d > kMaxD ? wide_init_impl(A, n, d, X0, max_iters, tol, ws, (hipStream_t)stream, &c)
                 : init_impl(A, n, d, X0, max_iters, tol, ws, (hipStream_t)stream, &c, packed);
  if (info) {
    fill_info(c, d, info, st);
    info->iters = c.init_iters;
    info->converged = c.init_done && !c.init_bad;
    if (d > kMaxD) {
      const int st2 = read_wide_info(ws, n, d, A->fmt, info, (hipStream_t)stream);
      if (st2) return st2;
    }
  }
  return st;
}

int sync_solve(const nsrgs_matrix *A, int n, int d, double mu, int ns_steps, int max_iters,
               double tol, void *X, void *ws, size_t ws_bytes, void *stream,
               const nsrgs_solve_opts *opts, nsrgs_info *info) {
  int st;
  if (!A) return fail(NSRGS_ERR_INVALID_ARG, "A is NULL");
  nsrgs_solve_opts o{1, 60, 0.0, 0, nullptr, 16, 0, NSRGS_METHOD_NS_RGS, NSRGS_STOP_REL_CHANGE};
  if (opts) o = *opts;
  if ((st = check_common_wide(n, d, A->fmt))) return st;
  if ((st = check_matrix(A, n, d, o.symmetric == 1))) return st;
  if (!X || !aligned16(X)) return fail(NSRGS_ERR_INVALID_ARG, "X must be non-NULL and 16-byte aligned");
  if (ns_steps < 0 || ns_steps > 64) return fail(NSRGS_ERR_INVALID_ARG, "ns_steps must be in [0, 64]");
  if (max_iters < 0) return fail(NSRGS_ERR_INVALID_ARG, "max_iters must be >= 0");
  if (!std::isfinite(mu)) return fail(NSRGS_ERR_INVALID_ARG, "mu must be finite");
  if (o.check_every <= 0) o.check_every = 16;
  if (o.symmetric != 0 && o.symmetric != 1) return fail(NSRGS_ERR_INVALID_ARG, "symmetric must be 0 or 1");
  if (o.method < NSRGS_METHOD_NS_RGS || o.method > NSRGS_METHOD_GPM)
    return fail(NSRGS_ERR_INVALID_ARG, "unknown method %d", (int)o.method);
  if (o.stop_rule != NSRGS_STOP_REL_CHANGE && o.stop_rule != NSRGS_STOP_OBJECTIVE)
    return fail(NSRGS_ERR_INVALID_ARG, "unknown stop rule %d", (int)o.stop_rule);
  // The matrix-core path runs d > 16, the exact-polar and GPM retractions and
  // the objective stop rule.
  const bool wide = d > kMaxD || o.method != NSRGS_METHOD_NS_RGS || o.stop_rule == NSRGS_STOP_OBJECTIVE ||
                    (!o.symmetric && ns_on_matrix_cores(A->fmt, d, ws_bytes, n) &&
                     (o.refine_iters <= 0 || !o.A_refine || wide_supported_fmt(o.A_refine->fmt)));
  if (wide) {
    if (!wide_supported_fmt(A->fmt))
      return fail(NSRGS_ERR_UNSUPPORTED, "d > 16, exact polar, GPM and the objective stop need F64 or F32 storage");
    if (o.symmetric) return fail(NSRGS_ERR_UNSUPPORTED, "the symmetric half-stream runs NS-RGS with d <= 16 only");
    if (o.refine_iters > 0 && o.A_refine && !wide_supported_fmt(o.A_refine->fmt))
      return fail(NSRGS_ERR_UNSUPPORTED, "A_refine must be F64 or F32 on this path");
    if (o.refine_iters > 0 && o.stop_rule == NSRGS_STOP_OBJECTIVE)
      return fail(NSRGS_ERR_UNSUPPORTED, "the objective stop rule does not combine with refinement");
  }
  if ((st = check_ws(ws, ws_bytes, n, d, A->fmt, wide))) return st;
  if (o.symmetric) {
    if ((st = sym_check(A, n, d, ws_bytes))) return st;
    if (o.refine_iters > 0 && o.A_refine && (st = sym_check(o.A_refine, n, d, ws_bytes))) return st;
  }
  const bool objective = o.stop_rule == NSRGS_STOP_OBJECTIVE;
  // one iteration on matrix M, with the solve's iteration index and stop rule
  // xs_ready: the previous launch of this phase was a matrix-core step (its
  // epilogue wrote this step's X in operand order); each phase's first step
  // stages X itself
  auto iterate = [&](const nsrgs_matrix *M, const void *xi, void *xo, int t, double tl, bool xs_ready) {
    if (wide)
      return wide_step_impl(M, n, d, mu, ns_steps, o.method, xi, xo, ws, (hipStream_t)stream, t, tl,
                            o.stop_rule, objective, true, true, xs_ready);
    return o.symmetric ? sym_step_launch(M, n, d, mu, ns_steps, xi, xo, ws, (hipStream_t)stream, t, tl, true)
                       : step_impl(M, n, d, mu, ns_steps, xi, xo, ws, (hipStream_t)stream, t, tl, true);
  };
  int refine = 0;
  if (o.refine_iters > 0 && o.A_refine) {
    if ((st = check_matrix(o.A_refine, n, d, o.symmetric == 1))) return st;
    if (xbytes(o.A_refine->fmt) != xbytes(A->fmt))
      return fail(NSRGS_ERR_INVALID_ARG, "A_refine must use the same iterate precision as A");
    if ((st = check_ws(ws, ws_bytes, n, d, o.A_refine->fmt, wide))) return st;
    refine = std::min(o.refine_iters, max_iters);
  } else if (o.refine_iters > 0) {
    return fail(NSRGS_ERR_INVALID_ARG, "refine_iters > 0 needs A_refine");
  }
  hipStream_t s = (hipStream_t)stream;
  const WsLayout L = layout(n, d, A->fmt);
  void *buf[2] = {X, static_cast<char *>(ws) + L.xalt};
  DevCtl host{};
  int init_status = NSRGS_OK;
  if (o.init) {
    init_status = d > kMaxD ? wide_init_impl(A, n, d, X, o.init_iters, o.init_tol, ws, s, &host)
                            : init_impl(A, n, d, X, o.init_iters, o.init_tol, ws, s, &host, o.symmetric == 1);
    if (init_status != NSRGS_OK && init_status != NSRGS_ERR_NOT_CONVERGED) {
      if (info) fill_info(host, d, info, init_status);
      return init_status;
    }
  }
  NSRGS_HIP(launch_ctl_reset(static_cast<DevCtl *>(ws), 1, s), "ctl reset");
  if (wide) NSRGS_HIP(launch_wide_ctl_reset(wide_ctl(ws, n, d, A->fmt), s), "wide ctl reset");
  // Phase 1 on A (early stop allowed), phase 2 on A_refine (fixed count).
  const int phase1 = max_iters - refine;
  int t = 0;
  while (t < phase1) {
    const int tend = std::min(phase1, t + o.check_every);
    for (; t < tend; ++t)
      if ((st = iterate(A, buf[t & 1], buf[(t + 1) & 1], t, tol, t > 0))) return st;
    if ((st = read_ctl(ws, &host, s))) return st;
    if (host.done) break;
  }
  if ((st = read_ctl(ws, &host, s))) return st;
  int done_iters = host.iters;
  const bool stopped_nonfinite = host.nonfinite != 0;
  if (refine > 0 && !stopped_nonfinite) {
    NSRGS_HIP(launch_ctl_reset(static_cast<DevCtl *>(ws), 1, s), "ctl reset");
    for (int r = 0; r < refine; ++r) {
      const int tt = done_iters + r;
      if ((st = iterate(o.A_refine, buf[tt & 1], buf[(tt + 1) & 1], tt, 0.0, r > 0))) return st;
    }
    const int conv = host.converged;
    if ((st = read_ctl(ws, &host, s))) return st;
    done_iters = host.iters;
    host.converged = conv;
  }
  if (done_iters & 1)
    NSRGS_HIP(hipMemcpyAsync(X, buf[1], (size_t)n * d * d * xbytes(A->fmt),
                             hipMemcpyDeviceToDevice, s), "result copy");
  NSRGS_HIP(hipStreamSynchronize(s), "stream sync");
  int result = NSRGS_OK;
  if (host.nonfinite) result = fail(NSRGS_ERR_NONFINITE, "non-finite iterate at iteration %d", done_iters);
  else if (tol > 0.0 && !host.converged) result = NSRGS_ERR_NOT_CONVERGED;
  if (info) {
    fill_info(host, d, info, result);
    info->iters = done_iters;
    info->init_residual = host.init_res;
    if (wide && (st = read_wide_info(ws, n, d, A->fmt, info, s))) return st;
  }
  (void)init_status;
  return result;
}

// ---- block-sparse storage through the matrix-core epilogue ----------------
// The product is the block-sparse kernel (one column chunk, A_ii absent); the
// epilogue, finish, objective and initialization are the dense path's.
static WideArgs bsr_wide_args(int n, int d, void *ws) {
  const nsrgs_matrix shape{NSRGS_A_F32, nullptr, nullptr, nullptr, 0};
  WideArgs a = wide_args(&shape, n, d, ws);
  a.A = nullptr;
  a.ld = 0;
  a.no_diag = 1;
  a.g.ks = 1;
  a.g.rows_pad = n * d;
  a.g.row_tiles = n;          // one sum-of-squares partial per block row
  return a;
}

static double *bsr_sumsq(int n, int d, void *ws) {
  return reinterpret_cast<double *>(static_cast<char *>(ws) + layout(n, d, NSRGS_A_F32).wide +
                                    wide_layout(n, d, NSRGS_A_F32).sumsq);
}

static int bsr_step_launch(const nsrgs_bsr_matrix *A, int n, int d, double mu, int ns_steps, int method,
                           const void *X_in, void *X_out, void *ws, hipStream_t s, int iter, double tol,
                           int stop_rule, bool objective, bool check_done, bool sliced) {
  WideArgs a = bsr_wide_args(n, d, ws);
  a.X_in = X_in;
  a.X_out = X_out;
  a.mu = mu > 0.0 ? mu : 1.0 / n;
  a.ns_steps = ns_steps;
  a.method = method;
  a.mode = WIDE_STEP;
  a.iter = iter;
  a.tol = tol;
  a.stop_rule = stop_rule;
  a.objective = objective ? 1 : 0;
  a.sumsq = (objective && iter == 0) ? bsr_sumsq(n, d, ws) : nullptr;
  a.stop_flag = check_done ? &a.ctl->done : nullptr;
  if (objective) NSRGS_HIP(launch_wide_gram(NSRGS_A_F32, a, s), "gram launch");
  // the sliced product does not form the sum of squares the objective's
  // constant needs on the first iteration
  if (sliced && !a.sumsq)
    NSRGS_HIP(launch_bsr_slice_wide_product(*A, n, d, static_cast<const float *>(X_in), static_cast<float *>(a.part),
                                            ws, a.stop_flag, s), "block-sparse product launch");
  else
    NSRGS_HIP(launch_bsr_wide_product(*A, n, d, static_cast<const float *>(X_in), static_cast<float *>(a.part),
                                      a.sumsq, a.stop_flag, s), "block-sparse product launch");
  NSRGS_HIP(launch_wide_post(NSRGS_A_F32, a, s), "epilogue launch");
  return NSRGS_OK;
}

}  // extern "C"

namespace nsrgs {
int bsr_wide_step(const nsrgs_bsr_matrix *A, int n, int d, double mu, int ns_steps, const void *X_in,
                  void *X_out, void *ws, size_t ws_bytes, hipStream_t s) {
  const size_t need = layout(n, d, NSRGS_A_F32).total;
  if (ws_bytes < need)
    return fail(NSRGS_ERR_OUT_OF_MEMORY, "workspace too small for d = %d: %zu < %zu bytes (sync_workspace_bytes)",
                d, ws_bytes, need);
  return bsr_step_launch(A, n, d, mu, ns_steps, WIDE_NS, X_in, X_out, ws, s, 0, 0.0, 0, false, false, false);
}
}  // namespace nsrgs

extern "C" {

int sync_solve_bsr(const nsrgs_bsr_matrix *A, int n, int d, double mu, int ns_steps, int max_iters, double tol,
                   void *X, void *ws, size_t ws_bytes, void *stream, const nsrgs_solve_opts *opts,
                   nsrgs_info *info) {
  if (n < 2) return fail(NSRGS_ERR_INVALID_ARG, "n must be >= 2 (got %d)", n);
  if (d < 1 || d > kWideMaxD) return fail(NSRGS_ERR_INVALID_ARG, "d must be in [1, %d] (got %d)", kWideMaxD, d);
  if ((int64_t)n * d * d >= (int64_t)1 << 31) return fail(NSRGS_ERR_INVALID_ARG, "n*d*d too large");
  if (!A || !A->row_ptr || !A->col_idx || !A->values) return fail(NSRGS_ERR_INVALID_ARG, "NULL matrix pointer");
  if (A->fmt != NSRGS_A_F32 && A->fmt != NSRGS_A_BF16)
    return fail(NSRGS_ERR_UNSUPPORTED, "block-sparse values must be F32 or BF16");
  if (!X || !aligned16(X)) return fail(NSRGS_ERR_INVALID_ARG, "X must be non-NULL and 16-byte aligned");
  if (ns_steps < 0 || ns_steps > 64) return fail(NSRGS_ERR_INVALID_ARG, "ns_steps must be in [0, 64]");
  if (max_iters < 0) return fail(NSRGS_ERR_INVALID_ARG, "max_iters must be >= 0");
  if (!std::isfinite(mu)) return fail(NSRGS_ERR_INVALID_ARG, "mu must be finite");
  int st;
  if ((st = check_ws(ws, ws_bytes, n, d, NSRGS_A_F32, true))) return st;
  nsrgs_solve_opts o{1, 60, 0.0, 0, nullptr, 16, 0, NSRGS_METHOD_NS_RGS, NSRGS_STOP_REL_CHANGE};
  if (opts) o = *opts;
  if (o.check_every <= 0) o.check_every = 16;
  if (o.method == NSRGS_METHOD_GPM)
    return fail(NSRGS_ERR_UNSUPPORTED, "GPM needs the diagonal blocks, which block-sparse storage omits");
  if (o.method != NSRGS_METHOD_NS_RGS && o.method != NSRGS_METHOD_POLAR)
    return fail(NSRGS_ERR_INVALID_ARG, "unknown method %d", (int)o.method);
  if (o.stop_rule != NSRGS_STOP_REL_CHANGE && o.stop_rule != NSRGS_STOP_OBJECTIVE)
    return fail(NSRGS_ERR_INVALID_ARG, "unknown stop rule %d", (int)o.stop_rule);
  if (o.symmetric || o.refine_iters > 0)
    return fail(NSRGS_ERR_UNSUPPORTED, "block-sparse solves take neither the symmetric step nor refinement");
  hipStream_t s = (hipStream_t)stream;
  const bool objective = o.stop_rule == NSRGS_STOP_OBJECTIVE;
  const WsLayout L = layout(n, d, NSRGS_A_F32);
  void *buf[2] = {X, static_cast<char *>(ws) + L.xalt};
  DevCtl host{};
  // d <= 6 with the larger workspace: every product runs sliced, on one
  // bounds table for the whole call (A does not change during it)
  const bool sliced = bsr_sliced(n, d, ws_bytes);
  if (sliced) NSRGS_HIP(launch_bsr_slice_bounds(*A, n, d, ws, s), "block-sparse bounds launch");
  if (o.init) {
    const int ist = wide_init_loop(NSRGS_A_F32, n, d, X, o.init_iters, o.init_tol, ws, s, &host,
                                   bsr_wide_args(n, d, ws), [&](const WideArgs &a) {
                                     const float *Y = static_cast<const float *>(a.X_in);
                                     float *P = static_cast<float *>(a.part);
                                     hipError_t e = sliced ? launch_bsr_slice_wide_product(*A, n, d, Y, P, ws,
                                                                                          a.stop_flag, s)
                                                           : launch_bsr_wide_product(*A, n, d, Y, P, nullptr,
                                                                                     a.stop_flag, s);
                                     return e != hipSuccess ? e : launch_wide_init_post(NSRGS_A_F32, a, s);
                                   });
    if (ist != NSRGS_OK && ist != NSRGS_ERR_NOT_CONVERGED) {
      if (info) fill_info(host, d, info, ist);
      return ist;
    }
  }
  NSRGS_HIP(launch_ctl_reset(static_cast<DevCtl *>(ws), 1, s), "ctl reset");
  NSRGS_HIP(launch_wide_ctl_reset(wide_ctl(ws, n, d, NSRGS_A_F32), s), "wide ctl reset");
  // NS-RGS with the relative-change rule on the sliced product takes the
  // sliced step's own epilogue (16 blocks per workgroup): at small d the
  // matrix-core epilogue's workgroup per block costs more than the product
  const bool narrow = sliced && o.method == NSRGS_METHOD_NS_RGS && !objective;
  int t = 0;
  while (t < max_iters) {
    const int tend = std::min(max_iters, t + o.check_every);
    for (; t < tend; ++t) {
      st = narrow ? bsr_sliced_iterate(*A, n, d, mu, ns_steps, buf[t & 1], buf[(t + 1) & 1], ws, s, t, tol)
                  : bsr_step_launch(A, n, d, mu, ns_steps, o.method, buf[t & 1], buf[(t + 1) & 1], ws, s, t, tol,
                                    o.stop_rule, objective, true, sliced);
      if (st) return st;
    }
    if ((st = read_ctl(ws, &host, s))) return st;
    if (host.done) break;
  }
  if ((st = read_ctl(ws, &host, s))) return st;
  const int done_iters = host.iters;
  if (done_iters & 1)
    NSRGS_HIP(hipMemcpyAsync(X, buf[1], (size_t)n * d * d * sizeof(float), hipMemcpyDeviceToDevice, s), "result copy");
  NSRGS_HIP(hipStreamSynchronize(s), "stream sync");
  int result = NSRGS_OK;
  if (host.nonfinite) result = fail(NSRGS_ERR_NONFINITE, "non-finite iterate at iteration %d", done_iters);
  else if (tol > 0.0 && !host.converged) result = NSRGS_ERR_NOT_CONVERGED;
  if (info) {
    fill_info(host, d, info, result);
    info->iters = done_iters;
    info->init_residual = host.init_res;
    if (!narrow && (st = read_wide_info(ws, n, d, NSRGS_A_F32, info, s))) return st;
  }
  return result;
}

int nsrgs_set_tuning(const nsrgs_tune_entry *entries, int count) {
  if (count < 0 || (count > 0 && !entries)) return fail(NSRGS_ERR_INVALID_ARG, "bad tuning table");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.assign(entries, entries + count);
  return NSRGS_OK;
}

int nsrgs_get_tuning(nsrgs_tune_entry *entries, int max_count) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const int n = (int)g_tune.size();
  for (int i = 0; i < n && i < max_count; ++i) entries[i] = g_tune[i];
  return n;
}

int nsrgs_step_variants(int d, int32_t *blocks_per_panel, int32_t *unroll, int max_count) {
  StreamConfig v[16];
  const int nv = stream_variants(d, v, 16);
  if (max_count > 0 && (!blocks_per_panel || !unroll)) {
    fail(NSRGS_ERR_INVALID_ARG, "NULL output arrays");
    return -1;
  }
  for (int i = 0; i < nv && i < max_count; ++i) {
    blocks_per_panel[i] = v[i].blocks_per_panel;
    unroll[i] = v[i].unroll;
  }
  return nv;
}

int nsrgs_generate_measurement(const double *Z, int n, int d, double sigma, uint64_t seed,
                               int zero_diag_blocks, double p, int fmt, void *A, int64_t ld,
                               void *stream) {
  int st;
  if (fmt != NSRGS_A_F64 && fmt != NSRGS_A_F32)
    return fail(NSRGS_ERR_INVALID_ARG, "generator writes F64 or F32 only");
  if ((st = check_common_wide(n, d, fmt))) return st;
  if (!Z || !A) return fail(NSRGS_ERR_INVALID_ARG, "Z / A is NULL");
  if (ld != NSRGS_LD_PACKED && ld < (int64_t)n * d) return fail(NSRGS_ERR_INVALID_ARG, "ld < n*d");
  if (!std::isfinite(sigma) || !(p > 0.0) || p > 1.0) return fail(NSRGS_ERR_INVALID_ARG, "bad sigma or p");
  NSRGS_HIP(launch_generate(Z, n, d, sigma, seed, zero_diag_blocks, p, fmt, A, ld, (hipStream_t)stream),
            "generate");
  return NSRGS_OK;
}

int nsrgs_convert(const float *A32, int nd, int64_t ld, const nsrgs_matrix *out, void *stream) {
  if (!A32 || !out || !out->data) return fail(NSRGS_ERR_INVALID_ARG, "NULL argument");
  if (nd < 1 || ld < nd) return fail(NSRGS_ERR_INVALID_ARG, "bad nd / ld");
  if (out->ld != ld) return fail(NSRGS_ERR_INVALID_ARG, "out->ld must equal ld");
  if (out->fmt == NSRGS_A_BF16_SPLIT && !out->data_lo) return fail(NSRGS_ERR_INVALID_ARG, "data_lo is NULL");
  if (out->fmt == NSRGS_A_FP8_E4M3 && !out->row_scale) return fail(NSRGS_ERR_INVALID_ARG, "row_scale is NULL");
  if (out->fmt != NSRGS_A_BF16 && out->fmt != NSRGS_A_BF16_SPLIT && out->fmt != NSRGS_A_FP8_E4M3)
    return fail(NSRGS_ERR_INVALID_ARG, "conversion target must be BF16, BF16_SPLIT or FP8_E4M3");
  NSRGS_HIP(launch_convert(A32, nd, ld, *out, (hipStream_t)stream), "convert");
  return NSRGS_OK;
}

int64_t nsrgs_packed_elems(int n, int d) {
  if (n < 1 || d < 1 || d > kWideMaxD || (int64_t)n * d >= (int64_t)1 << 31) return 0;
  return packed_elems(n, d);
}

int nsrgs_convert_packed(const float *A32, int n, int d, const nsrgs_matrix *out, void *stream) {
  if (!A32 || !out || !out->data) return fail(NSRGS_ERR_INVALID_ARG, "NULL argument");
  const int64_t count = nsrgs_packed_elems(n, d);
  if (count == 0) return fail(NSRGS_ERR_INVALID_ARG, "bad n / d");
  if (out->ld != NSRGS_LD_PACKED) return fail(NSRGS_ERR_INVALID_ARG, "out->ld must be NSRGS_LD_PACKED");
  if (out->fmt == NSRGS_A_FP8_E4M3)
    return fail(NSRGS_ERR_UNSUPPORTED, "packed storage serves the symmetric step, which does not read FP8");
  if (out->fmt != NSRGS_A_BF16 && out->fmt != NSRGS_A_BF16_SPLIT)
    return fail(NSRGS_ERR_INVALID_ARG, "conversion target must be BF16 or BF16_SPLIT");
  if (out->fmt == NSRGS_A_BF16_SPLIT && !out->data_lo) return fail(NSRGS_ERR_INVALID_ARG, "data_lo is NULL");
  NSRGS_HIP(launch_convert_flat(A32, count, *out, (hipStream_t)stream), "convert");
  return NSRGS_OK;
}

}  // extern "C"
