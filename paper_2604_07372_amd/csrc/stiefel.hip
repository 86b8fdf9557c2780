// C ABI of NS-RGS on the Stiefel manifold St(p, d)^n (the extension of the
// method the paper names as future work, Sec. 6): argument checks, workspace
// carve-up, the solve loop and the rounding to O(d)^n.  The kernels are the
// matrix-core path's product and the Stiefel epilogue in wide.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "device.h"
#include "host.h"
#include "kernels.h"
#include "nsrgs.h"
#include "wide.h"

namespace nsrgs {
namespace {

size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }

// The single-problem workspace of (n, d, fmt), then the Stiefel areas: the
// p x p Gram partials and the basis of the rounding, and the second iterate
// buffer of the solve (n d x p).
struct StLayout {
  size_t gram, basis, salt, total;
};

StLayout st_layout(int n, int d, int p, int fmt) {
  StLayout L{};
  size_t off = step_ws_bytes(n, d, fmt);
  L.gram = off;  off += a256((size_t)kWideGramGroups * p * p * sizeof(double));
  L.basis = off; off += a256((size_t)p * d * sizeof(double));
  L.salt = off;  off += a256((size_t)n * d * p * xbytes(fmt));
  L.total = off;
  return L;
}

int check_sizes(int n, int d, int p, int fmt) {
  if (n < 2) return fail(NSRGS_ERR_INVALID_ARG, "n must be >= 2 (got %d)", n);
  if (d < 1 || p < d || p > kWideMaxD)
    return fail(NSRGS_ERR_INVALID_ARG, "need 1 <= d <= p <= %d (got d = %d, p = %d)", kWideMaxD, d, p);
  if ((int64_t)n * d * p >= (int64_t)1 << 31) return fail(NSRGS_ERR_INVALID_ARG, "n*d*p too large");
  if (!valid_fmt(fmt)) return fail(NSRGS_ERR_INVALID_ARG, "unknown format %d", fmt);
  if (!wide_supported_fmt(fmt)) return fail(NSRGS_ERR_UNSUPPORTED, "the Stiefel step needs F64 or F32 storage");
  return NSRGS_OK;
}

int check_ws_st(const void *ws, size_t ws_bytes, int n, int d, int p, int fmt) {
  if (!ws || ((uintptr_t)ws & 255u)) return fail(NSRGS_ERR_INVALID_ARG, "workspace must be non-NULL and 256-byte aligned");
  const size_t need = st_layout(n, d, p, fmt).total;
  if (ws_bytes < need)
    return fail(NSRGS_ERR_OUT_OF_MEMORY, "workspace too small for the Stiefel calls: %zu < %zu bytes", ws_bytes, need);
  return NSRGS_OK;
}

int check_step(const nsrgs_matrix *A, int n, int d, int p, double mu, int ns_steps, const void *S_in,
               const void *S_out) {
  int st;
  if (!A) return fail(NSRGS_ERR_INVALID_ARG, "A is NULL");
  if ((st = check_sizes(n, d, p, A->fmt))) return st;
  if ((st = check_matrix(A, n, d))) return st;
  if (!S_in || !S_out || !aligned16(S_in) || !aligned16(S_out))
    return fail(NSRGS_ERR_INVALID_ARG, "S buffers must be non-NULL and 16-byte aligned");
  if (ns_steps < 0 || ns_steps > 64) return fail(NSRGS_ERR_INVALID_ARG, "ns_steps must be in [0, 64]");
  if (!std::isfinite(mu)) return fail(NSRGS_ERR_INVALID_ARG, "mu must be finite");
  const uintptr_t x = (uintptr_t)S_in, y = (uintptr_t)S_out;
  const size_t bytes = (size_t)n * d * p * xbytes(A->fmt);
  if (x < y + bytes && y < x + bytes) return fail(NSRGS_ERR_INVALID_ARG, "S_in and S_out overlap");
  return NSRGS_OK;
}

// One step launch; iter / tol / check_done as in the solve.
int st_step_launch(const nsrgs_matrix *A, int n, int d, int p, double mu, int ns_steps, const void *S_in,
                   void *S_out, void *ws, hipStream_t s, int iter, double tol, bool check_done) {
  WideArgs a = wide_args(A, n, d, ws);
  a.p = p;
  a.g.nt = p <= 16 ? 1 : 2;
  a.X_in = S_in;
  a.X_out = S_out;
  a.mu = mu > 0.0 ? mu : 1.0 / n;
  a.ns_steps = ns_steps;
  a.method = WIDE_NS;
  a.mode = WIDE_STEP;
  a.iter = iter;
  a.tol = tol;
  a.stop_rule = 0;
  a.objective = 0;
  a.stop_flag = check_done ? &a.ctl->done : nullptr;
  NSRGS_HIP(launch_wide_stiefel_step(A->fmt, a, s), "Stiefel step launch");
  return NSRGS_OK;
}

int read_back(const void *ws, DevCtl *host, hipStream_t s) {
  NSRGS_HIP(hipMemcpyAsync(host, ws, sizeof(DevCtl), hipMemcpyDeviceToHost, s), "ctl readback");
  NSRGS_HIP(hipStreamSynchronize(s), "stream sync");
  return NSRGS_OK;
}

}  // namespace
}  // namespace nsrgs

using namespace nsrgs;

extern "C" {

size_t sync_stiefel_workspace_bytes(int n, int d, int p, int fmt) {
  if (n < 2 || d < 1 || p < d || p > kWideMaxD || !valid_fmt(fmt) || !wide_supported_fmt(fmt)) return 0;
  if ((int64_t)n * d * p >= (int64_t)1 << 31) return 0;
  return st_layout(n, d, p, fmt).total;
}

int sync_step_stiefel(const nsrgs_matrix *A, int n, int d, int p, double mu, int ns_steps, const void *S_in,
                      void *S_out, void *ws, size_t ws_bytes, void *stream) {
  int st;
  if ((st = check_step(A, n, d, p, mu, ns_steps, S_in, S_out))) return st;
  if ((st = check_ws_st(ws, ws_bytes, n, d, p, A->fmt))) return st;
  return st_step_launch(A, n, d, p, mu, ns_steps, S_in, S_out, ws, (hipStream_t)stream, 0, 0.0, false);
}

int sync_solve_stiefel(const nsrgs_matrix *A, int n, int d, int p, double mu, int ns_steps, int max_iters,
                       double tol, void *S, void *ws, size_t ws_bytes, void *stream, nsrgs_info *info) {
  int st;
  if (!A) return fail(NSRGS_ERR_INVALID_ARG, "A is NULL");
  if ((st = check_sizes(n, d, p, A->fmt))) return st;
  if ((st = check_ws_st(ws, ws_bytes, n, d, p, A->fmt))) return st;
  void *alt = static_cast<char *>(ws) + st_layout(n, d, p, A->fmt).salt;
  if ((st = check_step(A, n, d, p, mu, ns_steps, S, alt))) return st;
  if (max_iters < 0) return fail(NSRGS_ERR_INVALID_ARG, "max_iters must be >= 0");
  hipStream_t s = (hipStream_t)stream;
  void *buf[2] = {S, alt};
  DevCtl host{};
  NSRGS_HIP(launch_ctl_reset(static_cast<DevCtl *>(ws), 1, s), "ctl reset");
  const int check_every = 16;
  int t = 0;
  while (t < max_iters) {
    const int tend = std::min(max_iters, t + check_every);
    for (; t < tend; ++t)
      if ((st = st_step_launch(A, n, d, p, mu, ns_steps, buf[t & 1], buf[(t + 1) & 1], ws, s, t, tol, true)))
        return st;
    if ((st = read_back(ws, &host, s))) return st;
    if (host.done) break;
  }
  if ((st = read_back(ws, &host, s))) return st;
  const int done_iters = host.iters;
  if (done_iters & 1)
    NSRGS_HIP(hipMemcpyAsync(S, buf[1], (size_t)n * d * p * xbytes(A->fmt), hipMemcpyDeviceToDevice, s),
              "result copy");
  NSRGS_HIP(hipStreamSynchronize(s), "stream sync");
  int result = NSRGS_OK;
  if (host.nonfinite) result = fail(NSRGS_ERR_NONFINITE, "non-finite iterate at iteration %d", done_iters);
  else if (tol > 0.0 && !host.converged) result = NSRGS_ERR_NOT_CONVERGED;
  if (info) {
    memset(info, 0, sizeof(*info));
    info->iters = done_iters;
    info->nonfinite = host.nonfinite;
    info->converged = host.converged;
    info->status = result;
    info->rel_change = host.rel_change;
    info->max_orth_defect = host.max_defect;
    info->init_residual = NAN;
    info->ritz_next = NAN;
    info->objective = NAN;
    info->objective_ratio = NAN;
  }
  return result;
}

int sync_stiefel_round(const void *S, int n, int d, int p, int fmt, void *X, void *ws, size_t ws_bytes,
                       void *stream) {
  int st;
  if ((st = check_sizes(n, d, p, fmt))) return st;
  if ((st = check_ws_st(ws, ws_bytes, n, d, p, fmt))) return st;
  if (!S || !X || !aligned16(S) || !aligned16(X))
    return fail(NSRGS_ERR_INVALID_ARG, "S / X must be non-NULL and 16-byte aligned");
  const uintptr_t x = (uintptr_t)S, y = (uintptr_t)X;
  const size_t sb = (size_t)n * d * p * xbytes(fmt), xb = (size_t)n * d * d * xbytes(fmt);
  if (x < y + xb && y < x + sb) return fail(NSRGS_ERR_INVALID_ARG, "S and X overlap");
  hipStream_t s = (hipStream_t)stream;
  const StLayout L = st_layout(n, d, p, fmt);
  char *base = static_cast<char *>(ws);
  DevCtl *ctl = static_cast<DevCtl *>(ws);
  NSRGS_HIP(launch_ctl_reset(ctl, 2, s), "ctl reset");
  NSRGS_HIP(launch_stiefel_round(fmt, S, n, d, p, reinterpret_cast<double *>(base + L.gram),
                                 reinterpret_cast<double *>(base + L.basis), X, ctl, s), "rounding launch");
  DevCtl host{};
  if ((st = read_back(ws, &host, s))) return st;
  if (host.init_bad) return fail(NSRGS_ERR_NONFINITE, "rounding: a block S_i V is singular or not finite");
  return NSRGS_OK;
}

}  // extern "C"
