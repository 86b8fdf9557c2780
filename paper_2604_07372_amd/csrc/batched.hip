// Many independent NS-RGS problems of uneven size (n, d) per launch.
//
// One launch runs one iteration of every active problem: each workgroup takes
// one (problem, panel) unit of a unit table, runs the same per-panel work as
// sync_step (stream the panel's rows of A, fused Riemannian step and
// Newton-Schulz retraction) and the last panel of each problem to arrive
// reduces that problem's monitors, advances its iteration counter and applies
// its stop rule (tolerance, budget, non-finite).  The iteration barrier of
// each problem is the launch boundary; no workgroup ever waits for another, so
// the host can enqueue a whole budget of launches without synchronizing.
// Problems that have stopped keep their units in the table; those workgroups
// return at once.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "host.h"
#include "stream_impl.h"

namespace nsrgs {

struct GroupInst {
  const void *A;
  const void *A_lo;
  const float *scale;
  int64_t ld;
  void *X[2];             // X^t lives in X[t & 1]
  PanelStat *stats;       // one per panel
  int n, d, nd, panels;
  int iters;              // iteration budget
  int pad0;
  double mu;
  double tol;             // > 0: stop after the first iteration with rel. change <= tol
  // kept by the device
  int t;                  // iterations completed
  int active;             // 1 while the problem still iterates
  unsigned arrive;        // panels done in the current launch (0 between launches)
  int converged;
  int nonfinite;
  int pad1;
  double rel_change;
  double max_defect;
};

struct GroupUnit {
  int inst;
  int panel;
};

struct GroupArgs {
  GroupInst *inst;
  const GroupUnit *units;
  int ns_steps;
};

// Rows per panel of the batched kernel for each d (B blocks of d rows).
__host__ __device__ constexpr int batch_blocks(int d) {
  return d == 1 ? 8 : d == 2 ? 4 : d == 3 ? 4 : d == 4 ? 2 : 1;
}

// Largest LDS need over the d handled by a kernel of class DMAX.
template <int FMT, int DMAX>
constexpr int batch_lds_bytes() {
  int m = 0;
#define NSRGS_BL(DD) \
  if (DD <= DMAX && panel_lds_bytes<FMT, DD, batch_blocks(DD)>() > m) m = panel_lds_bytes<FMT, DD, batch_blocks(DD)>();
  NSRGS_BL(1) NSRGS_BL(2) NSRGS_BL(3) NSRGS_BL(4) NSRGS_BL(5) NSRGS_BL(6) NSRGS_BL(7) NSRGS_BL(8)
  NSRGS_BL(9) NSRGS_BL(10) NSRGS_BL(11) NSRGS_BL(12) NSRGS_BL(13) NSRGS_BL(14) NSRGS_BL(15) NSRGS_BL(16)
#undef NSRGS_BL
  return m;
}

template <int FMT, int DMAX>
__device__ __forceinline__ void run_panel(int d, const PanelJob &job, char *lds) {
#define NSRGS_BP(DD)                                                            \
  if constexpr (DD <= DMAX)                                                     \
    if (d == DD) {                                                              \
      panel_compute<FMT, DD, batch_blocks(DD), 1, 0>(job, lds);                 \
      return;                                                                   \
    }
  NSRGS_BP(1) NSRGS_BP(2) NSRGS_BP(3) NSRGS_BP(4) NSRGS_BP(5) NSRGS_BP(6) NSRGS_BP(7)
  NSRGS_BP(8) NSRGS_BP(9) NSRGS_BP(10) NSRGS_BP(11) NSRGS_BP(12) NSRGS_BP(13) NSRGS_BP(14)
  NSRGS_BP(15) NSRGS_BP(16)
#undef NSRGS_BP
}

// Last panel of problem I in this launch: monitors, iteration counter, stop rule.
__device__ inline void finish_problem(GroupInst &I, double *s_scr) {
  const int tid = threadIdx.x;
  double a = 0.0, b = 0.0, m = 0.0, f = 0.0;
  for (int p = tid; p < I.panels; p += blockDim.x) {
    const PanelStat q = I.stats[p];
    a += q.dx2;
    b += q.x2;
    m = q.dmax > m ? q.dmax : m;
    f = q.nonfinite > f ? q.nonfinite : f;
  }
  a = block_sum(a, s_scr);
  b = block_sum(b, s_scr);
  m = block_max(m, s_scr);
  f = block_max(f, s_scr);
  if (tid == 0) {
    const double rel = b > 0.0 ? sqrt(a / b) : 0.0;
    I.rel_change = rel;
    I.max_defect = m;
    I.t = I.t + 1;
    if (f != 0.0 || !isfinite(rel)) {
      I.nonfinite = 1;
      I.active = 0;
    } else if (I.tol > 0.0 && rel <= I.tol) {
      I.converged = 1;
      I.active = 0;
    } else if (I.t >= I.iters) {
      I.active = 0;
    }
    I.arrive = 0u;
  }
}

template <int FMT, int DMAX>
__global__ void __launch_bounds__(kWave * kMaxWaves) grouped_kernel(GroupArgs args) {
  __shared__ double s_scr[kMaxWaves];
  __shared__ int s_last;
  __shared__ __attribute__((aligned(16))) char lds[batch_lds_bytes<FMT, DMAX>()];
  const GroupUnit unit = args.units[blockIdx.x];
  GroupInst &I = args.inst[unit.inst];
  if (!I.active) return;                              // uniform: set by an earlier launch
  const int t = I.t;
  PanelJob job;
  job.A = I.A;
  job.A_lo = I.A_lo;
  job.scale = I.scale;
  job.ld = I.ld;
  job.X_in = I.X[t & 1];
  job.X_out = I.X[(t + 1) & 1];
  job.n = I.n;
  job.nd = I.nd;
  job.panel = unit.panel;
  job.mu = I.mu;
  job.ns_steps = args.ns_steps;
  job.stat = I.stats + unit.panel;
  job.gram = nullptr;
  run_panel<FMT, DMAX>(I.d, job, lds);
  __threadfence();
  if (threadIdx.x == 0) s_last = (atomicAdd(&I.arrive, 1u) == (unsigned)I.panels - 1u);
  __syncthreads();
  if (s_last) {
    __threadfence();
    finish_problem(I, s_scr);
  }
}

__global__ void group_reset_kernel(GroupInst *inst, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) {
    inst[i].active = inst[i].t < inst[i].iters ? 1 : 0;
    inst[i].arrive = 0u;
    inst[i].converged = 0;
    inst[i].nonfinite = 0;
    inst[i].rel_change = 0.0;
    inst[i].max_defect = 0.0;
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
// Kernel classes: every d <= 4, d <= 10 or d <= 16 handled by one inlined kernel
// (a batch takes the smallest class that holds its largest d).
static int dclass(int dmax) { return dmax <= 4 ? 4 : dmax <= 10 ? 10 : 16; }

template <int FMT, int DMAX>
static hipError_t launch_g(const GroupArgs &a, int grid, int waves, hipStream_t s) {
  hipLaunchKernelGGL((grouped_kernel<FMT, DMAX>), dim3(grid), dim3(kWave * waves), 0, s, a);
  return hipGetLastError();
}

static hipError_t launch_group(int fmt, int dmax, const GroupArgs &a, int grid, int waves, hipStream_t s) {
  const int c = dclass(dmax);
#define NSRGS_LG(F)                                         \
  if (fmt == F) {                                           \
    if (c == 4) return launch_g<F, 4>(a, grid, waves, s);   \
    if (c == 10) return launch_g<F, 10>(a, grid, waves, s); \
    return launch_g<F, 16>(a, grid, waves, s);              \
  }
  NSRGS_LG(NSRGS_A_F64) NSRGS_LG(NSRGS_A_F32) NSRGS_LG(NSRGS_A_BF16)
#undef NSRGS_LG
  return hipErrorInvalidValue;
}

int batch_rows_per_panel(int d) { return batch_blocks(d) * d; }

int batch_panels(int n, int d) {
  const int R = batch_rows_per_panel(d);
  return (n * d + R - 1) / R;
}

// Unit order: 0 = problem-major, largest problems first (their long panels
// start earliest); 1 = panels of all problems interleaved.
static void build_units(const int *panels, int count, int order, std::vector<GroupUnit> &units) {
  units.clear();
  if (order == 1) {
    int maxp = 0;
    for (int k = 0; k < count; ++k) maxp = std::max(maxp, panels[k]);
    for (int p = 0; p < maxp; ++p)
      for (int k = 0; k < count; ++k)
        if (p < panels[k]) units.push_back(GroupUnit{k, p});
  } else {
    std::vector<int> idx(count);
    for (int k = 0; k < count; ++k) idx[k] = k;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return panels[a] > panels[b]; });
    for (int k : idx)
      for (int p = 0; p < panels[k]; ++p) units.push_back(GroupUnit{k, p});
  }
}

size_t group_control_bytes(int count, size_t units) {
  return align256((size_t)count * sizeof(GroupInst)) + align256(units * sizeof(GroupUnit));
}

// Upload descriptors (problem k resumes at iteration specs[k].t0, its
// iterate in X[t0 & 1]), then up to `launches` grouped launches (every
// `check_every` launches the descriptors are read back and the loop ends early
// once no problem is active).  Reads the final state into `out`.
int run_grouped(int fmt, const std::vector<GroupSpec> &specs, void *ctl, int launches, int ns_steps,
                int waves, int order, int check_every, hipStream_t s, std::vector<BatchResult> &out) {
  const int count = (int)specs.size();
  int dmax = 0;
  std::vector<GroupInst> host(count);
  std::vector<int> panels(count);
  for (int k = 0; k < count; ++k) {
    const GroupSpec &g = specs[k];
    GroupInst I{};
    I.A = g.A.data;
    I.A_lo = g.A.fmt == NSRGS_A_BF16_SPLIT ? g.A.data_lo : nullptr;
    I.scale = g.A.fmt == NSRGS_A_FP8_E4M3 ? g.A.row_scale : nullptr;
    I.ld = g.A.ld;
    I.X[0] = g.X0;
    I.X[1] = g.X1;
    I.stats = static_cast<PanelStat *>(g.stats);
    I.n = g.n;
    I.d = g.d;
    I.nd = g.n * g.d;
    I.panels = batch_panels(g.n, g.d);
    I.iters = g.iters;
    I.t = g.t0;
    I.mu = g.mu > 0.0 ? g.mu : 1.0 / g.n;
    I.tol = g.tol;
    host[k] = I;
    panels[k] = I.panels;
    dmax = std::max(dmax, g.d);
  }
  std::vector<GroupUnit> units;
  build_units(panels.data(), count, order, units);
  char *base = static_cast<char *>(ctl);
  GroupInst *dinst = reinterpret_cast<GroupInst *>(base);
  GroupUnit *dunits = reinterpret_cast<GroupUnit *>(base + align256((size_t)count * sizeof(GroupInst)));
  NSRGS_HIP(hipMemcpyAsync(dinst, host.data(), host.size() * sizeof(GroupInst), hipMemcpyHostToDevice, s),
            "batch descriptors");
  NSRGS_HIP(hipMemcpyAsync(dunits, units.data(), units.size() * sizeof(GroupUnit), hipMemcpyHostToDevice, s),
            "batch units");
  hipLaunchKernelGGL(group_reset_kernel, dim3((count + 255) / 256), dim3(256), 0, s, dinst, count);
  NSRGS_HIP(hipGetLastError(), "batch reset");
  GroupArgs a{dinst, dunits, ns_steps};
  if (check_every <= 0) check_every = std::max(launches, 1);
  std::vector<GroupInst> back(host);
  for (int it = 0; it < launches;) {
    const int end = std::min(launches, it + check_every);
    for (; it < end; ++it)
      NSRGS_HIP(launch_group(fmt, dmax, a, (int)units.size(), waves, s), "grouped launch");
    NSRGS_HIP(hipMemcpyAsync(back.data(), dinst, back.size() * sizeof(GroupInst), hipMemcpyDeviceToHost, s),
              "batch readback");
    NSRGS_HIP(hipStreamSynchronize(s), "stream sync");
    bool any = false;
    for (const GroupInst &I : back) any = any || I.active;
    if (!any) break;
  }
  if (launches <= 0) {
    NSRGS_HIP(hipMemcpyAsync(back.data(), dinst, back.size() * sizeof(GroupInst), hipMemcpyDeviceToHost, s),
              "batch readback");
    NSRGS_HIP(hipStreamSynchronize(s), "stream sync");
  }
  out.resize(count);
  for (int k = 0; k < count; ++k) {
    out[k].iters = back[k].t;
    out[k].converged = back[k].converged;
    out[k].nonfinite = back[k].nonfinite;
    out[k].panels = back[k].panels;
    out[k].rel_change = back[k].rel_change;
    out[k].max_defect = back[k].max_defect;
    out[k].active = back[k].active;
  }
  return NSRGS_OK;
}

}  // namespace nsrgs

using namespace nsrgs;

namespace {

struct BatchLayout {
  size_t ctl, init, total;
  std::vector<size_t> xalt_off, stats_off;
};

int batch_check(const nsrgs_problem *probs, int count, int *fmt, int *dmax) {
  if (!probs || count < 1) return fail(NSRGS_ERR_INVALID_ARG, "need at least one problem");
  *fmt = probs[0].A.fmt;
  *dmax = 0;
  for (int k = 0; k < count; ++k) {
    const nsrgs_problem &P = probs[k];
    int st;
    if ((st = check_common(P.n, P.d))) return fail(st, "problem %d: %s", k, nsrgs_last_error());
    if ((st = check_matrix(&P.A, P.n, P.d))) return fail(st, "problem %d: %s", k, nsrgs_last_error());
    if (P.A.fmt != *fmt) return fail(NSRGS_ERR_INVALID_ARG, "problem %d: all problems must share one format", k);
    if (!P.X || !aligned16(P.X)) return fail(NSRGS_ERR_INVALID_ARG, "problem %d: X must be 16-byte aligned", k);
    if (!std::isfinite(P.mu) || !std::isfinite(P.tol)) return fail(NSRGS_ERR_INVALID_ARG, "problem %d: bad mu/tol", k);
    *dmax = std::max(*dmax, P.d);
  }
  if (*fmt != NSRGS_A_F64 && *fmt != NSRGS_A_F32 && *fmt != NSRGS_A_BF16)
    return fail(NSRGS_ERR_UNSUPPORTED, "batched solves take F64, F32 or BF16 storage");
  return NSRGS_OK;
}

BatchLayout batch_layout(const nsrgs_problem *probs, int count, int with_init) {
  BatchLayout L;
  size_t units = 0;
  for (int k = 0; k < count; ++k) units += (size_t)batch_panels(probs[k].n, probs[k].d);
  size_t off = 0;
  L.ctl = off;
  off += group_control_bytes(count, units);
  L.xalt_off.resize(count);
  L.stats_off.resize(count);
  const size_t xb = xbytes(probs[0].A.fmt);
  size_t init_need = 0;
  for (int k = 0; k < count; ++k) {
    const size_t nd = (size_t)probs[k].n * probs[k].d;
    L.xalt_off[k] = off;
    off += align256(nd * probs[k].d * xb);
    L.stats_off[k] = off;
    off += align256((size_t)batch_panels(probs[k].n, probs[k].d) * sizeof(PanelStat));
    if (with_init) init_need = std::max(init_need, sync_workspace_bytes(probs[k].n, probs[k].d, probs[k].A.fmt));
  }
  L.init = off;
  off += align256(init_need);
  L.total = off;
  return L;
}

}  // namespace

extern "C" {

size_t sync_batch_workspace_bytes(const nsrgs_problem *probs, int count, int with_init) {
  int fmt, dmax;
  if (batch_check(probs, count, &fmt, &dmax)) return 0;
  return batch_layout(probs, count, with_init).total;
}

int sync_solve_batched(const nsrgs_problem *probs, int count, int ns_steps, int max_iters, void *ws,
                       size_t ws_bytes, void *stream, const nsrgs_batch_opts *opts,
                       nsrgs_problem_info *infos) {
  int fmt, dmax, st;
  if ((st = batch_check(probs, count, &fmt, &dmax))) return st;
  if (ns_steps < 0 || ns_steps > 64) return fail(NSRGS_ERR_INVALID_ARG, "ns_steps must be in [0, 64]");
  if (max_iters < 0) return fail(NSRGS_ERR_INVALID_ARG, "max_iters must be >= 0");
  nsrgs_batch_opts o{};
  if (opts) o = *opts;
  if (o.persistent)
    return fail(NSRGS_ERR_UNSUPPORTED,
                "the persistent single-launch schedule is switched off in this build; "
                "batches run as one grouped launch per iteration");
  if (o.waves < 0 || o.waves > kMaxWaves) return fail(NSRGS_ERR_INVALID_ARG, "waves must be in [0, %d]", kMaxWaves);
  if (o.waves == 0) o.waves = tuned_batch_waves(fmt, dmax);
  const BatchLayout L = batch_layout(probs, count, o.init);
  if (!ws || ((uintptr_t)ws & 255u)) return fail(NSRGS_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (ws_bytes < L.total) return fail(NSRGS_ERR_OUT_OF_MEMORY, "workspace too small: %zu < %zu", ws_bytes, L.total);
  hipStream_t s = (hipStream_t)stream;
  char *base = static_cast<char *>(ws);
  if (o.init) {
    void *iws = base + L.init;
    const size_t iwb = L.total - L.init;
    for (int k = 0; k < count; ++k) {
      NSRGS_HIP(launch_ctl_reset(static_cast<DevCtl *>(iws), 0, s), "ctl reset");
      st = sync_init_spectral(&probs[k].A, probs[k].n, probs[k].d, probs[k].X, 0, 0.0, iws, iwb, stream,
                              nullptr);
      if (st != NSRGS_OK && st != NSRGS_ERR_NOT_CONVERGED) return st;
    }
  }
  std::vector<GroupSpec> specs(count);
  bool any_tol = false;
  for (int k = 0; k < count; ++k) {
    const nsrgs_problem &P = probs[k];
    GroupSpec &g = specs[k];
    g.A = P.A;
    g.n = P.n;
    g.d = P.d;
    g.iters = P.iters > 0 ? std::min(P.iters, max_iters) : max_iters;
    g.X0 = P.X;
    g.X1 = base + L.xalt_off[k];
    g.stats = base + L.stats_off[k];
    g.mu = P.mu;
    g.tol = P.tol;
    g.t0 = 0;
    any_tol = any_tol || P.tol > 0.0;
  }
  std::vector<BatchResult> res;
  const int check_every = o.check_every > 0 ? o.check_every : (any_tol ? 8 : max_iters);
  if ((st = run_grouped(fmt, specs, base + L.ctl, max_iters, ns_steps, o.waves, o.order, check_every, s, res)))
    return st;
  int result = NSRGS_OK;
  for (int k = 0; k < count; ++k) {
    const nsrgs_problem &P = probs[k];
    const BatchResult &r = res[k];
    if (r.iters & 1)
      NSRGS_HIP(hipMemcpyAsync(P.X, specs[k].X1, (size_t)P.n * P.d * P.d * xbytes(fmt),
                               hipMemcpyDeviceToDevice, s), "result copy");
    int pst = NSRGS_OK;
    if (r.nonfinite) pst = NSRGS_ERR_NONFINITE;
    else if (P.tol > 0.0 && !r.converged) pst = NSRGS_ERR_NOT_CONVERGED;
    if (pst == NSRGS_ERR_NONFINITE) result = NSRGS_ERR_NONFINITE;
    if (infos) {
      infos[k].iters = r.iters;
      infos[k].converged = r.converged;
      infos[k].nonfinite = r.nonfinite;
      infos[k].status = pst;
      infos[k].rel_change = r.rel_change;
      infos[k].max_orth_defect = r.max_defect;
    }
  }
  NSRGS_HIP(hipStreamSynchronize(s), "stream sync");
  if (result == NSRGS_ERR_NONFINITE) return fail(result, "a problem of the batch became non-finite");
  return result;
}

}  // extern "C"
