// Many independent NS-RGS problems of uneven size (n, d) per launch: host
// side (descriptor upload, unit tables, the two schedules' drivers and the
// C ABI).  The structures, kernels and the schedules' rules are in
// batched_impl.h; the kernels are instantiated per format in batched_*.hip.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "batched_impl.h"

namespace nsrgs {

extern template hipError_t launch_group_fmt<NSRGS_A_F64>(int, const GroupArgs &, int, int, hipStream_t);
extern template hipError_t launch_persistent_fmt<NSRGS_A_F64>(int, const PersistArgs &, int, hipStream_t);
extern template hipError_t launch_group_fmt<NSRGS_A_F32>(int, const GroupArgs &, int, int, hipStream_t);
extern template hipError_t launch_persistent_fmt<NSRGS_A_F32>(int, const PersistArgs &, int, hipStream_t);
extern template hipError_t launch_group_fmt<NSRGS_A_BF16>(int, const GroupArgs &, int, int, hipStream_t);
extern template hipError_t launch_persistent_fmt<NSRGS_A_BF16>(int, const PersistArgs &, int, hipStream_t);

static hipError_t launch_group(int fmt, int dmax, const GroupArgs &a, int grid, int waves, hipStream_t s) {
  switch (fmt) {
    case NSRGS_A_F64: return launch_group_fmt<NSRGS_A_F64>(dmax, a, grid, waves, s);
    case NSRGS_A_F32: return launch_group_fmt<NSRGS_A_F32>(dmax, a, grid, waves, s);
    case NSRGS_A_BF16: return launch_group_fmt<NSRGS_A_BF16>(dmax, a, grid, waves, s);
    default: return hipErrorInvalidValue;
  }
}

static hipError_t launch_persistent(int fmt, int dmax, const PersistArgs &a, int waves, hipStream_t s) {
  switch (fmt) {
    case NSRGS_A_F64: return launch_persistent_fmt<NSRGS_A_F64>(dmax, a, waves, s);
    case NSRGS_A_F32: return launch_persistent_fmt<NSRGS_A_F32>(dmax, a, waves, s);
    case NSRGS_A_BF16: return launch_persistent_fmt<NSRGS_A_BF16>(dmax, a, waves, s);
    default: return hipErrorInvalidValue;
  }
}

// Grouped schedule, second launch of an iteration: each active problem's
// monitors, iteration counter and stop rule (one workgroup per problem).
__global__ void __launch_bounds__(256) group_finish_kernel(GroupInst *inst) {
  __shared__ double s_scr[kMaxWaves];
  GroupInst &I = inst[blockIdx.x];
  if (!I.active) return;                              // uniform
  finish_problem<false>(I, s_scr, I.t + 1);
}

__global__ void persist_reset_kernel(PersistCtl *pc) {
  if (threadIdx.x == 0) {
    pc->next = 0u;
    pc->abort = 0;
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


int batch_rows_per_panel(int d) { return batch_blocks(d) * d; }

int batch_panels(int n, int d) {
  const int R = batch_rows_per_panel(d);
  return (n * d + R - 1) / R;
}

// Unit order: 0 = problem-major, largest problems first (their long panels
// start earliest); 1 = units of all problems interleaved.  chunk[k] panels of
// problem k form one unit (the last unit of a problem may hold fewer).
static void build_units(const int *panels, const int *chunk, int count, int order,
                        std::vector<GroupUnit> &units) {
  units.clear();
  auto add = [&](int k, int p) { units.push_back(GroupUnit{k, p, std::min(chunk[k], panels[k] - p), 0}); };
  if (order == 1) {
    int maxu = 0;
    for (int k = 0; k < count; ++k) maxu = std::max(maxu, (panels[k] + chunk[k] - 1) / chunk[k]);
    for (int u = 0; u < maxu; ++u)
      for (int k = 0; k < count; ++k)
        if (u * chunk[k] < panels[k]) add(k, u * chunk[k]);
  } else {
    std::vector<int> idx(count);
    for (int k = 0; k < count; ++k) idx[k] = k;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return panels[a] > panels[b]; });
    for (int k : idx)
      for (int p = 0; p < panels[k]; p += chunk[k]) add(k, p);
  }
}

size_t group_control_bytes(int count, size_t units) {
  return align256((size_t)count * sizeof(GroupInst)) + align256(units * sizeof(GroupUnit)) +
         sizeof(PersistCtl);
}

// Problem descriptors and the unit table of one batch, uploaded to the
// control area (problem k resumes at iteration specs[k].t0 with its iterate in
// X[t0 & 1]); device state reset.
struct BatchDev {
  std::vector<GroupInst> host;
  std::vector<GroupUnit> units;
  GroupInst *dinst = nullptr;
  GroupUnit *dunits = nullptr;
  PersistCtl *pc = nullptr;
  int dmax = 0;
};

static int upload_batch(const std::vector<GroupSpec> &specs, void *ctl, int order, size_t min_unit_bytes,
                        hipStream_t s, BatchDev &B) {
  const int count = (int)specs.size();
  B.host.assign(count, GroupInst{});
  std::vector<int> panels(count), chunk(count, 1);
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
    I.t0 = g.t0;
    I.t = g.t0;
    I.mu = g.mu > 0.0 ? g.mu : 1.0 / g.n;
    I.tol = g.tol;
    B.host[k] = I;
    panels[k] = I.panels;
    if (min_unit_bytes > 0) {
      const size_t panel_bytes = (size_t)batch_rows_per_panel(g.d) * I.nd * elem_size(g.A.fmt);
      chunk[k] = (int)std::min<size_t>((size_t)I.panels, std::max<size_t>(1, (min_unit_bytes + panel_bytes - 1) / panel_bytes));
    }
    B.dmax = std::max(B.dmax, g.d);
  }
  build_units(panels.data(), chunk.data(), count, order, B.units);
  char *base = static_cast<char *>(ctl);
  B.dinst = reinterpret_cast<GroupInst *>(base);
  B.dunits = reinterpret_cast<GroupUnit *>(base + align256((size_t)count * sizeof(GroupInst)));
  B.pc = reinterpret_cast<PersistCtl *>(base + align256((size_t)count * sizeof(GroupInst)) +
                                        align256(B.units.size() * sizeof(GroupUnit)));
  NSRGS_HIP(hipMemcpyAsync(B.dinst, B.host.data(), B.host.size() * sizeof(GroupInst), hipMemcpyHostToDevice, s),
            "batch descriptors");
  NSRGS_HIP(hipMemcpyAsync(B.dunits, B.units.data(), B.units.size() * sizeof(GroupUnit), hipMemcpyHostToDevice, s),
            "batch units");
  hipLaunchKernelGGL(group_reset_kernel, dim3((count + 255) / 256), dim3(256), 0, s, B.dinst, count);
  NSRGS_HIP(hipGetLastError(), "batch reset");
  return NSRGS_OK;
}

static void copy_results(const std::vector<GroupInst> &back, std::vector<BatchResult> &out) {
  out.resize(back.size());
  for (size_t k = 0; k < back.size(); ++k) {
    out[k].iters = back[k].t;
    out[k].converged = back[k].converged;
    out[k].nonfinite = back[k].nonfinite;
    out[k].panels = back[k].panels;
    out[k].rel_change = back[k].rel_change;
    out[k].max_defect = back[k].max_defect;
    out[k].active = back[k].active;
  }
}

// Up to `launches` grouped launches; every `check_every` launches the
// descriptors are read back and the loop ends early once no problem is
// active.  Reads the final state into `out`.
int run_grouped(int fmt, const std::vector<GroupSpec> &specs, void *ctl, int launches, int ns_steps,
                int waves, int order, int check_every, hipStream_t s, std::vector<BatchResult> &out) {
  BatchDev B;
  int st;
  if ((st = upload_batch(specs, ctl, order, 0, s, B))) return st;
  GroupInst *dinst = B.dinst;
  const int dmax = B.dmax;
  const std::vector<GroupUnit> &units = B.units;
  const std::vector<GroupInst> &host = B.host;
  GroupArgs a{dinst, B.dunits, ns_steps};
  if (check_every <= 0) check_every = std::max(launches, 1);
  std::vector<GroupInst> back(host);
  for (int it = 0; it < launches;) {
    const int end = std::min(launches, it + check_every);
    for (; it < end; ++it) {
      NSRGS_HIP(launch_group(fmt, dmax, a, (int)units.size(), waves, s), "grouped launch");
      hipLaunchKernelGGL(group_finish_kernel, dim3((unsigned)host.size()), dim3(256), 0, s, dinst);
      NSRGS_HIP(hipGetLastError(), "grouped finish");
    }
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
  copy_results(back, out);
  return NSRGS_OK;
}

// One persistent launch for the whole remaining budget of every problem.
int run_persistent(int fmt, const std::vector<GroupSpec> &specs, void *ctl, int ns_steps, int waves,
                   int order, unsigned wait_polls, size_t min_ticket_bytes, hipStream_t s,
                   std::vector<BatchResult> &out) {
  BatchDev B;
  int st;
  if ((st = upload_batch(specs, ctl, order, min_ticket_bytes, s, B))) return st;
  int rounds = 0;
  for (const GroupSpec &g : specs) rounds = std::max(rounds, g.iters - g.t0);
  const double tickets = (double)B.units.size() * rounds;
  if (tickets > 2147483647.0)
    return fail(NSRGS_ERR_INVALID_ARG, "persistent schedule: %.0f tickets exceed 2^31 (fewer iterations per call)",
                tickets);
  hipLaunchKernelGGL(persist_reset_kernel, dim3(1), dim3(64), 0, s, B.pc);
  NSRGS_HIP(hipGetLastError(), "persistent reset");
  if (rounds > 0 && !B.units.empty()) {
    PersistArgs a{B.dinst, B.dunits, (int)B.units.size(), rounds, ns_steps, wait_polls, B.pc};
    NSRGS_HIP(launch_persistent(fmt, B.dmax, a, waves, s), "persistent launch");
  }
  std::vector<GroupInst> back(B.host);
  PersistCtl pc{};
  NSRGS_HIP(hipMemcpyAsync(back.data(), B.dinst, back.size() * sizeof(GroupInst), hipMemcpyDeviceToHost, s),
            "batch readback");
  NSRGS_HIP(hipMemcpyAsync(&pc, B.pc, sizeof(PersistCtl), hipMemcpyDeviceToHost, s), "persistent readback");
  NSRGS_HIP(hipStreamSynchronize(s), "stream sync");
  copy_results(back, out);
  if (pc.abort)
    return fail(NSRGS_ERR_DEVICE,
                "persistent schedule: a dependency wait exceeded %u polls and the launch was abandoned", wait_polls);
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
    if (with_init) init_need = std::max(init_need, narrow_ws_bytes(probs[k].n, probs[k].d, probs[k].A.fmt));
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
  if (o.persistent < 0 || o.persistent > 1) return fail(NSRGS_ERR_INVALID_ARG, "persistent must be 0 or 1");
  if (o.order < 0 || o.order > 1) return fail(NSRGS_ERR_INVALID_ARG, "order must be 0 or 1");
  if (o.wait_polls < 0) return fail(NSRGS_ERR_INVALID_ARG, "wait_polls must be >= 0");
  if (o.ticket_kb < 0) return fail(NSRGS_ERR_INVALID_ARG, "ticket_kb must be >= 0");
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
  if (o.persistent)
    st = run_persistent(fmt, specs, base + L.ctl, ns_steps, o.waves, o.order,
                        o.wait_polls > 0 ? (unsigned)o.wait_polls : kDefaultWaitPolls,
                        (size_t)(o.ticket_kb > 0 ? o.ticket_kb : kDefaultTicketKiB) * 1024, s, res);
  else
    st = run_grouped(fmt, specs, base + L.ctl, max_iters, ns_steps, o.waves, o.order, check_every, s, res);
  if (st) return st;
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
