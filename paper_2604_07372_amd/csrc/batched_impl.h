// Many independent NS-RGS problems of uneven size (n, d) per launch: the
// structures, device code and kernels (host side in batched.hip).
//
// Work unit: one (problem, panel) pair.  A workgroup runs the same per-panel
// work as sync_step (stream the panel's rows of A, fused Riemannian step and
// Newton-Schulz retraction), and the last panel of each problem to arrive
// reduces that problem's monitors, advances its iteration counter and applies
// its stop rule (tolerance, budget, non-finite).  Two schedules:
//
// * grouped: per iteration, one launch over every unit and one small launch
//   (a workgroup per problem) that reduces each problem's monitors and
//   applies its stop rule.  The iteration barrier of each problem is the
//   launch boundary; no workgroup waits for another, so the host enqueues a
//   whole budget of launches without synchronizing.
// * persistent: one launch for the whole budget.  Workgroups take tickets
//   from one counter; ticket k is round k / U of unit k mod U (U units per
//   round), so tickets go out round by round.  Before computing round r of a
//   problem, a workgroup waits until that problem has published iteration
//   t0 + r (or has stopped).  Every ticket it can wait on was handed out
//   earlier, to a workgroup that is already running, so by induction on r
//   every wait ends whatever the number of resident workgroups.  Each wait is
//   also bounded: after `wait_polls` polls it raises a launch-wide abort flag,
//   every other wait then gives up at once, and the grid drains.
#pragma once
#include <algorithm>

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
  int t0;                 // iterations done before this launch sequence (static)
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

// Work unit: panels [panel, panel + npanels) of problem inst (grouped
// launches use npanels = 1; persistent tickets merge small panels).
struct GroupUnit {
  int inst;
  int panel;
  int npanels;
  int pad;
};

struct GroupArgs {
  GroupInst *inst;
  const GroupUnit *units;
  int ns_steps;
};

// Control words of the persistent schedule (zeroed before the launch).
struct alignas(256) PersistCtl {
  unsigned next;          // next ticket
  int abort;              // a dependency wait ran out of polls
  int pad[62];
};

// Polls per dependency wait before a persistent launch gives up (each poll
// sleeps ~500 cycles, so about 2^21 polls is a few seconds: far longer than
// one iteration of any problem that fits in memory).
constexpr unsigned kDefaultWaitPolls = 1u << 21;
// Smallest amount of A per persistent ticket: panels of small problems are
// merged so that the per-ticket overhead (one device-wide atomic, one poll,
// two fences) stays small against the streaming time.
constexpr int kDefaultTicketKiB = 512;

struct PersistArgs {
  GroupInst *inst;
  const GroupUnit *units;
  int nunits;             // units per round
  int rounds;             // rounds of tickets (largest remaining budget)
  int ns_steps;
  unsigned wait_polls;    // polls per dependency wait before the launch aborts
  PersistCtl *pc;
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

// Last panel of problem I to arrive for the iteration that ends with t_new
// iterations done: monitors, iteration counter, stop rule.  PUBLISH (the
// persistent schedule) writes the stop state first and then releases t, so a
// workgroup that acquires the new t also sees whether the problem stopped.
template <bool PUBLISH>
__device__ inline void finish_problem(GroupInst &I, double *s_scr, int t_new) {
  (void)s_scr;
  const int tid = threadIdx.x;
  // Wave 0 alone reduces (fixed 64-lane stride, then a fixed butterfly), so
  // the monitors are bitwise the same whatever the workgroup size of the
  // launch that runs this (the grouped and persistent schedules differ).
  if (tid >= kWave) return;
  double a = 0.0, b = 0.0, m = 0.0, f = 0.0;
  for (int p = tid; p < I.panels; p += kWave) {
    const PanelStat q = I.stats[p];
    a += q.dx2;
    b += q.x2;
    m = q.dmax > m ? q.dmax : m;
    f = q.nonfinite > f ? q.nonfinite : f;
  }
  a = wave_sum(a);
  b = wave_sum(b);
  m = wave_max(m);
  f = wave_max(f);
  if (tid == 0) {
    const double rel = b > 0.0 ? sqrt(a / b) : 0.0;
    I.rel_change = rel;
    I.max_defect = m;
    int act = 1;
    if (f != 0.0 || !isfinite(rel)) {
      I.nonfinite = 1;
      act = 0;
    } else if (I.tol > 0.0 && rel <= I.tol) {
      I.converged = 1;
      act = 0;
    } else if (t_new >= I.iters) {
      act = 0;
    }
    if constexpr (PUBLISH) {
      __hip_atomic_store(&I.arrive, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&I.active, act, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&I.t, t_new, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      I.arrive = 0u;
      I.active = act;
      I.t = t_new;
    }
  }
}

// Grouped schedule, one launch per iteration: the panels of every active
// problem.  The per-problem reduction and stop rule run in a second launch
// (group_finish_kernel), after the kernel boundary has ordered all panel writes.
template <int FMT, int DMAX>
__global__ void __launch_bounds__(kWave * kMaxWaves) grouped_kernel(GroupArgs args) {
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
}

// Persistent schedule: one launch for the whole budget (see the top of the file).
// Thread 0 fetches the next ticket while the current one is computed; a
// workgroup's prefetched ticket is always larger than its current one, so the
// induction over tickets that makes every wait end still holds.
template <int FMT, int DMAX>
__global__ void __launch_bounds__(kWave * kMaxWaves) persistent_kernel(PersistArgs args) {
  __shared__ double s_scr[kMaxWaves];
  __shared__ unsigned s_ticket;
  __shared__ int s_go, s_last;
  __shared__ __attribute__((aligned(16))) char lds[batch_lds_bytes<FMT, DMAX>()];
  const unsigned total = (unsigned)args.nunits * (unsigned)args.rounds;
  unsigned next = 0;
  if (threadIdx.x == 0) next = atomicAdd(&args.pc->next, 1u);
  for (;;) {
    if (threadIdx.x == 0) s_ticket = next;
    __syncthreads();
    const unsigned tk = s_ticket;
    __syncthreads();                                  // s_ticket is rewritten next time round
    if (tk >= total) break;                           // uniform
    if (threadIdx.x == 0) next = atomicAdd(&args.pc->next, 1u);   // consumed next time round
    const int round = (int)(tk / (unsigned)args.nunits);
    const GroupUnit unit = args.units[tk % (unsigned)args.nunits];
    GroupInst &I = args.inst[unit.inst];
    const int t = I.t0 + round;                       // the iteration this ticket computes
    if (t >= I.iters) continue;                       // past this problem's budget (uniform)
    if (threadIdx.x == 0) {
      // Wait for iteration t - 1 of this problem to be published, or for it to stop.
      int go = 0;
      for (unsigned poll = 0;; ++poll) {
        const int done = __hip_atomic_load(&I.t, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        const int act = __hip_atomic_load(&I.active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (!act) break;                              // stopped: nothing left to compute
        if (done >= t) {
          go = 1;
          break;
        }
        if (__hip_atomic_load(&args.pc->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
        if (poll >= args.wait_polls) {
          __hip_atomic_store(&args.pc->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        __builtin_amdgcn_s_sleep(8);
      }
      s_go = go;
    }
    __syncthreads();
    const int go = s_go;
    if (!go) continue;                                // uniform; s_go is rewritten after two barriers
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // X^t written by other workgroups
    PanelJob job;
    job.A = I.A;
    job.A_lo = I.A_lo;
    job.scale = I.scale;
    job.ld = I.ld;
    job.X_in = I.X[t & 1];
    job.X_out = I.X[(t + 1) & 1];
    job.n = I.n;
    job.nd = I.nd;
    job.mu = I.mu;
    job.ns_steps = args.ns_steps;
    job.gram = nullptr;
    for (int q = 0; q < unit.npanels; ++q) {
      job.panel = unit.panel + q;
      job.stat = I.stats + job.panel;
      run_panel<FMT, DMAX>(I.d, job, lds);            // ends with a barrier
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // this ticket's X^{t+1} rows and monitors
    if (threadIdx.x == 0)
      s_last = (atomicAdd(&I.arrive, (unsigned)unit.npanels) + (unsigned)unit.npanels == (unsigned)I.panels);
    __syncthreads();
    if (s_last) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // every panel's monitors
      finish_problem<true>(I, s_scr, t + 1);
    }
    __syncthreads();                                  // s_last and LDS are reused next time round
  }
}

// Kernel classes: every d <= 4, d <= 10 or d <= 16 handled by one inlined kernel
// (a batch takes the smallest class that holds its largest d).
inline int dclass(int dmax) { return dmax <= 4 ? 4 : dmax <= 10 ? 10 : 16; }

template <int FMT, int DMAX>
hipError_t launch_g(const GroupArgs &a, int grid, int waves, hipStream_t s) {
  hipLaunchKernelGGL((grouped_kernel<FMT, DMAX>), dim3(grid), dim3(kWave * waves), 0, s, a);
  return hipGetLastError();
}


// Persistent launch: as many workgroups as fit on the device at once (more
// would only wait for a slot; fewer leave CUs idle), at most one per ticket.
template <int FMT, int DMAX>
hipError_t launch_p(const PersistArgs &a, int waves, hipStream_t s) {
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persistent_kernel<FMT, DMAX>, kWave * waves, 0);
  if (e != hipSuccess) return e;
  const long long tickets = (long long)a.nunits * a.rounds;
  long long grid = (long long)std::max(1, cus) * std::max(1, per_cu);
  grid = std::max(1LL, std::min(grid, tickets));
  hipLaunchKernelGGL((persistent_kernel<FMT, DMAX>), dim3((unsigned)grid), dim3(kWave * waves), 0, s, a);
  return hipGetLastError();
}


// Per-format entry points (explicitly instantiated, one translation unit per
// format, so the kernels of the three formats compile in parallel).
template <int FMT>
hipError_t launch_group_fmt(int dmax, const GroupArgs &a, int grid, int waves, hipStream_t s) {
  const int c = dclass(dmax);
  if (c == 4) return launch_g<FMT, 4>(a, grid, waves, s);
  if (c == 10) return launch_g<FMT, 10>(a, grid, waves, s);
  return launch_g<FMT, 16>(a, grid, waves, s);
}

template <int FMT>
hipError_t launch_persistent_fmt(int dmax, const PersistArgs &a, int waves, hipStream_t s) {
  const int c = dclass(dmax);
  if (c == 4) return launch_p<FMT, 4>(a, waves, s);
  if (c == 10) return launch_p<FMT, 10>(a, waves, s);
  return launch_p<FMT, 16>(a, waves, s);
}

}  // namespace nsrgs
