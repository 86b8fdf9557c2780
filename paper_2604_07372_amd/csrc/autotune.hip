// Autotuner: measures launch shapes on the caller's own problem and reports
// them fastest first.  The caller installs what it wants with
// nsrgs_set_tuning (the Python package's autotune module keeps the table in a
// JSON file).  Host code only; the kernels are the ones every entry point
// uses, with the shape forced.
#include <algorithm>
#include <chrono>
#include <vector>

#include "host.h"
#include "kernels.h"

using namespace nsrgs;

namespace {

constexpr int kTuneWaves[] = {1, 2, 4, 8};

int sort_and_copy(std::vector<nsrgs_tune_result> &r, nsrgs_tune_result *out, int max_out, int *count) {
  std::stable_sort(r.begin(), r.end(),
                   [](const nsrgs_tune_result &a, const nsrgs_tune_result &b) { return a.ms < b.ms; });
  for (int i = 0; i < (int)r.size() && i < max_out; ++i) out[i] = r[i];
  if (count) *count = (int)r.size();
  return NSRGS_OK;
}

}  // namespace

extern "C" {

int nsrgs_autotune_step(const nsrgs_matrix *A, int n, int d, const void *X_in, void *X_out, void *ws,
                        size_t ws_bytes, void *stream, int reps, nsrgs_tune_result *results,
                        int max_results, int *count) {
  int st;
  if ((st = check_step_args(A, n, d, 3, X_in, X_out, ws, ws_bytes))) return st;
  if (reps < 1 || reps > 10000) return fail(NSRGS_ERR_INVALID_ARG, "reps must be in [1, 10000]");
  if (max_results > 0 && !results) return fail(NSRGS_ERR_INVALID_ARG, "results is NULL");
  hipStream_t s = (hipStream_t)stream;
  StreamConfig v[16];
  const int nv = stream_variants(d, v, 16);
  hipEvent_t e0, e1;
  NSRGS_HIP(hipEventCreate(&e0), "event create");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(NSRGS_ERR_DEVICE, "event create");
  }
  std::vector<nsrgs_tune_result> r;
  st = NSRGS_OK;
  for (int i = 0; i < nv && st == NSRGS_OK; ++i) {
    for (int W : kTuneWaves) {
      if (v[i].unroll == 0 && W > kPipeMaxWaves) continue;   // launched with kPipeMaxWaves
      const StreamConfig cfg{v[i].blocks_per_panel, W, v[i].unroll};
      // one untimed launch, then reps timed launches on the stream
      if ((st = step_with_config(A, n, d, 0.0, 3, X_in, X_out, ws, s, cfg))) break;
      if (hipEventRecord(e0, s) != hipSuccess) { st = fail(NSRGS_ERR_DEVICE, "event record"); break; }
      for (int k = 0; k < reps && st == NSRGS_OK; ++k) st = step_with_config(A, n, d, 0.0, 3, X_in, X_out, ws, s, cfg);
      if (st) break;
      float ms = 0.0f;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        st = fail(NSRGS_ERR_DEVICE, "event timing");
        break;
      }
      nsrgs_tune_result t{};
      t.blocks_per_panel = cfg.blocks_per_panel;
      t.unroll = cfg.unroll;
      t.waves = W;
      t.ms = (double)ms / reps;
      r.push_back(t);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) return st;
  return sort_and_copy(r, results, max_results, count);
}

int nsrgs_autotune_batched(const nsrgs_problem *probs, int count, int ns_steps, int iters, void *ws,
                           size_t ws_bytes, void *stream, nsrgs_tune_result *results, int max_results,
                           int *n_results) {
  if (count < 1 || !probs) return fail(NSRGS_ERR_INVALID_ARG, "no problems");
  if (iters < 1 || iters > 10000) return fail(NSRGS_ERR_INVALID_ARG, "iters must be in [1, 10000]");
  if (max_results > 0 && !results) return fail(NSRGS_ERR_INVALID_ARG, "results is NULL");
  // Fixed budgets, no tolerance: every candidate does the same work.
  std::vector<nsrgs_problem> p(probs, probs + count);
  for (nsrgs_problem &q : p) {
    q.iters = iters;
    q.tol = 0.0;
  }
  struct Cand { int persistent, order, waves, ticket_kb; };
  std::vector<Cand> cands;
  for (int order : {0, 1})
    for (int W : {1, 2, 4}) {
      cands.push_back(Cand{0, order, W, 0});
      for (int kb : {128, 512, 2048}) cands.push_back(Cand{1, order, W, kb});
    }
  std::vector<nsrgs_tune_result> r;
  int st;
  for (const Cand &c : cands) {
    nsrgs_batch_opts o{};
    o.waves = c.waves;
    o.order = c.order;
    o.persistent = c.persistent;
    o.ticket_kb = c.ticket_kb;
    // one untimed pass, then the timed one (the call waits for the stream)
    if ((st = sync_solve_batched(p.data(), count, ns_steps, 1, ws, ws_bytes, stream, &o, nullptr))) return st;
    const auto t0 = std::chrono::steady_clock::now();
    if ((st = sync_solve_batched(p.data(), count, ns_steps, iters, ws, ws_bytes, stream, &o, nullptr))) return st;
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    nsrgs_tune_result t{};
    t.waves = c.waves;
    t.order = c.order;
    t.persistent = c.persistent;
    t.ticket_kb = c.ticket_kb;
    t.ms = ms / iters;
    r.push_back(t);
  }
  return sort_and_copy(r, results, max_results, n_results);
}

}  // extern "C"
