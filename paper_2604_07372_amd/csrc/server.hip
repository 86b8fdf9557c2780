// Serving: a request loop with continuous batching.
//
// Requests (n, d, sigma, seed, ground truth Z, tolerance) arrive at any time.
// The scheduler admits them in arrival order as device memory (a pool carved
// once at creation, first-fit with coalescing) and solve slots allow; ingest
// workers (threads with a stream each) generate each admitted request's A on
// the device in row chunks (FP32 staging rows converted to the storage
// format) and run its spectral initialization, so ingest overlaps the solves
// and other ingests on the device.  The scheduler thread runs "ticks": a few grouped
// launches (batched.hip) over every request that is ready, each request at its
// own iteration count; requests that became ready since the last tick join the
// next one, finished requests (tolerance met, budget spent, non-finite) leave,
// return their result and free their memory.  A request's arithmetic does not
// depend on what else is in the batch: its result is bitwise the same alone
// and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "device.h"
#include "host.h"
#include "kernels.h"
#include "nsrgs.h"

namespace nsrgs {

// ---------------------------------------------------------------------------
// Device memory pool: one allocation, first-fit free list, coalescing frees.
// ---------------------------------------------------------------------------
class DevicePool {
 public:
  hipError_t init(size_t bytes) {
    total_ = bytes & ~(size_t)255;
    hipError_t e = hipMalloc(&base_, total_);
    if (e != hipSuccess) {
      base_ = nullptr;
      return e;
    }
    free_[0] = total_;
    return hipSuccess;
  }
  ~DevicePool() {
    if (base_) (void)hipFree(base_);
  }
  void *alloc(size_t bytes) {
    bytes = align256(std::max<size_t>(bytes, 256));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t off = it->first, sz = it->second;
      free_.erase(it);
      if (sz > bytes) free_[off + bytes] = sz - bytes;
      used_[off] = bytes;
      inuse_ += bytes;
      peak_ = std::max(peak_, inuse_);
      return base_ + off;
    }
    return nullptr;
  }
  void release(void *p) {
    if (!p) return;
    const size_t off = static_cast<char *>(p) - base_;
    auto u = used_.find(off);
    if (u == used_.end()) return;
    size_t start = off, sz = u->second;
    inuse_ -= sz;
    used_.erase(u);
    auto nx = free_.lower_bound(start);
    if (nx != free_.end() && nx->first == start + sz) {
      sz += nx->second;
      free_.erase(nx);
    }
    auto pv = free_.lower_bound(start);
    if (pv != free_.begin()) {
      --pv;
      if (pv->first + pv->second == start) {
        start = pv->first;
        sz += pv->second;
        free_.erase(pv);
      }
    }
    free_[start] = sz;
  }
  // Would a set of allocations fit now (first-fit, in order)?
  bool fits(const std::vector<size_t> &sizes) const {
    std::map<size_t, size_t> f = free_;
    for (size_t b : sizes) {
      b = align256(std::max<size_t>(b, 256));
      bool ok = false;
      for (auto it = f.begin(); it != f.end(); ++it) {
        if (it->second < b) continue;
        const size_t off = it->first, sz = it->second;
        f.erase(it);
        if (sz > b) f[off + b] = sz - b;
        ok = true;
        break;
      }
      if (!ok) return false;
    }
    return true;
  }
  size_t total() const { return total_; }
  size_t peak() const { return peak_; }
  size_t in_use() const { return inuse_; }

 private:
  char *base_ = nullptr;
  size_t total_ = 0, inuse_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_, used_;
};

enum ReqState { kPending, kIngest, kReady, kActive, kDone };

struct Request {
  int64_t id = 0;
  nsrgs_request r{};
  std::vector<double> Z;
  ReqState state = kPending;
  double t_submit = 0, t_admit = 0, t_start = 0, t_done = 0;
  int status = NSRGS_OK;
  int t = 0, converged = 0, nonfinite = 0;
  double rel_change = 0;
  // device memory (pool)
  nsrgs_matrix A{};
  void *a_mem = nullptr, *x0 = nullptr, *x1 = nullptr, *stats = nullptr;
  void *zdev = nullptr, *stage = nullptr, *iws = nullptr;
  size_t a_bytes = 0, x_bytes = 0, stats_bytes = 0, z_bytes = 0, stage_bytes = 0, iws_bytes = 0;
  int stage_rows = 0;
};

static constexpr size_t kStageBytes = (size_t)256 << 20;   // FP32 staging rows per chunk

struct Server {
  nsrgs_server_opts o{};
  int device = 0;
  DevicePool pool;
  hipStream_t solve_stream = nullptr;
  std::vector<hipStream_t> ingest_streams;   // one per ingest worker
  void *ctl = nullptr;                 // grouped-launch control block (not from the pool)
  size_t ctl_bytes = 0;
  std::chrono::steady_clock::time_point t0;

  std::mutex mu;
  std::condition_variable cv;          // wakes the scheduler
  std::condition_variable ingest_cv;   // wakes the ingest thread
  std::condition_variable idle_cv;     // wakes wait_idle
  bool stop = false;
  int64_t next_id = 1;
  std::deque<std::shared_ptr<Request>> pending, ingest_q, ready;
  std::vector<std::shared_ptr<Request>> active;
  std::deque<nsrgs_result> results;
  std::vector<double> latencies;
  int64_t submitted = 0, completed = 0, rejected = 0;
  int ingesting = 0, max_active_seen = 0;
  double first_submit = -1, last_done = 0;
  std::thread sched;
  std::vector<std::thread> ingest;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

static size_t a_elem_bytes(int fmt) { return fmt == NSRGS_A_F32 ? 4 : 2; }

static void plan_memory(const Server &S, Request &q) {
  const int nd = q.r.n * q.r.d;
  const int64_t ld = ((int64_t)nd + 15) / 16 * 16;
  q.a_bytes = (size_t)nd * ld * a_elem_bytes(S.o.fmt);
  q.x_bytes = (size_t)nd * q.r.d * sizeof(float);
  q.stats_bytes = (size_t)batch_panels(q.r.n, q.r.d) * sizeof(PanelStat);
  q.z_bytes = (size_t)nd * q.r.d * sizeof(double);
  q.stage_rows = S.o.fmt == NSRGS_A_F32 ? 0 : (int)std::max<int64_t>(1, std::min<int64_t>(nd, kStageBytes / (ld * 4)));
  q.stage_bytes = (size_t)q.stage_rows * ld * 4;
  q.iws_bytes = narrow_ws_bytes(q.r.n, q.r.d, NSRGS_A_F32);
  q.A.fmt = S.o.fmt;
  q.A.ld = ld;
}

static std::vector<size_t> footprint(const Request &q) {
  return {q.a_bytes, q.x_bytes, q.x_bytes, q.stats_bytes, q.z_bytes, q.stage_bytes, q.iws_bytes};
}

static void free_transient(Server &S, Request &q) {
  S.pool.release(q.zdev);
  S.pool.release(q.stage);
  S.pool.release(q.iws);
  q.zdev = q.stage = q.iws = nullptr;
}

static void free_all(Server &S, Request &q) {
  free_transient(S, q);
  S.pool.release(q.a_mem);
  S.pool.release(q.x0);
  S.pool.release(q.x1);
  S.pool.release(q.stats);
  q.a_mem = q.x0 = q.x1 = q.stats = nullptr;
}

// Called with S.mu held.
static void finish(Server &S, const std::shared_ptr<Request> &q, int status) {
  q->status = status;
  q->state = kDone;
  q->t_done = S.now();
  nsrgs_result res{};
  res.id = q->id;
  res.status = status;
  res.iters = q->t;
  res.converged = q->converged;
  res.t_submit = q->t_submit;
  res.t_admit = q->t_admit;
  res.t_start = q->t_start;
  res.t_done = q->t_done;
  res.rel_change = q->rel_change;
  S.results.push_back(res);
  if (status == NSRGS_OK || status == NSRGS_ERR_NOT_CONVERGED) {
    S.latencies.push_back(q->t_done - q->t_submit);
    S.completed += 1;
    S.last_done = q->t_done;
  } else {
    S.rejected += 1;
  }
  S.idle_cv.notify_all();
}

// Generate A on the device (row chunks), then the spectral initialization.
static int ingest_steps(Server &S, Request &q, hipStream_t s) {
  const int n = q.r.n, d = q.r.d, nd = n * d;
  NSRGS_HIP(hipMemcpyAsync(q.zdev, q.Z.data(), q.z_bytes, hipMemcpyHostToDevice, s), "Z upload");
  if (S.o.fmt == NSRGS_A_F32) {
    NSRGS_HIP(launch_generate_rows(static_cast<double *>(q.zdev), n, d, q.r.sigma, q.r.seed, 0, 1.0,
                                   NSRGS_A_F32, q.a_mem, q.A.ld, 0, nd, s), "generate");
  } else {
    for (int r0 = 0; r0 < nd; r0 += q.stage_rows) {
      const int rows = std::min(q.stage_rows, nd - r0);
      NSRGS_HIP(launch_generate_rows(static_cast<double *>(q.zdev), n, d, q.r.sigma, q.r.seed, 0, 1.0,
                                     NSRGS_A_F32, q.stage, q.A.ld, r0, rows, s), "generate");
      NSRGS_HIP(launch_convert_rows(static_cast<float *>(q.stage), nd, q.A.ld, q.A, r0, rows, s), "convert");
    }
  }
  NSRGS_HIP(launch_ctl_reset(static_cast<DevCtl *>(q.iws), 0, s), "ctl reset");
  const int st = sync_init_spectral(&q.A, n, d, q.x0, 0, 0.0, q.iws, q.iws_bytes, s, nullptr);
  if (st != NSRGS_OK && st != NSRGS_ERR_NOT_CONVERGED) return st;
  NSRGS_HIP(hipStreamSynchronize(s), "ingest sync");
  return NSRGS_OK;
}

// ingest_steps, and on any error a wait for the stream before returning: the
// caller then releases the request's buffers to the pool, and no kernel or
// copy enqueued above may still be writing them.
static int ingest_one(Server &S, Request &q, hipStream_t s) {
  const int st = ingest_steps(S, q, s);
  if (st != NSRGS_OK) (void)hipStreamSynchronize(s);
  return st;
}

static void ingest_loop(Server *S, int worker) {
  (void)hipSetDevice(S->device);
  hipStream_t stream = S->ingest_streams[worker];
  for (;;) {
    std::shared_ptr<Request> q;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->ingest_cv.wait(lk, [&] { return S->stop || !S->ingest_q.empty(); });
      if (S->stop) return;
      q = S->ingest_q.front();
      S->ingest_q.pop_front();
    }
    const int st = ingest_one(*S, *q, stream);
    std::lock_guard<std::mutex> lk(S->mu);
    free_transient(*S, *q);
    S->ingesting -= 1;
    if (st != NSRGS_OK) {
      free_all(*S, *q);
      finish(*S, q, st);
    } else {
      q->state = kReady;
      S->ready.push_back(q);
    }
    S->cv.notify_all();
  }
}

// Admit pending requests in arrival order while memory and slots allow
// (a request that does not fit yet does not block smaller ones behind it).
// Called with S.mu held.
static void admit(Server &S) {
  for (auto it = S.pending.begin(); it != S.pending.end();) {
    const int slots = (int)S.active.size() + (int)S.ready.size() + S.ingesting;
    if (slots >= S.o.max_active) break;
    Request &q = **it;
    if (!S.pool.fits(footprint(q))) {
      ++it;
      continue;
    }
    q.a_mem = S.pool.alloc(q.a_bytes);
    q.x0 = S.pool.alloc(q.x_bytes);
    q.x1 = S.pool.alloc(q.x_bytes);
    q.stats = S.pool.alloc(q.stats_bytes);
    q.zdev = S.pool.alloc(q.z_bytes);
    q.stage = q.stage_bytes ? S.pool.alloc(q.stage_bytes) : nullptr;
    q.iws = S.pool.alloc(q.iws_bytes);
    q.A.data = q.a_mem;
    q.state = kIngest;
    q.t_admit = S.now();
    S.ingesting += 1;
    S.ingest_q.push_back(*it);
    it = S.pending.erase(it);
    S.ingest_cv.notify_all();
  }
}

static int ensure_ctl(Server &S, int count, size_t units) {
  const size_t need = group_control_bytes(count, units);
  if (need <= S.ctl_bytes) return NSRGS_OK;
  if (S.ctl) NSRGS_HIP(hipFree(S.ctl), "control free");
  S.ctl = nullptr;
  S.ctl_bytes = 0;
  NSRGS_HIP(hipMalloc(&S.ctl, need * 2), "control alloc");
  S.ctl_bytes = need * 2;
  return NSRGS_OK;
}

static void schedule_loop(Server *S) {
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    if (S->stop) {
      // shutting down: active requests end without a result
      for (auto &q : S->active) {
        free_all(*S, *q);
        finish(*S, q, NSRGS_ERR_NOT_CONVERGED);
      }
      S->active.clear();
      return;
    }
    admit(*S);
    while (!S->ready.empty()) {
      auto q = S->ready.front();
      S->ready.pop_front();
      q->state = kActive;
      q->t_start = S->now();
      S->active.push_back(q);
    }
    S->max_active_seen = std::max(S->max_active_seen, (int)S->active.size());
    if (S->active.empty()) {
      S->cv.wait_for(lk, std::chrono::milliseconds(50));
      continue;
    }
    // One tick over the active requests (the lock is released while the
    // device works; new submissions and ingest completions queue up).
    std::vector<std::shared_ptr<Request>> batch = S->active;
    lk.unlock();
    std::vector<GroupSpec> specs(batch.size());
    size_t units = 0;
    for (size_t k = 0; k < batch.size(); ++k) {
      const Request &q = *batch[k];
      GroupSpec &g = specs[k];
      g.A = q.A;
      g.n = q.r.n;
      g.d = q.r.d;
      g.iters = q.r.max_iters;
      g.t0 = q.t;
      g.X0 = q.x0;
      g.X1 = q.x1;
      g.stats = q.stats;
      g.mu = 0.0;
      g.tol = q.r.tol;
      units += (size_t)batch_panels(q.r.n, q.r.d);
    }
    std::vector<BatchResult> res;
    int st = ensure_ctl(*S, (int)batch.size(), units);
    if (st == NSRGS_OK)
      st = run_grouped(S->o.fmt, specs, S->ctl, S->o.iters_per_tick, S->o.ns_steps, S->o.waves, 0,
                       S->o.iters_per_tick, S->solve_stream, res);
    // Results of finished requests go to the caller's host buffers.
    std::vector<int> done(batch.size(), 0);
    for (size_t k = 0; k < batch.size(); ++k) {
      Request &q = *batch[k];
      if (st != NSRGS_OK) {
        done[k] = 1;
        continue;
      }
      q.t = res[k].iters;
      q.converged = res[k].converged;
      q.nonfinite = res[k].nonfinite;
      q.rel_change = res[k].rel_change;
      if (!res[k].active) {
        done[k] = 1;
        if (q.r.X_out)
          (void)hipMemcpyAsync(q.r.X_out, (q.t & 1) ? q.x1 : q.x0, q.x_bytes, hipMemcpyDeviceToHost,
                               S->solve_stream);
      }
    }
    (void)hipStreamSynchronize(S->solve_stream);
    lk.lock();
    std::vector<std::shared_ptr<Request>> keep;
    for (size_t k = 0; k < batch.size(); ++k) {
      auto &q = batch[k];
      if (!done[k]) {
        keep.push_back(q);
        continue;
      }
      int status = st;
      if (status == NSRGS_OK) {
        if (q->nonfinite) status = NSRGS_ERR_NONFINITE;
        else if (!q->converged) status = NSRGS_ERR_NOT_CONVERGED;
      }
      free_all(*S, *q);
      finish(*S, q, status);
    }
    // Requests that became ready during the tick wait in S->ready and join
    // at the top of the loop.
    S->active = keep;
  }
}

}  // namespace nsrgs

using namespace nsrgs;

struct nsrgs_server {
  Server impl;
};

extern "C" {

int nsrgs_server_create(const nsrgs_server_opts *opts, nsrgs_server **out) {
  if (!out) return fail(NSRGS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  nsrgs_server_opts o{};
  if (opts) o = *opts;
  if (o.fmt == 0 && !opts) o.fmt = NSRGS_A_BF16;
  if (o.fmt != NSRGS_A_BF16 && o.fmt != NSRGS_A_F32)
    return fail(NSRGS_ERR_INVALID_ARG, "server storage format must be BF16 or F32");
  if (o.max_active <= 0) o.max_active = 64;
  if (o.iters_per_tick <= 0) o.iters_per_tick = 4;
  if (o.ns_steps < 0 || o.ns_steps > 64) return fail(NSRGS_ERR_INVALID_ARG, "ns_steps must be in [0, 64]");
  if (o.ns_steps == 0) o.ns_steps = 3;
  if (o.waves < 0 || o.waves > kMaxWaves) return fail(NSRGS_ERR_INVALID_ARG, "waves must be in [0, %d]", kMaxWaves);
  if (o.waves == 0) o.waves = tuned_batch_waves(o.fmt, 4);
  if (o.ingest_workers <= 0) o.ingest_workers = 4;
  if (o.ingest_workers > 16) return fail(NSRGS_ERR_INVALID_ARG, "at most 16 ingest workers");
  std::unique_ptr<nsrgs_server> srv(new nsrgs_server());
  Server &S = srv->impl;
  NSRGS_HIP(hipGetDevice(&S.device), "get device");
  if (o.pool_bytes == 0) {
    size_t fr = 0, tot = 0;
    NSRGS_HIP(hipMemGetInfo(&fr, &tot), "memory info");
    o.pool_bytes = fr / 2;
  }
  S.o = o;
  hipError_t e = S.pool.init(o.pool_bytes);
  if (e != hipSuccess) return fail(NSRGS_ERR_OUT_OF_MEMORY, "server pool of %zu bytes: %s", (size_t)o.pool_bytes,
                                   hipGetErrorString(e));
  NSRGS_HIP(hipStreamCreateWithFlags(&S.solve_stream, hipStreamNonBlocking), "stream");
  S.ingest_streams.resize(o.ingest_workers);
  for (auto &st : S.ingest_streams) NSRGS_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "stream");
  S.t0 = std::chrono::steady_clock::now();
  S.sched = std::thread(schedule_loop, &S);
  for (int w = 0; w < o.ingest_workers; ++w) S.ingest.emplace_back(ingest_loop, &S, w);
  *out = srv.release();
  return NSRGS_OK;
}

int nsrgs_server_submit(nsrgs_server *srv, const nsrgs_request *req, int64_t *id) {
  if (!srv || !req) return fail(NSRGS_ERR_INVALID_ARG, "NULL server or request");
  Server &S = srv->impl;
  int st;
  if ((st = check_common(req->n, req->d))) return st;
  if (!req->Z) return fail(NSRGS_ERR_INVALID_ARG, "request needs the ground truth Z to generate A");
  if (!std::isfinite(req->sigma)) return fail(NSRGS_ERR_INVALID_ARG, "bad sigma");
  auto q = std::make_shared<Request>();
  q->r = *req;
  if (q->r.tol <= 0.0) q->r.tol = 1e-6;
  if (q->r.max_iters <= 0) q->r.max_iters = 300;
  const size_t nz = (size_t)req->n * req->d * req->d;
  q->Z.assign(req->Z, req->Z + nz);
  plan_memory(S, *q);
  size_t need = 0;
  for (size_t b : footprint(*q)) need += align256(b);
  std::lock_guard<std::mutex> lk(S.mu);
  if (S.stop) return fail(NSRGS_ERR_INVALID_ARG, "server is shutting down");
  q->id = S.next_id++;
  q->t_submit = S.now();
  if (S.first_submit < 0) S.first_submit = q->t_submit;
  S.submitted += 1;
  if (id) *id = q->id;
  if (need > S.pool.total()) {
    finish(S, q, fail(NSRGS_ERR_OUT_OF_MEMORY, "request needs %zu bytes, the pool holds %zu", need,
                      S.pool.total()));
    return NSRGS_OK;
  }
  S.pending.push_back(q);
  S.cv.notify_all();
  return NSRGS_OK;
}

int nsrgs_server_poll(nsrgs_server *srv, nsrgs_result *results, int max, int *count) {
  if (!srv || !count || (max > 0 && !results)) return fail(NSRGS_ERR_INVALID_ARG, "bad poll arguments");
  Server &S = srv->impl;
  std::lock_guard<std::mutex> lk(S.mu);
  int k = 0;
  while (k < max && !S.results.empty()) {
    results[k++] = S.results.front();
    S.results.pop_front();
  }
  *count = k;
  return NSRGS_OK;
}

int nsrgs_server_wait_idle(nsrgs_server *srv, double timeout_s) {
  if (!srv) return fail(NSRGS_ERR_INVALID_ARG, "NULL server");
  Server &S = srv->impl;
  std::unique_lock<std::mutex> lk(S.mu);
  auto idle = [&] {
    return S.pending.empty() && S.ingest_q.empty() && S.ready.empty() && S.active.empty() && S.ingesting == 0;
  };
  if (timeout_s <= 0) {
    S.idle_cv.wait(lk, idle);
    return NSRGS_OK;
  }
  if (!S.idle_cv.wait_for(lk, std::chrono::duration<double>(timeout_s), idle))
    return fail(NSRGS_ERR_NOT_CONVERGED, "server not idle after %.1f s", timeout_s);
  return NSRGS_OK;
}

int nsrgs_server_get_stats(nsrgs_server *srv, nsrgs_server_stats *st) {
  if (!srv || !st) return fail(NSRGS_ERR_INVALID_ARG, "NULL argument");
  Server &S = srv->impl;
  std::lock_guard<std::mutex> lk(S.mu);
  memset(st, 0, sizeof(*st));
  st->submitted = S.submitted;
  st->completed = S.completed;
  st->rejected = S.rejected;
  st->active = (int32_t)S.active.size();
  st->max_active_seen = S.max_active_seen;
  std::vector<double> l = S.latencies;
  std::sort(l.begin(), l.end());
  auto pct = [&](double p) {
    if (l.empty()) return 0.0;
    const double pos = p * (l.size() - 1);
    const size_t i = (size_t)pos;
    const double f = pos - i;
    return i + 1 < l.size() ? l[i] * (1 - f) + l[i + 1] * f : l[i];
  };
  st->p50_latency_s = pct(0.50);
  st->p99_latency_s = pct(0.99);
  double sum = 0;
  for (double v : l) sum += v;
  st->mean_latency_s = l.empty() ? 0.0 : sum / l.size();
  const double span = S.last_done - std::max(0.0, S.first_submit);
  st->solves_per_s = (span > 0 && S.completed > 0) ? S.completed / span : 0.0;
  st->pool_bytes = S.pool.total();
  st->pool_peak_bytes = S.pool.peak();
  return NSRGS_OK;
}

double nsrgs_server_clock(const nsrgs_server *srv) { return srv ? srv->impl.now() : 0.0; }

int nsrgs_server_destroy(nsrgs_server *srv) {
  if (!srv) return NSRGS_OK;
  Server &S = srv->impl;
  {
    std::lock_guard<std::mutex> lk(S.mu);
    S.stop = true;
    S.cv.notify_all();
    S.ingest_cv.notify_all();
  }
  for (auto &t : S.ingest)
    if (t.joinable()) t.join();
  if (S.sched.joinable()) S.sched.join();
  {
    std::lock_guard<std::mutex> lk(S.mu);
    for (auto *q : {&S.pending, &S.ingest_q, &S.ready}) {
      for (auto &r : *q) {
        free_all(S, *r);
        finish(S, r, NSRGS_ERR_NOT_CONVERGED);
      }
      q->clear();
    }
  }
  if (S.solve_stream) (void)hipStreamSynchronize(S.solve_stream);
  for (auto st : S.ingest_streams) (void)hipStreamSynchronize(st);
  if (S.ctl) (void)hipFree(S.ctl);
  if (S.solve_stream) (void)hipStreamDestroy(S.solve_stream);
  for (auto st : S.ingest_streams) (void)hipStreamDestroy(st);
  delete srv;
  return NSRGS_OK;
}

}  // extern "C"
