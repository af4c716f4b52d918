// Many-problem runtime of libhotrg: a pool of worker contexts, each with its
// own HIP stream and device workspace, fed from one queue.  Used by
// hotrg_run_batch (a batch of temperatures / couplings / D_cut values) and by
// the serving calls hotrg_submit / poll / wait / cancel (continuous
// batching: problems arriving while others run are admitted as soon as a
// worker is free and their device footprint fits the HBM budget).
//
// Admission.  The footprint of a problem is the sum over the context's
// grow-only buffers of their largest size over the problem's steps (the
// dimension schedule is known on the host).  The queue is served in arrival
// order; when the oldest problem does not fit next to the running ones, a
// later one that fits may go first, but the oldest is skipped at most
// kMaxSkips times before admission waits for it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "admit.h"
#include "internal.h"
#include "precision.h"

namespace hotrg {
size_t topk_workspace_doubles(int n, int p);
}

namespace {

using namespace hotrg;

constexpr size_t kSolverMargin = 256ull << 20;  // rocBLAS / rocSOLVER internal workspace

enum ReqState { Q_QUEUED = 0, Q_RUNNING = 1, Q_DONE = 2 };

struct Request {
  uint64_t id = 0;
  hotrg_model_params params{};
  std::vector<double> raw;
  hotrg_opts opts{};
  hotrg_result* out = nullptr;
  std::atomic<bool> cancel{false};
  int state = Q_QUEUED;
  hotrg_status status = HOTRG_ERR_NOT_READY;
  std::string err;
  size_t footprint = 0;
  int skips = 0;
  bool retried = false;
};

struct Server {
  hotrg_ctx* parent = nullptr;
  std::vector<hotrg_ctx*> workers;
  std::vector<std::thread> threads;
  std::mutex mu;
  std::condition_variable cv;       // work available / capacity freed
  std::condition_variable done_cv;  // a request finished
  std::deque<std::shared_ptr<Request>> queue;
  std::unordered_map<uint64_t, std::shared_ptr<Request>> all;
  std::vector<size_t> hold;         // bytes held by each idle worker
  size_t budget = 0;
  size_t reserved = 0;
  size_t peak_reserved = 0;
  uint64_t next_id = 1;
  uint64_t admitted = 0;
  uint64_t stalls = 0;
  bool stop = false;
};

// ---------------------------------------------------------------- footprint --
struct Dims {
  int dx, dy, dn;
};

bool initial_dims(const hotrg_model_params* p, int* dx, int* dy) {
  switch (p->model) {
    case HOTRG_ISING:
      *dx = *dy = 2;
      return true;
    case HOTRG_XY:
      *dx = *dy = 2 * p->n_max + 1;
      return p->n_max >= 0;
    case HOTRG_POTTS:
      *dx = *dy = p->q;
      return p->q >= 2;
    case HOTRG_GXY:
      *dx = *dy = 2 * p->n_max + 1;
      return p->n_max >= 0;
    case HOTRG_RAW:
      *dx = p->raw_dx;
      *dy = p->raw_dy;
      return p->raw_dx >= 1 && p->raw_dy >= 1;
    default:
      return false;
  }
}

// HOTRG_PREC_AUTO resolved as run_problem resolves it
hotrg_opts resolved(const hotrg_model_params* p, const hotrg_opts* o) {
  hotrg_opts r = *o;
  int dx = 0, dy = 0;
  if (r.prec == HOTRG_PREC_AUTO && initial_dims(p, &dx, &dy))
    r.prec = r.isometry == HOTRG_ISO_TWO_SIDED
                 ? HOTRG_FP64
                 : plan_auto(r.tol, dx, dy, r.d_cut, r.n_steps).prec;
  return r;
}

size_t footprint_of(const hotrg_model_params* p, const hotrg_opts* o_in) {
  int dx = 0, dy = 0;
  if (!initial_dims(p, &dx, &dy)) return 0;
  const hotrg_opts ro = resolved(p, o_in);
  const hotrg_opts* o = &ro;
  const int k0 = first_reduced_step(o->prec, o->tol);
  std::map<std::string, size_t> peak;
  auto need = [&](const char* name, double bytes) {
    size_t b = (size_t)bytes;
    if (b > peak[name]) peak[name] = b;
  };
  auto pad = [](long long k) { return (double)((k + 31) / 32 * 32); };
  need("state", 3.0 * dx * dy * dx * dy * 8);
  for (int k = 0; k < o->n_steps; ++k) {
    const double n = (double)dx * dx, P = (double)dx * dy;
    const int dn = (int)std::min<long long>(o->d_cut, (long long)dx * dx);
    const double X = (double)dn * dx * dx * dy * dy;
    const bool red = step_is_reduced(o->prec, k + 1, dx, dy, o->d_cut, k0);
    need("M", n * n * 8);
    need("WE", 2 * n * 8);
    need("U", 3 * n * dn * 8);
    const int p = std::min(128, std::max(2 * dn, dn + 17));
    need("eig", (double)topk_workspace_doubles((int)n, (p + 15) / 16 * 16) * 8 + (double)p * n * 8);
    need("dense", n > 128 ? n * n * 8 : 0);  // dsyevd fallback workspace
    if (o->isometry == HOTRG_ISO_TWO_SIDED && dn < n) {
      // mirrored operands, right environment, its eigenpairs
      need("side", 2.0 * dx * dy * dx * dy * 8 + n * n * 8 + n * 8 + (double)p * n * 8);
    }
    if (!red) {
      need("A12", 2 * P * P * 8);
      need("X12", 2 * X * 8);
      need("Tt", (double)dn * dy * dn * dy * 8);
    } else {
      const double es = 4;  // FP32, or two bf16 arrays
      need("rA12", 2 * n * pad((long long)dy * dy) * es);
      need("rX12", (double)dn * dy * dx * pad((long long)dx * dy) * es +
                       (double)dn * dy * dy * pad((long long)dx * dx) * es);
      need("rU", (double)dn * dx * pad(dx) * es + (double)dn * pad((long long)dx * dx) * es);
      need("Tt", (double)dn * dy * dn * dy * 4);
      need("rstate", 4 * (double)dy * dn * dy * dn * 8);
    }
    // next state (both generations exist while the operands are rebuilt)
    need("state", 6.0 * dy * dn * dy * dn * 8);
    const int ndx = dy;
    dy = dn;
    dx = ndx;
  }
  size_t total = kSolverMargin;
  for (auto& kv : peak) total += kv.second;
  return total;
}

// ------------------------------------------------------------------ server --
// S->reserved counts the footprint of every running problem plus the bytes
// each idle worker context still holds (its grow-only buffers are kept
// between problems so that equal-sized problems do not re-allocate).  A
// problem runs on worker w either next to w's held buffers (held + footprint
// is a bound on what w holds while it runs) or after w has released them; an
// idle worker that holds memory while a queued problem does not fit releases
// its buffers, so every problem within the budget is admitted eventually.
void worker_loop(Server* S, int w) {
  hotrg_ctx* c = S->workers[w];
  size_t& hold = S->hold[w];
  for (;;) {
    std::shared_ptr<Request> r;
    bool release = false;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      for (;;) {
        if (S->stop) return;
        const size_t others = S->reserved - hold;
        const AdmitChoice ch = admit_choice(
            S->queue, [](const std::shared_ptr<Request>& q) { return q->footprint; },
            [](const std::shared_ptr<Request>& q) { return q->skips; }, others, hold, S->budget);
        if (ch.action == ADMIT_RELEASE) {
          release = true;  // release this worker's buffers, then decide again
          break;
        }
        if (ch.action == ADMIT_RUN) {
          if (ch.index > 0) {
            ++S->queue.front()->skips;
            ++S->stalls;
          }
          r = S->queue[ch.index];
          S->queue.erase(S->queue.begin() + (long)ch.index);
          break;
        }
        if (!S->queue.empty()) ++S->stalls;
        S->cv.wait(lk);
      }
      if (r) {
        r->state = Q_RUNNING;
        S->reserved += r->footprint;
        S->peak_reserved = std::max(S->peak_reserved, S->reserved);
        ++S->admitted;
        r->out->t_start = ctx_seconds(S->parent);
      }
    }
    if (release) {
      ctx_trim(c);
      std::lock_guard<std::mutex> lk(S->mu);
      S->reserved -= hold;
      hold = 0;
      S->cv.notify_all();
    }
    if (!r) continue;
    hotrg_status st = run_problem(c, &r->params, &r->opts, r->out, &r->cancel);
    r->out->prec_used = r->opts.prec;
    std::string err = st == HOTRG_OK ? "" : last_error_text();
    const size_t held = hotrg_ctx_bytes_in_use(c);
    const bool retry = st == HOTRG_ERR_NUMERIC && r->opts.prec != HOTRG_FP64 && !r->retried &&
                       !r->cancel.load();
    hotrg_opts o64 = r->opts;
    o64.prec = HOTRG_FP64;
    const size_t f64 = retry ? footprint_of(&r->params, &o64) : 0;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->reserved -= r->footprint + hold;
      hold = held;
      S->reserved += hold;
      // a cancel that arrived while the request ran found it Q_RUNNING and did
      // not take it off the queue: it must not be queued again
      if (retry && f64 <= S->budget && !r->cancel.load()) {
        // reduced-precision noise drove the run off: queue it once more in FP64
        r->opts = o64;
        r->footprint = f64;
        r->retried = true;
        r->state = Q_QUEUED;
        r->skips = 0;
        S->queue.push_front(r);
        S->cv.notify_all();
        continue;
      }
      r->out->t_end = ctx_seconds(S->parent);
      r->status = st;
      r->err = err;
      r->state = Q_DONE;
    }
    S->cv.notify_all();
    S->done_cv.notify_all();
  }
}

Server* server_of(hotrg_ctx* c, bool create) {
  void*& slot = ctx_sched(c);
  if (slot || !create) return (Server*)slot;
  auto* S = new Server();
  S->parent = c;
  size_t budget = ctx_budget(c);
  if (budget == 0) {
    size_t free_b = 0, total_b = 0;
    (void)hipSetDevice(ctx_device(c));
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = 1ull << 34;
    budget = (size_t)(0.9 * (double)free_b);
  }
  S->budget = budget;
  const int nw = std::max(1, ctx_workers(c));
  for (int i = 0; i < nw; ++i) {
    hotrg_ctx* w = nullptr;
    if (hotrg_ctx_create(ctx_device(c), nullptr, 0, &w) != HOTRG_OK) break;
    ctx_test_fail_step(w) = ctx_test_fail_step(c);
    S->workers.push_back(w);
  }
  if (S->workers.empty()) {
    delete S;
    return nullptr;
  }
  S->hold.assign(S->workers.size(), 0);
  for (int i = 0; i < (int)S->workers.size(); ++i) S->threads.emplace_back(worker_loop, S, i);
  slot = S;
  return S;
}

double now_s(hotrg_ctx* c) { return ctx_seconds(c); }

}  // namespace

namespace hotrg {

void sched_shutdown(hotrg_ctx* c) {
  Server* S = server_of(c, false);
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    for (auto& kv : S->all) kv.second->cancel = true;
  }
  S->cv.notify_all();
  for (auto& t : S->threads) t.join();
  for (hotrg_ctx* w : S->workers) hotrg_ctx_destroy(w);
  delete S;
  ctx_sched(c) = nullptr;
}

}  // namespace hotrg

extern "C" {

hotrg_status hotrg_ctx_set_workers(hotrg_ctx* ctx, int n_workers) {
  if (!ctx || n_workers < 1 || n_workers > 64) {
    set_last_error("n_workers must be in [1, 64]");
    return HOTRG_ERR_INVALID;
  }
  if (ctx_sched(ctx)) {
    set_last_error("workers are already running");
    return HOTRG_ERR_INVALID;
  }
  ctx_workers(ctx) = n_workers;
  return HOTRG_OK;
}

hotrg_status hotrg_footprint(const hotrg_model_params* params, const hotrg_opts* opts,
                             size_t* bytes) {
  if (!params || !opts || !bytes) {
    set_last_error("NULL argument");
    return HOTRG_ERR_INVALID;
  }
  size_t b = footprint_of(params, opts);
  if (b == 0) {
    set_last_error("unknown model or bad dimensions");
    return HOTRG_ERR_INVALID;
  }
  *bytes = b;
  return HOTRG_OK;
}

hotrg_status hotrg_submit(hotrg_ctx* ctx, const hotrg_model_params* params, const hotrg_opts* opts,
                          hotrg_result* result, uint64_t* ticket) {
  if (!ctx || !params || !opts || !result || !ticket) {
    set_last_error("NULL argument");
    return HOTRG_ERR_INVALID;
  }
  if (opts->d_cut < 1 || opts->n_steps < 0) {
    set_last_error("d_cut must be >= 1 and n_steps >= 0");
    return HOTRG_ERR_INVALID;
  }
  auto r = std::make_shared<Request>();
  r->params = *params;
  if (params->model == HOTRG_RAW) {
    if (!params->raw || params->raw_dx < 1 || params->raw_dy < 1) {
      set_last_error("raw tensor: need raw != NULL and positive dims");
      return HOTRG_ERR_INVALID;
    }
    const size_t ne = (size_t)params->raw_dx * params->raw_dy * params->raw_dx * params->raw_dy;
    r->raw.assign(params->raw, params->raw + ne);
    r->params.raw = r->raw.data();
  }
  if (opts->prec == HOTRG_PREC_AUTO && !(opts->tol > 0.0)) {
    set_last_error("HOTRG_PREC_AUTO needs tol > 0");
    return HOTRG_ERR_INVALID;
  }
  // the precision is chosen at admission: the cheapest that meets tol
  r->opts = resolved(params, opts);
  r->out = result;
  r->footprint = footprint_of(params, &r->opts);
  if (r->footprint == 0) {
    set_last_error("unknown model or bad dimensions");
    return HOTRG_ERR_INVALID;
  }
  Server* S = server_of(ctx, true);
  if (!S) {
    set_last_error("could not start workers");
    return HOTRG_ERR_DEVICE;
  }
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (r->footprint > S->budget) {
      set_last_error("problem footprint exceeds the HBM budget");
      return HOTRG_ERR_OOM;
    }
    r->id = S->next_id++;
    result->t_submit = now_s(ctx);
    result->t_start = result->t_end = -1.0;
    S->all[r->id] = r;
    S->queue.push_back(r);
    *ticket = r->id;
  }
  S->cv.notify_all();
  return HOTRG_OK;
}

static hotrg_status status_locked(Server* S, uint64_t ticket, std::shared_ptr<Request>* out) {
  auto it = S->all.find(ticket);
  if (it == S->all.end()) return HOTRG_ERR_INVALID;
  if (out) *out = it->second;
  return it->second->state == Q_DONE ? it->second->status : HOTRG_ERR_NOT_READY;
}

hotrg_status hotrg_poll(hotrg_ctx* ctx, uint64_t ticket) {
  Server* S = ctx ? server_of(ctx, false) : nullptr;
  if (!S) {
    set_last_error("no such ticket");
    return HOTRG_ERR_INVALID;
  }
  std::shared_ptr<Request> r;
  hotrg_status st;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    st = status_locked(S, ticket, &r);
  }
  if (st == HOTRG_ERR_INVALID) set_last_error("no such ticket");
  else if (st != HOTRG_OK && st != HOTRG_ERR_NOT_READY) set_last_error(r->err.c_str());
  return st;
}

hotrg_status hotrg_wait(hotrg_ctx* ctx, uint64_t ticket, double timeout_s) {
  Server* S = ctx ? server_of(ctx, false) : nullptr;
  if (!S) {
    set_last_error("no such ticket");
    return HOTRG_ERR_INVALID;
  }
  std::shared_ptr<Request> r;
  hotrg_status st;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    auto ready = [&] { return status_locked(S, ticket, &r) != HOTRG_ERR_NOT_READY; };
    if (timeout_s < 0)
      S->done_cv.wait(lk, ready);
    else
      S->done_cv.wait_for(lk, std::chrono::duration<double>(timeout_s), ready);
    st = status_locked(S, ticket, &r);
  }
  if (st == HOTRG_ERR_INVALID) set_last_error("no such ticket");
  else if (st != HOTRG_OK && st != HOTRG_ERR_NOT_READY) set_last_error(r->err.c_str());
  return st;
}

hotrg_status hotrg_cancel(hotrg_ctx* ctx, uint64_t ticket) {
  Server* S = ctx ? server_of(ctx, false) : nullptr;
  if (!S) {
    set_last_error("no such ticket");
    return HOTRG_ERR_INVALID;
  }
  {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) {
      set_last_error("no such ticket");
      return HOTRG_ERR_INVALID;
    }
    auto& r = it->second;
    r->cancel = true;
    if (r->state == Q_QUEUED) {
      S->queue.erase(std::remove(S->queue.begin(), S->queue.end(), r), S->queue.end());
      r->state = Q_DONE;
      r->status = HOTRG_ERR_CANCELLED;
      r->err = "cancelled";
      r->out->t_end = now_s(ctx);
    }
  }
  S->cv.notify_all();
  S->done_cv.notify_all();
  return HOTRG_OK;
}

hotrg_status hotrg_release(hotrg_ctx* ctx, uint64_t ticket) {
  Server* S = ctx ? server_of(ctx, false) : nullptr;
  if (!S) {
    set_last_error("no such ticket");
    return HOTRG_ERR_INVALID;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) {
    set_last_error("no such ticket");
    return HOTRG_ERR_INVALID;
  }
  if (it->second->state != Q_DONE) {
    set_last_error("problem still queued or running");
    return HOTRG_ERR_NOT_READY;
  }
  S->all.erase(it);
  return HOTRG_OK;
}

hotrg_status hotrg_run_batch(hotrg_ctx* ctx, int n, const hotrg_model_params* params,
                             const hotrg_opts* opts, hotrg_result* results,
                             hotrg_status* statuses) {
  if (!ctx || n < 0 || (n > 0 && (!params || !opts || !results))) {
    set_last_error("NULL argument");
    return HOTRG_ERR_INVALID;
  }
  // largest problems first, for load balance over the workers
  std::vector<int> order(n);
  std::vector<size_t> cost(n);
  for (int i = 0; i < n; ++i) {
    order[i] = i;
    cost[i] = footprint_of(&params[i], &opts[i]);
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<uint64_t> tickets(n, 0);
  std::vector<hotrg_status> st(n, HOTRG_OK);
  for (int i : order) {
    st[i] = hotrg_submit(ctx, &params[i], &opts[i], &results[i], &tickets[i]);
  }
  hotrg_status first = HOTRG_OK;
  std::string first_err;
  for (int i = 0; i < n; ++i) {
    if (st[i] == HOTRG_OK) {
      st[i] = hotrg_wait(ctx, tickets[i], -1.0);
      (void)hotrg_release(ctx, tickets[i]);
    }
    if (statuses) statuses[i] = st[i];
    if (st[i] != HOTRG_OK && first == HOTRG_OK) {
      first = st[i];
      first_err = last_error_text();
    }
  }
  if (first != HOTRG_OK) set_last_error(first_err.c_str());
  return first;
}

hotrg_status hotrg_thermo(hotrg_ctx* ctx, const hotrg_model_params* params,
                          const hotrg_opts* opts, double dbeta, double* out) {
  if (!ctx || !params || !opts || !out) {
    set_last_error("NULL argument");
    return HOTRG_ERR_INVALID;
  }
  if (params->model == HOTRG_RAW) {
    set_last_error("thermo needs a model whose tensor depends on beta");
    return HOTRG_ERR_INVALID;
  }
  if (!(dbeta > 0.0) || !(params->beta - 2.0 * dbeta >= 0.0)) {
    set_last_error("need dbeta > 0 and beta - 2 dbeta >= 0");
    return HOTRG_ERR_INVALID;
  }
  // ln Z/N at beta + j dbeta, j = -2 .. 2, on the worker pool
  hotrg_model_params P[5];
  hotrg_opts O[5];
  hotrg_result R[5];
  hotrg_status S[5];
  for (int j = 0; j < 5; ++j) {
    P[j] = *params;
    P[j].beta = params->beta + (j - 2) * dbeta;
    O[j] = *opts;
    std::memset(&R[j], 0, sizeof(hotrg_result));
  }
  const hotrg_status st = hotrg_run_batch(ctx, 5, P, O, R, S);
  if (st != HOTRG_OK) return st;
  double f[5];
  for (int j = 0; j < 5; ++j) f[j] = R[j].lnz_per_site;
  // five-point central differences, error O(dbeta^4)
  const double d1 = (f[0] - 8.0 * f[1] + 8.0 * f[3] - f[4]) / (12.0 * dbeta);
  const double d2 = (-f[0] + 16.0 * f[1] - 30.0 * f[2] + 16.0 * f[3] - f[4]) / (12.0 * dbeta * dbeta);
  out[0] = f[2];
  out[1] = -d1;
  out[2] = params->beta * params->beta * d2;
  return HOTRG_OK;
}

hotrg_status hotrg_ctx_sched_stats(hotrg_ctx* ctx, uint64_t* admitted, uint64_t* stalls,
                                   size_t* peak_reserved) {
  Server* S = ctx ? server_of(ctx, false) : nullptr;
  if (!S) {
    if (admitted) *admitted = 0;
    if (stalls) *stalls = 0;
    if (peak_reserved) *peak_reserved = 0;
    return ctx ? HOTRG_OK : HOTRG_ERR_INVALID;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  if (admitted) *admitted = S->admitted;
  if (stalls) *stalls = S->stalls;
  if (peak_reserved) *peak_reserved = S->peak_reserved;
  return HOTRG_OK;
}

}  // extern "C"
