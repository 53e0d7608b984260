// Serving form: continuous batching of independent space-time solves.
//
// A server owns a device byte budget, a small set of HIP streams and one
// worker thread.  Requests wait in arrival order.  Whenever a slot is free and
// the head request's context fits in the budget, the worker admits it,
// together with up to max_batch - 1 waiting requests of the same (J, K,
// precision) and a similar tolerance, if the problem is small: they become
// the right-hand sides of one batched context, so every operator of the
// group is one launch.  Admitted groups run at the
// same time on different streams: the worker advances every group by one
// unit of device work (one PCG iteration, or a refinement step) as soon as
// its previous unit has completed, so work of groups admitted at different
// times overlaps on the device.  A finished group writes its solutions,
// releases its slot at once, and its context is kept for reuse by a later
// group of the same shape (or freed when the budget needs the room).
//
// Each right-hand side of a batched context computes exactly what a solo
// solve computes (per right-hand side scalars, tolerance and stopping), so a
// result does not depend on what else runs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "solver.h"

using namespace stp;

namespace {

using Clock = std::chrono::steady_clock;

double seconds_since(Clock::time_point t0, Clock::time_point t1) {
  return std::chrono::duration<double>(t1 - t0).count();
}

struct Request {
  uint64_t id = 0;
  stp_request req{};
  Clock::time_point t_submit, t_start, t_done;
  int state = 0;  // 0 waiting, 1 running, 2 finished
  stp_status status = STP_OK;
  stp_stats stats{};
  std::string error;
};

struct Group {
  stp_ctx* ctx = nullptr;
  size_t bytes = 0;
  std::vector<std::shared_ptr<Request>> reqs;
};

struct Cached {
  stp_ctx* ctx;
  size_t bytes;
  int J, K, prec, nrhs;
};

// Requests whose single context is larger than this are never grouped.
constexpr size_t kGroupMaxBytes = size_t(2) << 30;

int pow2_floor(int n) {
  int p = 1;
  while (p * 2 <= n) p *= 2;
  return p;
}

}  // namespace

struct stp_server {
  size_t budget = 0;
  int max_slots = 1;
  int max_batch = 1;
  stp_options opt{};
  int device = 0;
  std::vector<hipStream_t> streams;
  int next_stream = 0;

  std::mutex mu;
  std::condition_variable cv_work;  // worker: new requests or stop
  std::condition_variable cv_done;  // callers: a request finished
  std::deque<std::shared_ptr<Request>> waiting;
  std::map<uint64_t, std::shared_ptr<Request>> table;
  uint64_t next_id = 1;
  bool stop = false;
  int unfinished = 0;

  // owned by the worker thread
  std::vector<Group> running;
  std::list<Cached> cache;  // most recently used first
  size_t bytes_in_use = 0;  // running + cached contexts
  size_t peak_bytes = 0;
  std::thread worker;

  // statistics (under mu)
  size_t stat_in_use = 0, stat_peak = 0;
  int stat_running = 0;
  int64_t stat_groups = 0, stat_batched = 0;
};

namespace {

void finish_request(stp_server* s, const std::shared_ptr<Request>& r, stp_status st,
                    const std::string& err) {
  std::lock_guard<std::mutex> lk(s->mu);
  r->status = st;
  r->error = err;
  r->t_done = Clock::now();
  r->state = 2;
  s->unfinished -= 1;
  s->cv_done.notify_all();
}

void release_ctx(stp_server* s, stp_ctx* c, size_t bytes, bool keep) {
  if (keep) {
    s->cache.push_front(Cached{c, bytes, c->J, c->K, c->prec, c->nrhs});
  } else {
    stp_destroy(c);
    s->bytes_in_use -= bytes;
  }
}

// Evict cached contexts (least recently used first) until `need` bytes fit.
bool make_room(stp_server* s, size_t need) {
  while (s->bytes_in_use + need > s->budget && !s->cache.empty()) {
    Cached c = s->cache.back();
    s->cache.pop_back();
    stp_destroy(c.ctx);
    s->bytes_in_use -= c.bytes;
  }
  return s->bytes_in_use + need <= s->budget;
}

// A context for (J, K, prec, nrhs): from the cache, or newly created.
stp_status get_ctx(stp_server* s, int J, int K, int prec, int nrhs, stp_ctx** out, size_t* bytes) {
  for (auto it = s->cache.begin(); it != s->cache.end(); ++it) {
    if (it->J == J && it->K == K && it->prec == prec && it->nrhs == nrhs) {
      *out = it->ctx;
      *bytes = it->bytes;
      s->cache.erase(it);
      return STP_OK;
    }
  }
  size_t need = 0;
  STP_TRY(stp_footprint(J, K, nrhs, prec, &need));
  if (!make_room(s, need)) {
    set_error("the request does not fit in the server's device budget");
    return STP_E_OUT_OF_MEMORY;
  }
  hipStream_t st = s->streams[s->next_stream];
  s->next_stream = (s->next_stream + 1) % (int)s->streams.size();
  STP_TRY(stp_create(J, K, nrhs, prec, &s->opt, st, out));
  *bytes = (*out)->bytes;
  s->bytes_in_use += *bytes;
  s->peak_bytes = std::max(s->peak_bytes, s->bytes_in_use);
  return STP_OK;
}

// Bytes a new context would add, after what the cache can give back.
bool fits(stp_server* s, int J, int K, int prec, int nrhs) {
  for (const Cached& c : s->cache)
    if (c.J == J && c.K == K && c.prec == prec && c.nrhs == nrhs) return true;
  size_t need = 0;
  if (stp_footprint(J, K, nrhs, prec, &need) != STP_OK) return false;
  size_t cached = 0;
  for (const Cached& c : s->cache) cached += c.bytes;
  return s->bytes_in_use - cached + need <= s->budget;
}

// Admit waiting requests while a slot is free and the head request fits.
void admit(stp_server* s) {
  while ((int)s->running.size() < s->max_slots) {
    std::vector<std::shared_ptr<Request>> grp;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (s->waiting.empty()) return;
      const stp_request& h = s->waiting.front()->req;
      // requests of the same shape and a tolerance within a factor of 10 of
      // the head's (so the group's right-hand sides need similar iteration
      // counts) join the head request, up to max_batch of them -- for small
      // problems only, whose launches are too short to fill the device; a
      // large one fills it alone and grouping would only hold device memory
      std::vector<size_t> idx{0};
      size_t one = 0;
      const bool small = stp_footprint(h.J, h.K, 1, h.precision, &one) == STP_OK &&
                         one <= kGroupMaxBytes;
      for (size_t i = 1; small && i < s->waiting.size() && (int)idx.size() < s->max_batch; ++i) {
        const stp_request& q = s->waiting[i]->req;
        if (q.J == h.J && q.K == h.K && q.precision == h.precision &&
            q.rel_tol <= 10.0 * h.rel_tol && h.rel_tol <= 10.0 * q.rel_tol)
          idx.push_back(i);
      }
      int nb = pow2_floor((int)idx.size());
      while (nb > 1 && !fits(s, h.J, h.K, h.precision, nb)) nb /= 2;
      if (!fits(s, h.J, h.K, h.precision, nb)) {
        if (!s->running.empty()) return;  // wait for memory to free up
        nb = 1;                           // nothing runs: let get_ctx report the failure
      }
      idx.resize(nb);
      for (size_t k = idx.size(); k-- > 0;) {
        grp.insert(grp.begin(), s->waiting[idx[k]]);
        s->waiting.erase(s->waiting.begin() + (long)idx[k]);
      }
      for (auto& r : grp) {
        r->state = 1;
        r->t_start = Clock::now();
      }
    }
    const stp_request& h = grp.front()->req;
    const int nb = (int)grp.size();
    Group g;
    g.reqs = grp;
    auto start = [&]() -> stp_status {
      STP_TRY(get_ctx(s, h.J, h.K, h.precision, nb, &g.ctx, &g.bytes));
      std::vector<double> tol(nb);
      for (int b = 0; b < nb; ++b) {
        const stp_request& q = grp[b]->req;
        STP_TRY(stp_set_u0(g.ctx, b, q.u0, q.on_device));
        STP_TRY(stp_set_g(g.ctx, b, q.g, q.on_device));
        tol[b] = q.rel_tol;
      }
      STP_TRY(drive_begin(g.ctx, tol.data()));
      return STP_OK;
    };
    const stp_status st = start();
    if (st < 0) {
      const std::string err = stp_last_error();
      if (g.ctx) {
        g.ctx->drv.phase = stp_ctx::kIdle;
        release_ctx(s, g.ctx, g.bytes, false);
      }
      for (auto& r : grp) finish_request(s, r, st, err);
      continue;
    }
    s->running.push_back(std::move(g));
    std::lock_guard<std::mutex> lk(s->mu);
    s->stat_groups += 1;
    s->stat_batched += nb;
  }
}

// Write the solutions of a finished group and release its slot.
void complete(stp_server* s, Group& g) {
  stp_status err_st = STP_OK;
  std::string err;
  for (size_t b = 0; b < g.reqs.size(); ++b) {
    const stp_request& q = g.reqs[b]->req;
    if (q.u) {
      const stp_status st = stp_get_solution(g.ctx, (int)b, q.u, q.on_device);
      if (st < 0 && err_st == STP_OK) {
        err_st = st;
        err = stp_last_error();
      }
    }
  }
  const bool ok = hipStreamSynchronize(g.ctx->stream) == hipSuccess && err_st == STP_OK;
  for (size_t b = 0; b < g.reqs.size(); ++b) {
    g.reqs[b]->stats = g.ctx->stats[b];
    finish_request(s, g.reqs[b], ok ? g.ctx->stats[b].status : (err_st < 0 ? err_st : STP_E_DEVICE),
                   ok ? std::string() : (err.empty() ? std::string("stream error") : err));
  }
  g.ctx->drv.phase = stp_ctx::kIdle;
  release_ctx(s, g.ctx, g.bytes, ok);
  g.ctx = nullptr;
}

void worker_main(stp_server* s) {
  (void)hipSetDevice(s->device);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (s->running.empty())
        s->cv_work.wait(lk, [&] { return s->stop || !s->waiting.empty(); });
      if (s->stop && s->waiting.empty() && s->running.empty()) break;
    }
    admit(s);
    bool progressed = false;
    for (size_t i = 0; i < s->running.size();) {
      Group& g = s->running[i];
      if (!drive_ready(g.ctx)) {
        ++i;
        continue;
      }
      progressed = true;
      const stp_status st = drive_next(g.ctx);
      if (st < 0) {
        const std::string err = stp_last_error();
        for (auto& r : g.reqs) finish_request(s, r, st, err);
        g.ctx->drv.phase = stp_ctx::kIdle;
        release_ctx(s, g.ctx, g.bytes, false);
        s->running.erase(s->running.begin() + (long)i);
        continue;
      }
      if (g.ctx->drv.phase == stp_ctx::kDone) {
        complete(s, g);
        s->running.erase(s->running.begin() + (long)i);
        continue;
      }
      ++i;
    }
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stat_in_use = s->bytes_in_use;
      s->stat_peak = s->peak_bytes;
      s->stat_running = (int)s->running.size();
    }
    if (!progressed && !s->running.empty()) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
  for (Cached& c : s->cache) stp_destroy(c.ctx);
  s->cache.clear();
}

stp_status check_request(const stp_request* q) {
  if (!q) {
    set_error("NULL request");
    return STP_E_INVALID_ARG;
  }
  if (q->J < 0 || q->J > kMaxJ || q->K < 1 || q->K > kMaxK ||
      (q->precision != STP_FP64 && q->precision != STP_MIXED) || !(q->rel_tol >= 0.0) ||
      q->rel_tol >= 1.0) {
    set_error("request needs 0 <= J <= 14, 1 <= K <= 10, a valid precision and 0 <= rel_tol < 1");
    return STP_E_INVALID_ARG;
  }
  return STP_OK;
}

}  // namespace

extern "C" {

stp_status stp_server_create(size_t hbm_budget_bytes, int max_slots, int max_batch,
                             const stp_options* opt, stp_server** out) {
  if (!out || hbm_budget_bytes == 0 || max_slots < 1 || max_slots > 64 || max_batch < 1 ||
      max_batch > 64) {
    set_error("stp_server_create: need an output pointer, a nonzero budget, 1 <= max_slots <= 64 "
              "and 1 <= max_batch <= 64");
    return STP_E_INVALID_ARG;
  }
  if (opt && (opt->nested > 0 || opt->dim == 3)) {
    set_error("stp_server_create: nested iteration and the 3D problem are not offered by the "
              "server");
    return STP_E_UNSUPPORTED;
  }
  *out = nullptr;
  std::unique_ptr<stp_server> s(new (std::nothrow) stp_server());
  if (!s) {
    set_error("host allocation failed");
    return STP_E_OUT_OF_MEMORY;
  }
  s->budget = hbm_budget_bytes;
  s->max_slots = max_slots;
  s->max_batch = max_batch;
  if (opt) s->opt = *opt;
  if (hipGetDevice(&s->device) != hipSuccess) {
    set_error("no HIP device");
    return STP_E_DEVICE;
  }
  const int nstreams = std::min(max_slots, 4);
  for (int i = 0; i < nstreams; ++i) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t t : s->streams) (void)hipStreamDestroy(t);
      set_error("hipStreamCreate failed");
      return STP_E_DEVICE;
    }
    s->streams.push_back(st);
  }
  stp_server* raw = s.release();
  raw->worker = std::thread(worker_main, raw);
  *out = raw;
  return STP_OK;
}

stp_status stp_server_submit(stp_server* s, const stp_request* req, uint64_t* id) {
  if (!s || !id) {
    set_error("NULL server or id");
    return STP_E_INVALID_ARG;
  }
  STP_TRY(check_request(req));
  size_t need = 0;
  STP_TRY(stp_footprint(req->J, req->K, 1, req->precision, &need));
  if (need > s->budget) {
    set_error("request footprint " + std::to_string(need) + " bytes exceeds the server budget");
    return STP_E_OUT_OF_MEMORY;
  }
  auto r = std::make_shared<Request>();
  r->req = *req;
  r->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    r->id = s->next_id++;
    s->table[r->id] = r;
    s->waiting.push_back(r);
    s->unfinished += 1;
  }
  s->cv_work.notify_one();
  *id = r->id;
  return STP_OK;
}

stp_status stp_server_poll(stp_server* s, uint64_t id, stp_stats* stats, double* latency_seconds) {
  if (!s) {
    set_error("NULL server");
    return STP_E_INVALID_ARG;
  }
  std::shared_ptr<Request> r;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->table.find(id);
    if (it == s->table.end()) {
      set_error("unknown request id (never submitted, or already collected)");
      return STP_E_INVALID_ARG;
    }
    r = it->second;
    if (r->state != 2) return STP_E_BUSY;
    s->table.erase(it);
  }
  if (stats) *stats = r->stats;
  if (latency_seconds) *latency_seconds = seconds_since(r->t_submit, r->t_done);
  if (r->status < 0) set_error(r->error);
  return r->status;
}

stp_status stp_server_drain(stp_server* s) {
  if (!s) {
    set_error("NULL server");
    return STP_E_INVALID_ARG;
  }
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->unfinished == 0; });
  return STP_OK;
}

stp_status stp_server_info(stp_server* s, stp_server_stats* out) {
  if (!s || !out) {
    set_error("NULL server or output");
    return STP_E_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  out->waiting = (int)s->waiting.size();
  out->running_groups = s->stat_running;
  out->unfinished = s->unfinished;
  out->bytes_in_use = s->stat_in_use;
  out->peak_bytes = s->stat_peak;
  out->groups_started = s->stat_groups;
  out->requests_started = s->stat_batched;
  return STP_OK;
}

stp_status stp_server_destroy(stp_server* s) {
  if (!s) return STP_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (hipStream_t t : s->streams) (void)hipStreamDestroy(t);
  delete s;
  return STP_OK;
}

}  // extern "C"
