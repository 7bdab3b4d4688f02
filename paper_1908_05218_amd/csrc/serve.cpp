// Serving: a request loop per context with continuous batching.  Each request
// builds an H^2 matrix (h2_build) and computes C = A A (h2_mmp, Sections
// III-IV).  The loop owns `serve_slots` slot contexts (same device, each with
// its own stream and pool) and one worker thread per slot, so up to that many
// requests are on the device at once: while one request waits on the host
// (rank read-backs between levels, allocation), the kernels of another fill
// the device.  Requests are taken in submission order; the request at the
// head of the queue is admitted once a slot is free and its device-memory
// estimate fits the context's budget next to the bytes of the results still
// held (results stay resident until h2_release) and the estimates of the
// requests in flight.  The estimate is kappa N^1.5 bytes: the product's
// intermediates grow with the ranks of the upper levels, so the peak grows
// faster than N; kappa starts from measured peaks of the cube and plate
// families and is raised by every completed request's measured peak.  A
// request that runs out of device memory while sharing the device is retried
// once, alone.  The kernels are deterministic, so a result does not depend on
// what ran beside it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <deque>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.h"

namespace h2 {

h2_status build_impl(h2_ctx ctx, const double* xyz, int64_t n, const h2_kernel* kernel,
                     const h2_build_opts* opts, h2_mat share, h2_mat* out);

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

// starting kappa (bytes per N^1.5) by precision: FP64, FP32-bulk; measured
// peaks of the build plus the product at Chebyshev order 3 reach about 8300
// (FP64) and 6400 (FP32-bulk) for the unit cube at eps 1e-6, less for plates
constexpr double kKappa0[2] = {9000.0, 7000.0};

struct Job {
  h2_request req{};
  std::vector<double> xyz;
  size_t est = 0;         // estimate charged while in flight
  size_t held_bytes = 0;  // device bytes of the result while held
  bool alone = false;     // retry after running out of memory: run alone
  bool done = false;
  h2_result res{};
  Clock::time_point t_submit;
};

}  // namespace

struct Server {
  h2_ctx ctx = nullptr;         // the context the requests were submitted to
  std::vector<h2_ctx> slots;    // one context per concurrent request
  std::mutex m;                 // guards the fields below (never held across device work)
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, Job> jobs;  // node-based: Job references stay valid
  size_t held = 0;      // bytes of the finished, unreleased results
  size_t inflight = 0;  // estimates of the running requests
  int running = 0;
  double kappa[2] = {kKappa0[0], kKappa0[1]};
  uint64_t next = 1;
  bool stop = false;
  std::vector<std::thread> workers;

  size_t estimate(const Job& j) const {
    const double p = j.req.opts.cheb_order / 3.0;
    const double nn = (double)j.req.n;
    return (size_t)(kappa[j.req.precision] * nn * std::sqrt(nn) * p * p * p) + ((size_t)64 << 20);
  }

  // under m: may the request at the head of the queue start now?
  bool admissible(const Job& j) const {
    if (j.alone) return running == 0;
    if (!ctx->budget || (held == 0 && running == 0)) return true;
    return held + inflight + estimate(j) <= ctx->budget;
  }

  void run(h2_ctx sc) {
    for (;;) {
      uint64_t t;
      Job* j;
      bool shared;
      {
        std::unique_lock<std::mutex> lk(m);
        cv_work.wait(lk, [&] {
          return stop || (!queue.empty() && admissible(jobs.at(queue.front())));
        });
        if (stop) return;
        t = queue.front();
        queue.pop_front();
        j = &jobs.at(t);
        j->est = estimate(*j);
        inflight += j->est;
        shared = running > 0;
        ++running;
      }
      const auto t0 = Clock::now();
      h2_result r{};
      r.queue_ms = ms_between(j->t_submit, t0);
      h2_mat A = nullptr, C = nullptr;
      size_t live0, peak;
      {
        std::lock_guard<std::recursive_mutex> lk(sc->mu);
        live0 = sc->live_bytes;
        sc->mark();
      }
      r.status = build_impl(sc, j->xyz.data(), j->req.n, &j->req.kernel, &j->req.opts, nullptr, &A);
      const auto t1 = Clock::now();
      r.build_ms = ms_between(t0, t1);
      size_t build_peak;
      {
        std::lock_guard<std::recursive_mutex> lk(sc->mu);
        build_peak = sc->peak_live;
      }
      if (r.status == H2_OK) {
        r.status = h2_mmp(sc, A, A, j->req.eps, j->req.trunc_mode, j->req.precision, nullptr, &C);
        if (r.status != H2_OK) {
          h2_free(A);
          A = nullptr;
        }
      }
      const auto t2 = Clock::now();
      if (r.status != H2_OK) std::snprintf(r.message, sizeof(r.message), "%s", h2_last_error());
      r.mmp_ms = ms_between(t1, t2);
      r.total_ms = ms_between(j->t_submit, t2);
      r.A = A;
      r.C = C;
      size_t live1;
      {
        std::lock_guard<std::recursive_mutex> lk(sc->mu);
        const size_t top = std::max(build_peak, sc->peak_live);
        peak = top > live0 ? top - live0 : 0;
        live1 = sc->live_bytes;
        // under a budget the slot keeps no cached blocks between requests:
        // admission counts only held results and requests in flight
        if (ctx->budget) sc->trim(0);
      }
      {
        std::lock_guard<std::mutex> lk(m);
        inflight -= j->est;
        --running;
        if (r.status == H2_ERR_OOM && !j->alone && (shared || running > 0)) {
          // the device was shared: run it again once nothing else runs
          j->alone = true;
          queue.push_front(t);
        } else {
          if (r.status == H2_OK) {
            j->held_bytes = live1 > live0 ? live1 - live0 : 0;
            held += j->held_bytes;
            r.bytes = (int64_t)j->held_bytes;
            const double nn = (double)j->req.n;
            const double p = j->req.opts.cheb_order / 3.0;
            const double k = (double)peak / (nn * std::sqrt(nn) * p * p * p);
            kappa[j->req.precision] = std::max(kappa[j->req.precision], k);
          }
          j->res = r;
          j->done = true;
        }
      }
      cv_done.notify_all();
      cv_work.notify_all();
    }
  }
};

void stop_server(h2_ctx ctx) {
  Server* s = ctx->server;
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->m);
    s->stop = true;
  }
  s->cv_work.notify_all();
  s->cv_done.notify_all();
  for (auto& w : s->workers)
    if (w.joinable()) w.join();
  for (auto& kv : s->jobs) {
    if (kv.second.done) {
      h2_free(kv.second.res.C);
      h2_free(kv.second.res.A);
    }
  }
  for (h2_ctx sc : s->slots) h2_ctx_destroy(sc);
  delete s;
  ctx->server = nullptr;
}

}  // namespace h2

extern "C" {

h2_status h2_serve_slots(h2_ctx ctx, int slots) {
  using namespace h2;
  if (!ctx || slots < 1 || slots > 8) return set_error(H2_ERR_ARG, "need 1 <= slots <= 8");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  if (ctx->server) return set_error(H2_ERR_BUSY, "the serving loop has already started");
  ctx->serve_slots = slots;
  return H2_OK;
}

h2_status h2_submit(h2_ctx ctx, const h2_request* req, uint64_t* ticket) {
  using namespace h2;
  if (!ctx || !req || !ticket || !req->xyz) return set_error(H2_ERR_ARG, "null argument");
  if (ctx->parent) return set_error(H2_ERR_ARG, "not a user context");
  if (req->n < 1 || req->opts.leaf_size < 1 || !(req->opts.eta > 0.0) ||
      req->opts.cheb_order < 1 || req->opts.cheb_order > 6)
    return set_error(H2_ERR_ARG, "invalid request sizes or options");
  if (!(req->eps >= 0.0) || req->trunc_mode < 0 || req->trunc_mode > 3 || req->precision < 0 ||
      req->precision > 1)
    return set_error(H2_ERR_ARG, "invalid eps, mode or precision");
  if (req->kernel.kind != H2_KERNEL_LAPLACE)
    return set_error(H2_ERR_UNSUPPORTED, "unsupported kernel");
  Job j;
  j.req = *req;
  j.xyz.assign(req->xyz, req->xyz + 3 * req->n);
  j.req.xyz = nullptr;
  j.t_submit = std::chrono::steady_clock::now();
  {
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (!ctx->server) {
      auto* s = new Server();
      s->ctx = ctx;
      for (int w = 0; w < ctx->serve_slots; ++w) {
        h2_ctx sc = nullptr;
        if (h2_ctx_create(ctx->device, ctx->budget, ctx->has_hook ? &ctx->hook : nullptr, &sc) != H2_OK) {
          for (h2_ctx c : s->slots) h2_ctx_destroy(c);
          delete s;
          return H2_ERR_DEVICE;  // message set by h2_ctx_create
        }
        sc->parent = ctx;
        sc->profiling = ctx->profiling;
        s->slots.push_back(sc);
      }
      for (h2_ctx sc : s->slots)
        s->workers.emplace_back([s, sc] {
          hipSetDevice(sc->device);
          s->run(sc);
        });
      ctx->server = s;
    }
  }
  Server* s = ctx->server;
  {
    std::lock_guard<std::mutex> lk(s->m);
    const size_t est = s->estimate(j);
    if (ctx->budget && est > ctx->budget)
      return set_error(H2_ERR_OOM, "request estimate of " + std::to_string(est) +
                                       " bytes exceeds the context budget");
    const uint64_t t = s->next++;
    s->jobs.emplace(t, std::move(j));
    s->queue.push_back(t);
    *ticket = t;
  }
  s->cv_work.notify_all();
  return H2_OK;
}

h2_status h2_poll(h2_ctx ctx, uint64_t ticket) {
  using namespace h2;
  if (!ctx || !ctx->server) return set_error(H2_ERR_ARG, "unknown ticket");
  Server* s = ctx->server;
  std::lock_guard<std::mutex> lk(s->m);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return set_error(H2_ERR_ARG, "unknown ticket");
  return it->second.done ? H2_OK : H2_ERR_BUSY;
}

h2_status h2_wait(h2_ctx ctx, uint64_t ticket, h2_result* out) {
  using namespace h2;
  if (!ctx || !out || !ctx->server) return set_error(H2_ERR_ARG, "unknown ticket or null out");
  Server* s = ctx->server;
  std::unique_lock<std::mutex> lk(s->m);
  if (s->jobs.find(ticket) == s->jobs.end()) return set_error(H2_ERR_ARG, "unknown ticket");
  s->cv_done.wait(lk, [&] {
    auto f = s->jobs.find(ticket);
    return f == s->jobs.end() || f->second.done || s->stop;
  });
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end() || !it->second.done) return set_error(H2_ERR_ARG, "request dropped");
  *out = it->second.res;
  return H2_OK;
}

h2_status h2_release(h2_ctx ctx, uint64_t ticket) {
  using namespace h2;
  if (!ctx || !ctx->server) return set_error(H2_ERR_ARG, "unknown ticket");
  Server* s = ctx->server;
  h2_mat A = nullptr, C = nullptr;
  {
    std::lock_guard<std::mutex> lk(s->m);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) return set_error(H2_ERR_ARG, "unknown ticket");
    if (!it->second.done) return set_error(H2_ERR_BUSY, "request not finished");
    A = it->second.res.A;
    C = it->second.res.C;
    s->held -= it->second.held_bytes;
    s->jobs.erase(it);
  }
  h2_ctx home = C ? C->ctx : A ? A->ctx : nullptr;
  h2_free(C);
  h2_free(A);
  if (home && ctx->budget) {
    std::lock_guard<std::recursive_mutex> lk(home->mu);
    home->trim(0);
  }
  s->cv_work.notify_all();
  return H2_OK;
}

}  // extern "C"
