// Serving: a request loop per context.  Each request builds an H^2 matrix
// (h2_build) and computes C = A A (h2_mmp, Sections III-IV); one worker thread
// runs them in submission order.  A request is admitted once its device
// memory estimate fits the context's budget next to the results still held
// (results stay resident until h2_release), so concurrent submitters never
// drive the device out of memory; the context lock serialises the worker
// with every other entry point of the context.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <condition_variable>
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

// device bytes one request may need: about 80 KB per point at rank 27
// (operand, product and the product's per-level intermediates), scaled by the
// rank p^3
size_t estimate_bytes(const h2_request& r) {
  const double p3 = (double)r.opts.cheb_order * r.opts.cheb_order * r.opts.cheb_order;
  return (size_t)((double)r.n * 80e3 * (p3 / 27.0)) + ((size_t)64 << 20);
}

struct Job {
  h2_request req{};
  std::vector<double> xyz;
  size_t est = 0;
  bool done = false;
  h2_result res{};
  Clock::time_point t_submit;
};

}  // namespace

struct Server {
  h2_ctx ctx = nullptr;
  std::mutex m;  // guards the fields below (never held across device work)
  std::condition_variable cv_work, cv_done, cv_mem;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, Job> jobs;
  size_t held = 0;  // estimates of the finished, unreleased requests
  uint64_t next = 1;
  bool stop = false;
  std::thread worker;

  void run() {
    for (;;) {
      uint64_t t;
      Job* j;
      {
        std::unique_lock<std::mutex> lk(m);
        cv_work.wait(lk, [&] { return stop || !queue.empty(); });
        if (stop) return;
        t = queue.front();
        j = &jobs.at(t);
        // admission: wait until the estimate fits next to the held results
        if (ctx->budget) {
          cv_mem.wait(lk, [&] { return stop || held == 0 || held + j->est <= ctx->budget; });
          if (stop) return;
        }
        queue.pop_front();
      }
      const auto t0 = Clock::now();
      h2_result r{};
      r.queue_ms = ms_between(j->t_submit, t0);
      h2_mat A = nullptr, C = nullptr;
      r.status = build_impl(ctx, j->xyz.data(), j->req.n, &j->req.kernel, &j->req.opts, nullptr, &A);
      const auto t1 = Clock::now();
      r.build_ms = ms_between(t0, t1);
      if (r.status == H2_OK) {
        r.status = h2_mmp(ctx, A, A, j->req.eps, j->req.trunc_mode, j->req.precision, &C);
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
      {
        std::lock_guard<std::mutex> lk(m);
        j->res = r;
        j->done = true;
        if (r.status == H2_OK) held += j->est;
      }
      cv_done.notify_all();
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
  s->cv_mem.notify_all();
  s->cv_done.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (auto& kv : s->jobs) {
    if (kv.second.done) {
      h2_free(kv.second.res.C);
      h2_free(kv.second.res.A);
    }
  }
  delete s;
  ctx->server = nullptr;
}

}  // namespace h2

extern "C" {

h2_status h2_submit(h2_ctx ctx, const h2_request* req, uint64_t* ticket) {
  using namespace h2;
  if (!ctx || !req || !ticket || !req->xyz) return set_error(H2_ERR_ARG, "null argument");
  if (req->n < 1 || req->opts.leaf_size < 1 || !(req->opts.eta > 0.0) ||
      req->opts.cheb_order < 1 || req->opts.cheb_order > 6)
    return set_error(H2_ERR_ARG, "invalid request sizes or options");
  if (!(req->eps >= 0.0) || req->trunc_mode < 0 || req->trunc_mode > 2 || req->precision < 0 ||
      req->precision > 1)
    return set_error(H2_ERR_ARG, "invalid eps, mode or precision");
  if (req->kernel.kind != H2_KERNEL_LAPLACE)
    return set_error(H2_ERR_UNSUPPORTED, "unsupported kernel");
  Job j;
  j.req = *req;
  j.xyz.assign(req->xyz, req->xyz + 3 * req->n);
  j.req.xyz = nullptr;
  j.est = estimate_bytes(*req);
  if (ctx->budget && j.est > ctx->budget)
    return set_error(H2_ERR_OOM, "request estimate of " + std::to_string(j.est) +
                                     " bytes exceeds the context budget");
  j.t_submit = std::chrono::steady_clock::now();
  {
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (!ctx->server) {
      ctx->server = new Server();
      ctx->server->ctx = ctx;
      Server* s = ctx->server;
      s->worker = std::thread([s] {
        hipSetDevice(s->ctx->device);
        s->run();
      });
    }
  }
  Server* s = ctx->server;
  {
    std::lock_guard<std::mutex> lk(s->m);
    const uint64_t t = s->next++;
    s->jobs.emplace(t, std::move(j));
    s->queue.push_back(t);
    *ticket = t;
  }
  s->cv_work.notify_one();
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
  // look the job up afresh on every wake-up: other submissions may rehash
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
    if (it->second.res.status == H2_OK) s->held -= it->second.est;
    s->jobs.erase(it);
  }
  h2_free(C);
  h2_free(A);
  s->cv_mem.notify_all();
  return H2_OK;
}

}  // extern "C"
