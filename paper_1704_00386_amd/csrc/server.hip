// server.hip -- a request loop with continuous batching.
//
// Callers submit graphs; a worker thread admits them while a slot is free and
// their preparation (incidence lists, tau buffers) fits the context's
// device-memory budget, adds them to the running batch of their kind, mode
// and tau width (batch.hip), and keeps sweeping every batch one chunk of
// epochs at a time.  A request that converges (or hits its sweep cap, or is
// cancelled) is retired at the next poll: its result is copied to the
// caller's buffer, its device memory released and its slot given to the next
// waiting request.  Waiting requests therefore join while others are on the
// GPU, and their sweeps share launches.  Results equal those of a lone
// nd_decompose (SND iterates do not depend on what else is in a launch; AND
// converges to the same unique fixed point).
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>

#include "api_util.h"
#include "batch.h"

namespace nd {

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t ticket = 0;
  nd_graph *g = nullptr;
  nd_kind kind = ND_KCORE;
  nd_opts opts{};
  int32_t *kappa = nullptr;  // caller's host buffer
  Clock::time_point t_submit, t_done;
  bool admitted = false, done = false, cancelled = false;
  nd_status status = ND_OK;
  nd_result res{};
  Member *member = nullptr;
  Batch *batch = nullptr;
  std::string error;
};

}  // namespace nd

struct nd_server {
  nd_ctx *ctx = nullptr;
  int32_t max_slots = 1, max_queue = 1;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<nd::Request *> queue;
  std::map<uint64_t, std::unique_ptr<nd::Request>> reqs;
  std::thread worker;
  bool stop = false;
  int active = 0;
  uint64_t next_ticket = 1;
  hipStream_t stream = nullptr;
  // one batch per (kind, mode, tau width, frontier)
  std::unique_ptr<nd::Batch> batches[nd::kNumKinds][2][2][2];
};

namespace nd {

namespace {

void finish(nd_server *srv, Request *r, nd_status st) {
  std::lock_guard<std::mutex> lk(srv->mu);
  r->status = st;
  r->t_done = Clock::now();
  r->done = true;
  if (r->admitted) srv->active--;
  srv->cv_done.notify_all();
  srv->cv_work.notify_all();
}

void release_graph(Request *r) {
  if (r->g) {
    nd_graph_destroy(r->g);
    r->g = nullptr;
  }
}

// Retire a finished member: copy its result out and free its memory.
void retire(nd_server *srv, Batch &b, std::unique_ptr<Member> m) {
  Request *r = (Request *)m->user;
  nd_status st = ND_OK;
  const KindState &ks = r->g->ks[r->kind];
  try {
    StreamScope scope(b.stream());
    if (ks.nr > 0 && !r->cancelled) {
      DArr<int32_t> tmp(srv->ctx->alloc, ks.nr);
      to_original(ks, b.result_tau(*m), b.tau16(), tmp.p, b.stream());
      ND_HIP(hipMemcpyAsync(r->kappa, tmp.p, sizeof(int32_t) * ks.nr,
                            hipMemcpyDeviceToHost, b.stream()));
      ND_HIP(hipStreamSynchronize(b.stream()));
    }
    nd_result &res = r->res;
    memset(&res, 0, sizeof res);
    res.sweeps = (int32_t)m->sweeps;
    res.converged = m->converged ? 1 : 0;
    res.n_rcliques = ks.nr;
    res.n_incidence = ks.P;
    res.updates = ks.bin_lo[kBinZero] * m->sweeps;
    res.ms_prep = ks.ms_prep;
    res.max_sdegree = ks.max_ds;
    res.tau_bytes = b.tau16() ? 2 : 4;
    st = r->cancelled ? ND_ERR_CANCELLED
                      : (m->converged ? ND_OK : ND_ERR_NOT_CONVERGED);
  } catch (const Err &e) {
    st = e.code;
    r->error = nd_last_error();
  }
  {
    StreamScope scope(b.stream());
    m.reset();  // tau buffers and counters back to the allocator
  }
  release_graph(r);
  finish(srv, r, st);
}

// Prepare and add one waiting request; false when it must wait for memory.
bool admit(nd_server *srv, Request *r) {
  try {
    StreamScope scope(srv->stream);
    prepare(r->g, r->kind, srv->stream);
    const KindState &ks = r->g->ks[r->kind];
    const int mi = r->opts.mode == ND_AND ? 1 : 0;
    const int wi = ks.tau16 ? 1 : 0;
    const int fi = r->opts.use_frontier ? 1 : 0;
    auto &slot = srv->batches[r->kind][mi][wi][fi];
    if (!slot)
      slot = std::make_unique<Batch>(srv->ctx, r->kind, r->opts.mode, ks.tau16,
                                     fi != 0, srv->stream);
    r->member = slot->add(r->g, r->opts.max_iters, r);
    r->batch = slot.get();
    return true;
  } catch (const Err &e) {
    if (e.code == ND_ERR_OOM) {
      // others hold memory (this request already counts as active): wait
      std::lock_guard<std::mutex> lk(srv->mu);
      if (srv->active > 1) return false;
    }
    r->error = nd_last_error();
    release_graph(r);
    finish(srv, r, e.code);
    return true;
  }
}

void worker_main(nd_server *srv) {
  (void)hipSetDevice(srv->ctx->device);
  int chunk = 1;
  for (;;) {
    // ------------------------------------------------ admission
    for (;;) {
      Request *r = nullptr;
      {
        std::unique_lock<std::mutex> lk(srv->mu);
        srv->cv_work.wait(lk, [&] {
          return srv->stop || srv->active > 0 || !srv->queue.empty();
        });
        if (srv->stop) return;
        if (srv->queue.empty() || srv->active >= srv->max_slots) break;
        r = srv->queue.front();
        srv->queue.pop_front();
        if (r->cancelled) {
          lk.unlock();
          release_graph(r);
          finish(srv, r, ND_ERR_CANCELLED);
          continue;
        }
        r->admitted = true;
        srv->active++;
      }
      if (!admit(srv, r)) {
        std::lock_guard<std::mutex> lk(srv->mu);
        r->admitted = false;
        srv->active--;
        srv->queue.push_front(r);
        break;
      }
      chunk = 1;  // newcomers: poll soon
    }
    // ------------------------------------------------ sweep
    bool any = false;
    for (auto &bk : srv->batches)
      for (auto &bm : bk)
        for (auto &bw : bm)
          for (auto &b : bw) {
          if (!b || b->size() == 0) continue;
          any = true;
          try {
            // cancelled running requests stop at this poll
            {
              std::lock_guard<std::mutex> lk(srv->mu);
              for (auto &kv : srv->reqs) {
                Request *r = kv.second.get();
                if (r->admitted && !r->done && r->cancelled && r->batch == b.get() &&
                    r->member)
                  r->member->finished = true;
              }
            }
            StreamScope scope(b->stream());
            b->run_epochs(chunk);
            b->poll(chunk);
            for (auto &m : b->take_finished()) retire(srv, *b, std::move(m));
          } catch (const Err &e) {
            // a device failure ends every request of this batch
            for (auto &m : b->take_finished()) retire(srv, *b, std::move(m));
            std::lock_guard<std::mutex> lk(srv->mu);
            for (auto &kv : srv->reqs) {
              Request *r = kv.second.get();
              if (r->batch == b.get() && !r->done) r->member->finished = true;
            }
            (void)e;
          }
        }
    if (any) chunk = std::min(chunk * 2, Batch::kGraphEpochs);
  }
}

}  // namespace

}  // namespace nd

using namespace nd;

extern "C" {

nd_status nd_server_create(nd_ctx *ctx, int32_t max_slots, int32_t max_queue,
                           nd_server **out) {
  return guarded([&] {
    ND_REQUIRE(ctx && out, ND_ERR_INVALID, "NULL argument");
    ND_REQUIRE(max_slots >= 1 && max_queue >= 1, ND_ERR_INVALID,
               "max_slots and max_queue must be positive");
    ND_HIP(hipSetDevice(ctx->device));
    auto srv = std::make_unique<nd_server>();
    srv->ctx = ctx;
    ctx->retain();
    srv->max_slots = max_slots;
    srv->max_queue = max_queue;
    ND_HIP(hipStreamCreateWithFlags(&srv->stream, hipStreamNonBlocking));
    nd_server *raw = srv.release();
    raw->worker = std::thread(worker_main, raw);
    *out = raw;
  });
}

nd_status nd_server_submit(nd_server *srv, nd_graph *g, nd_kind kind,
                           const nd_opts *opts, int32_t *kappa,
                           uint64_t *ticket) {
  return guarded([&] {
    ND_REQUIRE(srv && g && ticket, ND_ERR_INVALID, "NULL argument");
    ND_REQUIRE(g->ctx == srv->ctx, ND_ERR_INVALID,
               "graph belongs to another context");
    ND_REQUIRE(kind_valid(kind),
               ND_ERR_UNSUPPORTED, "unknown kind");
    nd_opts o;
    nd_opts_init(&o);
    if (opts) o = *opts;
    ND_REQUIRE(o.mode == ND_SND || o.mode == ND_AND, ND_ERR_INVALID,
               "unknown mode");
    ND_REQUIRE(!o.on_iter && o.stop_active_ratio == 0, ND_ERR_UNSUPPORTED,
               "served requests support mode, max_iters and use_frontier");
    auto r = std::make_unique<Request>();
    r->g = g;
    r->kind = kind;
    r->opts = o;
    r->kappa = kappa;
    r->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(srv->mu);
    ND_REQUIRE((int32_t)srv->queue.size() < srv->max_queue, ND_ERR_BUSY,
               "server queue is full (%d waiting)", (int)srv->queue.size());
    r->ticket = srv->next_ticket++;
    *ticket = r->ticket;
    srv->queue.push_back(r.get());
    srv->reqs[r->ticket] = std::move(r);
    srv->cv_work.notify_all();
  });
}

nd_status nd_server_wait(nd_server *srv, uint64_t ticket, int64_t timeout_us,
                         nd_result *res, double *latency_ms) {
  if (!srv) {
    set_error("server is NULL");
    return ND_ERR_INVALID;
  }
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) {
    set_error("unknown ticket %llu", (unsigned long long)ticket);
    return ND_ERR_INVALID;
  }
  Request *r = it->second.get();
  auto ready = [&] { return r->done; };
  if (timeout_us < 0) {
    srv->cv_done.wait(lk, ready);
  } else if (!srv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us),
                                    ready)) {
    set_error("request %llu still running", (unsigned long long)ticket);
    return ND_ERR_TIMEOUT;
  }
  if (res) *res = r->res;
  if (latency_ms)
    *latency_ms =
        std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
  const nd_status st = r->status;
  if (st != ND_OK) set_error("%s", r->error.empty() ? nd_status_str(st) : r->error.c_str());
  srv->reqs.erase(it);
  return st;
}

nd_status nd_server_cancel(nd_server *srv, uint64_t ticket) {
  if (!srv) {
    set_error("server is NULL");
    return ND_ERR_INVALID;
  }
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) {
    set_error("unknown ticket %llu", (unsigned long long)ticket);
    return ND_ERR_INVALID;
  }
  it->second->cancelled = true;
  srv->cv_work.notify_all();
  return ND_OK;
}

void nd_server_destroy(nd_server *srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
    srv->cv_work.notify_all();
  }
  if (srv->worker.joinable()) srv->worker.join();
  (void)hipSetDevice(srv->ctx->device);
  for (auto &bk : srv->batches)
    for (auto &bm : bk)
      for (auto &bw : bm)
        for (auto &b : bw) b.reset();
  for (auto &kv : srv->reqs) release_graph(kv.second.get());
  srv->reqs.clear();
  srv->ctx->alloc.forget_stream(srv->stream);
  (void)hipStreamDestroy(srv->stream);
  nd_ctx *ctx = srv->ctx;
  delete srv;
  ctx->release();
}

}  // extern "C"
