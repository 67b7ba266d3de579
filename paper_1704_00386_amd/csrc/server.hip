// server.hip -- a request loop with continuous batching.
//
// Callers submit graphs.  Host threads serve them, each with its own
// stream:
//   * kPrepThreads preparation threads take waiting requests while a slot is
//     free and build what their kind needs (r-cliques, incidence lists, d_s)
//     on their streams, so that the short, launch-bound build phases of
//     several newcomers overlap.  Admission is by device memory: the
//     builders' allocations are charged to the context's budget, the
//     incidence lists at their exact size from the count pass.  A request
//     that does not fit releases what it built and is retried on its own
//     (no other build running); if it still does not fit it waits for a
//     running request to retire, and fails when nothing else holds memory.
//     Preparing here keeps the sweep loop running while newcomers are built;
//   * two worker threads add prepared requests to the running batch of their
//     size class, kind, mode, tau width and frontier setting (batch.hip) and
//     keep sweeping every batch of their class a chunk of epochs at a time.
//     Small requests (fewer than kSmallWork incidence entries) have a worker
//     and batches of their own: in a batch every member advances one sweep
//     per epoch, and an epoch lasts as long as its largest member's sweep,
//     so a small request batched with large ones would wait for them at
//     every sweep.  A request that
//     converges (or hits its sweep cap, or is cancelled) is retired at the
//     next poll: its result is copied into host memory the server owns, its
//     device memory released and its slot given to the next waiting request.
// Waiting requests therefore join while others are on the GPU and their
// sweeps share launches.  Results equal those of a lone nd_decompose (SND
// iterates do not depend on what else is in a launch; AND converges to the
// same unique fixed point).
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
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
  Clock::time_point t_submit, t_done;
  bool admitted = false;  // holds a slot (preparing, ready or running)
  bool retry_alone = false;  // did not fit beside other builds
  int cls = 0;               // size class, set once prepared
  bool done = false, cancelled = false;
  nd_status status = ND_OK;
  nd_result res{};
  nd_serve_info info{};
  Member *member = nullptr;
  Batch *batch = nullptr;
  // the result: kappa in pinned host memory owned by the server (a pooled
  // buffer of host_cap bytes), complete once `copied` has fired
  void *host = nullptr;
  size_t host_cap = 0;
  int64_t n_result = 0;
  hipEvent_t copied = nullptr;
  std::string error;
};

}  // namespace nd

struct nd_server {
  nd_ctx *ctx = nullptr;
  int32_t max_slots = 1, max_queue = 1;
  std::mutex mu;
  std::condition_variable cv_work, cv_prep, cv_done;
  std::deque<nd::Request *> queue;  // submitted, not yet being prepared
  std::deque<nd::Request *> ready;  // prepared, not yet in a batch
  std::map<uint64_t, std::unique_ptr<nd::Request>> reqs;
  std::thread workers[2];  // size classes: small, large
  std::vector<std::thread> preps;
  bool stop = false;
  int admitted = 0;         // requests holding a slot
  int preparing = 0;        // builds in progress
  bool alone = false;       // a retried build runs with no other build
  size_t build_bytes = 0;   // largest graph a build has produced so far
  int running = 0;          // requests in a batch
  int running_cls[2] = {0, 0};  // of them, per size class
  uint64_t retired = 0;     // retirements so far (memory may have freed)
  uint64_t next_ticket = 1;
  std::atomic<int64_t> epochs{0};  // epochs run over all batches
  hipStream_t streams[2] = {nullptr, nullptr};  // the workers
  std::vector<hipStream_t> prep_streams;  // one per preparation thread
  // pinned result buffers not in use, by capacity (guarded by mu)
  std::multimap<size_t, void *> pinned_free;
  // one batch per (size class, kind, mode, tau width, frontier)
  std::unique_ptr<nd::Batch> batches[2][nd::kNumKinds][2][2][2];
};

namespace nd {

namespace {

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

// Mark r finished with status st (lock held by the caller).
void finish_locked(nd_server *srv, Request *r, nd_status st) {
  r->status = st;
  r->t_done = Clock::now();
  r->done = true;
  r->info.latency_ms = ms_between(r->t_submit, r->t_done);
  if (r->admitted) {
    srv->admitted--;
    r->admitted = false;
  }
  srv->cv_done.notify_all();
  srv->cv_prep.notify_all();
  srv->cv_work.notify_all();
}

// Free r's graph; its last device work was ordered on s (the server's
// threads never wait for the whole device, which would stall the sweeps
// behind a preparation or the other way round).
void release_graph(Request *r, hipStream_t s, bool wait = true) {
  if (r->g) {
    destroy_graph(r->g, s, wait);
    r->g = nullptr;
  }
}

// A pinned buffer of at least `bytes` from the pool (or a new one, in power
// of two sizes from 64 KiB), and its return.
void *take_pinned(nd_server *srv, size_t bytes, size_t *cap) {
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->pinned_free.lower_bound(bytes);
    if (it != srv->pinned_free.end()) {
      void *p = it->second;
      *cap = it->first;
      srv->pinned_free.erase(it);
      return p;
    }
  }
  size_t c = (size_t)64 << 10;
  while (c < bytes) c <<= 1;
  void *p = nullptr;
  ND_HIP(hipHostMalloc(&p, c, hipHostMallocDefault));
  *cap = c;
  return p;
}

// Give r's result buffer and event back (lock held).
void drop_result_locked(nd_server *srv, Request *r) {
  if (r->copied) {
    (void)hipEventSynchronize(r->copied);
    (void)hipEventDestroy(r->copied);
    r->copied = nullptr;
  }
  if (r->host) {
    srv->pinned_free.emplace(r->host_cap, r->host);
    r->host = nullptr;
  }
}

// Retire a finished member (worker thread): queue the copy of its result
// into a pinned buffer (the caller's nd_server_result waits for it) and free
// its device memory, all without waiting for the device.
void retire(nd_server *srv, Batch &b, std::unique_ptr<Member> m) {
  Request *r = (Request *)m->user;
  nd_status st = ND_OK;
  const KindState &ks = r->g->ks[r->kind];
  try {
    StreamScope scope(b.stream());
    if (ks.nr > 0 && !r->cancelled) {
      const size_t bytes = sizeof(int32_t) * (size_t)ks.nr;
      r->host = take_pinned(srv, bytes, &r->host_cap);
      r->n_result = ks.nr;
      DArr<int32_t> tmp(srv->ctx->alloc, ks.nr);
      to_original(ks, b.result_tau(*m), b.tau16() ? 2 : 4, tmp.p, b.stream());
      ND_HIP(hipMemcpyAsync(r->host, tmp.p, bytes, hipMemcpyDeviceToHost,
                            b.stream()));
      ND_HIP(hipEventCreateWithFlags(&r->copied, hipEventDisableTiming));
      ND_HIP(hipEventRecord(r->copied, b.stream()));
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
    r->info.epoch_done = b.epoch();
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
  release_graph(r, b.stream(), /*wait=*/false);
  std::lock_guard<std::mutex> lk(srv->mu);
  srv->running--;
  srv->running_cls[r->cls]--;
  srv->retired++;
  finish_locked(srv, r, st);
}

constexpr int kPrepThreads = 4;
constexpr int64_t kSmallWork = (int64_t)1 << 20;  // incidence entries

int server_prep_threads() {
  const char *v = getenv("ND_PREP_THREADS");
  const int x = v ? atoi(v) : kPrepThreads;
  return x < 1 ? 1 : x > 16 ? 16 : x;
}

// May a build start now (lock held)?  One build always may (the budget
// admits or rejects it as it allocates).  Another starts beside running
// builds only while the free budget holds twice the largest graph built so
// far for each of them and the newcomer, so that concurrent builds do not
// take the memory the callers' own graphs need.  A request marked
// retry_alone starts only when no other build runs, and none starts beside it.
bool may_start_build(nd_server *srv) {
  if (srv->queue.empty() || srv->admitted >= srv->max_slots || srv->alone)
    return false;
  if (srv->preparing == 0) return true;
  if (srv->queue.front()->retry_alone || srv->build_bytes == 0) return false;
  const Allocator &al = srv->ctx->alloc;
  const size_t live = al.live_bytes();
  const size_t free_b = al.budget() > live ? al.budget() - live : 0;
  return free_b / 2 / (size_t)(srv->preparing + 1) >= srv->build_bytes;
}

// A preparation thread: build waiting requests while slots are free.
void prep_main(nd_server *srv, int t) {
  (void)hipSetDevice(srv->ctx->device);
  hipStream_t ps = srv->prep_streams[t];
  for (;;) {
    Request *r = nullptr;
    uint64_t retired0 = 0;
    int64_t epochs0 = 0;
    bool alone = false;
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      srv->cv_prep.wait(lk, [&] { return srv->stop || may_start_build(srv); });
      if (srv->stop) return;
      r = srv->queue.front();
      srv->queue.pop_front();
      if (r->cancelled) {
        lk.unlock();
        release_graph(r, ps);
        lk.lock();
        finish_locked(srv, r, ND_ERR_CANCELLED);
        continue;
      }
      r->admitted = true;
      srv->admitted++;
      srv->preparing++;
      alone = r->retry_alone;
      srv->alone = alone;
      retired0 = srv->retired;
      epochs0 = srv->epochs.load();
    }
    const Clock::time_point t0 = Clock::now();
    nd_status code = ND_OK;
    try {
      Phase phase("nd.server.prepare");
      StreamScope scope(ps);
      prepare(r->g, r->kind, ps);
    } catch (const Err &e) {
      code = e.code;
      r->error = nd_last_error();
      // give back what the failed build holds
      StreamScope scope(ps);
      (void)hipStreamSynchronize(ps);
      r->g->ks[r->kind] = KindState{};
    }
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->preparing--;
    if (alone) srv->alone = false;
    srv->cv_prep.notify_all();
    r->info.prep_ms += ms_between(t0, Clock::now());
    r->info.epochs_during_prep += srv->epochs.load() - epochs0;
    if (code == ND_OK) {
      srv->build_bytes = std::max(srv->build_bytes, r->g->bytes());
      r->cls = r->g->ks[r->kind].P < kSmallWork ? 0 : 1;
      srv->ready.push_back(r);
      srv->cv_work.notify_all();
      continue;
    }
    if (code == ND_ERR_OOM) {
      bool retry = false;
      if (!alone) {
        retry = true;  // other builds held memory too: retry on its own
      } else if (srv->running > 0 || !srv->ready.empty()) {
        // others hold memory: wait for one of them to retire (or for all
        // of them to be gone), then retry
        srv->cv_prep.wait(lk, [&] {
          return srv->stop || srv->retired != retired0 ||
                 (srv->running == 0 && srv->ready.empty());
        });
        retry = !srv->stop;
      }
      if (retry) {
        r->admitted = false;
        srv->admitted--;
        r->retry_alone = true;
        r->error.clear();
        srv->queue.push_front(r);
        srv->cv_prep.notify_all();
        continue;
      }
    }
    lk.unlock();
    release_graph(r, ps);
    lk.lock();
    finish_locked(srv, r, code);
  }
}

// Add a prepared request to its batch (worker thread of its class).
// Returns false when it has to wait for memory.
bool add_ready(nd_server *srv, Request *r) {
  hipStream_t ws = srv->streams[r->cls];
  try {
    StreamScope scope(ws);
    const KindState &ks = r->g->ks[r->kind];
    const int mi = r->opts.mode == ND_AND ? 1 : 0;
    const int wi = ks.tau16 ? 1 : 0;
    const int fi = r->opts.use_frontier ? 1 : 0;
    auto &slot = srv->batches[r->cls][r->kind][mi][wi][fi];
    if (!slot)
      slot = std::make_unique<Batch>(srv->ctx, r->kind, r->opts.mode, ks.tau16,
                                     fi != 0, ws);
    int running_before = 0;
    for (Member *m : slot->live()) running_before += m->sweeps > 0 ? 1 : 0;
    r->info.epoch_joined = slot->epoch();
    r->info.joined_running = running_before > 0 ? 1 : 0;
    r->member = slot->add(r->g, r->opts.max_iters, r);
    r->batch = slot.get();
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->running++;
    srv->running_cls[r->cls]++;
    return true;
  } catch (const Err &e) {
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      if (e.code == ND_ERR_OOM && srv->running > 0) return false;
    }
    r->error = nd_last_error();
    release_graph(r, ws);
    std::lock_guard<std::mutex> lk(srv->mu);
    finish_locked(srv, r, e.code);
    return true;
  }
}

// The worker of size class c.
void worker_main(nd_server *srv, int c) {
  (void)hipSetDevice(srv->ctx->device);
  int chunk = 1;
  for (;;) {
    std::deque<Request *> newcomers;
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      auto mine = [&] {
        for (Request *r : srv->ready)
          if (r->cls == c) return true;
        return false;
      };
      srv->cv_work.wait(lk, [&] {
        return srv->stop || srv->running_cls[c] > 0 || mine();
      });
      if (srv->stop) return;
      for (auto it = srv->ready.begin(); it != srv->ready.end();) {
        if ((*it)->cls == c) {
          newcomers.push_back(*it);
          it = srv->ready.erase(it);
        } else {
          ++it;
        }
      }
    }
    while (!newcomers.empty()) {
      Request *r = newcomers.front();
      if (r->cancelled) {
        newcomers.pop_front();
        release_graph(r, srv->streams[c]);
        std::lock_guard<std::mutex> lk(srv->mu);
        finish_locked(srv, r, ND_ERR_CANCELLED);
        continue;
      }
      if (!add_ready(srv, r)) break;  // wait for a retirement
      newcomers.pop_front();
      chunk = 1;  // newcomers: poll soon
    }
    if (!newcomers.empty()) {
      std::lock_guard<std::mutex> lk(srv->mu);
      srv->ready.insert(srv->ready.begin(), newcomers.begin(), newcomers.end());
    }
    bool any = false;
    for (auto &bk : srv->batches[c])
      for (auto &bm : bk)
        for (auto &bw : bm)
          for (auto &b : bw) {
            if (!b || b->size() == 0) continue;
            any = true;
            try {
              // cancelled running requests stop at this poll
              {
                std::lock_guard<std::mutex> lk(srv->mu);
                for (Member *m : b->live())
                  if (((Request *)m->user)->cancelled) m->finished = true;
              }
              StreamScope scope(b->stream());
              Phase phase("nd.server.epochs");
              const std::vector<Member *> live = b->live();
              b->run_epochs(chunk);
              srv->epochs += chunk;
              b->poll(chunk);
              for (Member *m : live) {
                Request *r = (Request *)m->user;
                r->info.peak_members =
                    std::max<int32_t>(r->info.peak_members, (int32_t)live.size());
              }
              for (auto &m : b->take_finished()) retire(srv, *b, std::move(m));
            } catch (const Err &e) {
              // a device failure ends every request of this batch
              for (Member *m : b->live()) {
                m->finished = true;
                ((Request *)m->user)->error = nd_last_error();
              }
              for (auto &m : b->take_finished()) retire(srv, *b, std::move(m));
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
    srv->max_slots = max_slots;
    srv->max_queue = max_queue;
    auto drop_streams = [&] {
      for (hipStream_t q : srv->prep_streams) (void)hipStreamDestroy(q);
      for (hipStream_t q : srv->streams)
        if (q) (void)hipStreamDestroy(q);
    };
    for (hipStream_t &ws : srv->streams) {
      const hipError_t e = hipStreamCreateWithFlags(&ws, hipStreamNonBlocking);
      if (e != hipSuccess) {
        ws = nullptr;
        drop_streams();
        ND_HIP(e);
      }
    }
    const int npt = server_prep_threads();
    for (int t = 0; t < npt; t++) {
      hipStream_t ps = nullptr;
      const hipError_t e = hipStreamCreateWithFlags(&ps, hipStreamNonBlocking);
      if (e != hipSuccess) {
        drop_streams();
        ND_HIP(e);
      }
      srv->prep_streams.push_back(ps);
    }
    ctx->retain();
    nd_server *raw = srv.release();
    for (int c = 0; c < 2; c++) raw->workers[c] = std::thread(worker_main, raw, c);
    for (int t = 0; t < npt; t++)
      raw->preps.emplace_back(prep_main, raw, t);
    *out = raw;
  });
}

nd_status nd_server_submit(nd_server *srv, nd_graph *g, nd_kind kind,
                           const nd_opts *opts, uint64_t *ticket) {
  return guarded([&] {
    ND_REQUIRE(srv && g && ticket, ND_ERR_INVALID, "NULL argument");
    ND_REQUIRE(g->ctx == srv->ctx, ND_ERR_INVALID,
               "graph belongs to another context");
    ND_REQUIRE(kind_valid(kind), ND_ERR_UNSUPPORTED, "unknown kind");
    nd_opts o;
    nd_opts_init(&o);
    if (opts) o = *opts;
    ND_REQUIRE(o.mode == ND_SND || o.mode == ND_AND, ND_ERR_INVALID,
               "unknown mode");
    ND_REQUIRE(!o.on_iter && o.stop_active_ratio == 0 && !o.count_active,
               ND_ERR_UNSUPPORTED,
               "served requests support mode, max_iters and use_frontier");
    auto r = std::make_unique<Request>();
    r->g = g;
    r->kind = kind;
    r->opts = o;
    r->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(srv->mu);
    ND_REQUIRE((int32_t)srv->queue.size() < srv->max_queue, ND_ERR_BUSY,
               "server queue is full (%d waiting)", (int)srv->queue.size());
    r->ticket = srv->next_ticket++;
    *ticket = r->ticket;
    srv->queue.push_back(r.get());
    srv->reqs[r->ticket] = std::move(r);
    srv->cv_prep.notify_all();
  });
}

nd_status nd_server_wait(nd_server *srv, uint64_t ticket, int64_t timeout_us,
                         nd_result *res, nd_serve_info *info) {
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
  if (info) *info = r->info;
  const nd_status st = r->status;
  if (st != ND_OK)
    set_error("%s", r->error.empty() ? nd_status_str(st) : r->error.c_str());
  // a result stays until nd_server_result collects it
  if (st != ND_OK && st != ND_ERR_NOT_CONVERGED) {
    drop_result_locked(srv, r);
    srv->reqs.erase(it);
  }
  return st;
}

nd_status nd_server_result(nd_server *srv, uint64_t ticket, int32_t *kappa,
                           int64_t capacity) {
  return guarded([&] {
    ND_REQUIRE(srv, ND_ERR_INVALID, "server is NULL");
    std::unique_ptr<Request> r;
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      auto it = srv->reqs.find(ticket);
      ND_REQUIRE(it != srv->reqs.end(), ND_ERR_INVALID, "unknown ticket %llu",
                 (unsigned long long)ticket);
      ND_REQUIRE(it->second->done, ND_ERR_INVALID,
                 "request %llu has not finished", (unsigned long long)ticket);
      ND_REQUIRE(!kappa || capacity >= it->second->n_result, ND_ERR_INVALID,
                 "kappa holds %lld entries, the result %lld",
                 (long long)capacity, (long long)it->second->n_result);
      r = std::move(it->second);
      srv->reqs.erase(it);
    }
    // the copy was queued at retirement; wait for it outside the lock
    if (r->copied) ND_HIP(hipEventSynchronize(r->copied));
    if (kappa && r->n_result)
      memcpy(kappa, r->host, sizeof(int32_t) * (size_t)r->n_result);
    std::lock_guard<std::mutex> lk(srv->mu);
    drop_result_locked(srv, r.get());
  });
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
  srv->cv_prep.notify_all();
  return ND_OK;
}

void nd_server_destroy(nd_server *srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
    srv->cv_work.notify_all();
    srv->cv_prep.notify_all();
  }
  for (auto &th : srv->preps)
    if (th.joinable()) th.join();
  for (auto &w : srv->workers)
    if (w.joinable()) w.join();
  (void)hipSetDevice(srv->ctx->device);
  for (auto &bc : srv->batches)
    for (auto &bk : bc)
      for (auto &bm : bk)
        for (auto &bw : bm)
          for (auto &b : bw) b.reset();
  (void)hipDeviceSynchronize();
  for (auto &kv : srv->reqs) {
    release_graph(kv.second.get(), srv->streams[0]);
    drop_result_locked(srv, kv.second.get());
  }
  srv->reqs.clear();
  for (auto &kv : srv->pinned_free) (void)hipHostFree(kv.second);
  srv->pinned_free.clear();
  for (hipStream_t ws : srv->streams) srv->ctx->alloc.forget_stream(ws);
  for (hipStream_t ps : srv->prep_streams) srv->ctx->alloc.forget_stream(ps);
  for (hipStream_t ws : srv->streams) (void)hipStreamDestroy(ws);
  for (hipStream_t ps : srv->prep_streams) (void)hipStreamDestroy(ps);
  nd_ctx *ctx = srv->ctx;
  delete srv;
  ctx->release();
}

}  // extern "C"
