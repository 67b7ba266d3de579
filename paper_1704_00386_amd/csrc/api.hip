// api.hip -- the C ABI declared in include/nd.h: contexts, the caching
// allocator, graph construction and preparation, nd_update and the status
// plumbing.  Decomposition drivers are in driver.hip, batching in batch.hip,
// serving in server.hip.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "api_util.h"
#include "internal.h"

namespace nd {

// ------------------------------------------------------------ errors

static thread_local char g_last_error[512];

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
  va_end(ap);
}

// ------------------------------------------------- static workspace

// The workspace of nd_decompose_noalloc.  In host code `scratch` names a
// host-side stand-in, not device memory: its device address on each device
// is looked up once (hipGetSymbolAddress, with that device current) and only
// that address is ever handed to kernels or copies.  Every device keeps its
// own copy of the array, held until the process ends.
static __device__ __align__(256) uint8_t scratch[kNoallocWorkspaceBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// With `device` current: look up its workspace address (once per device).
static void noalloc_setup(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  ND_REQUIRE(device >= 0 && device < kMaxDevices, ND_ERR_UNSUPPORTED,
             "device %d: at most %d devices are supported", device, kMaxDevices);
  if (g_scratch_ptr[device]) return;
  void *p = nullptr;
  ND_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  ND_REQUIRE(p != nullptr, ND_ERR_DEVICE,
             "no device address for the static workspace on device %d", device);
  g_scratch_ptr[device] = p;
}

void *noalloc_workspace(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

// ------------------------------------------------------------ streams

static thread_local hipStream_t g_stream = nullptr;

hipStream_t current_stream() { return g_stream; }
StreamScope::StreamScope(hipStream_t s) : prev(g_stream) { g_stream = s; }
StreamScope::~StreamScope() { g_stream = prev; }

// ---------------------------------------------------------- allocator

Allocator::~Allocator() {
  std::lock_guard<std::mutex> lk(mu_);
  trim_locked();
}

void Allocator::trim_locked() {
  for (auto &kv : cache_) {
    try {
      if (!kv.second.idle) (void)hipStreamSynchronize(kv.second.s);
      (void)hipFree(kv.second.p);
    } catch (...) {
      // runtime already torn down (process exit): leave the block
    }
  }
  cache_.clear();
  cache_total_ = 0;
}

void Allocator::forget_stream(hipStream_t s) {
  std::lock_guard<std::mutex> lk(mu_);
  (void)hipStreamSynchronize(s);
  for (auto &kv : cache_)
    if (kv.second.s == s) {
      kv.second.idle = true;
      kv.second.s = nullptr;
    }
}

void Allocator::trim() {
  std::lock_guard<std::mutex> lk(mu_);
  trim_locked();
}

static size_t round_bytes(size_t b) {
  const size_t q = 256;
  b = b < q ? q : b;
  return (b + q - 1) / q * q;
}

void *Allocator::alloc(size_t bytes) {
  bytes = round_bytes(bytes);
  const hipStream_t s = current_stream();
  std::lock_guard<std::mutex> lk(mu_);
  // Best fit among cached blocks no more than twice the request.  A block is
  // taken at once when no pending work can touch it: idle, last used on this
  // stream (stream order protects it), or on a stream that has drained.
  // Waiting for another stream is the last resort, after a fresh block
  // within the budget: a server's sweep loop must not wait for a
  // preparation running on another thread's stream.
  auto take = [&](std::multimap<size_t, Cached>::iterator it) {
    void *p = it->second.p;
    const size_t sz = it->first;
    cache_.erase(it);
    cache_total_ -= sz;
    live_[p] = sz;
    live_total_ += sz;
    return p;
  };
  for (int pass = 0; pass < 2; pass++) {
    auto it = cache_.lower_bound(bytes);
    for (; it != cache_.end() && it->first <= 2 * bytes; ++it) {
      const bool free_now =
          it->second.idle || it->second.s == s ||
          (pass == 1 && hipStreamQuery(it->second.s) == hipSuccess);
      if (free_now) return take(it);
    }
  }
  (void)hipGetLastError();  // a query of a busy stream is not an error
  if (!budget_ || live_total_ + cache_total_ + bytes <= budget_) {
    void *p = nullptr;
    if (hipMalloc(&p, bytes) == hipSuccess) {
      live_[p] = bytes;
      live_total_ += bytes;
      return p;
    }
    (void)hipGetLastError();
  }
  {
    auto it = cache_.lower_bound(bytes);
    if (it != cache_.end() && it->first <= 2 * bytes) {
      ND_HIP(hipStreamSynchronize(it->second.s));
      return take(it);
    }
  }
  if (budget_ && live_total_ + cache_total_ + bytes > budget_) trim_locked();
  ND_REQUIRE(!budget_ || live_total_ + bytes <= budget_, ND_ERR_OOM,
             "device-memory budget exceeded: %zu live + %zu requested > %zu",
             live_total_, bytes, budget_);
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    trim_locked();
    e = hipMalloc(&p, bytes);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error("hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    throw Err(ND_ERR_OOM);
  }
  live_[p] = bytes;
  live_total_ += bytes;
  return p;
}

void Allocator::release(void *p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(mu_);
  auto it = live_.find(p);
  if (it == live_.end()) return;
  const size_t sz = it->second;
  live_.erase(it);
  live_total_ -= sz;
  cache_.emplace(sz, Cached{p, current_stream(), false});
  cache_total_ += sz;
}

size_t Allocator::live_bytes() const {
  std::lock_guard<std::mutex> lk(mu_);
  return live_total_;
}

size_t Allocator::cached_bytes() const {
  std::lock_guard<std::mutex> lk(mu_);
  return cache_total_;
}

size_t KindState::bytes() const {
  size_t b = 0;
  if (perm.p) b += perm.bytes();
  if (inv.p) b += inv.bytes();
  if (ds.p) b += ds.bytes();
  if (inc_off.p) b += inc_off.bytes();
  if (inc_ids.p) b += inc_ids.bytes();
  return b;
}

// ------------------------------------------------------- preparation

namespace {

__global__ void k_iota(int32_t *p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (int32_t)i;
}

__global__ void k_tri_verts(const int32_t *__restrict__ ev,
                            const int32_t *__restrict__ tri_e,
                            const int32_t *__restrict__ tri_w, int64_t nt,
                            int32_t *__restrict__ out) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  const int32_t e = tri_e[t];
  out[3 * t] = ev[2 * (int64_t)e];
  out[3 * t + 1] = ev[2 * (int64_t)e + 1];
  out[3 * t + 2] = tri_w[t];
}

// Every listed id must name another r-clique: a cheap guard that turns a
// builder fault into an error instead of an out-of-range gather.
// Reads 16 bytes a lane (ids is 256-byte aligned), the tail one id a lane.
__global__ void k_check_incidence(const int32_t *__restrict__ ids,
                                  int64_t nids, int64_t nr,
                                  int32_t *__restrict__ err) {
  bool bad = false;
  const uint32_t lim = (uint32_t)nr;  // ids below 0 wrap above it
  const int64_t n4 = nids / 4;
  const int4 *v = reinterpret_cast<const int4 *>(ids);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t j = t0; j < n4; j += stride) {
    const int4 x = v[j];
    bad |= (uint32_t)x.x >= lim || (uint32_t)x.y >= lim ||
           (uint32_t)x.z >= lim || (uint32_t)x.w >= lim;
  }
  for (int64_t j = 4 * n4 + t0; j < nids; j += stride)
    bad |= (uint32_t)ids[j] >= lim;
  if (ballot(bad) && lane_id() == 0) atomicOr(err, 1);
}

// tau given in r-clique-id order must satisfy 0 <= tau <= d_s.
__global__ void k_check_tau(const int32_t *__restrict__ tau,
                            const int32_t *__restrict__ perm,
                            const int32_t *__restrict__ ds, int64_t n,
                            int32_t *__restrict__ err) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const int32_t t = tau[perm[i]];
    if (t < 0 || t > ds[i]) atomicOr(err, 1);
  }
}

}  // namespace

static void prepare_kind(nd_graph *g, nd_kind kind, hipStream_t s) {
  KindState &ks = g->ks[kind];
  if (ks.ready) return;
  static const char *const kPhase[kNumKinds] = {
      "nd.prepare.core", "nd.prepare.truss", "nd.prepare.nucleus34",
      "nd.prepare.nucleus13", "nd.prepare.nucleus24"};
  Phase phase(kPhase[kind]);
  hipEvent_t e0, e1;
  ND_HIP(hipEventCreate(&e0));
  ND_HIP(hipEventCreate(&e1));
  ND_HIP(hipEventRecord(e0, s));
  const KindRS rs = kind_rs(kind);
  ks.r = rs.r; ks.s = rs.s; ks.k = rs.k;
  switch (kind) {
    case ND_KCORE:
      // (1,2): the s-cliques containing vertex u are its edges and the other
      // r-clique of each is the neighbour: the incidence is the CSR.
      build_incidence_core(g, ks, s);
      break;
    case ND_KTRUSS:
      build_incidence_truss(g, ks, s);
      break;
    case ND_NUCLEUS34:
      build_incidence_n34(g, ks, s);
      break;
    case ND_NUCLEUS13:
      build_incidence_n13(g, ks, s);
      break;
    case ND_NUCLEUS24:
      build_incidence_n24(g, ks, s);
      break;
    default:
      ND_REQUIRE(false, ND_ERR_UNSUPPORTED, "unknown kind %d", (int)kind);
  }
  ND_REQUIRE((int64_t)ks.max_ds < ((int64_t)1 << 28), ND_ERR_UNSUPPORTED,
             "an S-degree of %d exceeds the 2^28 supported per r-clique",
             ks.max_ds);
  {
    DArr<int32_t> err(g->ctx->alloc, 1);
    fill_i32(err.p, 0, 1, s);
    const int64_t nids = ks.P * ks.k;
    if (nids > 0) {
      const unsigned grid = (unsigned)std::min<int64_t>(grid_for((nids + 3) / 4, 256), 65536);
      k_check_incidence<<<grid, 256, 0, s>>>(ks.inc_ids.p, nids, ks.nr, err.p);
      ND_LAUNCHED();
    }
    const int32_t h = *PinnedChunk().read(err.p, 1, s);
    ND_REQUIRE(h == 0, ND_ERR_DEVICE,
               "internal error: incidence list holds an invalid r-clique id");
  }
  ND_HIP(hipEventRecord(e1, s));
  ND_HIP(hipEventSynchronize(e1));
  float ms = 0;
  ND_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ks.ms_prep = ms;
  ks.ready = true;
}

void prepare(nd_graph *g, nd_kind kind, hipStream_t s) {
  ND_REQUIRE(kind_valid(kind), ND_ERR_UNSUPPORTED, "unknown kind %d",
             (int)kind);
  prepare_kind(g, kind, s);
}

void check_tau_range(nd_graph *g, const KindState &ks, const int32_t *tau,
                     hipStream_t s) {
  DArr<int32_t> err(g->ctx->alloc, 1);
  fill_i32(err.p, 0, 1, s);
  if (ks.nr > 0) {
    k_check_tau<<<grid_for(ks.nr, 256), 256, 0, s>>>(tau, ks.perm.p, ks.ds.p,
                                                      ks.nr, err.p);
    ND_LAUNCHED();
  }
  const int32_t h = *PinnedChunk().read(err.p, 1, s);
  ND_REQUIRE(h == 0, ND_ERR_INVALID, "tau must satisfy 0 <= tau <= d_s");
}

}  // namespace nd

size_t nd_graph::bytes() const {
  size_t b = 0;
  auto add = [&](size_t x, const void *p) { if (p) b += x; };
  add(row_off.bytes(), row_off.p);
  add(col.bytes(), col.p);
  add(rowid.bytes(), rowid.p);
  add(nlow.bytes(), nlow.p);
  add(eoff.bytes(), eoff.p);
  add(eid.bytes(), eid.p);
  add(ev.bytes(), ev.p);
  add(toff.bytes(), toff.p);
  add(tri_w.bytes(), tri_w.p);
  add(tri_e.bytes(), tri_e.p);
  for (const auto &k : ks) b += k.bytes();
  return b;
}

using namespace nd;

// ------------------------------------------------------------------ ABI

extern "C" {

const char *nd_status_str(nd_status s) {
  switch (s) {
    case ND_OK: return "ok";
    case ND_ERR_INVALID: return "invalid argument";
    case ND_ERR_OOM: return "out of device memory";
    case ND_ERR_DEVICE: return "device error";
    case ND_ERR_UNSUPPORTED: return "unsupported";
    case ND_ERR_NOT_CONVERGED: return "not converged";
    case ND_ERR_BUSY: return "busy";
    case ND_ERR_CANCELLED: return "cancelled";
    case ND_ERR_TIMEOUT: return "timeout";
  }
  return "unknown status";
}

const char *nd_last_error(void) { return g_last_error; }

void nd_opts_init(nd_opts *o) {
  if (!o) return;
  memset(o, 0, sizeof *o);
  o->mode = ND_SND;
  o->max_iters = -1;
}

nd_status nd_ctx_create(int device, size_t hbm_budget_bytes, nd_ctx **out) {
  return guarded([&] {
    ND_REQUIRE(out, ND_ERR_INVALID, "out is NULL");
    int count = 0;
    ND_HIP(hipGetDeviceCount(&count));
    ND_REQUIRE(device >= 0 && device < count, ND_ERR_INVALID,
               "device %d not present (%d devices)", device, count);
    ND_HIP(hipSetDevice(device));
    std::unique_ptr<nd_ctx> c(new nd_ctx(device, hbm_budget_bytes));
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount,
                              device) == hipSuccess && cu > 0)
      c->num_cu = cu;
    // what a decomposition needs besides its device buffers, made once
    ND_HIP(hipHostMalloc(&c->host_stats, sizeof(SweepStats) * kHostStatsRing,
                         hipHostMallocDefault));
    for (hipEvent_t &e : c->ev) ND_HIP(hipEventCreate(&e));
    noalloc_setup(device);
    *out = c.release();
  });
}

void nd_ctx_destroy(nd_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  ctx->release();
}

size_t nd_ctx_bytes_in_use(const nd_ctx *ctx) {
  return ctx ? ctx->alloc.live_bytes() + ctx->alloc.cached_bytes() : 0;
}

nd_status nd_graph_from_edges(nd_ctx *ctx, int32_t n, int64_t m,
                              const int32_t *src, const int32_t *dst,
                              int on_device, void *stream, nd_graph **out) {
  nd_graph *g = nullptr;
  nd_status st = guarded([&] {
    ND_REQUIRE(ctx && out, ND_ERR_INVALID, "ctx/out is NULL");
    ND_REQUIRE(n >= 0 && m >= 0, ND_ERR_INVALID, "negative size");
    ND_REQUIRE(m == 0 || (src && dst), ND_ERR_INVALID, "src/dst is NULL");
    Phase phase("nd.graph_from_edges");
    ND_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    StreamScope scope(s);
    g = new nd_graph();
    g->ctx = ctx;
    ctx->retain();
    g->n = n;
    DArr<int32_t> hs, hd;
    const int32_t *ds = src, *dd = dst;
    if (!on_device && m > 0) {
      hs.reset(ctx->alloc, m);
      hd.reset(ctx->alloc, m);
      ND_HIP(hipMemcpyAsync(hs.p, src, sizeof(int32_t) * m, hipMemcpyHostToDevice, s));
      ND_HIP(hipMemcpyAsync(hd.p, dst, sizeof(int32_t) * m, hipMemcpyHostToDevice, s));
      ds = hs.p;
      dd = hd.p;
    }
    build_from_edges(g, m, ds, dd, s);
    ND_HIP(hipStreamSynchronize(s));
    *out = g;
  });
  if (st != ND_OK && g) {
    (void)hipStreamSynchronize((hipStream_t)stream);
    nd_graph_destroy(g);
  }
  return st;
}

nd_status nd_graphs_from_edges(nd_ctx *ctx, int32_t count, const int32_t *n,
                               const int64_t *m, const int32_t *const *src,
                               const int32_t *const *dst, int on_device,
                               void *stream, nd_graph **out) {
  std::vector<nd_graph *> built;
  hipStream_t s = (hipStream_t)stream;
  nd_status st = guarded([&] {
    ND_REQUIRE(ctx && (count == 0 || (n && m && src && dst && out)),
               ND_ERR_INVALID, "NULL argument");
    ND_REQUIRE(count >= 0, ND_ERR_INVALID, "negative count");
    for (int i = 0; i < count; i++) {
      ND_REQUIRE(n[i] >= 0 && m[i] >= 0, ND_ERR_INVALID, "graph %d: negative size", i);
      ND_REQUIRE(m[i] == 0 || (src[i] && dst[i]), ND_ERR_INVALID,
                 "graph %d: src/dst is NULL", i);
      out[i] = nullptr;
    }
    if (count == 0) return;
    ND_HIP(hipSetDevice(ctx->device));
    built.assign(count, nullptr);
    // graph i built on stream bs (its own copies, validation and CSR)
    auto build = [&](int i, hipStream_t bs) {
      Phase phase("nd.graph_from_edges");
      StreamScope scope(bs);
      nd_graph *g = new nd_graph();
      g->ctx = ctx;
      ctx->retain();
      g->n = n[i];
      built[i] = g;
      DArr<int32_t> hs, hd;
      const int32_t *ds = src[i], *dd = dst[i];
      if (!on_device && m[i] > 0) {
        hs.reset(ctx->alloc, m[i]);
        hd.reset(ctx->alloc, m[i]);
        ND_HIP(hipMemcpyAsync(hs.p, src[i], sizeof(int32_t) * m[i],
                              hipMemcpyHostToDevice, bs));
        ND_HIP(hipMemcpyAsync(hd.p, dst[i], sizeof(int32_t) * m[i],
                              hipMemcpyHostToDevice, bs));
        ds = hs.p;
        dd = hd.p;
      }
      build_from_edges(g, m[i], ds, dd, bs);
      ND_HIP(hipStreamSynchronize(bs));
    };
    const int nt = std::min(prep_threads(), count);
    if (nt <= 1) {
      StreamScope scope(s);
      for (int i = 0; i < count; i++) build(i, s);
    } else {
      hipEvent_t start;
      ND_HIP(hipEventCreateWithFlags(&start, hipEventDisableTiming));
      ND_HIP(hipEventRecord(start, s));
      std::vector<hipStream_t> streams;
      for (int t = 0; t < nt; t++) {
        hipStream_t bs = nullptr;
        const hipError_t e = hipStreamCreateWithFlags(&bs, hipStreamNonBlocking);
        if (e != hipSuccess) break;
        streams.push_back(bs);
        (void)hipStreamWaitEvent(bs, start, 0);
      }
      (void)hipEventDestroy(start);
      std::atomic<int> next{0};
      std::mutex mu;
      nd_status code = ND_OK;
      std::string msg;
      std::vector<std::thread> threads;
      for (size_t t = 0; t < streams.size(); t++)
        threads.emplace_back([&, t] {
          try {
            ND_HIP(hipSetDevice(ctx->device));
            for (int i; (i = next++) < count;) {
              {
                std::lock_guard<std::mutex> lk(mu);
                if (code != ND_OK) return;
              }
              build(i, streams[t]);
            }
          } catch (const Err &e) {
            std::lock_guard<std::mutex> lk(mu);
            if (code == ND_OK) {
              code = e.code;
              msg = nd_last_error();
            }
          } catch (const std::exception &e) {
            std::lock_guard<std::mutex> lk(mu);
            if (code == ND_OK) {
              code = ND_ERR_DEVICE;
              msg = e.what();
            }
          }
        });
      for (auto &th : threads) th.join();
      for (hipStream_t bs : streams) {
        ctx->alloc.forget_stream(bs);  // waits for it
        (void)hipStreamDestroy(bs);
      }
      ND_REQUIRE(!streams.empty(), ND_ERR_DEVICE, "no stream for the builders");
      if (code != ND_OK) {
        set_error("%s", msg.c_str());
        throw Err(code);
      }
    }
    for (int i = 0; i < count; i++) out[i] = built[i];
  });
  if (st != ND_OK) {
    (void)hipStreamSynchronize(s);
    for (nd_graph *g : built)
      if (g) nd_graph_destroy(g);
  }
  return st;
}

nd_status nd_graph_from_csr(nd_ctx *ctx, int32_t n, int64_t nnz,
                            const int64_t *row_off, const int32_t *col,
                            int on_device, void *stream, nd_graph **out) {
  nd_graph *g = nullptr;
  nd_status st = guarded([&] {
    ND_REQUIRE(ctx && out && row_off, ND_ERR_INVALID, "NULL argument");
    ND_REQUIRE(n >= 0 && nnz >= 0, ND_ERR_INVALID, "negative size");
    ND_REQUIRE(nnz == 0 || col, ND_ERR_INVALID, "col is NULL");
    Phase phase("nd.graph_from_csr");
    ND_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    StreamScope scope(s);
    g = new nd_graph();
    g->ctx = ctx;
    ctx->retain();
    g->n = n;
    g->nnz = nnz;
    g->row_off.reset(ctx->alloc, (int64_t)n + 1);
    g->col.reset(ctx->alloc, nnz);
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    ND_HIP(hipMemcpyAsync(g->row_off.p, row_off, sizeof(int64_t) * ((size_t)n + 1), kind, s));
    if (nnz > 0)
      ND_HIP(hipMemcpyAsync(g->col.p, col, sizeof(int32_t) * nnz, kind, s));
    validate_csr(g, s);
    ND_HIP(hipStreamSynchronize(s));
    *out = g;
  });
  if (st != ND_OK && g) {
    (void)hipStreamSynchronize((hipStream_t)stream);
    nd_graph_destroy(g);
  }
  return st;
}

}  // extern "C"

namespace nd {

// Free a graph whose last device work was ordered on stream s (the server's
// retirement): waits for s only (or not at all), never for the whole device,
// and returns the graph's memory to the allocator tagged with s.
void destroy_graph(nd_graph *g, hipStream_t s, bool wait) {
  if (!g) return;
  nd_ctx *ctx = g->ctx;
  (void)hipSetDevice(ctx->device);
  if (wait) (void)hipStreamSynchronize(s);
  {
    StreamScope scope(s);
    delete g;
  }
  ctx->release();
}

}  // namespace nd

extern "C" {

void nd_graph_destroy(nd_graph *g) {
  if (!g) return;
  nd_ctx *ctx = g->ctx;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  {
    StreamScope scope(nullptr);
    delete g;
  }
  ctx->release();
}

nd_status nd_graph_dims(const nd_graph *g, int32_t *n, int64_t *nnz) {
  return guarded([&] {
    ND_REQUIRE(g, ND_ERR_INVALID, "graph is NULL");
    if (n) *n = g->n;
    if (nnz) *nnz = g->nnz;
  });
}

nd_status nd_graph_csr(nd_graph *g, int64_t *row_off, int32_t *col,
                       int on_device, void *stream) {
  return guarded([&] {
    ND_REQUIRE(g && row_off && (col || g->nnz == 0), ND_ERR_INVALID,
               "NULL argument");
    ND_HIP(hipSetDevice(g->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    ND_HIP(hipMemcpyAsync(row_off, g->row_off.p, sizeof(int64_t) * ((size_t)g->n + 1), kind, s));
    if (g->nnz > 0)
      ND_HIP(hipMemcpyAsync(col, g->col.p, sizeof(int32_t) * g->nnz, kind, s));
    ND_HIP(hipStreamSynchronize(s));
  });
}

nd_status nd_prepare(nd_graph *g, nd_kind kind, void *stream) {
  return guarded([&] {
    ND_REQUIRE(g, ND_ERR_INVALID, "graph is NULL");
    ND_HIP(hipSetDevice(g->ctx->device));
    StreamScope scope((hipStream_t)stream);
    prepare(g, kind, (hipStream_t)stream);
  });
}

nd_status nd_sizes(nd_graph *g, nd_kind kind, int64_t *n_rcliques,
                   int64_t *n_incidence, size_t *dev_bytes) {
  return guarded([&] {
    ND_REQUIRE(g, ND_ERR_INVALID, "graph is NULL");
    ND_REQUIRE(kind_valid(kind), ND_ERR_UNSUPPORTED, "unknown kind %d",
               (int)kind);
    const int r = kind_rs(kind).r;
    if (!n_incidence && !dev_bytes && !g->ks[kind].ready && r <= 2) {
      // |R| without building anything: vertices, or edges (the CSR is
      // symmetric and simple, so every edge is stored twice)
      if (n_rcliques) *n_rcliques = r == 1 ? (int64_t)g->n : g->nnz / 2;
      return;
    }
    ND_HIP(hipSetDevice(g->ctx->device));
    StreamScope scope(nullptr);
    prepare(g, kind, nullptr);
    if (n_rcliques) *n_rcliques = g->ks[kind].nr;
    if (n_incidence) *n_incidence = g->ks[kind].P;
    if (dev_bytes) *dev_bytes = g->bytes();
  });
}

nd_status nd_rcliques(nd_graph *g, nd_kind kind, int32_t *verts, int on_device,
                      void *stream) {
  return guarded([&] {
    ND_REQUIRE(g, ND_ERR_INVALID, "graph is NULL");
    ND_HIP(hipSetDevice(g->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    StreamScope scope(s);
    prepare(g, kind, s);
    const KindState &ks = g->ks[kind];
    const int r = ks.r;
    const int64_t cnt = ks.nr * r;
    ND_REQUIRE(verts || cnt == 0, ND_ERR_INVALID, "verts is NULL");
    if (cnt == 0) return;
    DArr<int32_t> tmp(g->ctx->alloc, cnt);
    const int32_t *src = tmp.p;
    if (r == 1) {
      k_iota<<<grid_for(cnt, 256), 256, 0, s>>>(tmp.p, cnt);
      ND_LAUNCHED();
    } else if (r == 2) {
      src = g->ev.p;
    } else {
      k_tri_verts<<<grid_for(ks.nr, 256), 256, 0, s>>>(
          g->ev.p, g->tri_e.p, g->tri_w.p, ks.nr, tmp.p);
      ND_LAUNCHED();
    }
    ND_HIP(hipMemcpyAsync(verts, src, sizeof(int32_t) * cnt,
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    ND_HIP(hipStreamSynchronize(s));
  });
}

nd_status nd_incidence(nd_graph *g, nd_kind kind, int64_t *off, int32_t *ids,
                       int on_device, void *stream) {
  return guarded([&] {
    ND_REQUIRE(g && off, ND_ERR_INVALID, "NULL argument");
    ND_HIP(hipSetDevice(g->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    StreamScope scope(s);
    prepare(g, kind, s);
    const KindState &ks = g->ks[kind];
    const int64_t nid = ks.P * ks.k;
    ND_REQUIRE(ids || nid == 0, ND_ERR_INVALID, "ids is NULL");
    Allocator &al = g->ctx->alloc;
    DArr<int64_t> doff;
    DArr<int32_t> dids;
    int64_t *po = off;
    int32_t *pi = ids;
    if (!on_device) {
      doff.reset(al, ks.nr + 1);
      dids.reset(al, nid);
      po = doff.p;
      pi = dids.p;
    }
    incidence_original(g, ks, po, pi, s);
    if (!on_device) {
      ND_HIP(hipMemcpyAsync(off, po, sizeof(int64_t) * (ks.nr + 1), hipMemcpyDeviceToHost, s));
      if (nid > 0) ND_HIP(hipMemcpyAsync(ids, pi, sizeof(int32_t) * nid, hipMemcpyDeviceToHost, s));
    }
    ND_HIP(hipStreamSynchronize(s));
  });
}

nd_status nd_sdegree(nd_graph *g, nd_kind kind, int32_t *ds, int on_device,
                     void *stream) {
  return guarded([&] {
    ND_REQUIRE(g, ND_ERR_INVALID, "graph is NULL");
    ND_HIP(hipSetDevice(g->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    StreamScope scope(s);
    prepare(g, kind, s);
    const KindState &ks = g->ks[kind];
    ND_REQUIRE(ds || ks.nr == 0, ND_ERR_INVALID, "ds is NULL");
    if (ks.nr == 0) return;
    DArr<int32_t> tmp;
    int32_t *out = ds;
    if (!on_device) {
      tmp.reset(g->ctx->alloc, ks.nr);
      out = tmp.p;
    }
    sdegree_original(ks, out, s);
    if (!on_device)
      ND_HIP(hipMemcpyAsync(ds, out, sizeof(int32_t) * ks.nr, hipMemcpyDeviceToHost, s));
    ND_HIP(hipStreamSynchronize(s));
  });
}

nd_status nd_update(nd_graph *g, nd_kind kind, const int32_t *tau_in,
                    int32_t *tau_out, int on_device, void *stream) {
  return guarded([&] {
    ND_REQUIRE(g, ND_ERR_INVALID, "graph is NULL");
    ND_HIP(hipSetDevice(g->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    StreamScope scope(s);
    prepare(g, kind, s);
    const KindState &ks = g->ks[kind];
    if (ks.nr == 0) return;
    ND_REQUIRE(tau_in && tau_out, ND_ERR_INVALID, "tau is NULL");
    Allocator &al = g->ctx->alloc;
    DArr<int32_t> din, dout;
    const int32_t *pin = tau_in;
    int32_t *pout = tau_out;
    if (!on_device) {
      din.reset(al, ks.nr);
      dout.reset(al, ks.nr);
      ND_HIP(hipMemcpyAsync(din.p, tau_in, sizeof(int32_t) * ks.nr, hipMemcpyHostToDevice, s));
      pin = din.p;
      pout = dout.p;
    }
    check_tau_range(g, ks, pin, s);
    const size_t tb = (size_t)ks.tau_bytes;
    DArr<uint8_t> ta(al, (int64_t)(tb * ks.nr)), tbuf(al, (int64_t)(tb * ks.nr));
    to_internal(ks, pin, ta.p, ks.tau_bytes, s);
    DArr<SweepStats> st(al, 1);
    ND_HIP(hipMemsetAsync(st.p, 0, sizeof(SweepStats), s));
    SweepArgs a{};
    a.inc_off = ks.inc_off.p;
    a.inc_ids = ks.inc_ids.p;
    a.tau_in = ta.p;
    a.tau_out = tbuf.p;
    a.stats = st.p;
    a.prev = nullptr;
    a.cap_by_tau = 0;
    launch_sweep(ks, a, false, s);
    to_original(ks, tbuf.p, ks.tau_bytes, pout, s);
    if (!on_device)
      ND_HIP(hipMemcpyAsync(tau_out, pout, sizeof(int32_t) * ks.nr, hipMemcpyDeviceToHost, s));
    ND_HIP(hipStreamSynchronize(s));
  });
}

}  // extern "C"
