// internal.h -- library-internal types: context, caching allocator, graph
// state and the host entry points of each kernel family.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <map>
#include <mutex>
#include <vector>

#include "common.h"

namespace nd {

// ------------------------------------------------------------ allocator

// The stream that work issued by the current thread is ordered on.  Set at
// every ABI entry (StreamScope); the allocator tags blocks with it.
hipStream_t current_stream();
struct StreamScope {
  hipStream_t prev;
  explicit StreamScope(hipStream_t s);
  ~StreamScope();
};

// Device allocator with a byte budget and a cache of freed blocks, so that
// repeated decompositions do not pay hipMalloc/hipFree (which synchronises the
// device) on every call.  A freed block remembers the stream it was last used
// on: the same stream may reuse it at once (stream order protects it), any
// other stream only after synchronising that stream.  Thread-safe.
class Allocator {
 public:
  Allocator(int device, size_t budget) : device_(device), budget_(budget) {}
  ~Allocator();
  void *alloc(size_t bytes);  // throws Err(ND_ERR_OOM)
  void release(void *p);      // back to the cache, tagged current_stream()
  void trim();                // return cached blocks to the device
  // Before destroying stream s: wait for it and mark its cached blocks free
  // for any stream (no handle of a destroyed stream is ever used again).
  void forget_stream(hipStream_t s);
  size_t live_bytes() const;
  size_t cached_bytes() const;
  size_t budget() const { return budget_; }
  int device() const { return device_; }

 private:
  struct Cached {
    void *p;
    hipStream_t s;
    bool idle;  // no pending work may touch it: reusable without a wait
  };
  void trim_locked();
  int device_;
  size_t budget_;
  mutable std::mutex mu_;
  std::map<void *, size_t> live_;
  std::multimap<size_t, Cached> cache_;
  size_t live_total_ = 0, cache_total_ = 0;
};

// Owning device array of T.
template <typename T>
struct DArr {
  T *p = nullptr;
  int64_t n = 0;
  Allocator *a = nullptr;
  DArr() = default;
  DArr(Allocator &al, int64_t count) { reset(al, count); }
  DArr(const DArr &) = delete;
  DArr &operator=(const DArr &) = delete;
  DArr(DArr &&o) noexcept : p(o.p), n(o.n), a(o.a) { o.p = nullptr; o.n = 0; }
  DArr &operator=(DArr &&o) noexcept {
    if (this != &o) {
      free();
      p = o.p; n = o.n; a = o.a;
      o.p = nullptr; o.n = 0;
    }
    return *this;
  }
  ~DArr() { free(); }
  void reset(Allocator &al, int64_t count) {
    free();
    a = &al;
    n = count;
    p = (T *)al.alloc(sizeof(T) * (size_t)(count > 0 ? count : 1));
  }
  void free() {
    if (p && a) a->release(p);
    p = nullptr;
    n = 0;
  }
  size_t bytes() const { return sizeof(T) * (size_t)(n > 0 ? n : 1); }
};

// -------------------------------------------------------------- context

}  // namespace nd

// A context lives until nd_ctx_destroy has been called and every graph made
// from it has been destroyed, whatever the order of those calls.
struct nd_ctx {
  int device = 0;
  nd::Allocator alloc;
  int num_cu = 256;
  // Made once at creation, so that the sweep loop creates nothing on the
  // host (nd_decompose_noalloc relies on it): the pinned read-back ring of
  // the sweep counters (kHostStatsRing entries) and the timing events of the
  // sweep loop (whole loop, one sweep).
  void *host_stats = nullptr;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  std::atomic<int> refs{1};    // the owner's reference + one per graph
  nd_ctx(int dev, size_t budget) : device(dev), alloc(dev, budget) {}
  ~nd_ctx() {
    if (host_stats) (void)hipHostFree(host_stats);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  void retain() { refs.fetch_add(1); }
  void release() {
    if (refs.fetch_sub(1) == 1) delete this;
  }
};

namespace nd {

// ---------------------------------------------------------- sweep bins

// r-cliques are numbered internally by sweep bin, ascending id within a bin,
// so every sweep bin is a contiguous range of internal ids, r-cliques that
// share vertices stay close together (their gathers hit nearby cache lines),
// and zero-degree r-cliques (never swept) sit at the end.  Bins in internal
// order, with their d_s ranges:
enum SweepBin : int {
  kBinBlock = 0,  // d_s >= 2048:  one workgroup per r-clique, LDS histogram
  kBinWave,       // 1025..2047:   one wave, 32 values per lane in registers
  kBinWave16,     // 513..1024:    one wave, 16 values per lane
  kBinWave8,      // 257..512:     one wave, 8 values per lane
  kBinG64,        // 65..256:      one wave, 4 values per lane
  kBinG16,        // 17..64:       16 lanes
  kBinG4,         // 5..16:        4 lanes
  kBinG1,         // 1..4:         one lane
  kBinZero,       // 0:            tau stays 0
  kNumBins
};
// kBinWave16 .. kBinG1: the bins swept by one launch (k_sweep_small)
constexpr int kFirstSmall = kBinWave16;
constexpr int kNumSmall = kBinZero - kFirstSmall;

// Per-kind state of a graph: internal numbering, incidence lists, schedule.
struct KindState {
  bool ready = false;
  int r = 0, s = 0, k = 0;  // k = C(s,r) - 1
  int64_t nr = 0;           // |R|
  int64_t P = 0;            // sum_R d_s(R)
  DArr<int32_t> perm;       // internal id -> r-clique id
  DArr<int32_t> inv;        // r-clique id -> internal id
  DArr<int32_t> ds;         // d_s, internal order
  // incidence, internal order and ids: r-clique i owns the s-cliques
  // inc_off[i] .. inc_off[i+1]; s-clique j lists inc_ids[k*j .. k*j+k)
  DArr<int64_t> inc_off;
  DArr<int32_t> inc_ids;
  int64_t bin_lo[kNumBins] = {0}, bin_hi[kNumBins] = {0};
  int32_t max_ds = 0;
  bool tau16 = false;       // tau fits uint16 (max d_s < 32768)
  // bytes per tau value in the one-graph sweeps: 1 (max d_s < 256), 2 or 4
  // (batches and the server hold 2 or 4, by tau16)
  int tau_bytes = 4;
  double ms_prep = 0;
  size_t bytes() const;
};

}  // namespace nd

struct nd_graph {
  nd_ctx *ctx = nullptr;
  int32_t n = 0;
  int64_t nnz = 0;
  nd::DArr<int64_t> row_off;  // n+1
  nd::DArr<int32_t> col;      // nnz, ascending per row
  nd::DArr<int32_t> rowid;    // nnz: row of each entry
  // edge numbering (r = 2): edges u<v lexicographic
  bool edges_ready = false;
  int64_t ne = 0;
  nd::DArr<int32_t> ev;       // 2*ne: endpoints (u, v) of each edge
  nd::DArr<int32_t> nlow;     // n: neighbours below u
  nd::DArr<int64_t> eoff;     // n+1: first edge id of u
  nd::DArr<int32_t> eid;      // nnz: id of the edge of each entry
  // triangle numbering (r = 3): triangles u<v<w lexicographic
  bool tris_ready = false;
  int64_t nt = 0;
  nd::DArr<int64_t> toff;     // ne+1: first triangle id of edge (u,v)
  nd::DArr<int32_t> tri_w;    // nt: third vertex w
  nd::DArr<int32_t> tri_e;    // nt: edge id of (u,v)
  nd::KindState ks[nd::kNumKinds];
  double ms_build = 0;
  size_t bytes() const;
};

namespace nd {

// Free a graph whose last device work was ordered on stream s, returning
// its memory to the allocator tagged with s (waits for s first when `wait`;
// nd_graph_destroy waits for the device).  Without waiting this is still
// safe for the graph's own arrays: the allocator hands a block tagged with s
// to another stream only once s has drained.
void destroy_graph(nd_graph *g, hipStream_t s, bool wait = true);

// ------------------------------------------------------- primitives

// out[i] = sum_{j<i} in[j] for i <= n (out has n+1 entries).
void exclusive_scan_i32(const int32_t *in, int64_t *out, int64_t n,
                        hipStream_t s, Allocator &al);
void exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n,
                        hipStream_t s, Allocator &al);
// Stable LSD radix sort of keys by bits [lo_bit, hi_bit); returns whichever
// of keys/tmp holds the result.
uint64_t *radix_sort_u64(uint64_t *keys, uint64_t *tmp, int64_t n, int lo_bit,
                         int hi_bit, hipStream_t s, Allocator &al);
// items[] = 0..n-1 grouped by bin[i] (stable), offsets[b] = first index of
// bin b (host, nbins+1 entries).  nbins <= 256.
void partition_by_bin(const uint8_t *bin, int64_t n, int nbins, int32_t *items,
                      int64_t *offsets, hipStream_t s, Allocator &al);
void fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
void fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t s);
void fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t s);
void iota_i32(int32_t *p, int64_t n, hipStream_t s);  // p[i] = i
int64_t read_i64(const int64_t *dev, hipStream_t s);  // synchronous

// A 4 KiB pinned host chunk taken from a pool for the life of the object,
// for reading a few words back from the device: a copy into pageable memory
// goes through the runtime's staging path instead of straight to its
// destination.  Chunks return to the pool, never to the runtime.
class PinnedChunk {
 public:
  static constexpr size_t kBytes = 4096;
  PinnedChunk();
  ~PinnedChunk();
  PinnedChunk(const PinnedChunk &) = delete;
  PinnedChunk &operator=(const PinnedChunk &) = delete;
  template <class T>
  T *as() const { return static_cast<T *>(p_); }
  // Copy n words of T from the device (ordered on s, waits for it).
  template <class T>
  const T *read(const T *dev, size_t n, hipStream_t s) {
    ND_REQUIRE(n * sizeof(T) <= kBytes, ND_ERR_INVALID, "read-back too large");
    ND_HIP(hipMemcpyAsync(p_, dev, n * sizeof(T), hipMemcpyDeviceToHost, s));
    ND_HIP(hipStreamSynchronize(s));
    return as<T>();
  }

 private:
  void *p_ = nullptr;
};

// ------------------------------------------------------------ graph prep

// Canonical CSR from raw device pairs (validates ids; ND_ERR_INVALID).
void build_from_edges(nd_graph *g, int64_t m, const int32_t *src,
                      const int32_t *dst, hipStream_t s);
// Check a device CSR already copied into g (ND_ERR_INVALID when malformed).
void validate_csr(nd_graph *g, hipStream_t s);
void build_rowid(nd_graph *g, hipStream_t s);
void build_edges(nd_graph *g, hipStream_t s);
void build_triangles(nd_graph *g, hipStream_t s);
// Incidence lists in the internal numbering (each calls build_layout once
// the S-degrees are counted, then writes the lists in place).
void build_incidence_core(nd_graph *g, KindState &ks, hipStream_t s);
void build_incidence_truss(nd_graph *g, KindState &ks, hipStream_t s);
void build_incidence_n34(nd_graph *g, KindState &ks, hipStream_t s);
void build_incidence_n13(nd_graph *g, KindState &ks, hipStream_t s);
void build_incidence_n24(nd_graph *g, KindState &ks, hipStream_t s);
// From S-degrees in r-clique-id order: perm, inv, ds, inc_off, bins.
void build_layout(nd_graph *g, KindState &ks, const int32_t *cnt,
                  hipStream_t s);
// Re-index between internal and r-clique-id order; the internal side holds
// `bytes` (1, 2 or 4) per value.
void to_internal(const KindState &ks, const int32_t *in, void *out, int bytes,
                 hipStream_t s);
void to_original(const KindState &ks, const void *in, int bytes, int32_t *out,
                 hipStream_t s);
// Incidence lists in r-clique-id order with r-clique ids (off[nr+1]).
void incidence_original(nd_graph *g, const KindState &ks, int64_t *off,
                        int32_t *ids, hipStream_t s);
void sdegree_original(const KindState &ks, int32_t *ds, hipStream_t s);
// tau_0 = d_s in the internal numbering, `bytes` (1, 2 or 4) per value.
void init_tau(const KindState &ks, void *tau, int bytes, hipStream_t s);

// ---------------------------------------------------------------- sweeps

// Per-sweep counters.  Every wave adds its counts atomically; with one
// counter all those atomics would queue on a single L2 channel, so the counts
// are split over kStatParts parts, one 128-byte line each, and summed by the
// reader.
constexpr int kStatParts = 16;
struct alignas(128) StatPart {
  unsigned long long changed;
  unsigned long long evaluated;
  unsigned long long pad[14];
};
struct SweepStats {
  StatPart part[kStatParts];
  unsigned long long notified;  // 1: this sweep set the next sweep's flags
  unsigned long long active;    // r-cliques flagged for the next sweep
                                // (counted after the sweep when asked for)
  unsigned long long pad[14];
  __host__ __device__ unsigned long long changed_total() const {
    unsigned long long s = 0;
    for (int i = 0; i < kStatParts; i++) s += part[i].changed;
    return s;
  }
  __host__ __device__ unsigned long long evaluated_total() const {
    unsigned long long s = 0;
    for (int i = 0; i < kStatParts; i++) s += part[i].evaluated;
    return s;
  }
};

struct SweepArgs {
  const int64_t *inc_off;
  const int32_t *inc_ids;
  const void *tau_in;      // SND: tau_t; AND: the in-place array
  void *tau_out;           // SND: tau_{t+1}; AND: same as tau_in
  SweepStats *stats;       // this sweep's counters
  const SweepStats *prev;  // previous sweep's counters (skip when converged)
  int cap_by_tau;          // 1: clamp at tau_in(R) (iterates); 0: at d_s
  // Frontier (Section 4.3 notifications), both NULL when off: only
  // r-cliques with act[R] != 0 are recomputed; a changed one sets act_next
  // for every neighbour whose value is above its new value.
  const uint8_t *act;       // flags of this sweep (stamps, see sweep_dev.h)
  uint8_t *act_next;
  // one stamp per 64 r-cliques, set with any flag of the group (NULL: none)
  const uint8_t *act_sum;
  uint8_t *act_sum_next;
  uint8_t stamp;            // this sweep's stamp
  // Notifications start once a sweep changes at most this many r-cliques
  // (before that nearly everything is active and notifying costs as much as
  // the gathers it would save); from then on every sweep notifies and the
  // next one recomputes only flagged r-cliques.
  unsigned long long notify_below;
  // 1: the first sweep notifies too (notify_below only applies from the
  // second sweep on otherwise).
  int notify_first;
  // 1: flags are written and counted but never used to skip r-cliques (the
  // active-ratio indicator without the frontier).
  int flags_unused;
  // PartialAND (Section 4.3, end): act marks a fixed set (stamp 1) that is
  // the only thing recomputed, every sweep, and nothing notifies.
  int fixed_set;
  // At most this many workgroups per lanes-per-r-clique kernel (they stride
  // over the rest of the bin); 0: one pass, no cap.
  int grid_cap;
  // Nonzero: a notifying sweep whose previous sweep changed at least this
  // many r-cliques writes flags but no group summaries (many of its
  // notifications would store the same summary byte); launch_group_sums
  // rebuilds them after it from the flags.
  unsigned long long sums_after;
};

// The static device workspace of nd_decompose_noalloc: one array per device
// (api.hip), its address looked up when the first context on the device is
// created; NULL before that.
constexpr size_t kNoallocWorkspaceBytes = ND_NOALLOC_WORKSPACE_BYTES;
void *noalloc_workspace(int device);

// Entries of the pinned host ring that receives the sweep counters.
constexpr int kHostStatsRing = 1024;

// Launch one sweep over every bin of ks (internal numbering, tau of
// ks.tau_bytes per value).  `and_mode` selects in-place reads.
void launch_sweep(const KindState &ks, const SweepArgs &a, bool and_mode,
                  hipStream_t s);
// After the sweep of a (same arguments): the group summaries of the flags it
// wrote, when a.sums_after made it skip them; nothing otherwise.
void launch_group_sums(const KindState &ks, const SweepArgs &a, hipStream_t s);

// Host threads (each with a stream) that build or prepare several graphs
// at once: 2, or ND_PREP_THREADS.
int prep_threads();

// Frontier switch: notifications start once a sweep changes at most
// 1/d of the swept r-cliques; d = 8 for SND and AND (measured on the three
// benchmark workloads), ND_FRONTIER_SWITCH overrides it (0: from the first
// sweep on).
int frontier_switch(bool and_mode);

}  // namespace nd
