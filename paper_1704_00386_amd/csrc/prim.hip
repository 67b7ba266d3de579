// prim.hip -- device primitives used by graph preparation: exclusive scan,
// stable LSD radix sort of 64-bit keys, stable partition by a small key, and
// fills.  All integer, all deterministic.
#include <algorithm>
#include <mutex>
#include <vector>

#include "internal.h"

namespace nd {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;  // 2048

// Inclusive scan of one value per lane across the wave.
__device__ __forceinline__ int64_t wave_inclusive_scan(int64_t x) {
  const int lane = lane_id();
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    int64_t y = __shfl_up(x, off, kWave);
    if (lane >= off) x += y;
  }
  return x;
}

// Block-wide exclusive prefix of one value per thread (256 threads).
// Returns the prefix and writes the block total to *total.
__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v,
                                                        int64_t *total) {
  __shared__ int64_t wsum[kScanThreads / kWave];
  const int lane = lane_id();
  const int wid = threadIdx.x / kWave;
  int64_t inc = wave_inclusive_scan(v);
  if (lane == kWave - 1) wsum[wid] = inc;
  __syncthreads();
  int64_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kScanThreads / kWave; w++) {
    if (w < wid) before += wsum[w];
    all += wsum[w];
  }
  *total = all;
  __syncthreads();  // wsum may be reused by a following call
  return before + inc - v;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(
    const T *__restrict__ in, int64_t n, int64_t *__restrict__ partial) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int64_t sum = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; j++) {
    int64_t i = base + j;
    if (i < n) sum += (int64_t)in[i];
  }
  int64_t total;
  block_exclusive_scan(sum, &total);
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// out[i] = offset(block) + exclusive prefix within the tile.  The last block
// also writes out[n] (the grand total).
template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_tile(
    const T *__restrict__ in, int64_t n, const int64_t *__restrict__ block_off,
    int64_t *__restrict__ out) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int64_t v[kScanItems];
  int64_t sum = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; j++) {
    int64_t i = base + j;
    v[j] = i < n ? (int64_t)in[i] : 0;
    sum += v[j];
  }
  int64_t total;
  int64_t run = block_exclusive_scan(sum, &total);
  const int64_t off = block_off ? block_off[blockIdx.x] : 0;
  run += off;
#pragma unroll
  for (int j = 0; j < kScanItems; j++) {
    int64_t i = base + j;
    if (i < n) out[i] = run;
    run += v[j];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = off + total;
}

// Up to this many tiles, one workgroup scans them in turn, carrying the
// running total: one launch instead of three (the scans of graph
// preparation are mostly this short, and launches dominate them).
constexpr int64_t kScanLoopTiles = 64;

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_loop(
    const T *__restrict__ in, int64_t n, int64_t *__restrict__ out) {
  int64_t carry = 0;
  for (int64_t base0 = 0; base0 < n; base0 += kScanTile) {
    const int64_t base = base0 + threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t sum = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
      const int64_t i = base + j;
      v[j] = i < n ? (int64_t)in[i] : 0;
      sum += v[j];
    }
    int64_t total;
    int64_t run = carry + block_exclusive_scan(sum, &total);
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
      const int64_t i = base + j;
      if (i < n) out[i] = run;
      run += v[j];
    }
    carry += total;
  }
  if (threadIdx.x == 0) out[n] = carry;
}

template <typename T>
void exclusive_scan_impl(const T *in, int64_t *out, int64_t n, hipStream_t s,
                         Allocator &al) {
  const int64_t nb = ceil_div(std::max<int64_t>(n, 0), kScanTile);
  if (nb <= kScanLoopTiles) {  // n == 0 too: writes out[0] = 0
    k_scan_loop<T><<<1, kScanThreads, 0, s>>>(in, std::max<int64_t>(n, 0), out);
    ND_LAUNCHED();
    return;
  }
  DArr<int64_t> partial(al, nb), pscan(al, nb + 1);
  k_scan_reduce<T><<<(unsigned)nb, kScanThreads, 0, s>>>(in, n, partial.p);
  ND_LAUNCHED();
  exclusive_scan_impl<int64_t>(partial.p, pscan.p, nb, s, al);
  k_scan_tile<T><<<(unsigned)nb, kScanThreads, 0, s>>>(in, n, pscan.p, out);
  ND_LAUNCHED();
}

// ------------------------------------------------------------ radix sort

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;  // 4096 keys per block
constexpr int kSortWaves = kSortThreads / kWave;

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(
    const uint64_t *__restrict__ keys, int64_t n, int shift,
    int32_t *__restrict__ hist, int64_t nb) {
  __shared__ int32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll 4
  for (int it = 0; it < kSortItems; it++) {
    int64_t i = base + it * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: keys of the tile are ranked in input order (round, wave,
// lane); equal digits within a wave are matched with 8 ballots.
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const uint64_t *__restrict__ in, uint64_t *__restrict__ out, int64_t n,
    int shift, const int64_t *__restrict__ offs, int64_t nb) {
  __shared__ int64_t run[256];
  __shared__ int32_t cnt[kSortWaves][256];
  const int tid = threadIdx.x;
  const int wid = tid / kWave;
  run[tid] = offs[(int64_t)tid * nb + blockIdx.x];
#pragma unroll
  for (int w = 0; w < kSortWaves; w++) cnt[w][tid] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int it = 0; it < kSortItems; it++) {
    const int64_t i = base + it * kSortThreads + tid;
    const bool valid = i < n;
    const uint64_t key = valid ? in[i] : 0;
    const int d = (int)((key >> shift) & 255);
    uint64_t peers = ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; b++) {
      const bool bit = (d >> b) & 1;
      const uint64_t m = ballot(bit);
      peers &= bit ? m : ~m;
    }
    const int rank = lanes_below(peers);
    if (valid && rank == 0) cnt[wid][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int64_t pos = run[d] + rank;
      for (int w = 0; w < wid; w++) pos += cnt[w][d];
      out[pos] = key;
    }
    __syncthreads();
    int32_t add = 0;
#pragma unroll
    for (int w = 0; w < kSortWaves; w++) {
      add += cnt[w][tid];
      cnt[w][tid] = 0;
    }
    run[tid] += add;
    __syncthreads();
  }
}

// ------------------------------------------------------------- misc

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_u8(uint8_t *p, uint8_t v, int64_t n) {
  // four bytes per thread where aligned
  int64_t i = 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
  if (i + 3 < n && ((uintptr_t)(p + i) & 3) == 0) {
    const uint32_t w = 0x01010101u * v;
    *reinterpret_cast<uint32_t *>(p + i) = w;
  } else {
    for (int64_t j = i; j < i + 4 && j < n; j++) p[j] = v;
  }
}

__global__ void k_fill_u64(uint64_t *p, uint64_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Keys bin<<32 | i, and the bin sizes: counted per block in LDS first, so
// that the global counters see one atomic per (block, bin) rather than one
// per item (a handful of bins would otherwise serialise every thread).
__global__ __launch_bounds__(256) void k_bin_keys(
    const uint8_t *__restrict__ bin, int64_t n, int nbins,
    uint64_t *__restrict__ keys, unsigned long long *__restrict__ counts) {
  __shared__ unsigned int h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * 256 * 8;
  for (int j = 0; j < 8; j++) {
    const int64_t i = base + j * 256 + threadIdx.x;
    if (i < n) {
      const uint8_t b = bin[i];
      keys[i] = ((uint64_t)b << 32) | (uint64_t)i;
      atomicAdd(&h[b], 1u);
    }
  }
  __syncthreads();
  if (threadIdx.x < nbins && h[threadIdx.x])
    atomicAdd(&counts[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

__global__ void k_low32(const uint64_t *__restrict__ keys, int64_t n,
                        int32_t *__restrict__ items) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) items[i] = (int32_t)(keys[i] & 0xffffffffu);
}

}  // namespace

void exclusive_scan_i32(const int32_t *in, int64_t *out, int64_t n,
                        hipStream_t s, Allocator &al) {
  exclusive_scan_impl<int32_t>(in, out, n, s, al);
}

void exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n,
                        hipStream_t s, Allocator &al) {
  exclusive_scan_impl<int64_t>(in, out, n, s, al);
}

uint64_t *radix_sort_u64(uint64_t *keys, uint64_t *tmp, int64_t n, int lo_bit,
                         int hi_bit, hipStream_t s, Allocator &al) {
  if (n <= 1 || hi_bit <= lo_bit) return keys;
  const int64_t nb = ceil_div(n, kSortTile);
  ND_REQUIRE(nb * 256 < (int64_t)1 << 31, ND_ERR_INVALID,
             "radix sort: %lld keys is too many", (long long)n);
  DArr<int32_t> hist(al, 256 * nb);
  DArr<int64_t> offs(al, 256 * nb + 1);
  uint64_t *src = keys, *dst = tmp;
  for (int shift = lo_bit; shift < hi_bit; shift += 8) {
    k_radix_hist<<<(unsigned)nb, kSortThreads, 0, s>>>(src, n, shift, hist.p,
                                                        nb);
    ND_LAUNCHED();
    exclusive_scan_i32(hist.p, offs.p, 256 * nb, s, al);
    k_radix_scatter<<<(unsigned)nb, kSortThreads, 0, s>>>(src, dst, n, shift,
                                                           offs.p, nb);
    ND_LAUNCHED();
    uint64_t *t = src;
    src = dst;
    dst = t;
  }
  return src;
}

void partition_by_bin(const uint8_t *bin, int64_t n, int nbins, int32_t *items,
                      int64_t *offsets, hipStream_t s, Allocator &al) {
  ND_REQUIRE(nbins >= 1 && nbins <= 256, ND_ERR_INVALID, "bad bin count");
  for (int b = 0; b <= nbins; b++) offsets[b] = 0;
  if (n <= 0) return;
  DArr<uint64_t> keys(al, n), tmp(al, n);
  DArr<unsigned long long> counts(al, nbins);
  ND_HIP(hipMemsetAsync(counts.p, 0, sizeof(unsigned long long) * nbins, s));
  k_bin_keys<<<grid_for(n, 256 * 8), 256, 0, s>>>(bin, n, nbins, keys.p,
                                                   counts.p);
  ND_LAUNCHED();
  uint64_t *sorted = radix_sort_u64(keys.p, tmp.p, n, 32, 40, s, al);
  k_low32<<<grid_for(n, 256), 256, 0, s>>>(sorted, n, items);
  ND_LAUNCHED();
  PinnedChunk pc;
  const unsigned long long *h = pc.read(counts.p, (size_t)nbins, s);
  for (int b = 0; b < nbins; b++) offsets[b + 1] = offsets[b] + (int64_t)h[b];
}

void fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_fill_i32<<<grid_for(n, 256), 256, 0, s>>>(p, v, n);
  ND_LAUNCHED();
}

namespace {
__global__ void k_iota_i32(int32_t *__restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (int32_t)i;
}
}  // namespace

void iota_i32(int32_t *p, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_iota_i32<<<grid_for(n, 256), 256, 0, s>>>(p, n);
  ND_LAUNCHED();
}

void fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_fill_u8<<<grid_for(ceil_div(n, 4), 256), 256, 0, s>>>(p, v, n);
  ND_LAUNCHED();
}

void fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_fill_u64<<<grid_for(n, 256), 256, 0, s>>>(p, v, n);
  ND_LAUNCHED();
}

namespace {
std::mutex g_pinned_mu;
std::vector<void *> g_pinned_free;
}  // namespace

PinnedChunk::PinnedChunk() {
  {
    std::lock_guard<std::mutex> lk(g_pinned_mu);
    if (!g_pinned_free.empty()) {
      p_ = g_pinned_free.back();
      g_pinned_free.pop_back();
      return;
    }
  }
  ND_HIP(hipHostMalloc(&p_, kBytes, hipHostMallocDefault));
}

PinnedChunk::~PinnedChunk() {
  std::lock_guard<std::mutex> lk(g_pinned_mu);
  g_pinned_free.push_back(p_);
}

int64_t read_i64(const int64_t *dev, hipStream_t s) {
  PinnedChunk h;
  return *h.read(dev, 1, s);
}

}  // namespace nd
