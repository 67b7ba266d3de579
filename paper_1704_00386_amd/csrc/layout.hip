// layout.hip -- the internal numbering of r-cliques.
//
// Sweeps run over r-cliques grouped by sweep bin (the lanes per r-clique
// chosen from d_s: d_s >= 2048 first, d_s = 0 last), each group in ascending
// id order.  Both choices serve the memory hierarchy, not the method:
//   * each bin becomes a contiguous id range, so no per-bin index lists are
//     read and the incidence lists are one sequential stream;
//   * within a bin, ids keep the lexicographic order of the r-cliques, so
//     r-cliques swept by neighbouring lanes share vertices, and the tau
//     values they gather (r-cliques of their common s-cliques, which share
//     those vertices too) sit in nearby cache lines.  Measured on a power-law
//     k-truss workload this beats ordering by exact d_s (which packs the most
//     gathered values together but scatters each lane group's neighbours) by
//     about 30% per sweep;
//   * r-cliques with d_s = 0 (never swept) go to the end.
// Results are un-permuted on the way out; nothing observable depends on the
// internal order (SND iterates are order-independent by definition).
#include "internal.h"

namespace nd {

namespace {

int bits_for(int64_t x) {
  int b = 1;
  while (b < 62 && ((int64_t)1 << b) <= x) b++;
  return b;
}

__device__ __forceinline__ int bin_of(int64_t d) {
  return d >= 2048 ? kBinBlock
       : d >= 1025 ? kBinWave
       : d >= 513 ? kBinWave16
       : d >= 257 ? kBinWave8
       : d >= 65  ? kBinG64
       : d >= 17  ? kBinG16
       : d >= 5   ? kBinG4
       : d >= 1   ? kBinG1
                  : kBinZero;
}

// Maximum degree and bin sizes: counts per thread in registers over a
// grid-stride share, then per block in LDS, then one global atomic per block
// and bin (atomics from every wave onto the same few words serialise).
constexpr int kStatsBlocks = 4096;

__global__ __launch_bounds__(256) void k_layout_stats(
    const int32_t *__restrict__ cnt, int64_t nr, int32_t *__restrict__ maxd,
    unsigned long long *__restrict__ bins) {
  __shared__ unsigned int h[kNumBins];
  __shared__ int32_t hm;
  if (threadIdx.x < kNumBins) h[threadIdx.x] = 0;
  if (threadIdx.x == 0) hm = 0;
  __syncthreads();
  int32_t m = 0;
  unsigned int c[kNumBins];
#pragma unroll
  for (int b = 0; b < kNumBins; b++) c[b] = 0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i0 = (int64_t)blockIdx.x * 256 + threadIdx.x; i0 < nr;
       i0 += 4 * stride) {
    int32_t d[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int64_t i = i0 + j * stride;
      d[j] = i < nr ? cnt[i] : -1;
    }
#pragma unroll
    for (int j = 0; j < 4; j++) {
      if (d[j] < 0) continue;
      m = max(m, d[j]);
      const int bd = bin_of(d[j]);
#pragma unroll
      for (int b = 0; b < kNumBins; b++) c[b] += bd == b;
    }
  }
#pragma unroll
  for (int b = 0; b < kNumBins; b++) {
    unsigned int v = c[b];
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    if (lane_id() == 0 && v) atomicAdd(&h[b], v);
  }
  for (int o = kWave / 2; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, kWave));
  if (lane_id() == 0) atomicMax(&hm, m);
  __syncthreads();
  if (threadIdx.x < kNumBins && h[threadIdx.x])
    atomicAdd(&bins[threadIdx.x], (unsigned long long)h[threadIdx.x]);
  if (threadIdx.x == kNumBins) atomicMax(maxd, hm);
}

// Sort key: sweep bin, then ascending id.
__global__ void k_layout_keys(const int32_t *__restrict__ cnt, int64_t nr,
                              int rb, uint64_t *__restrict__ keys) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nr) keys[i] = ((uint64_t)bin_of(cnt[i]) << rb) | (uint64_t)i;
}

__global__ void k_layout_perm(const uint64_t *__restrict__ keys, int64_t nr,
                              int rb, const int32_t *__restrict__ cnt,
                              int32_t *__restrict__ perm,
                              int32_t *__restrict__ inv,
                              int32_t *__restrict__ ds) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nr) return;
  const int32_t R = (int32_t)(keys[i] & (((uint64_t)1 << rb) - 1));
  perm[i] = R;
  inv[R] = (int32_t)i;
  ds[i] = cnt[R];
}

template <typename T>
__global__ void k_to_internal(const int32_t *__restrict__ in,
                              const int32_t *__restrict__ perm, int64_t nr,
                              T *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nr) out[i] = (T)in[perm[i]];
}

template <typename T>
__global__ void k_to_original(const T *__restrict__ in,
                              const int32_t *__restrict__ inv, int64_t nr,
                              int32_t *__restrict__ out) {
  const int64_t R = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (R < nr) out[R] = (int32_t)in[inv[R]];
}

// List of r-clique R (original numbering) with original ids, G lanes each.
template <int G>
__global__ __launch_bounds__(256) void k_incidence_original(
    const int64_t *__restrict__ in_off, const int32_t *__restrict__ in_ids,
    const int32_t *__restrict__ inv, const int32_t *__restrict__ perm, int k,
    int64_t nr, const int64_t *__restrict__ out_off,
    int32_t *__restrict__ out_ids) {
  const int sl = lane_id() % G;
  const int64_t nsub = (int64_t)gridDim.x * blockDim.x / G;
  for (int64_t R = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
       R < nr; R += nsub) {
    const int32_t i = inv[R];
    const int64_t b = in_off[i] * k, e = in_off[i + 1] * k, o = out_off[R] * k;
    for (int64_t j = b + sl; j < e; j += G) out_ids[o + (j - b)] = perm[in_ids[j]];
  }
}

template <typename T>
__global__ void k_init_tau(const int32_t *__restrict__ ds, int64_t nr,
                           T *__restrict__ tau) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nr) tau[i] = (T)ds[i];
}

}  // namespace

void init_tau(const KindState &ks, void *tau, int bytes, hipStream_t s) {
  if (ks.nr == 0) return;
  const unsigned grid = grid_for(ks.nr, 256);
  if (bytes == 1)
    k_init_tau<uint8_t><<<grid, 256, 0, s>>>(ks.ds.p, ks.nr, (uint8_t *)tau);
  else if (bytes == 2)
    k_init_tau<uint16_t><<<grid, 256, 0, s>>>(ks.ds.p, ks.nr, (uint16_t *)tau);
  else
    k_init_tau<int32_t><<<grid, 256, 0, s>>>(ks.ds.p, ks.nr, (int32_t *)tau);
  ND_LAUNCHED();
}

void build_layout(nd_graph *g, KindState &ks, const int32_t *cnt,
                  hipStream_t s) {
  Phase phase("nd.layout");
  Allocator &al = g->ctx->alloc;
  const int64_t nr = ks.nr;
  ND_REQUIRE(nr < ((int64_t)1 << 31), ND_ERR_INVALID,
             "%lld r-cliques: ids must fit int32", (long long)nr);
  DArr<int32_t> maxd(al, 1);
  DArr<unsigned long long> bins(al, kNumBins);
  fill_i32(maxd.p, 0, 1, s);
  fill_u64((uint64_t *)bins.p, 0, kNumBins, s);
  if (nr > 0) {
    const unsigned grid =
        (unsigned)std::min<int64_t>(grid_for(nr, 256 * 4), kStatsBlocks);
    k_layout_stats<<<grid, 256, 0, s>>>(cnt, nr, maxd.p, bins.p);
    ND_LAUNCHED();
  }
  PinnedChunk pc;
  unsigned long long *hb = pc.as<unsigned long long>();
  int32_t *hmaxp = reinterpret_cast<int32_t *>(hb + kNumBins);
  ND_HIP(hipMemcpyAsync(hmaxp, maxd.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  ND_HIP(hipMemcpyAsync(hb, bins.p, sizeof(unsigned long long) * kNumBins,
                        hipMemcpyDeviceToHost, s));
  ND_HIP(hipStreamSynchronize(s));
  const int32_t hmax = *hmaxp;
  ks.max_ds = hmax;
  ks.tau16 = hmax < 32768;
  ks.tau_bytes = hmax < 256 ? 1 : ks.tau16 ? 2 : 4;
  int64_t at = 0;
  for (int b = 0; b < kNumBins; b++) {
    ks.bin_lo[b] = at;
    at += (int64_t)hb[b];
    ks.bin_hi[b] = at;
  }
  ks.perm.reset(al, nr);
  ks.inv.reset(al, nr);
  ks.ds.reset(al, nr);
  ks.inc_off.reset(al, nr + 1);
  if (nr > 0) {
    const int rb = bits_for(nr - 1);
    DArr<uint64_t> keys(al, nr), tmp(al, nr);
    k_layout_keys<<<grid_for(nr, 256), 256, 0, s>>>(cnt, nr, rb, keys.p);
    ND_LAUNCHED();
    static_assert(kNumBins <= 16, "bin index must fit 4 key bits");
    // the keys are in id order already and the sort is stable, so sorting
    // by the bin bits alone (one pass) orders them by (bin, id)
    uint64_t *sorted = radix_sort_u64(keys.p, tmp.p, nr, rb, rb + 4, s, al);
    k_layout_perm<<<grid_for(nr, 256), 256, 0, s>>>(sorted, nr, rb, cnt,
                                                     ks.perm.p, ks.inv.p,
                                                     ks.ds.p);
    ND_LAUNCHED();
  }
  exclusive_scan_i32(ks.ds.p, ks.inc_off.p, nr, s, al);
  ks.P = read_i64(ks.inc_off.p + nr, s);
}

void to_internal(const KindState &ks, const int32_t *in, void *out, int bytes,
                 hipStream_t s) {
  if (ks.nr == 0) return;
  const unsigned grid = grid_for(ks.nr, 256);
  if (bytes == 1)
    k_to_internal<uint8_t><<<grid, 256, 0, s>>>(in, ks.perm.p, ks.nr, (uint8_t *)out);
  else if (bytes == 2)
    k_to_internal<uint16_t><<<grid, 256, 0, s>>>(in, ks.perm.p, ks.nr, (uint16_t *)out);
  else
    k_to_internal<int32_t><<<grid, 256, 0, s>>>(in, ks.perm.p, ks.nr, (int32_t *)out);
  ND_LAUNCHED();
}

void to_original(const KindState &ks, const void *in, int bytes, int32_t *out,
                 hipStream_t s) {
  if (ks.nr == 0) return;
  const unsigned grid = grid_for(ks.nr, 256);
  if (bytes == 1)
    k_to_original<uint8_t><<<grid, 256, 0, s>>>((const uint8_t *)in, ks.inv.p, ks.nr, out);
  else if (bytes == 2)
    k_to_original<uint16_t><<<grid, 256, 0, s>>>((const uint16_t *)in, ks.inv.p, ks.nr, out);
  else
    k_to_original<int32_t><<<grid, 256, 0, s>>>((const int32_t *)in, ks.inv.p, ks.nr, out);
  ND_LAUNCHED();
}

void sdegree_original(const KindState &ks, int32_t *ds, hipStream_t s) {
  to_original(ks, ks.ds.p, 4, ds, s);
}

void incidence_original(nd_graph *g, const KindState &ks, int64_t *off,
                        int32_t *ids, hipStream_t s) {
  Allocator &al = g->ctx->alloc;
  DArr<int32_t> dso(al, ks.nr);
  sdegree_original(ks, dso.p, s);
  exclusive_scan_i32(dso.p, off, ks.nr, s, al);
  if (ks.nr == 0 || ks.P == 0) return;
  k_incidence_original<16><<<grid_stride(ks.nr, 16), 256, 0, s>>>(
      ks.inc_off.p, ks.inc_ids.p, ks.inv.p, ks.perm.p, ks.k, ks.nr, off, ids);
  ND_LAUNCHED();
}

}  // namespace nd
