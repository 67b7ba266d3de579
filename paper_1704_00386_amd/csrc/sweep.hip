// sweep.hip -- one application of the update operator U to every r-clique
// (Section 3, Defn. of U; the parallel loop of Alg. 2 and Alg. 3):
//
//   rho(S,R)  = min over the k other r-cliques R' of S of tau(R')  (gather+min)
//   tau'(R)   = H({rho(S,R)} over the d_s(R) s-cliques S containing R)
//   changed  += (tau'(R) != tau(R))                         (convergence flag)
//
// r-cliques are in the internal numbering (descending d_s), so each bin is a
// contiguous id range and the incidence lists are read in one sequential,
// coalesced stream; the tau reads are the random part.  tau is stored as
// uint16 when every d_s fits (then every tau does: tau <= d_s), halving the
// bytes of the gathered array.
//
// H is computed exactly with a cap c (Section 4.4 "can the current value be
// preserved" check, made exact):
//   * H(min(K,c)) = min(H(K), c) for any multiset K and any c >= 0, and
//     H(K) <= |K| = d_s(R), so with c = d_s(R) the cap never changes H.
//   * For the iterates of SND/AND, U tau(R) <= tau(R) (Theorem 1, and the same
//     argument for in-place sweeps, whose inputs only decrease), so c = tau(R)
//     is exact there too and keeps the work small.
//   * If #{rho >= c} >= c then H = c (the preserve check).  Otherwise H is
//     the largest x < c with #{rho >= x} >= x, found by binary search on x
//     with counts reduced across the lanes that hold the rho values.
//
// Mappings by S-degree bin:
//   d_s <= 256     G = 1/4/16/64 lanes per r-clique, 4 rho values per lane
//   257..2047      one wave per r-clique, 32 rho values per lane
//   >= 2048        one 256-thread workgroup per r-clique; LDS histogram of
//                  min(rho, c) in up to 16384 bins; for larger c the values
//                  are binned coarsely and the coarse bin holding H is refined
//                  with a second gather.
// SND reads tau_t and writes tau_{t+1} (double buffer, race free, so every
// iterate is deterministic).  AND reads and writes one array in place; its
// neighbour reads bypass the per-CU cache so that they see other workgroups'
// recent writes, which only ever lower values (Section 4.2).
#include "internal.h"

namespace nd {

namespace {

constexpr int kBlockThreads = 256;
constexpr int kBlockHistBins = 16384;  // 64 KiB of LDS

template <typename T, bool AND>
__device__ __forceinline__ int32_t load_tau(const T *p) {
  if constexpr (AND) {
    return (int32_t)__hip_atomic_load(p, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
  } else {
    return (int32_t)*p;
  }
}

template <typename T, bool AND>
__device__ __forceinline__ void store_tau(T *p, int32_t h, bool changed) {
  if constexpr (AND) {
    if (changed)
      __hip_atomic_store(p, (T)h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    *p = (T)h;
  }
}

// rho for the s-clique j of the incidence list (k = K ids per s-clique).
template <int K, typename T, bool AND>
__device__ __forceinline__ int32_t gather_rho(const int32_t *__restrict__ ids,
                                              int64_t j, const T *tau) {
  if constexpr (K == 1) {
    return load_tau<T, AND>(tau + ids[j]);
  } else if constexpr (K == 2) {
    const int2 p = *reinterpret_cast<const int2 *>(ids + 2 * j);
    return min(load_tau<T, AND>(tau + p.x), load_tau<T, AND>(tau + p.y));
  } else {
    const int32_t *q = ids + 3 * j;
    const int32_t x = q[0], y = q[1], z = q[2];
    return min(min(load_tau<T, AND>(tau + x), load_tau<T, AND>(tau + y)),
               load_tau<T, AND>(tau + z));
  }
}

template <int G>
__device__ __forceinline__ int subgroup_sum(int x) {
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, G);
  return x;
}

__device__ __forceinline__ bool converged_before(const SweepStats *prev) {
  return prev != nullptr && prev->changed == 0;
}

__device__ __forceinline__ void count_changed(SweepStats *st, bool changed) {
  const uint64_t m = ballot(changed);
  if (lane_id() == 0 && m) atomicAdd(&st->changed, (unsigned long long)__popcll(m));
}

// Largest x in [0, c-1] with #{rho >= x} >= x, given that x = 0 satisfies it;
// G lanes of a subgroup each hold M values (absent values are -1).
template <int G, int M>
__device__ __forceinline__ int32_t hindex_search(const int32_t (&rho)[M],
                                                 int32_t c) {
  int32_t lo = 0, hi = c - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    int cm = 0;
#pragma unroll
    for (int m = 0; m < M; m++) cm += rho[m] >= mid;
    cm = subgroup_sum<G>(cm);
    if (cm >= mid)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// ------------------------------------------- registers, G lanes per R

template <int K, int G, int M, typename T, bool AND>
__global__ __launch_bounds__(256) void k_sweep_regs(SweepArgs a, int64_t lo,
                                                    int64_t hi) {
  if (converged_before(a.prev)) return;
  const T *tau_in = (const T *)a.tau_in;
  T *tau_out = (T *)a.tau_out;
  const int64_t R = lo + ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const int sl = lane_id() % G;
  const bool active = R < hi;
  int32_t told = 0, c = 0;
  int64_t b = 0, d = 0;
  if (active) {
    b = a.inc_off[R];
    d = a.inc_off[R + 1] - b;
    told = (int32_t)tau_in[R];
    c = a.cap_by_tau ? told : (int32_t)d;
  }
  int32_t rho[M];
#pragma unroll
  for (int m = 0; m < M; m++) {
    const int64_t j = sl + (int64_t)m * G;
    rho[m] = (j < d) ? gather_rho<K, T, AND>(a.inc_ids, b + j, tau_in) : -1;
  }
  int cnt = 0;
#pragma unroll
  for (int m = 0; m < M; m++) cnt += rho[m] >= c;
  cnt = subgroup_sum<G>(cnt);
  const int32_t h = cnt >= c ? c : hindex_search<G, M>(rho, c);
  const bool lead = active && sl == 0;
  const bool changed = lead && h != told;
  if (lead) store_tau<T, AND>(tau_out + R, h, changed);
  count_changed(a.stats, changed);
}

// ------------------------------------------- workgroup per R (LDS)

// Bins hist[0..nb) count values, bin i standing for the value x0 + i*scale.
// Returns the largest i with base + sum_{i' >= i} hist[i'] >= x0 + i*scale,
// or -1 if there is none.  All NT threads of the block call it.
template <int NT>
__device__ int suffix_search(const int32_t *hist, int nb, int64_t base,
                             int64_t x0, int64_t scale) {
  __shared__ int64_t part[NT];
  __shared__ int best_s;
  const int t = threadIdx.x;
  const int chunk = (nb + NT - 1) / NT;
  const int lo = min(nb, t * chunk), hi = min(nb, lo + chunk);
  int64_t mine = 0;
  for (int i = lo; i < hi; i++) mine += hist[i];
  part[t] = mine;
  if (t == 0) best_s = -1;
  __syncthreads();
  int64_t above = base;  // the chunks above mine
  for (int q = t + 1; q < NT; q++) above += part[q];
  int found = -1;
  int64_t run = above;
  for (int i = hi - 1; i >= lo; i--) {
    run += hist[i];
    if (run >= x0 + (int64_t)i * scale) {
      found = i;
      break;
    }
  }
  if (found >= 0) atomicMax(&best_s, found);
  __syncthreads();
  const int r = best_s;
  __syncthreads();
  return r;
}

__device__ __forceinline__ int64_t block_sum(int64_t x) {
  __shared__ int64_t ws[kBlockThreads / kWave];
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
  if (lane_id() == 0) ws[threadIdx.x / kWave] = x;
  __syncthreads();
  int64_t s = 0;
#pragma unroll
  for (int w = 0; w < kBlockThreads / kWave; w++) s += ws[w];
  __syncthreads();
  return s;
}

template <int K, typename T, bool AND>
__global__ __launch_bounds__(kBlockThreads) void k_sweep_block(SweepArgs a,
                                                               int64_t lo,
                                                               int64_t hi) {
  __shared__ int32_t hist[kBlockHistBins];
  if (converged_before(a.prev)) return;
  const T *tau_in = (const T *)a.tau_in;
  T *tau_out = (T *)a.tau_out;
  const int t = threadIdx.x;
  for (int64_t R = lo + blockIdx.x; R < hi; R += gridDim.x) {
    const int64_t b = a.inc_off[R];
    const int64_t d = a.inc_off[R + 1] - b;
    const int32_t told = (int32_t)tau_in[R];
    const int32_t c = a.cap_by_tau ? told : (int32_t)d;
    // bin width: 1 when c+1 bins fit, else coarse
    const int64_t w = ((int64_t)c + kBlockHistBins) / kBlockHistBins;
    const int nb = (int)(((int64_t)c + w) / w);  // bins for values 0..c
    for (int x = t; x < nb; x += kBlockThreads) hist[x] = 0;
    __syncthreads();
    int64_t ge = 0;
    for (int64_t j = t; j < d; j += kBlockThreads) {
      const int32_t rho = gather_rho<K, T, AND>(a.inc_ids, b + j, tau_in);
      ge += rho >= c;
      atomicAdd(&hist[min(rho, c) / w], 1);
    }
    ge = block_sum(ge);
    int32_t h = c;
    if (ge < c) {
      const int i = suffix_search<kBlockThreads>(hist, nb, 0, 0, w);
      if (w == 1) {
        h = i;
      } else {
        // H lies in [i*w, i*w + w - 1]: histogram those values exactly and
        // count the ones above the range, with a second gather.
        const int64_t x0 = (int64_t)i * w;
        const int64_t x1 = min(x0 + w, (int64_t)c + 1);  // exclusive
        const int nfine = (int)(x1 - x0);
        for (int x = t; x < nfine; x += kBlockThreads) hist[x] = 0;
        __syncthreads();
        int64_t above = 0;
        for (int64_t j = t; j < d; j += kBlockThreads) {
          const int32_t rho =
              min(gather_rho<K, T, AND>(a.inc_ids, b + j, tau_in), c);
          if (rho >= x1)
            above++;
          else if (rho >= x0)
            atomicAdd(&hist[rho - x0], 1);
        }
        above = block_sum(above);
        const int f = suffix_search<kBlockThreads>(hist, nfine, above, x0, 1);
        h = (int32_t)(x0 + f);
      }
    }
    const bool changed = t == 0 && h != told;
    if (t == 0) store_tau<T, AND>(tau_out + R, h, changed);
    count_changed(a.stats, changed);
    __syncthreads();
  }
}

template <typename T>
__global__ void k_zero_range(T *__restrict__ tau, int64_t lo, int64_t hi) {
  const int64_t i = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < hi) tau[i] = 0;
}

template <int K, typename T, bool AND>
void launch_bins(const KindState &ks, const SweepArgs &a, hipStream_t s) {
  for (int bin = kBinBlock; bin < kBinZero; bin++) {
    const int64_t lo = ks.bin_lo[bin], hi = ks.bin_hi[bin], n = hi - lo;
    if (n == 0) continue;
    switch (bin) {
      case kBinG1:
        k_sweep_regs<K, 1, 4, T, AND><<<grid_for(n, 256), 256, 0, s>>>(a, lo, hi);
        break;
      case kBinG4:
        k_sweep_regs<K, 4, 4, T, AND><<<grid_for(n * 4, 256), 256, 0, s>>>(a, lo, hi);
        break;
      case kBinG16:
        k_sweep_regs<K, 16, 4, T, AND><<<grid_for(n * 16, 256), 256, 0, s>>>(a, lo, hi);
        break;
      case kBinG64:
        k_sweep_regs<K, 64, 4, T, AND><<<grid_for(n * 64, 256), 256, 0, s>>>(a, lo, hi);
        break;
      case kBinWave:
        k_sweep_regs<K, 64, 32, T, AND><<<grid_for(n * 64, 256), 256, 0, s>>>(a, lo, hi);
        break;
      default: {
        const unsigned grid = (unsigned)(n < 65536 ? n : 65536);
        k_sweep_block<K, T, AND><<<grid, kBlockThreads, 0, s>>>(a, lo, hi);
        break;
      }
    }
    ND_LAUNCHED();
  }
}

template <typename T>
void launch_typed(const KindState &ks, const SweepArgs &a, bool and_mode,
                  hipStream_t s) {
  if (!a.cap_by_tau) {
    // plain U on an arbitrary tau: r-cliques in no s-clique get H({}) = 0
    const int64_t lo = ks.bin_lo[kBinZero], hi = ks.bin_hi[kBinZero];
    if (hi > lo) {
      k_zero_range<T><<<grid_for(hi - lo, 256), 256, 0, s>>>((T *)a.tau_out, lo, hi);
      ND_LAUNCHED();
    }
  }
  switch (ks.k * 2 + (and_mode ? 1 : 0)) {
    case 2: launch_bins<1, T, false>(ks, a, s); break;
    case 3: launch_bins<1, T, true>(ks, a, s); break;
    case 4: launch_bins<2, T, false>(ks, a, s); break;
    case 5: launch_bins<2, T, true>(ks, a, s); break;
    case 6: launch_bins<3, T, false>(ks, a, s); break;
    case 7: launch_bins<3, T, true>(ks, a, s); break;
    default:
      ND_REQUIRE(false, ND_ERR_UNSUPPORTED, "no sweep kernel for k=%d", ks.k);
  }
}

}  // namespace

void launch_sweep(const KindState &ks, const SweepArgs &a, bool and_mode,
                  hipStream_t s) {
  if (ks.tau16)
    launch_typed<uint16_t>(ks, a, and_mode, s);
  else
    launch_typed<int32_t>(ks, a, and_mode, s);
}

}  // namespace nd
