// partial.hip -- ego-network estimates by PartialAND (the set-restricted AND
// of Section 4.3, end, applied as in Section 5.3): for a
// query r-clique q, AND recomputes only the r-cliques of
//   P(q) = {q} + every r-clique sharing an s-clique with q
// (for k-core: q and its neighbours; for k-truss: q and the other edges of
// its triangles), every other r-clique keeping tau_0 = d_s, until a sweep
// changes nothing; the estimate is q's resulting value, an upper bound on
// kappa(q).
//
// The restricted operator is monotone and tau_0 lies above its image, so
// in-place sweeps in any order reach the same limit -- the largest fixed
// point below tau_0 -- and each query's result is deterministic although the
// sweeps inside a workgroup race.
//
// Many queries run in one launch, one workgroup each (the many-small-
// problems shape of serving): P(q) is sorted into LDS together with the
// members' current values; a gathered id is looked up there by binary search
// and, when absent, read as d_s from global memory.  One wave recomputes one
// member at a time, its rho values in registers (d_s <= 2048) or re-gathered
// per probe of the h-index search (larger d_s).  Queries whose P(q) does not
// fit the LDS table run one at a time through the global sweep kernels.
#include <limits.h>
#include <string.h>

#include <vector>

#include "api_util.h"
#include "internal.h"
#include "sweep_dev.h"

namespace nd {

nd_status decompose_impl(nd_graph *g, nd_kind kind, const nd_opts *opts_in,
                         int32_t *kappa, int on_device, hipStream_t s,
                         nd_result *res, const uint8_t *fixed_set);

namespace {

using namespace dev;

constexpr int kEgoCap = 4096;      // members of P(q) held in LDS
constexpr int kEgoThreads = 256;   // 4 waves
constexpr int kEgoWaves = kEgoThreads / kWave;

struct EgoArgs {
  const int64_t *inc_off;  // internal numbering
  const int32_t *inc_ids;
  const int32_t *ds;
  const int32_t *inv;      // original id -> internal id
  const int32_t *queries;  // original ids, already range-checked
  int64_t count;
  int32_t max_iters;
  int32_t *est;            // per query; -1 when P(q) is too large
  int32_t *sweeps;         // per query
  uint8_t *big;            // per query: 1 = run it through the fallback
  int32_t *not_converged;  // set when a query stopped at max_iters
};

__device__ __forceinline__ int ego_find(const int32_t *mem, int np, int32_t x) {
  int lo = 0, hi = np;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (mem[mid] < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < np && mem[lo] == x) ? lo : -1;
}

// Current value of r-clique x: its LDS slot when x is in P(q), else d_s.
__device__ __forceinline__ int32_t ego_val(const int32_t *mem, int32_t *tl,
                                           int np, const int32_t *ds,
                                           int32_t x) {
  const int p = ego_find(mem, np, x);
  return p >= 0 ? __hip_atomic_load(&tl[p], __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_WORKGROUP)
                : ds[x];
}

template <int K>
__device__ __forceinline__ int32_t ego_rho(const EgoArgs &a, const int32_t *mem,
                                           int32_t *tl, int np, int64_t j) {
  const int32_t *q = a.inc_ids + (int64_t)K * j;
  int32_t v = ego_val(mem, tl, np, a.ds, q[0]);
#pragma unroll
  for (int x = 1; x < K; x++) v = min(v, ego_val(mem, tl, np, a.ds, q[x]));
  return v;
}

__device__ __forceinline__ int wave_sum(int x) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
  return x;
}

// Ascending bitonic sort of v[0..n), n a power of two, by the whole block.
__device__ void block_bitonic(int32_t *v, int n) {
  for (int k = 2; k <= n; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int l = i ^ j;
        if (l > i) {
          const bool up = (i & k) == 0;
          const int32_t x = v[i], y = v[l];
          if ((x > y) == up) {
            v[i] = y;
            v[l] = x;
          }
        }
      }
      __syncthreads();
    }
  }
}

template <int K>
__global__ __launch_bounds__(kEgoThreads) void k_ego(EgoArgs a) {
  __shared__ int32_t mem[kEgoCap];
  __shared__ int32_t tl[kEgoCap];
  __shared__ int32_t wsum[kEgoWaves];
  __shared__ int s_np, s_changed;
  const int t = threadIdx.x, lane = lane_id(), w = t / kWave;
  for (int64_t qi = blockIdx.x; qi < a.count; qi += gridDim.x) {
    const int32_t R0 = a.inv[a.queries[qi]];
    const int64_t b0 = a.inc_off[R0];
    const int64_t d0 = a.inc_off[R0 + 1] - b0;
    const int64_t nraw = 1 + (int64_t)K * d0;
    if (nraw > kEgoCap) {  // uniform over the block
      if (t == 0) {
        a.big[qi] = 1;
        a.est[qi] = -1;
        a.sweeps[qi] = 0;
      }
      continue;
    }
    int n2 = 1;
    while (n2 < nraw) n2 <<= 1;
    for (int i = t; i < n2; i += kEgoThreads)
      mem[i] = i == 0 ? R0 : (i < nraw ? a.inc_ids[(int64_t)K * b0 + i - 1]
                                       : INT_MAX);
    __syncthreads();
    block_bitonic(mem, n2);
    // drop repeats (none arise from a simple graph, kept for safety): keep
    // the first of each run, compacted through tl
    int keep_cnt = 0;
    const int per = (n2 + kEgoThreads - 1) / kEgoThreads;
    const int lo = min(n2, t * per), hi = min(n2, lo + per);
    for (int i = lo; i < hi; i++)
      keep_cnt += mem[i] != INT_MAX && (i == 0 || mem[i] != mem[i - 1]);
    // block exclusive scan of keep_cnt
    int incl = keep_cnt;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const int y = __shfl_up(incl, off, kWave);
      if (lane >= off) incl += y;
    }
    if (lane == kWave - 1) wsum[w] = incl;
    __syncthreads();
    int base = 0;
    for (int q = 0; q < w; q++) base += wsum[q];
    int pos = base + incl - keep_cnt;
    for (int i = lo; i < hi; i++)
      if (mem[i] != INT_MAX && (i == 0 || mem[i] != mem[i - 1])) tl[pos++] = mem[i];
    if (t == kEgoThreads - 1) s_np = base + incl;
    __syncthreads();
    const int np = s_np;
    for (int i = t; i < np; i += kEgoThreads) mem[i] = tl[i];
    __syncthreads();
    for (int i = t; i < np; i += kEgoThreads) tl[i] = a.ds[mem[i]];
    __syncthreads();

    int sweeps = 0;
    bool changed_last = true;
    while (sweeps < a.max_iters) {
      if (t == 0) s_changed = 0;
      __syncthreads();
      for (int i = w; i < np; i += kEgoWaves) {
        const int32_t R = mem[i];
        const int64_t b = a.inc_off[R];
        const int64_t d = a.inc_off[R + 1] - b;
        const int32_t c = __hip_atomic_load(&tl[i], __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_WORKGROUP);
        int32_t h;
        if (d <= (int64_t)kWave * 32) {
          int32_t rho[32];
#pragma unroll
          for (int m = 0; m < 32; m++) {
            const int64_t j = lane + (int64_t)m * kWave;
            rho[m] = j < d ? ego_rho<K>(a, mem, tl, np, b + j) : -1;
          }
          const int cnt = count_ge<kWave, 32>(rho, c);
          h = cnt >= c ? c : hindex_search<kWave, 32>(rho, c);
        } else {
          // long list: count #{rho >= x} by a fresh pass per probe
          auto count = [&](int32_t x) {
            int n = 0;
            for (int64_t j = lane; j < d; j += kWave)
              n += ego_rho<K>(a, mem, tl, np, b + j) >= x;
            return wave_sum(n);
          };
          if (count(c) >= c) {
            h = c;
          } else {
            int32_t l = 0, r = c - 1;
            while (l < r) {
              const int32_t mid = (l + r + 1) >> 1;
              if (count(mid) >= mid)
                l = mid;
              else
                r = mid - 1;
            }
            h = l;
          }
        }
        if (lane == 0 && h != c) {
          __hip_atomic_store(&tl[i], h, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
          s_changed = 1;
        }
      }
      __syncthreads();
      sweeps++;
      changed_last = s_changed != 0;
      __syncthreads();
      if (!changed_last) break;
    }
    if (t == 0) {
      a.est[qi] = tl[ego_find(mem, np, R0)];
      a.sweeps[qi] = sweeps;
      if (changed_last) *a.not_converged = 1;
    }
    __syncthreads();
  }
}

__global__ void k_check_queries(const int32_t *__restrict__ q, int64_t count,
                                int64_t nr, int32_t *__restrict__ err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count && (q[i] < 0 || q[i] >= nr)) *err = 1;
}

// mark[R0] = 1 and mark[x] = 1 for every id x in R0's incidence list.
__global__ void k_mark_ego(const int64_t *__restrict__ inc_off,
                           const int32_t *__restrict__ inc_ids, int k,
                           int32_t R0, uint8_t *__restrict__ mark) {
  const int64_t b = inc_off[R0] * k, e = inc_off[R0 + 1] * k;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) mark[R0] = 1;
  if (b + i < e) mark[inc_ids[b + i]] = 1;
}

}  // namespace

nd_status ego_estimate(nd_graph *g, nd_kind kind, const int32_t *queries,
                       int64_t count, int32_t max_iters, int32_t *est,
                       int32_t *sweeps, int on_device, hipStream_t s) {
  ND_REQUIRE(count >= 0 && (count == 0 || (queries && est)), ND_ERR_INVALID,
             "bad query list");
  prepare(g, kind, s);
  const KindState &ks = g->ks[kind];
  Allocator &al = g->ctx->alloc;
  if (count == 0) return ND_OK;
  if (max_iters < 0) max_iters = INT_MAX;
  DArr<int32_t> dq(al, count), dest(al, count), dsw(al, count), flags(al, 2);
  DArr<uint8_t> big(al, count);
  ND_HIP(hipMemcpyAsync(dq.p, queries, sizeof(int32_t) * count,
                        on_device ? hipMemcpyDeviceToDevice
                                  : hipMemcpyHostToDevice, s));
  fill_i32(flags.p, 0, 2, s);
  fill_u8(big.p, 0, count, s);
  k_check_queries<<<grid_for(count, 256), 256, 0, s>>>(dq.p, count, ks.nr,
                                                        flags.p);
  ND_LAUNCHED();
  int32_t herr[2] = {0, 0};
  ND_HIP(hipMemcpyAsync(herr, flags.p, sizeof herr, hipMemcpyDeviceToHost, s));
  ND_HIP(hipStreamSynchronize(s));
  ND_REQUIRE(herr[0] == 0, ND_ERR_INVALID,
             "a query id is outside [0, %lld)", (long long)ks.nr);
  EgoArgs a{};
  a.inc_off = ks.inc_off.p;
  a.inc_ids = ks.inc_ids.p;
  a.ds = ks.ds.p;
  a.inv = ks.inv.p;
  a.queries = dq.p;
  a.count = count;
  a.max_iters = max_iters;
  a.est = dest.p;
  a.sweeps = dsw.p;
  a.big = big.p;
  a.not_converged = flags.p + 1;
  const unsigned grid =
      (unsigned)std::min<int64_t>(count, (int64_t)g->ctx->num_cu * 8);
  switch (ks.k) {
    case 1: k_ego<1><<<grid, kEgoThreads, 0, s>>>(a); break;
    case 2: k_ego<2><<<grid, kEgoThreads, 0, s>>>(a); break;
    case 3: k_ego<3><<<grid, kEgoThreads, 0, s>>>(a); break;
    case 5: k_ego<5><<<grid, kEgoThreads, 0, s>>>(a); break;
    default: ND_REQUIRE(false, ND_ERR_UNSUPPORTED, "no ego kernel for k=%d", ks.k);
  }
  ND_LAUNCHED();
  std::vector<int32_t> hq(count), he(count), hs(count);
  std::vector<uint8_t> hb(count);
  ND_HIP(hipMemcpyAsync(hq.data(), dq.p, sizeof(int32_t) * count,
                        hipMemcpyDeviceToHost, s));
  ND_HIP(hipMemcpyAsync(he.data(), dest.p, sizeof(int32_t) * count,
                        hipMemcpyDeviceToHost, s));
  ND_HIP(hipMemcpyAsync(hs.data(), dsw.p, sizeof(int32_t) * count,
                        hipMemcpyDeviceToHost, s));
  ND_HIP(hipMemcpyAsync(hb.data(), big.p, count, hipMemcpyDeviceToHost, s));
  ND_HIP(hipMemcpyAsync(herr, flags.p, sizeof herr, hipMemcpyDeviceToHost, s));
  ND_HIP(hipStreamSynchronize(s));
  bool not_conv = herr[1] != 0;
  // queries whose ego network does not fit one workgroup's table
  std::vector<int32_t> inv_h;
  for (int64_t i = 0; i < count; i++) {
    if (!hb[i]) continue;
    if (inv_h.empty()) {
      inv_h.resize(ks.nr);
      ND_HIP(hipMemcpyAsync(inv_h.data(), ks.inv.p, sizeof(int32_t) * ks.nr,
                            hipMemcpyDeviceToHost, s));
      ND_HIP(hipStreamSynchronize(s));
    }
    const int32_t R0 = inv_h[hq[i]];
    DArr<uint8_t> mark(al, ks.nr);
    fill_u8(mark.p, 0, ks.nr, s);
    int64_t hoff[2];
    ND_HIP(hipMemcpyAsync(hoff, ks.inc_off.p + R0, sizeof hoff,
                          hipMemcpyDeviceToHost, s));
    ND_HIP(hipStreamSynchronize(s));
    const int64_t len = (hoff[1] - hoff[0]) * ks.k;
    k_mark_ego<<<grid_for(std::max<int64_t>(len, 1), 256), 256, 0, s>>>(
        ks.inc_off.p, ks.inc_ids.p, ks.k, R0, mark.p);
    ND_LAUNCHED();
    DArr<int32_t> full(al, ks.nr);
    nd_opts o;
    nd_opts_init(&o);
    o.max_iters = max_iters;
    nd_result r{};
    const nd_status st = decompose_impl(g, kind, &o, full.p, 1, s, &r, mark.p);
    if (st == ND_ERR_NOT_CONVERGED)
      not_conv = true;
    else if (st != ND_OK)
      return st;
    ND_HIP(hipMemcpyAsync(&he[i], full.p + hq[i], sizeof(int32_t),
                          hipMemcpyDeviceToHost, s));
    ND_HIP(hipStreamSynchronize(s));
    hs[i] = r.sweeps;
  }
  if (on_device) {
    ND_HIP(hipMemcpyAsync(est, he.data(), sizeof(int32_t) * count,
                          hipMemcpyHostToDevice, s));
    if (sweeps)
      ND_HIP(hipMemcpyAsync(sweeps, hs.data(), sizeof(int32_t) * count,
                            hipMemcpyHostToDevice, s));
  } else {
    memcpy(est, he.data(), sizeof(int32_t) * count);
    if (sweeps) memcpy(sweeps, hs.data(), sizeof(int32_t) * count);
  }
  ND_HIP(hipStreamSynchronize(s));
  if (not_conv) {
    set_error("a query stopped at max_iters without converging");
    return ND_ERR_NOT_CONVERGED;
  }
  return ND_OK;
}

}  // namespace nd

using namespace nd;

extern "C" nd_status nd_ego_estimate(nd_graph *g, nd_kind kind,
                                     const int32_t *queries, int64_t count,
                                     int32_t max_iters, int32_t *est,
                                     int32_t *sweeps, int on_device,
                                     void *stream) {
  nd_status out = ND_OK;
  nd_status st = guarded([&] {
    ND_REQUIRE(g, ND_ERR_INVALID, "graph is NULL");
    ND_HIP(hipSetDevice(g->ctx->device));
    StreamScope scope((hipStream_t)stream);
    out = ego_estimate(g, kind, queries, count, max_iters, est, sweeps,
                       on_device, (hipStream_t)stream);
  });
  return st != ND_OK ? st : out;
}
