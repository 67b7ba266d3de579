// levels.hip -- degree levels (Defn. 4): L_0 holds the r-cliques of minimum
// S-degree; removing them removes every s-clique that contains one of them;
// L_1 holds the minimum-degree r-cliques of what is left, and so on.  Their
// number bounds the sweeps SND needs (level i is exact after i sweeps), the
// DL row of Table 3.
//
// Levels form a chain (each depends on the previous removal) and power-law
// graphs have hundreds of thousands of small ones, so a level must cost
// microseconds, not a scan of everything still present.  Degree buckets make
// each level proportional to its own work:
//   * I[d]: the r-cliques whose initial degree is d (one sort, up front);
//   * B[d]: r-cliques whose degree dropped to d at the end of some level,
//     appended then.  A degree only falls, so an r-clique enters B[d] at most
//     once for each d below its initial degree: B[d] needs at most
//     #{R : d_s(R) > d} slots, P slots in all;
//   * hist[d]: how many r-cliques still present have degree d.
// Level i with minimum m: the members of I[m] (first visit of m only) and of
// B[m] past what earlier visits of m consumed that are still present with
// degree m form L_i -- every present r-clique of degree m is there, and stale
// entries (degree fell further, or removed) are skipped.  Peeling L_i walks
// its incidence lists: an s-clique still present (no member removed at an
// earlier level) is counted once, by its L_i member of smallest id, and
// lowers the degree of each member still present by one.  The next minimum
// is the first non-empty bucket of hist from min(lowest new degree, m + 1):
// everything not lowered in level i has degree above m.
//
// The loop over levels runs in one workgroup (barriers between the phases of
// a level cost far less than kernel launches): most levels are small, and
// their cost is the chain of dependent memory accesses of their phases.  A
// level with many candidates (kBigLevel, ND_LEVELS_BIG) would keep one CU
// busy for long while the others idle, so the workgroup stops before it,
// leaving its state in a control block; that level runs as four grid-wide
// kernels (collect, peel, re-bucket, finish), and the workgroup resumes.
// Every loop has a hard bound and an inconsistency ends it with an error
// flag rather than a hang.
#include <limits.h>
#include <stdlib.h>

#include <algorithm>
#include <vector>

#include "api_util.h"
#include "internal.h"

namespace nd {

namespace {

constexpr int kLvThreads = 1024;
constexpr int kLvWaves = kLvThreads / kWave;
// A level with this many candidates runs on the whole grid (measured on the
// Chung-Lu k-core and k-truss workloads: 512 to 16384 all within 10% of each
// other, every one 1.3-3x faster than the workgroup alone).
constexpr int64_t kBigLevel = kLvThreads;

struct LevelArgs {
  const int64_t *inc_off;  // internal numbering
  const int32_t *inc_ids;
  int64_t nr;
  int32_t maxd;
  int32_t m0;             // minimum initial degree
  int32_t *deg;           // current degree (starts at d_s)
  int32_t *lvl;           // level, -1 while present
  int32_t *hist;          // [maxd + 1] present r-cliques per degree
  const int32_t *I;       // r-cliques by initial degree
  const int64_t *Ioff;    // [maxd + 2]
  int32_t *B;             // re-bucketed r-cliques
  const int64_t *Boff;    // [maxd + 1]
  int64_t *Bcnt;          // [maxd + 1] entries appended
  int64_t *Bused;         // [maxd + 1] entries consumed
  uint8_t *Iused;         // [maxd + 1] I[d] consumed
  int32_t *moved_at;      // per r-clique: last level that lowered it
  int32_t *F;             // frontier (this level), nr slots
  int32_t *MV;            // r-cliques lowered in this level, nr slots
  int32_t *out;           // [0] = number of levels, [1] = error code
  struct LevelCtl *ctl;   // state between launches
  int64_t big;            // candidates from which a level runs grid-wide
};

// The level loop's state between launches.
struct LevelCtl {
  int64_t alive;       // r-cliques not yet removed
  int64_t ilo, ilen;   // candidates of the pending big level: I part
  int64_t blo, blen;   //   and B part
  int32_t m;           // current minimum degree
  int32_t level;       // next level number
  int32_t err;
  int32_t big;         // 1: the level `level` (minimum m) is pending
  int32_t nf, nmv, dmin;
  int32_t pad;
};

template <int K>
__global__ __launch_bounds__(kLvThreads) void k_levels(LevelArgs a) {
  __shared__ int32_t s_m, s_nf, s_nmv, s_dmin, s_err, s_level;
  __shared__ int64_t s_alive, s_ilo, s_ilen, s_blo, s_blen;
  const int t = threadIdx.x, lane = lane_id(), w = t / kWave;
  if (t == 0) {
    s_m = a.ctl->m;
    s_alive = a.ctl->alive;
    s_err = a.ctl->err;
    s_level = a.ctl->level;
  }
  __syncthreads();
  for (int64_t guard = 0; guard <= a.nr; guard++) {
    if (s_alive <= 0 || s_err) break;  // uniform: read after a barrier
    const int32_t m = s_m, level = s_level;
    // ---- collect L_level
    if (t == 0) {
      s_ilo = a.Ioff[m];
      s_ilen = a.Iused[m] ? 0 : a.Ioff[m + 1] - a.Ioff[m];
      s_blo = a.Boff[m] + a.Bused[m];
      s_blen = a.Bcnt[m] - a.Bused[m];
      s_nf = 0;
      s_nmv = 0;
      s_dmin = INT_MAX;
    }
    __syncthreads();
    const int64_t ilo = s_ilo, ilen = s_ilen, blo = s_blo, blen = s_blen;
    if (ilen + blen >= a.big) {  // uniform: leave this level to the grid
      if (t == 0) {
        LevelCtl &c = *a.ctl;
        c.ilo = ilo;
        c.ilen = ilen;
        c.blo = blo;
        c.blen = blen;
        c.nf = 0;
        c.nmv = 0;
        c.dmin = INT_MAX;
        c.big = 1;
      }
      break;
    }
    for (int64_t x = t; x < ilen + blen; x += kLvThreads) {
      const int32_t R = x < ilen ? a.I[ilo + x] : a.B[blo + (x - ilen)];
      if (a.deg[R] == m && atomicCAS(&a.lvl[R], -1, level) == -1)
        a.F[atomicAdd(&s_nf, 1)] = R;
    }
    __syncthreads();
    const int32_t nf = s_nf;
    if (nf == 0) {  // the minimum bucket must hold a present r-clique
      if (t == 0) s_err = 1;
      __syncthreads();
      break;
    }
    if (t == 0) {
      a.Iused[m] = 1;
      a.Bused[m] += blen;
    }
    // ---- peel: one wave per r-clique of L_level
    for (int f = w; f < nf; f += kLvWaves) {
      const int32_t R = a.F[f];
      const int64_t b = a.inc_off[R], d = a.inc_off[R + 1] - b;
      for (int64_t j = lane; j < d; j += kWave) {
        const int32_t *o = a.inc_ids + (int64_t)K * (b + j);
        bool skip = false;
#pragma unroll
        for (int x = 0; x < K; x++) {
          const int32_t l = a.lvl[o[x]];
          skip |= (l >= 0 && l < level) || (l == level && o[x] < R);
        }
        if (skip) continue;
#pragma unroll
        for (int x = 0; x < K; x++) {
          const int32_t q = o[x];
          if (a.lvl[q] >= 0) continue;
          const int32_t old = atomicSub(&a.deg[q], 1);
          if (old < 1 || old > a.maxd) {  // a present s-clique counts in deg
            s_err = 4;
            continue;
          }
          atomicSub(&a.hist[old], 1);
          atomicAdd(&a.hist[old - 1], 1);
          atomicMin(&s_dmin, old - 1);
          if (atomicExch(&a.moved_at[q], level) != level)
            a.MV[atomicAdd(&s_nmv, 1)] = q;
        }
      }
    }
    __syncthreads();
    // ---- re-bucket what was lowered, at its final degree of this level
    const int32_t nmv = s_nmv;
    for (int x = t; x < nmv; x += kLvThreads) {
      const int32_t q = a.MV[x];
      const int32_t dq = a.deg[q];
      if (dq < 0 || dq > a.maxd) {
        s_err = 5;
        continue;
      }
      const int64_t p = (int64_t)atomicAdd((unsigned long long *)&a.Bcnt[dq], 1ull);
      if (a.Boff[dq] + p < a.Boff[dq + 1])  // a bucket never overflows
        a.B[a.Boff[dq] + p] = q;
      else
        s_err = 6;
    }
    if (t == 0) {
      atomicSub(&a.hist[m], nf);
      s_alive -= nf;
      s_level = level + 1;
    }
    __syncthreads();
    // ---- next minimum: first non-empty bucket from min(dmin, m + 1)
    if (w == 0 && s_alive > 0) {
      const int32_t lo = min(s_dmin, m + 1);
      int32_t found = -1;
      for (int32_t base = lo; base <= a.maxd && found < 0; base += kWave) {
        const int32_t dd = base + lane;
        const bool hit = dd <= a.maxd && a.hist[dd] > 0;
        const uint64_t bal = ballot(hit);
        if (bal) found = base + __ffsll((long long)bal) - 1;
      }
      if (lane == 0) {
        if (found < 0)
          s_err = 2;
        else
          s_m = found;
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    LevelCtl &c = *a.ctl;
    c.m = s_m;
    c.alive = s_alive;
    c.level = s_level;
    c.err = s_err;
    a.out[0] = s_level;
    a.out[1] = s_err ? s_err : (s_alive > 0 && !c.big ? 3 : 0);
  }
}

// ---- a big level on the whole grid (the same steps, counters in *ctl)

__global__ void k_lv_collect(LevelArgs a) {
  const LevelCtl &c = *a.ctl;
  if (!c.big) return;
  const int32_t m = c.m, level = c.level;
  const int64_t n = c.ilen + c.blen;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int32_t R = x < c.ilen ? a.I[c.ilo + x] : a.B[c.blo + (x - c.ilen)];
    if (a.deg[R] == m && atomicCAS(&a.lvl[R], -1, level) == -1)
      a.F[atomicAdd(&a.ctl->nf, 1)] = R;
  }
}

template <int K>
__global__ __launch_bounds__(256) void k_lv_peel(LevelArgs a) {
  LevelCtl &c = *a.ctl;
  if (!c.big) return;
  const int32_t m = c.m, level = c.level, nf = c.nf;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (nf == 0) c.err = 1;  // the minimum bucket must hold a present r-clique
    a.Iused[m] = 1;
    a.Bused[m] += c.blen;
  }
  const int lane = lane_id();
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
  int32_t dmin = INT_MAX;
  for (int64_t f = wave; f < nf; f += nwaves) {
    const int32_t R = a.F[f];
    const int64_t b = a.inc_off[R], d = a.inc_off[R + 1] - b;
    for (int64_t j = lane; j < d; j += kWave) {
      const int32_t *o = a.inc_ids + (int64_t)K * (b + j);
      bool skip = false;
#pragma unroll
      for (int x = 0; x < K; x++) {
        const int32_t l = a.lvl[o[x]];
        skip |= (l >= 0 && l < level) || (l == level && o[x] < R);
      }
      if (skip) continue;
#pragma unroll
      for (int x = 0; x < K; x++) {
        const int32_t q = o[x];
        if (a.lvl[q] >= 0) continue;
        const int32_t old = atomicSub(&a.deg[q], 1);
        if (old < 1 || old > a.maxd) {
          c.err = 4;
          continue;
        }
        atomicSub(&a.hist[old], 1);
        atomicAdd(&a.hist[old - 1], 1);
        dmin = min(dmin, old - 1);
        if (atomicExch(&a.moved_at[q], level) != level)
          a.MV[atomicAdd(&c.nmv, 1)] = q;
      }
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) dmin = min(dmin, __shfl_xor(dmin, off, kWave));
  if (lane == 0 && dmin != INT_MAX) atomicMin(&c.dmin, dmin);
}

__global__ void k_lv_rebucket(LevelArgs a) {
  LevelCtl &c = *a.ctl;
  if (!c.big) return;
  const int32_t nmv = c.nmv;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < nmv;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int32_t q = a.MV[x];
    const int32_t dq = a.deg[q];
    if (dq < 0 || dq > a.maxd) {
      c.err = 5;
      continue;
    }
    const int64_t p = (int64_t)atomicAdd((unsigned long long *)&a.Bcnt[dq], 1ull);
    if (a.Boff[dq] + p < a.Boff[dq + 1])
      a.B[a.Boff[dq] + p] = q;
    else
      c.err = 6;
  }
}

// One wave: close the level and find the next minimum, the first
// non-empty bucket from min(lowest degree produced, m + 1).
__global__ void k_lv_finish(LevelArgs a) {
  LevelCtl &c = *a.ctl;
  if (!c.big) return;
  const int lane = lane_id();
  const int32_t m = c.m, nf = c.nf;
  const int64_t alive = c.alive - nf;
  if (lane == 0) a.hist[m] -= nf;
  __syncthreads();
  int32_t found = -1;
  if (alive > 0) {
    const int32_t lo = min(c.dmin, m + 1);
    for (int32_t base = lo; base <= a.maxd && found < 0; base += kWave) {
      const int32_t dd = base + lane;
      const uint64_t bal = ballot(dd <= a.maxd && a.hist[dd] > 0);
      if (bal) found = base + __ffsll((long long)bal) - 1;
    }
  }
  if (lane == 0) {
    if (alive > 0 && found < 0) c.err = 2;
    if (found >= 0) c.m = found;
    c.alive = alive;
    c.level += 1;
    c.big = 0;
  }
}

// keys[i] = d_s(i) << rb | i
__global__ void k_deg_keys(const int32_t *__restrict__ ds, int64_t nr, int rb,
                           uint64_t *__restrict__ keys) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nr) keys[i] = ((uint64_t)ds[i] << rb) | (uint64_t)i;
}

// From the degree-sorted keys: I (ids), and Ioff[d] = first position of
// degree >= d, for d = 0 .. maxd + 1.
__global__ void k_deg_buckets(const uint64_t *__restrict__ keys, int64_t nr,
                              int rb, int32_t maxd, int32_t *__restrict__ I,
                              int64_t *__restrict__ Ioff) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j > nr) return;
  const int32_t dj = j < nr ? (int32_t)(keys[j] >> rb) : maxd + 1;
  const int32_t dp = j > 0 ? (int32_t)(keys[j - 1] >> rb) : -1;
  for (int32_t d = dp + 1; d <= dj; d++) Ioff[d] = j;
  if (j < nr) I[j] = (int32_t)(keys[j] & (((uint64_t)1 << rb) - 1));
}

// hist[d] = |I[d]|; cap[d] = #{R : d_s(R) > d} = nr - Ioff[d + 1].
__global__ void k_deg_hist(const int64_t *__restrict__ Ioff, int64_t nr,
                           int32_t maxd, int32_t *__restrict__ hist,
                           int64_t *__restrict__ cap) {
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d > maxd) return;
  hist[d] = (int32_t)(Ioff[d + 1] - Ioff[d]);
  cap[d] = nr - Ioff[d + 1];
}

int bits_for(int64_t x) {
  int b = 1;
  while (b < 62 && ((int64_t)1 << b) <= x) b++;
  return b;
}

}  // namespace

nd_status levels(nd_graph *g, nd_kind kind, int32_t *level_out,
                 int32_t *num_levels, int on_device, hipStream_t s) {
  prepare(g, kind, s);
  const KindState &ks = g->ks[kind];
  Allocator &al = g->ctx->alloc;
  const int64_t nr = ks.nr;
  ND_REQUIRE(num_levels, ND_ERR_INVALID, "num_levels is NULL");
  ND_REQUIRE(level_out || nr == 0, ND_ERR_INVALID, "level is NULL");
  if (nr == 0) {
    *num_levels = 0;
    return ND_OK;
  }
  const int32_t maxd = ks.max_ds;
  const int rb = bits_for(nr - 1);
  ND_REQUIRE(rb + bits_for(maxd + 1) <= 64, ND_ERR_UNSUPPORTED,
             "degree-level keys do not fit 64 bits");
  DArr<int32_t> deg(al, nr), lvl(al, nr), I(al, nr), moved(al, nr), F(al, nr),
      MV(al, nr), hist(al, maxd + 1), out(al, 2);
  DArr<int64_t> Ioff(al, maxd + 2), cap(al, maxd + 1), Boff(al, maxd + 2),
      Bcnt(al, maxd + 1), Bused(al, maxd + 1);
  DArr<uint8_t> Iused(al, maxd + 1);
  {
    DArr<uint64_t> keys(al, nr), tmp(al, nr);
    k_deg_keys<<<grid_for(nr, 256), 256, 0, s>>>(ks.ds.p, nr, rb, keys.p);
    ND_LAUNCHED();
    const uint64_t *sorted =
        radix_sort_u64(keys.p, tmp.p, nr, rb, rb + bits_for(maxd + 1), s, al);
    k_deg_buckets<<<grid_for(nr + 1, 256), 256, 0, s>>>(sorted, nr, rb, maxd,
                                                         I.p, Ioff.p);
    ND_LAUNCHED();
  }
  k_deg_hist<<<grid_for(maxd + 1, 256), 256, 0, s>>>(Ioff.p, nr, maxd, hist.p,
                                                      cap.p);
  ND_LAUNCHED();
  exclusive_scan_i64(cap.p, Boff.p, maxd + 1, s, al);
  const int64_t btotal = read_i64(Boff.p + maxd + 1, s);  // = P
  DArr<int32_t> B(al, std::max<int64_t>(btotal, 1));
  ND_HIP(hipMemcpyAsync(deg.p, ks.ds.p, sizeof(int32_t) * nr,
                        hipMemcpyDeviceToDevice, s));
  fill_i32(lvl.p, -1, nr, s);
  fill_i32(moved.p, -1, nr, s);
  fill_u64((uint64_t *)Bcnt.p, 0, maxd + 1, s);
  fill_u64((uint64_t *)Bused.p, 0, maxd + 1, s);
  fill_u8(Iused.p, 0, maxd + 1, s);
  fill_i32(out.p, 0, 2, s);
  // minimum initial degree: the first non-empty bucket
  std::vector<int64_t> hoff(maxd + 2);
  ND_HIP(hipMemcpyAsync(hoff.data(), Ioff.p, sizeof(int64_t) * (maxd + 2),
                        hipMemcpyDeviceToHost, s));
  ND_HIP(hipStreamSynchronize(s));
  int32_t m0 = 0;
  while (m0 <= maxd && hoff[m0 + 1] == hoff[m0]) m0++;
  ND_REQUIRE(m0 <= maxd, ND_ERR_DEVICE, "degree buckets are empty");
  DArr<LevelCtl> ctl(al, 1);
  LevelCtl c0{};
  c0.alive = nr;
  c0.m = m0;
  ND_HIP(hipMemcpyAsync(ctl.p, &c0, sizeof c0, hipMemcpyHostToDevice, s));
  LevelArgs a{};
  a.ctl = ctl.p;
  a.big = kBigLevel;
  if (const char *v = getenv("ND_LEVELS_BIG")) a.big = std::max<int64_t>(1, atoll(v));
  a.inc_off = ks.inc_off.p;
  a.inc_ids = ks.inc_ids.p;
  a.nr = nr;
  a.maxd = maxd;
  a.m0 = m0;
  a.deg = deg.p;
  a.lvl = lvl.p;
  a.hist = hist.p;
  a.I = I.p;
  a.Ioff = Ioff.p;
  a.B = B.p;
  a.Boff = Boff.p;
  a.Bcnt = Bcnt.p;
  a.Bused = Bused.p;
  a.Iused = Iused.p;
  a.moved_at = moved.p;
  a.F = F.p;
  a.MV = MV.p;
  a.out = out.p;
  ND_REQUIRE(ks.k == 1 || ks.k == 2 || ks.k == 3 || ks.k == 5, ND_ERR_UNSUPPORTED,
             "no level kernel for k=%d", ks.k);
  const unsigned grid = (unsigned)g->ctx->num_cu * 8;
  PinnedChunk pc;
  const LevelCtl *hc = nullptr;
  // the workgroup runs levels until it finishes or meets a big one, which
  // the grid then runs; each round removes at least one level
  for (int64_t round = 0; round <= nr; round++) {
    switch (ks.k) {
      case 1: k_levels<1><<<1, kLvThreads, 0, s>>>(a); break;
      case 2: k_levels<2><<<1, kLvThreads, 0, s>>>(a); break;
      case 3: k_levels<3><<<1, kLvThreads, 0, s>>>(a); break;
      default: k_levels<5><<<1, kLvThreads, 0, s>>>(a); break;
    }
    ND_LAUNCHED();
    hc = pc.read(ctl.p, 1, s);
    ND_REQUIRE(hc->err == 0, ND_ERR_DEVICE,
               "degree levels: inconsistent buckets (code %d)", hc->err);
    if (!hc->big) break;
    k_lv_collect<<<grid, 256, 0, s>>>(a);
    ND_LAUNCHED();
    switch (ks.k) {
      case 1: k_lv_peel<1><<<grid, 256, 0, s>>>(a); break;
      case 2: k_lv_peel<2><<<grid, 256, 0, s>>>(a); break;
      case 3: k_lv_peel<3><<<grid, 256, 0, s>>>(a); break;
      default: k_lv_peel<5><<<grid, 256, 0, s>>>(a); break;
    }
    ND_LAUNCHED();
    k_lv_rebucket<<<grid, 256, 0, s>>>(a);
    ND_LAUNCHED();
    k_lv_finish<<<1, kWave, 0, s>>>(a);
    ND_LAUNCHED();
  }
  ND_REQUIRE(hc && !hc->big && hc->alive == 0, ND_ERR_DEVICE,
             "degree levels: %lld r-cliques left without a level",
             hc ? (long long)hc->alive : (long long)nr);
  *num_levels = hc->level;
  if (on_device) {
    to_original(ks, lvl.p, 4, level_out, s);
  } else {
    DArr<int32_t> o(al, nr);
    to_original(ks, lvl.p, 4, o.p, s);
    ND_HIP(hipMemcpyAsync(level_out, o.p, sizeof(int32_t) * nr,
                          hipMemcpyDeviceToHost, s));
  }
  ND_HIP(hipStreamSynchronize(s));
  return ND_OK;
}

}  // namespace nd

using namespace nd;

extern "C" nd_status nd_levels(nd_graph *g, nd_kind kind, int32_t *level,
                               int32_t *num_levels, int on_device,
                               void *stream) {
  nd_status out = ND_OK;
  nd_status st = guarded([&] {
    ND_REQUIRE(g, ND_ERR_INVALID, "graph is NULL");
    ND_HIP(hipSetDevice(g->ctx->device));
    StreamScope scope((hipStream_t)stream);
    out = levels(g, kind, level, num_levels, on_device, (hipStream_t)stream);
  });
  return st != ND_OK ? st : out;
}
