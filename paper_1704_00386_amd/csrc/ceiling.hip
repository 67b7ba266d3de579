// ceiling.hip -- measurement kernels for the ceilings the benchmark reports
// beside the sweep's fraction of HBM peak.  Not part of the method and not
// linked into libnd.so: built as libndceil.so and loaded by the benchmark
// only.
//
//   ndc_read      streams n bytes (16-byte loads, summed): the achievable
//                 read bandwidth;
//   ndc_copy      copies n bytes (16-byte loads and stores);
//   ndc_gather    for every s-clique j: min over its k listed ids of tau[id]
//                 (tau 8-, 16- or 32-bit), summed -- the id stream and the random
//                 tau gathers of one sweep without the h-index: the ceiling of
//                 the gather pattern itself.  Each workgroup takes contiguous
//                 runs of the id stream (the mapping of the update kernel's
//                 full sweeps, which lets a CU's cache serve the values that
//                 neighbouring lists share); with the whole grid striding
//                 over the stream instead, the same gathers take about 1.7x
//                 longer on the block-model (3,4) workload.
// Each enqueues one kernel on `stream` between two events of its own and
// returns the kernel's device time in milliseconds (negative on error).
// The sums go to *sink so that no load is optimised away.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ void sink_add(unsigned long long *sink,
                                         unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if (__lane_id() == 0 && v) atomicAdd(sink, v);
}

__global__ __launch_bounds__(kThreads) void k_read(const uint4 *__restrict__ p,
                                                   int64_t n16,
                                                   unsigned long long *sink) {
  unsigned long long s = 0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n16;
       i += (int64_t)gridDim.x * kThreads) {
    const uint4 v = p[i];
    s += v.x ^ v.y ^ v.z ^ v.w;
  }
  sink_add(sink, s);
}

__global__ __launch_bounds__(kThreads) void k_copy(const uint4 *__restrict__ a,
                                                   uint4 *__restrict__ b,
                                                   int64_t n16) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n16;
       i += (int64_t)gridDim.x * kThreads)
    b[i] = a[i];
}

constexpr int64_t kGatherRun = 32768;  // s-cliques per workgroup run

template <int K, typename T>
__global__ __launch_bounds__(kThreads) void k_gather(
    const int32_t *__restrict__ ids, int64_t nsets, const T *__restrict__ tau,
    unsigned long long *sink) {
  unsigned long long s = 0;
  for (int64_t r = (int64_t)blockIdx.x * kGatherRun; r < nsets;
       r += (int64_t)gridDim.x * kGatherRun) {
    const int64_t end = r + kGatherRun < nsets ? r + kGatherRun : nsets;
    for (int64_t j = r + threadIdx.x; j < end; j += kThreads) {
      const int32_t *q = ids + K * j;
      uint32_t m = 0xffffffffu;
#pragma unroll
      for (int x = 0; x < K; x++) m = min(m, (uint32_t)tau[q[x]]);
      s += m;
    }
  }
  sink_add(sink, s);
}

template <class F>
float timed(hipStream_t s, F &&launch) {
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return -1;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return -1;
  }
  float ms = -1;
  if (hipEventRecord(a, s) == hipSuccess) {
    launch();
    if (hipGetLastError() == hipSuccess && hipEventRecord(b, s) == hipSuccess &&
        hipEventSynchronize(b) == hipSuccess)
      (void)hipEventElapsedTime(&ms, a, b);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return ms;
}

template <typename T>
struct Tag {
  using type = T;
};

unsigned grid_of(int64_t items, int cus) {
  const int64_t g = (items + kThreads - 1) / kThreads;
  const int64_t cap = (int64_t)cus * 32;
  return (unsigned)(g < 1 ? 1 : g > cap ? cap : g);
}

int num_cus() {
  int dev = 0, cu = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev);
  return cu > 0 ? cu : 256;
}

}  // namespace

extern "C" {

// bytes must be a multiple of 16 and p 16-byte aligned.
float ndc_read(const void *p, int64_t bytes, unsigned long long *sink,
               void *stream) {
  if (!p || bytes < 16 || bytes % 16 || !sink) return -1;
  const int64_t n16 = bytes / 16;
  hipStream_t s = (hipStream_t)stream;
  return timed(s, [&] {
    k_read<<<grid_of(n16, num_cus()), kThreads, 0, s>>>((const uint4 *)p, n16,
                                                        sink);
  });
}

float ndc_copy(const void *src, void *dst, int64_t bytes, void *stream) {
  if (!src || !dst || bytes < 16 || bytes % 16) return -1;
  const int64_t n16 = bytes / 16;
  hipStream_t s = (hipStream_t)stream;
  return timed(s, [&] {
    k_copy<<<grid_of(n16, num_cus()), kThreads, 0, s>>>((const uint4 *)src,
                                                        (uint4 *)dst, n16);
  });
}

// ids[k * nsets] (every id a valid index of tau), tau of tau_bytes 1, 2 or
// 4 bytes per value (8- and 16-bit unsigned, 32-bit signed); k in {1, 2, 3}.
float ndc_gather(const int32_t *ids, int64_t nsets, int k, const void *tau,
                 int tau_bytes, unsigned long long *sink, void *stream) {
  if (!ids || !tau || !sink || nsets < 1 || k < 1 || k > 3) return -1;
  if (tau_bytes != 1 && tau_bytes != 2 && tau_bytes != 4) return -1;
  hipStream_t s = (hipStream_t)stream;
  const int64_t runs = (nsets + kGatherRun - 1) / kGatherRun;
  const int64_t cap = (int64_t)num_cus() * 8;
  const unsigned grid = (unsigned)(runs < cap ? runs : cap);
  auto go = [&](auto kc, auto tc) {
    constexpr int K = decltype(kc)::value;
    using T = typename decltype(tc)::type;
    k_gather<K, T><<<grid, kThreads, 0, s>>>(ids, nsets, (const T *)tau, sink);
  };
  auto by_type = [&](auto kc) {
    if (tau_bytes == 1) go(kc, Tag<uint8_t>{});
    else if (tau_bytes == 2) go(kc, Tag<uint16_t>{});
    else go(kc, Tag<int32_t>{});
  };
  return timed(s, [&] {
    if (k == 1) by_type(std::integral_constant<int, 1>{});
    else if (k == 2) by_type(std::integral_constant<int, 2>{});
    else by_type(std::integral_constant<int, 3>{});
  });
}

}  // extern "C"
