// common.h -- shared host/device helpers for the gfx950 nucleus-decomposition
// library.  Internal header: not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>
#include <stdint.h>

#include <exception>
#include <string>

#include "../../include/nd.h"

namespace nd {

constexpr int kWave = 64;  // CDNA wavefront width

// ------------------------------------------------------------ error state

void set_error(const char *fmt, ...) __attribute__((format(printf, 1, 2)));

// Status carrier used inside the library; converted to nd_status at the ABI.
struct Err {
  nd_status code;
  explicit Err(nd_status c) : code(c) {}
};

// A HIP runtime call; failures (and C++ exceptions escaping the runtime)
// become an Err naming the call site.
#define ND_HIP(call)                                                        \
  do {                                                                      \
    hipError_t e_;                                                          \
    try {                                                                   \
      e_ = (call);                                                          \
    } catch (const std::exception &x_) {                                    \
      ::nd::set_error("%s threw at %s:%d: %s", #call, __FILE__, __LINE__,  \
                      x_.what());                                           \
      throw ::nd::Err(ND_ERR_DEVICE);                                       \
    }                                                                       \
    if (e_ != hipSuccess) {                                                 \
      ::nd::set_error("%s failed at %s:%d: %s", #call, __FILE__, __LINE__, \
                      hipGetErrorString(e_));                               \
      throw ::nd::Err(e_ == hipErrorOutOfMemory ? ND_ERR_OOM                \
                                                : ND_ERR_DEVICE);           \
    }                                                                       \
  } while (0)

#define ND_REQUIRE(cond, code, ...) \
  do {                              \
    if (!(cond)) {                  \
      ::nd::set_error(__VA_ARGS__); \
      throw ::nd::Err(code);        \
    }                               \
  } while (0)

// After a launch: surface launch-configuration errors immediately.
#define ND_LAUNCHED() ND_HIP(hipGetLastError())

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// A named range around a phase of the path (graph build, enumeration,
// incidence, layout, sweeps, output) for profilers that collect markers
// (rocprofv3 --marker-trace); nothing happens when none listens.
struct Phase {
  explicit Phase(const char *name) { roctxRangePushA(name); }
  ~Phase() { roctxRangePop(); }
  Phase(const Phase &) = delete;
  Phase &operator=(const Phase &) = delete;
};

// The (r,s) of every nd_kind and k = C(s,r) - 1, the number of other
// r-cliques listed per s-clique.
constexpr int kNumKinds = 5;
struct KindRS {
  int r, s, k;
};
inline bool kind_valid(int kind) { return kind >= 0 && kind < kNumKinds; }
inline KindRS kind_rs(int kind) {
  constexpr KindRS t[kNumKinds] = {
      {1, 2, 1},  // ND_KCORE
      {2, 3, 2},  // ND_KTRUSS
      {3, 4, 3},  // ND_NUCLEUS34
      {1, 3, 2},  // ND_NUCLEUS13
      {2, 4, 5},  // ND_NUCLEUS24
  };
  return t[kind];
}

// Grid size for `items` work items at `per_block` items per block, at least 1.
inline unsigned grid_for(int64_t items, int64_t per_block) {
  int64_t g = ceil_div(items, per_block);
  return (unsigned)(g < 1 ? 1 : g);
}

// Workgroups of 256 threads for `items` work items of `lanes` lanes each,
// at most kMaxStrideBlocks (2^28 threads).  Kernels launched with it stride
// over the items, so no launch exceeds the 32-bit dispatch size however many
// items there are (the (3,4) builders reach 4*10^8 triangles x 64 lanes).
constexpr int64_t kMaxStrideBlocks = 1 << 20;
inline unsigned grid_stride(int64_t items, int64_t lanes) {
  const int64_t g = ceil_div(items * lanes, 256);
  return (unsigned)(g < 1 ? 1 : g > kMaxStrideBlocks ? kMaxStrideBlocks : g);
}

// --------------------------------------------------------- device helpers

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Number of set bits of `mask` below this lane.
__device__ __forceinline__ int lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// First index in the ascending array a[lo, hi) whose value is >= x.
template <typename T>
__device__ __forceinline__ int64_t lower_bound(const T *__restrict__ a,
                                               int64_t lo, int64_t hi, T x) {
  while (lo < hi) {
    int64_t mid = lo + ((hi - lo) >> 1);
    if (a[mid] < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

}  // namespace nd
