// la_probe.hip -- plain HBM streams (read, write, copy).
//
// The attention kernels are bound by HBM traffic with a fixed mix of reads
// and writes (the summary reads only; the apply reads one tensor and writes
// one; the key backward reads two and writes two).  These three streams
// measure what a plain kernel of each mix reaches on the device at hand, so
// the attention kernels' rates can be read against a ceiling measured the
// same way rather than only against the nominal peak.  Reads and writes
// stream a contiguous chunk per wave (16-byte words, four in flight per
// lane); the copy sweeps the buffer with the whole grid, the form of the
// apply and key-backward kernels; in both the words past the last whole
// chunk or block are spread over all lanes.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/la.h"
#include "la_profile.h"

namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;   // four waves per workgroup
constexpr int kUnroll = 4;      // words in flight per lane
constexpr int64_t kStep = 64 * kUnroll;

struct Split {
  int64_t per_wave;  // words per wave, a multiple of kStep
  int64_t waves;     // waves with a chunk
  int64_t n;         // all words
};

template <bool NT>
__device__ __forceinline__ u32x4 load_word(const u32x4* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

template <bool NT>
__device__ __forceinline__ void store_word(u32x4 v, u32x4* p) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// the words [waves * per_wave, n), spread over every lane of the grid
__device__ __forceinline__ int64_t tail_begin(const Split& s) {
  return s.waves * s.per_wave + (int64_t)blockIdx.x * kThreads + threadIdx.x;
}

// Reads every word.  The XOR of a lane's words is stored only if it equals
// `key`, a value the host picks and never expects, so the loads stay live
// while (almost surely) nothing is written.
template <bool NT>
__global__ __launch_bounds__(kThreads) void stream_read_kernel(const u32x4* __restrict__ src, Split s,
                                                               u32x4 key, u32x4* __restrict__ sink) {
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  u32x4 acc = {0u, 0u, 0u, 0u};
  if (w < s.waves) {
    const u32x4* p = src + w * s.per_wave + lane;
    for (int64_t i = 0; i < s.per_wave; i += kStep) {
      u32x4 v[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) v[u] = load_word<NT>(p + i + 64 * u);
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) acc ^= v[u];
    }
  }
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t i = tail_begin(s); i < s.n; i += stride) acc ^= src[i];
  if (acc.x == key.x && acc.y == key.y && acc.z == key.z && acc.w == key.w) sink[0] = acc;
}

template <bool NT>
__global__ __launch_bounds__(kThreads) void stream_write_kernel(u32x4* __restrict__ dst, Split s,
                                                                uint32_t pattern) {
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const u32x4 v = {pattern, pattern, pattern, pattern};
  if (w < s.waves) {
    u32x4* q = dst + w * s.per_wave + lane;
    for (int64_t i = 0; i < s.per_wave; i += kStep) {
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) store_word<NT>(v, q + i + 64 * u);
    }
  }
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t i = tail_begin(s); i < s.n; i += stride) dst[i] = v;
}

// Copy with the grid sweeping the buffer together: consecutive waves take
// consecutive blocks of 64 * U words (one 16-byte word per lane per load),
// so the accesses in flight at any moment lie in a narrow window of the
// buffer; the words past the last whole block are spread over all lanes.
template <int U, bool NT>
__global__ __launch_bounds__(kThreads) void stream_copy_swept_kernel(const u32x4* __restrict__ src,
                                                                     u32x4* __restrict__ dst,
                                                                     int64_t n) {
  constexpr int64_t BLK = 64 * U;
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * kThreads + threadIdx.x) >> 6;
  const int64_t waves = (int64_t)gridDim.x * (kThreads / 64);
  const int64_t full = n / BLK * BLK;
  for (int64_t base = wave * BLK; base < full; base += waves * BLK) {
    u32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = load_word<NT>(src + base + 64 * u + lane);
#pragma unroll
    for (int u = 0; u < U; ++u) store_word<NT>(v[u], dst + base + 64 * u + lane);
  }
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t i = full + (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride)
    dst[i] = src[i];
}

// `waves` chunks of whole kStep groups; fewer waves when the buffer is small
Split split_words(int64_t n, int64_t waves) {
  Split s;
  s.n = n;
  s.waves = std::min<int64_t>(waves, n / kStep);
  s.per_wave = s.waves > 0 ? n / s.waves / kStep * kStep : 0;
  if (s.per_wave == 0) s.waves = 0;
  return s;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

}  // namespace

extern "C" la_status la_stream_probe(int32_t kind, const void* src, void* dst, size_t bytes,
                                     uint32_t pattern, la_stream stream) {
  if (bytes == 0 || bytes % 16 != 0 || (bytes >> 60) != 0) return LA_ERR_INVALID_ARG;
  if (!dst || !aligned16(dst)) return LA_ERR_INVALID_ARG;
  if (kind != LA_STREAM_WRITE && (!src || !aligned16(src))) return LA_ERR_INVALID_ARG;
  if (kind == LA_STREAM_COPY) {
    const char* s = (const char*)src;
    const char* d = (const char*)dst;
    if (s < d + bytes && d < s + bytes) return LA_ERR_INVALID_ARG;  // overlap
  }
  if (kind != LA_STREAM_READ && kind != LA_STREAM_WRITE && kind != LA_STREAM_COPY)
    return LA_ERR_INVALID_ARG;
  // Per kind, the fastest form measured on a 4 GiB buffer (one contiguous
  // chunk per wave at 2048 to 16384 waves, with and without nontemporal
  // accesses, bursts of 8 and 16 words per lane, and grid-swept forms):
  // reads with nontemporal loads at two waves per SIMD (7.02 TB/s), writes
  // with plain stores at two waves per SIMD (5.97 TB/s), copies grid-swept,
  // eight nontemporal words per lane, 8192 workgroups (5.49 TB/s; one
  // chunk per wave reached 5.21, bursts 5.31).
  const hipStream_t st = (hipStream_t)stream;
  const int64_t n = (int64_t)(bytes / 16);
  auto grid = [](const Split& s) { return dim3((unsigned)std::max<int64_t>(1, (s.waves + 3) / 4)); };
  if (kind == LA_STREAM_READ) {
    const Split s = split_words(n, 2048);
    la::ProfScope prof("stream_read", st);
    const u32x4 key = {0x9e3779b9u, 0x7f4a7c15u, 0xf39cc060u, 0x5ced1c5bu};
    hipLaunchKernelGGL(stream_read_kernel<true>, grid(s), dim3(kThreads), 0, st, (const u32x4*)src,
                       s, key, (u32x4*)dst);
  } else if (kind == LA_STREAM_WRITE) {
    const Split s = split_words(n, 2048);
    la::ProfScope prof("stream_write", st);
    hipLaunchKernelGGL(stream_write_kernel<false>, grid(s), dim3(kThreads), 0, st, (u32x4*)dst, s,
                       pattern);
  } else {
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(8192, n / (8 * 256)));
    la::ProfScope prof("stream_copy", st);
    hipLaunchKernelGGL((stream_copy_swept_kernel<8, true>), dim3((unsigned)blocks), dim3(kThreads),
                       0, st, (const u32x4*)src, (u32x4*)dst, n);
  }
  return hipGetLastError() == hipSuccess ? LA_OK : LA_ERR_HIP;
}
