// A plain device copy, timed with HIP events: the HBM bandwidth a streaming
// kernel reaches on this GPU, the ceiling that the step kernel's algorithmic
// bandwidth is read against beside the published peak.  Not part of the
// method; the bench calls it once.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

#include "sdem.h"

namespace sdem {
int set_error(int code, const char* msg);
}  // namespace sdem

namespace {

constexpr int kCopyThreads = 256;
constexpr int kCopyUnroll = 4;  // 16-byte words in flight per lane

typedef int v4i __attribute__((ext_vector_type(4)));

// Each workgroup moves its own kCopyThreads * kCopyUnroll consecutive 16-byte
// words (all loads issued before the stores), with nontemporal loads and
// stores: the fastest of the plain copies measured on MI355X (one workgroup
// per 16 KB rather than a grid-strided loop, 4 words per lane rather than 1,
// 2 or 8, nontemporal rather than cached: 6.3 TB/s on 1 GiB, against 5.3-6.2
// for the others and 5.0 for a device-to-device hipMemcpy).
__global__ __launch_bounds__(kCopyThreads) void k_copy_probe(const v4i* __restrict__ src,
                                                             v4i* __restrict__ dst, int64_t n16) {
  const int64_t b = (int64_t)blockIdx.x * kCopyThreads * kCopyUnroll + threadIdx.x;
  v4i v[kCopyUnroll];
#pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u) {
    const int64_t i = b + (int64_t)u * kCopyThreads;
    if (i < n16) v[u] = __builtin_nontemporal_load(src + i);
  }
#pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u) {
    const int64_t i = b + (int64_t)u * kCopyThreads;
    if (i < n16) __builtin_nontemporal_store(v[u], dst + i);
  }
}

int fail_hip(hipError_t e, const char* what) {
  char buf[256];
  snprintf(buf, sizeof buf, "%s failed: %s", what, hipGetErrorString(e));
  return sdem::set_error(SDEM_EHIP, buf);
}

}  // namespace

extern "C" int sdem_copy_probe(const void* src, void* dst, int64_t bytes, int32_t reps,
                               void* hip_stream, double* ms_per_copy) {
  if (!src || !dst || !ms_per_copy || bytes <= 0 || bytes % 16 != 0 || reps < 1 ||
      reinterpret_cast<uintptr_t>(src) % 16 != 0 || reinterpret_cast<uintptr_t>(dst) % 16 != 0)
    return sdem::set_error(SDEM_EINVAL,
                           "copy probe: src, dst 16-byte aligned, bytes > 0 a multiple of 16, "
                           "reps >= 1, ms_per_copy required");
  const char* s0 = static_cast<const char*>(src);
  const char* d0 = static_cast<const char*>(dst);
  if (s0 < d0 + bytes && d0 < s0 + bytes)
    return sdem::set_error(SDEM_EINVAL, "copy probe: src and dst overlap");
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  const int64_t n16 = bytes / 16;
  const int64_t per_block = (int64_t)kCopyThreads * kCopyUnroll;
  const int64_t blocks = (n16 + per_block - 1) / per_block;
  if (blocks > 0x7fffffffLL) return sdem::set_error(SDEM_EINVAL, "copy probe: too many bytes");
  const unsigned grid = (unsigned)blocks;
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipError_t e = hipEventCreate(&ev[0]);
  if (e == hipSuccess) e = hipEventCreate(&ev[1]);
  if (e == hipSuccess) {
    k_copy_probe<<<grid, kCopyThreads, 0, st>>>(static_cast<const v4i*>(src),
                                                 static_cast<v4i*>(dst), n16);  // untimed
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(ev[0], st);
  for (int r = 0; r < reps && e == hipSuccess; ++r) {
    k_copy_probe<<<grid, kCopyThreads, 0, st>>>(static_cast<const v4i*>(src),
                                                 static_cast<v4i*>(dst), n16);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(ev[1], st);
  if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  if (e != hipSuccess) return fail_hip(e, "copy probe");
  *ms_per_copy = (double)ms / reps;
  return SDEM_OK;
}
