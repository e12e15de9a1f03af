// Error plumbing, kernel timing and the calibration copy kernel.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <string>

#include "internal.hpp"

namespace bm25 {

// Fixed-size per-thread message buffer: reporting an error allocates nothing.
static thread_local char g_last_error[512];

int set_error(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
  return code;
}

void clear_error() { g_last_error[0] = '\0'; }

// Plain streaming copy, 16 bytes per lane per step; the tail (n % 16) is copied bytewise.
__global__ __launch_bounds__(256) void k_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                              int64_t n16, const uint8_t* __restrict__ src_tail,
                                              uint8_t* __restrict__ dst_tail, int tail) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    dst[i] = src[i];
  if (blockIdx.x == 0 && (int)threadIdx.x < tail) dst_tail[threadIdx.x] = src_tail[threadIdx.x];
}

}  // namespace bm25

using namespace bm25;

extern "C" const char* bm25_last_error(void) { return g_last_error; }

extern "C" int bm25_copy_bytes(void* dst, const void* src, int64_t n_bytes, void* stream) {
  clear_error();
  if (!dst || !src || n_bytes < 0) return set_error(BM25_E_INVAL, "bad copy arguments");
  if (((uintptr_t)dst | (uintptr_t)src) & 15u)
    return set_error(BM25_E_INVAL, "copy pointers must be 16-byte aligned");
  if (n_bytes == 0) return BM25_OK;
  const int64_t n16 = n_bytes / 16;
  const int tail = (int)(n_bytes % 16);
  int64_t blocks = (n16 + 255) / 256;
  if (blocks > 256 * 32) blocks = 256 * 32;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                     (const uint4*)src, (uint4*)dst, n16, (const uint8_t*)src + n16 * 16,
                     (uint8_t*)dst + n16 * 16, tail);
  BM25_HIP(hipGetLastError());
  return BM25_OK;
}

extern "C" int bm25_kernel_timing(bm25_index* index, int32_t enable) {
  clear_error();
  if (!index) return set_error(BM25_E_INVAL, "index is NULL");
  std::lock_guard<std::mutex> g(index->mu);
  index->timing = enable != 0;
  return BM25_OK;
}

extern "C" int bm25_kernel_time_read(bm25_index* index, double* total_ms, int64_t* launches) {
  clear_error();
  if (!index) return set_error(BM25_E_INVAL, "index is NULL");
  std::lock_guard<std::mutex> g(index->mu);
  double ms = index->timing_ms;
  int64_t n = index->timing_launches;
  for (auto& ev : index->timing_events) {
    BM25_HIP(hipEventSynchronize(ev.second));
    float t = 0.f;
    BM25_HIP(hipEventElapsedTime(&t, ev.first, ev.second));
    ms += t;
    ++n;
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  index->timing_events.clear();
  index->timing_ms = 0.0;
  index->timing_launches = 0;
  if (total_ms) *total_ms = ms;
  if (launches) *launches = n;
  return BM25_OK;
}
