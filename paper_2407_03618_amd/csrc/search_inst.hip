// Template instances of the gather and sweep kernels for one stored score type.
// Compiled once per type with -DBM25_ST=F32|F16|BF16 and -DBM25_ST_SUFFIX=f32|f16|bf16.
#include <hip/hip_runtime.h>

#include "search_kernels.hpp"

#ifndef BM25_ST
#error "BM25_ST must be defined"
#endif

#define BM25_CAT2(a, b) a##b
#define BM25_CAT(a, b) BM25_CAT2(a, b)

namespace bm25 {

using namespace bm25dev;

static constexpr int kMaxLds = 160 * 1024;

template <int W, int QPW, int KPL>
static hipError_t gather_one(dim3 g, size_t sh, hipStream_t s, const GatherArgs& a) {
  auto fn = k_gather<W, QPW, KPL, BM25_ST>;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       kMaxLds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(fn, g, dim3(W * 64), sh, s, a);
  return hipGetLastError();
}

template <int W, int KPL>
static hipError_t sweep_one(dim3 g, size_t sh, hipStream_t s, const SweepArgs& a) {
  auto fn = k_sweep<W, KPL, BM25_ST>;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       kMaxLds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(fn, g, dim3(W * 64), sh, s, a);
  return hipGetLastError();
}

hipError_t BM25_CAT(launch_gather_, BM25_ST_SUFFIX)(int W, int QPW, int KPL, dim3 g, size_t sh,
                                                  hipStream_t s, const GatherArgs& a) {
#define BM25_G(w, q)                                          \
  if (W == w && QPW == q) {                                   \
    switch (KPL) {                                            \
      case 1: return gather_one<w, q, 1>(g, sh, s, a);        \
      case 2: return gather_one<w, q, 2>(g, sh, s, a);        \
      case 4: return gather_one<w, q, 4>(g, sh, s, a);        \
      case 8: return gather_one<w, q, 8>(g, sh, s, a);        \
      case 16: return gather_one<w, q, 16>(g, sh, s, a);      \
      default: return hipErrorInvalidValue;                   \
    }                                                         \
  }
  BM25_G(4, 1)
  BM25_G(4, 2)
  BM25_G(4, 4)
  BM25_G(8, 1)
  BM25_G(8, 2)
  BM25_G(8, 4)
#undef BM25_G
  return hipErrorInvalidValue;
}

hipError_t BM25_CAT(launch_sweep_, BM25_ST_SUFFIX)(int W, int KPL, dim3 g, size_t sh,
                                                 hipStream_t s, const SweepArgs& a) {
#define BM25_S(w)                                          \
  if (W == w) {                                            \
    switch (KPL) {                                         \
      case 1: return sweep_one<w, 1>(g, sh, s, a);         \
      case 2: return sweep_one<w, 2>(g, sh, s, a);         \
      case 4: return sweep_one<w, 4>(g, sh, s, a);         \
      case 8: return sweep_one<w, 8>(g, sh, s, a);         \
      case 16: return sweep_one<w, 16>(g, sh, s, a);       \
      default: return hipErrorInvalidValue;                \
    }                                                      \
  }
  BM25_S(4)
  BM25_S(8)
#undef BM25_S
  return hipErrorInvalidValue;
}

}  // namespace bm25
