// Template instances of the gather and sweep kernels for one stored score type.
// Compiled once per type with -DBM25_ST=F32|F16|BF16 and -DBM25_ST_SUFFIX=f32|f16|bf16.
#include <hip/hip_runtime.h>

#include <atomic>

#include "search_kernels.hpp"

#ifndef BM25_ST
#error "BM25_ST must be defined"
#endif

#define BM25_CAT2(a, b) a##b
#define BM25_CAT(a, b) BM25_CAT2(a, b)

namespace bm25 {

using namespace bm25dev;

static constexpr int kMaxLds = 160 * 1024;

// Raises the kernel's dynamic LDS limit once per process (concurrent first calls may both set
// it, which is harmless).
template <typename F>
static hipError_t allow_lds(F fn, std::atomic<bool>& done) {
  if (done.load(std::memory_order_acquire)) return hipSuccess;
  hipError_t e =
      hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
  if (e == hipSuccess) done.store(true, std::memory_order_release);
  return e;
}

template <int W, int QT, int R, int KPL>
static hipError_t gather_one(dim3 g, size_t sh, hipStream_t s, const GatherArgs& a) {
  auto fn = k_gather<W, QT, R, KPL, BM25_ST>;
  static std::atomic<bool> attr{false};
  hipError_t e = allow_lds(fn, attr);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, g, dim3(W * 64), sh, s, a);
  return hipGetLastError();
}

// Built shapes (W, R): (8, 2) and (4, 4) give 1024-document tiles, (8, 4) 2048. Queries per
// tile QT = QPW * W with QPW in {1, 2, 4}; lists per wave QPW * KPL <= 8 registers when QPW > 1.
template <int W, int R>
static hipError_t gather_qt(int QT, int KPL, dim3 g, size_t sh, hipStream_t s,
                            const GatherArgs& a) {
#define BM25_Q(qpw, kpl) \
  if (QT == (qpw) * W && KPL == kpl) return gather_one<W, (qpw) * W, R, kpl>(g, sh, s, a);
  BM25_Q(1, 1)
  BM25_Q(1, 2)
  BM25_Q(1, 4)
  BM25_Q(1, 8)
  BM25_Q(1, 16)
  BM25_Q(2, 1)
  BM25_Q(2, 2)
  BM25_Q(2, 4)
  if constexpr (W * R <= 16) {
    BM25_Q(4, 1)
    BM25_Q(4, 2)
  }
#undef BM25_Q
  return hipErrorInvalidValue;
}

hipError_t BM25_CAT(launch_gather_, BM25_ST_SUFFIX)(int W, int QT, int R, int KPL, dim3 g,
                                                  size_t sh, hipStream_t s, const GatherArgs& a) {
  if (W == 8 && R == 2) return gather_qt<8, 2>(QT, KPL, g, sh, s, a);
  if (W == 4 && R == 4) return gather_qt<4, 4>(QT, KPL, g, sh, s, a);
  if (W == 8 && R == 4) return gather_qt<8, 4>(QT, KPL, g, sh, s, a);
  return hipErrorInvalidValue;
}

template <int W, int KPL>
static hipError_t sweep_one(dim3 g, size_t sh, hipStream_t s, const SweepArgs& a) {
  auto fn = k_sweep<W, 16, KPL, BM25_ST>;
  static std::atomic<bool> attr{false};
  hipError_t e = allow_lds(fn, attr);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, g, dim3(W * 64), sh, s, a);
  return hipGetLastError();
}

template <int W>
static hipError_t sweep_w(int KPL, dim3 g, size_t sh, hipStream_t s, const SweepArgs& a) {
  switch (KPL) {
    case 1: return sweep_one<W, 1>(g, sh, s, a);
    case 2: return sweep_one<W, 2>(g, sh, s, a);
    case 4: return sweep_one<W, 4>(g, sh, s, a);
    case 8: return sweep_one<W, 8>(g, sh, s, a);
    case 16: return sweep_one<W, 16>(g, sh, s, a);
    default: return hipErrorInvalidValue;
  }
}

// Sweeps with 1, 2, 4 or 8 waves per workgroup.
hipError_t BM25_CAT(launch_sweep_, BM25_ST_SUFFIX)(int W, int KPL, dim3 g, size_t sh,
                                                 hipStream_t s, const SweepArgs& a) {
  switch (W) {
    case 1: return sweep_w<1>(KPL, g, sh, s, a);
    case 2: return sweep_w<2>(KPL, g, sh, s, a);
    case 4: return sweep_w<4>(KPL, g, sh, s, a);
    case 8: return sweep_w<8>(KPL, g, sh, s, a);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace bm25
