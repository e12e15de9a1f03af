// Device-wide exclusive prefix sums (reduce, scan partials, apply), shared by the build and the
// search planner. Defined in index_build.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bm25 {

// out[i] = sum_{j<i} in[i] for i < n, computed in T; if total != nullptr, *total (device) =
// sum of all n values. `tmp` must hold scan_tmp_elems(n) values of T. in and out may alias.
template <typename T>
hipError_t scan_exclusive(const T* in, T* out, int64_t n, T* tmp, T* total, hipStream_t s);

int64_t scan_tmp_elems(int64_t n);

}  // namespace bm25
