// Host-side internals shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bm25.h"

namespace bm25 {

// Error plumbing: set_error stores a thread-local message and returns the code.
int set_error(int code, const char* fmt, ...);
void clear_error();

struct HipError {
  hipError_t err;
  const char* what;
};

#define BM25_HIP(call)                                                             \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) {                                                        \
      return ::bm25::set_error(BM25_E_HIP, "%s failed: %s", #call,               \
                               hipGetErrorString(e_));                             \
    }                                                                              \
  } while (0)

// Source of an index's device memory: the caller's allocator (bm25_allocator) or hipMalloc.
// `stream` is handed to the caller's callbacks; it is the stream of the call that allocates.
struct Alloc {
  bm25_allocator fn{};
  bool custom = false;
  hipStream_t stream = nullptr;

  hipError_t alloc(void** p, size_t n) const {
    if (!custom) return hipMalloc(p, n);
    *p = fn.alloc(n, (void*)stream, fn.ctx);
    if (!*p) return hipErrorOutOfMemory;
    if (((uintptr_t)*p & 255u) != 0) {  // the documented alignment is part of the contract
      fn.free(*p, (void*)stream, fn.ctx);
      *p = nullptr;
      return hipErrorInvalidValue;
    }
    return hipSuccess;
  }
  void free(void* p) const {
    if (!custom) (void)hipFree(p);
    else fn.free(p, (void*)stream, fn.ctx);
  }
};

// Device buffer owned by the library, allocated through `al` (hipMalloc when null).
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  const Alloc* al = nullptr;
  DevBuf() = default;
  explicit DevBuf(const Alloc* a) : al(a) {}
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (ptr) {
      if (al) al->free(ptr);
      else (void)hipFree(ptr);
    }
    ptr = nullptr;
    bytes = 0;
  }
  // Grows to at least n bytes (contents are not preserved). Returns hipSuccess or the error.
  hipError_t reserve(size_t n) {
    if (n <= bytes) return hipSuccess;
    release();
    size_t want = n < 256 ? 256 : n;
    hipError_t e = al ? al->alloc(&ptr, want) : hipMalloc(&ptr, want);
    if (e != hipSuccess) {
      ptr = nullptr;
      return e;
    }
    bytes = want;
    return hipSuccess;
  }
  template <typename T>
  T* as() const {
    return static_cast<T*>(ptr);
  }
};

// Pinned host buffer owned by the library.
struct PinnedBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  PinnedBuf() = default;
  PinnedBuf(const PinnedBuf&) = delete;
  PinnedBuf& operator=(const PinnedBuf&) = delete;
  ~PinnedBuf() { release(); }
  void release() {
    if (ptr) (void)hipHostFree(ptr);
    ptr = nullptr;
    bytes = 0;
  }
  hipError_t reserve(size_t n) {
    if (n <= bytes) return hipSuccess;
    release();
    size_t want = n < 4096 ? 4096 : n;
    hipError_t e = hipHostMalloc(&ptr, want, hipHostMallocDefault);
    if (e != hipSuccess) {
      ptr = nullptr;
      return e;
    }
    bytes = want;
    return hipSuccess;
  }
  template <typename T>
  T* as() const {
    return static_cast<T*>(ptr);
  }
};

// Documents per skip block. Rows with at least kLongRow entries keep, for every block j, the
// offset of their first entry whose document id is >= j * kSkipBlock, so a workgroup or a sweep
// that starts at a block boundary finds its cursor in such a row with one load (shorter rows take
// a binary search). About 28k rows and 1 GB of table at 8.8M documents, about 94k rows and
// 1.8 GB at 5M documents of 300 ids.
constexpr int64_t kSkipBlock = 1024;
constexpr int64_t kLongRow = 1024;
static_assert(kLongRow <= 64 * 64, "a row without a skip table is searched with 64 samples of 64");

// Rows of tokens present in at least 1/kDenseFraction of the documents are also kept as dense
// rows (one stored score per document, zero where the token is absent), at most kDenseBytes in
// total. Query-time accumulation reads them with coalesced loads into registers.
constexpr int64_t kDenseFraction = 16;
constexpr int64_t kDenseBytes = 4ll << 30;
constexpr int64_t kDensePad = 4096;

// Per-call device scratch of the search path: one arena, carved per call (layout in search.hip).
// The host plan (query offsets, k, tile bounds) is staged in host memory and copied to the
// arena's first region.
struct SearchScratch {
  DevBuf arena;                 // owned arena, grown on demand
  uint8_t* fixed = nullptr;     // or an arena lent by the caller (server lane, static scratch)
  size_t fixed_bytes = 0;
  PinnedBuf host;               // pinned staging of the host plan, grown on demand
  uint8_t* host_fixed = nullptr;  // or lent staging (pageable: the copy is staged by HIP)
  size_t host_fixed_bytes = 0;
  bool no_alloc = false;        // no allocation of any kind: no events, graphs or timing
  hipEvent_t host_free = nullptr;  // the pinned staging may be rewritten once this has fired
  hipEvent_t done = nullptr;    // recorded after the last call's launches, on that call's stream
  hipStream_t last_stream = nullptr;  // stream of the last call (valid once done was recorded)
  bool used = false;
  // graph mode: launches are recorded on cap_stream (capture only, nothing runs there) and the
  // instantiated graphs are kept for the next batches, updated in place while their topology
  // holds. Two are kept and used in turn, so a graph is only updated once its own previous
  // launch (two batches back) has finished, never the launch still in flight.
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
  hipEvent_t graph_done[2] = {nullptr, nullptr};
  std::array<int64_t, 10> graph_cfg[2]{};  // launch configuration each graph was captured with
  int graph_next = 0;
  int64_t graph_builds = 0;    // instantiations
  int64_t graph_updates = 0;   // in-place updates

  // Destroys the events, streams and graphs (device buffers free themselves).
  void release_handles() {
    for (int i = 0; i < 2; ++i) {
      if (graph_exec[i]) (void)hipGraphExecDestroy(graph_exec[i]);
      if (graph_done[i]) (void)hipEventDestroy(graph_done[i]);
      graph_exec[i] = nullptr;
      graph_done[i] = nullptr;
    }
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (host_free) (void)hipEventDestroy(host_free);
    if (done) (void)hipEventDestroy(done);
    cap_stream = nullptr;
    host_free = nullptr;
    done = nullptr;
  }
};

struct TileShape {
  int q_tile = 0;
  int waves = 0;
  int doc_tile = 0;
  int doc_groups = 0;
  int query_order = 0;  // 0 automatic, 1 grouped by frequent tokens, 2 as given
  int sparse_only = 0;
};

}  // namespace bm25

struct bm25_index {
  bm25::Alloc alloc;  // declared first: outlives every buffer below
  int device = 0;
  int64_t n_docs = 0;
  int64_t n_tokens = 0;
  int32_t vocab = 0;
  int64_t nnz = 0;
  int64_t sum_len = 0;
  double l_avg = 0.0;
  bm25_params params{};

  bm25::DevBuf indptr;    // int64[V+1]
  bm25::DevBuf indices;   // int32[nnz]
  bm25::DevBuf tf;        // int32[nnz]
  bm25::DevBuf data;      // store dtype[nnz]
  bm25::DevBuf df;        // int32[V]
  bm25::DevBuf idf;       // double[V]
  bm25::DevBuf theta;     // double[V]
  bm25::DevBuf theta32;   // float[V]
  bm25::DevBuf doclen;    // int32[N]
  bm25::DevBuf long_id;   // int32[V]: index among long rows, or -1
  bm25::DevBuf skip;      // uint32[n_long][n_blocks+1]
  int64_t n_long = 0;
  int64_t n_blocks = 0;   // ceil(N / kSkipBlock)
  bm25::DevBuf dense_id;  // int32[V]: dense row of the token, or -1
  bm25::DevBuf dense_rank;  // int32[n_dense]: rank of the row by document frequency (0 = most)
  bm25::DevBuf dense;     // store dtype[n_dense][n_pad]: S (or S_delta) per document, 0 if absent
  int64_t n_dense = 0;
  int64_t n_pad = 0;      // dense row length: N rounded up to kDensePad

  bm25::SearchScratch batch_scratch;
  bm25::SearchScratch plain_scratch;

  bool plan_fixed = false;
  bm25::TileShape fixed_plan;
  std::map<uint64_t, bm25::TileShape> tuned;  // shape class -> tuned plan

  bool use_graphs = false;  // batched searches run as one HIP graph launch each

  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> timing_events;
  double timing_ms = 0.0;
  int64_t timing_launches = 0;

  // stored values rounded to a subnormal, from non-zero to zero, and to infinity
  int64_t range_subnormal = 0;
  int64_t range_to_zero = 0;
  int64_t range_overflow = 0;

  std::mutex mu;

  // Every device buffer of the index and its scratch takes memory from `alloc`.
  void bind_alloc() {
    bm25::DevBuf* bufs[] = {&indptr, &indices, &tf, &data, &df, &idf, &theta, &theta32,
                            &doclen, &long_id, &skip, &dense_id, &dense_rank, &dense,
                            &batch_scratch.arena, &plain_scratch.arena};
    for (auto* b : bufs) b->al = &alloc;
  }
};

namespace bm25 {

// Search entry used by the server (host-planned batches).
int search_batch_impl(bm25_index* idx, const int32_t* q_ids_dev, const int64_t* q_off_host,
                      int32_t n, const int32_t* k_host, int32_t k_max, int32_t* out_ids,
                      float* out_scores, int32_t* out_count, hipStream_t stream,
                      SearchScratch& scratch, const TileShape* force);

// Launch shape bm25_search_batch uses for a batch (fixed plan, tuned plan or automatic).
TileShape batch_shape(const bm25_index* idx, int32_t n, int32_t max_qlen, int32_t k_max);

// Device arena bytes and host staging bytes a batch of n queries with `positions` ids (the
// longest holding max_qlen) and lists for k_max needs under bm25_search_batch's launch shape;
// an upper bound of what search_batch_impl carves.
size_t batch_arena_bytes(const bm25_index* idx, int32_t n, int64_t positions, int32_t max_qlen,
                         int32_t k_max);
size_t batch_staging_bytes(int32_t n);

TileShape choose_shape(const bm25_index* idx, int32_t n, int32_t max_qlen, int32_t k_max);

}  // namespace bm25
