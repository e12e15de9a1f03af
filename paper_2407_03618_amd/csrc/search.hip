// Host side of the search path: argument checks, tile planning, staging and launches.
#define BM25_SEARCH_MAIN 1
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.hpp"
#include "search_kernels.hpp"

namespace bm25 {

using namespace bm25dev;

hipError_t launch_gather_f32(int, int, int, int, dim3, size_t, hipStream_t, const GatherArgs&);
hipError_t launch_gather_f16(int, int, int, int, dim3, size_t, hipStream_t, const GatherArgs&);
hipError_t launch_gather_bf16(int, int, int, int, dim3, size_t, hipStream_t, const GatherArgs&);
hipError_t launch_sweep_f32(int, int, dim3, size_t, hipStream_t, const SweepArgs&);
hipError_t launch_sweep_f16(int, int, dim3, size_t, hipStream_t, const SweepArgs&);
hipError_t launch_sweep_bf16(int, int, dim3, size_t, hipStream_t, const SweepArgs&);

static constexpr int64_t kMaxLdsBytes = 160 * 1024;
// queries of the per-query form whose candidate lists are merged by one launch
static constexpr int32_t kPlainMergeBatch = 256;
static constexpr int64_t kPlainCandBytes = 512ll << 20;

static hipError_t launch_gather(int dtype, int W, int QT, int R, int KPL, dim3 g, size_t sh,
                                hipStream_t s, const GatherArgs& a) {
  switch (dtype) {
    case BM25_F32: return launch_gather_f32(W, QT, R, KPL, g, sh, s, a);
    case BM25_F16: return launch_gather_f16(W, QT, R, KPL, g, sh, s, a);
    default: return launch_gather_bf16(W, QT, R, KPL, g, sh, s, a);
  }
}

static hipError_t launch_sweep(int dtype, int W, int KPL, dim3 g, size_t sh, hipStream_t s,
                               const SweepArgs& a) {
  switch (dtype) {
    case BM25_F32: return launch_sweep_f32(W, KPL, g, sh, s, a);
    case BM25_F16: return launch_sweep_f16(W, KPL, g, sh, s, a);
    default: return launch_sweep_bf16(W, KPL, g, sh, s, a);
  }
}

static hipError_t launch_merge(int KPL, dim3 g, hipStream_t s, const MergeArgs& a) {
  switch (KPL) {
    case 1: hipLaunchKernelGGL(k_merge<1>, g, dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_merge<2>, g, dim3(256), 0, s, a); break;
    case 4: hipLaunchKernelGGL(k_merge<4>, g, dim3(256), 0, s, a); break;
    case 8: hipLaunchKernelGGL(k_merge<8>, g, dim3(256), 0, s, a); break;
    case 16: hipLaunchKernelGGL(k_merge<16>, g, dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

static int kpl_for(int k_max) {
  int kpl = 1;
  while (kpl * 64 < k_max) kpl *= 2;
  return kpl;
}

static IndexView index_view(const bm25_index* idx, bool sparse_only) {
  IndexView v;
  v.indptr = idx->indptr.as<int64_t>();
  v.indices = idx->indices.as<int32_t>();
  v.data = idx->data.ptr;
  v.long_id = idx->long_id.as<int32_t>();
  v.skip = idx->skip.as<uint32_t>();
  const int var = idx->params.variant;
  const bool shifted = var == BM25_BM25L || var == BM25_BM25PLUS || var == BM25_TFLDP;
  v.theta32 = shifted ? idx->theta32.as<float>() : nullptr;
  const bool dense = !sparse_only && idx->n_dense > 0;
  v.dense_id = dense ? idx->dense_id.as<int32_t>() : nullptr;
  v.dense_rank = dense ? idx->dense_rank.as<int32_t>() : nullptr;
  v.dense = idx->dense.ptr;
  v.n_docs = idx->n_docs;
  v.n_blocks = idx->n_blocks;
  v.n_pad = idx->n_pad;
  v.vocab = idx->vocab;
  return v;
}

struct BatchInfo {
  int32_t max_qlen = 0;
  int64_t positions = 0;
};

static int check_batch(const bm25_index* idx, const int32_t* q_ids, const int64_t* q_off,
                       int32_t n, const int32_t* k, int32_t k_max, const int32_t* out_ids,
                       const float* out_scores, const int32_t* out_count, BatchInfo& info) {
  if (!idx) return set_error(BM25_E_INVAL, "index is NULL");
  if (n < 0) return set_error(BM25_E_INVAL, "n_queries < 0");
  if (k_max < 1 || k_max > BM25_MAX_K)
    return set_error(BM25_E_INVAL, "k_max must lie in [1, %d]", BM25_MAX_K);
  if (n == 0) return BM25_OK;
  if (!q_off) return set_error(BM25_E_INVAL, "q_offsets is NULL");
  if (!out_ids || !out_scores || !out_count) return set_error(BM25_E_INVAL, "output is NULL");
  if (q_off[0] != 0) return set_error(BM25_E_INVAL, "q_offsets[0] must be 0");
  int64_t mx = 0;
  for (int32_t i = 0; i < n; ++i) {
    const int64_t len = q_off[i + 1] - q_off[i];
    if (len < 0) return set_error(BM25_E_INVAL, "q_offsets must be non-decreasing");
    if (len > BM25_MAX_QUERY_LEN)
      return set_error(BM25_E_INVAL, "query %d has %lld ids (limit %d)", i, (long long)len,
                       BM25_MAX_QUERY_LEN);
    mx = std::max(mx, len);
  }
  if (q_off[n] > (int64_t)INT32_MAX) return set_error(BM25_E_INVAL, "too many query positions");
  if (q_off[n] > 0 && !q_ids) return set_error(BM25_E_INVAL, "q_ids is NULL");
  if (k) {
    for (int32_t i = 0; i < n; ++i)
      if (k[i] < 1 || k[i] > k_max)
        return set_error(BM25_E_INVAL, "k[%d] = %d outside [1, k_max]", i, k[i]);
  }
  info.max_qlen = (int32_t)mx;
  info.positions = q_off[n];
  return BM25_OK;
}

// Built (waves, documents per lane) shapes and (queries per tile, list registers) pairs; see
// search_inst.hip.
static bool shape_ok(const TileShape& t, int k_max) {
  if (t.waves < 1 || t.doc_tile < 64 * t.waves || t.doc_tile % (64 * t.waves) != 0) return false;
  const int R = t.doc_tile / (64 * t.waves);
  const bool wr = (t.waves == 8 && R == 2) || (t.waves == 4 && R == 4) || (t.waves == 8 && R == 4);
  if (!wr) return false;
  if (t.q_tile < t.waves || t.q_tile % t.waves != 0) return false;
  const int qpw = t.q_tile / t.waves;
  const int kpl = kpl_for(k_max);
  const bool ok = qpw == 1 || (qpw == 2 && kpl <= 4) ||
                  (qpw == 4 && kpl <= 2 && t.waves * R <= 16);
  if (!ok) return false;
  if (t.doc_groups < 1 || t.doc_groups > 65536) return false;
  if (t.query_order < 0 || t.query_order > 2) return false;
  return true;
}

// Largest built q_tile for this list size and shape, not above `want`.
static int fit_q_tile(int want, int kpl, int waves, int R) {
  for (int qpw : {4, 2, 1}) {
    TileShape t;
    t.waves = waves;
    t.doc_tile = 64 * waves * R;
    t.q_tile = qpw * waves;
    t.doc_groups = 1;
    if ((t.q_tile <= want || qpw == 1) && shape_ok(t, kpl * 64)) return t.q_tile;
  }
  return waves;
}

// accumulators + entry state (static and one cursor copy) + member copy
// Largest multiplicity of one dense entry in the batched form: the gather adds 16-bit stored rows
// on the matrix cores with the multiplicity as a 16-bit operand, exact for integers up to 2^11
// (FP16) or 2^8 (BF16); FP32 rows are added on the vector units with no limit.
static int32_t dense_mult_max(const bm25_index* idx) {
  switch (idx->params.store_dtype) {
    case BM25_F16: return 2048;
    case BM25_BF16: return 256;
    default: return INT32_MAX;
  }
}

static int64_t gather_lds(const TileShape& t, int64_t ecap, int64_t pcap) {
  return (int64_t)t.q_tile * t.doc_tile * 4 + ecap * (kEntryStaticBytes + kEntryDynBytes) +
         pcap * 4 + 64;
}

TileShape choose_shape(const bm25_index* idx, int32_t n, int32_t max_qlen, int32_t k_max) {
  TileShape t;
  const int kpl = kpl_for(k_max);
  // measured best on the 8.8M-document index, for the benchmark's batches (up to 30 ids per
  // query, top-100) and the serving recipe's (up to 64 ids, top-10/100/1000) alike, at 1024 to
  // 4096 queries per batch: 4 waves, 4 documents per lane, 4 queries per tile (8-query tiles
  // were 20-40% slower)
  t.waves = 4;
  t.doc_tile = 1024;
  t.q_tile = fit_q_tile(4, kpl, 4, 4);
  // long queries: fewer queries per tile so that accumulators and entry state fit in LDS
  auto fits = [&](const TileShape& s) {
    const int64_t pc = std::min<int64_t>((int64_t)s.q_tile * max_qlen, kTileMaxPositions);
    return gather_lds(s, pc + s.waves, pc) <= 96 * 1024;
  };
  while (!fits(t) && t.q_tile > t.waves) t.q_tile = fit_q_tile(t.q_tile / 2, kpl, 4, 4);
  // document groups. Each group keeps and merges its own lists, which costs more the longer
  // they are, so long lists take fewer groups. Lists of up to 256 keys: about 4096 workgroups
  // in all (2048 for batches of fewer than 64 tiles) and at least 8 groups; 512 keys: 2048 and
  // at least 4; 1024 keys: 2048 (batches of 128 tiles and more) or 1024, and at least 4. Counts
  // of 8 and above are multiples of 8 (one share per XCD), smaller ones powers of two; at most
  // 2048 / (keys per list / 64). Measured best on the same index: top-10 and top-100 batches of
  // 256 to 4096 queries at 4096 workgroups and 8 groups or more, of 16 to 128 queries at 2048
  // (64 queries, top-100: 1.22 ms against 1.36 with 4096); top-500 batches of 1024, 2048 and
  // 4096 queries at 8, 4-8 and 4 groups; top-1000 batches of 64, 256, 512, 1024, 2048 and 4096
  // queries at 64, 16, 16, 8, 4 and 4 groups (4096 queries: 59.7 ms, against 66.3 with 2
  // groups and 68.5 with 8).
  const int64_t ntiles = std::max<int64_t>(1, (n + t.q_tile - 1) / t.q_tile);
  int64_t target = ntiles < 64 ? 2048 : 4096, gmin = 8;
  if (kpl == 8) {
    target = 2048;
    gmin = 4;
  } else if (kpl > 8) {
    target = ntiles >= 128 ? 2048 : 1024;
    gmin = 4;
  }
  int64_t g = std::max<int64_t>((target + ntiles - 1) / ntiles, gmin);
  if (g >= 8) {
    g = ((g + 7) / 8) * 8;
  } else {
    int64_t p2 = 1;
    while (p2 < g) p2 *= 2;
    g = p2;
  }
  g = std::min<int64_t>(g, std::min<int64_t>(512, 2048 / kpl));
  const int64_t tiles = std::max<int64_t>(1, (idx->n_docs + t.doc_tile - 1) / t.doc_tile);
  g = std::min<int64_t>(g, tiles);
  t.doc_groups = (int)g;
  t.query_order = 0;
  t.sparse_only = 0;
  return t;
}

static uint64_t shape_class(int32_t n, int32_t max_qlen, int32_t k_max) {
  auto lg = [](int64_t v) {
    int b = 0;
    while ((1ll << b) < v) ++b;
    return (uint64_t)b;
  };
  return (lg(n) << 32) | (lg(max_qlen) << 16) | (uint64_t)kpl_for(k_max);
}

template <typename T>
static T* carve(uint8_t*& p, size_t count) {
  uintptr_t u = ((uintptr_t)p + 15) & ~(uintptr_t)15;
  T* r = reinterpret_cast<T*>(u);
  p = reinterpret_cast<uint8_t*>(u + count * sizeof(T));
  return r;
}

// Host plan of one call, staged in host memory and copied to the first region of the arena.
// Tile arrays have room for n + 1 tiles (every tile holds at least one query).
struct Staged {
  int64_t* q_off;
  int32_t* q_k;
  int32_t* tile_q0;
  int64_t* tile_e0;
};

// Lays out (q_off, q_k, tile_q0, tile_e0) in `base`; returns the byte size.
static size_t stage_layout(uint8_t* base, int32_t n, Staged& s) {
  uint8_t* p = base;
  s.q_off = carve<int64_t>(p, (size_t)n + 1);
  s.q_k = carve<int32_t>(p, (size_t)n);
  s.tile_q0 = carve<int32_t>(p, (size_t)n + 2);
  s.tile_e0 = carve<int64_t>(p, (size_t)n + 2);
  return (size_t)(p - base) + 16;
}

size_t batch_staging_bytes(int32_t n) {
  Staged s;
  return stage_layout(nullptr, n, s) + 64;
}

// Regions of one call inside the search arena, each 256-byte aligned.
struct ArenaNeed {
  int32_t n = 0;            // queries
  int32_t n_tiles = 0;      // planner tiles (one per query in the per-query form)
  int32_t waves = 1;        // waves the planner deals entries to
  int64_t ent = 0;          // planner entry slots
  int64_t positions = 0;    // query ids of the call
  int64_t cand_keys = 0;    // candidate list keys
  bool ordered = false;     // tile cost and launch order
  bool grouped = false;     // grouped copy of the batch
};

struct ArenaLayout {
  size_t meta = 0, wave_e0 = 0, qstat = 0, entries = 0, members = 0, dense_ent = 0, dense_n = 0,
         cand = 0, tile_cost = 0, order = 0, perm = 0, ids2 = 0, off2 = 0, k2 = 0;
  size_t total = 0;
};

static ArenaLayout arena_layout(const ArenaNeed& a) {
  ArenaLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = (off + std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;
    return o;
  };
  const size_t pos = (size_t)std::max<int64_t>(a.positions, 1);
  L.meta = take(batch_staging_bytes(a.n));
  L.wave_e0 = take((size_t)a.n_tiles * (a.waves + 1) * 4);
  L.qstat = take((size_t)a.n * 4);
  L.entries = take((size_t)std::max<int64_t>(a.ent, 1) * sizeof(Entry));
  L.members = take(pos * 4);
  L.dense_ent = take(pos * sizeof(DenseEntry));
  L.dense_n = take((size_t)a.n_tiles * 4);
  L.cand = take((size_t)a.cand_keys * 8);
  if (a.ordered) {
    L.tile_cost = take((size_t)a.n_tiles * 4);
    L.order = take((size_t)a.n_tiles * 4);
  }
  if (a.grouped) {
    L.perm = take((size_t)a.n * 4);
    L.ids2 = take(pos * 4);
    L.off2 = take(((size_t)a.n + 1) * 8);
    L.k2 = take((size_t)a.n * 4);
  }
  L.total = off;
  return L;
}

#define BM25_RESERVE(buf, bytes)                                                       \
  do {                                                                                 \
    hipError_t e_ = (buf).reserve(bytes);                                              \
    if (e_ != hipSuccess)                                                              \
      return set_error(BM25_E_NOMEM, "allocation of %lld bytes failed: %s",           \
                       (long long)(bytes), hipGetErrorString(e_));                     \
  } while (0)

// Host staging for the plan of a call of n queries: the lent buffer (pageable; hipMemcpyAsync
// consumes it before returning), else the pinned buffer once the previous upload has read it.
static int acquire_staging(SearchScratch& sc, int32_t n, uint8_t** host) {
  const size_t bytes = batch_staging_bytes(n);
  if (sc.host_fixed) {
    if (bytes > sc.host_fixed_bytes)
      return set_error(BM25_E_NOMEM, "a batch of %d queries needs %zu bytes of host staging, "
                       "%zu are available", n, bytes, sc.host_fixed_bytes);
    *host = sc.host_fixed;
    return BM25_OK;
  }
  if (!sc.host_free) BM25_HIP(hipEventCreateWithFlags(&sc.host_free, hipEventDisableTiming));
  else BM25_HIP(hipEventSynchronize(sc.host_free));
  BM25_RESERVE(sc.host, bytes);
  *host = sc.host.as<uint8_t>();
  return BM25_OK;
}

// Device arena of `need` bytes: the lent one, or the owned one grown once the previous call's
// work on it has finished.
static int acquire_arena(SearchScratch& sc, size_t need, uint8_t** base) {
  if (sc.fixed) {
    if (need > sc.fixed_bytes)
      return set_error(BM25_E_NOMEM, "the call needs %zu bytes of search scratch, %zu are "
                       "available", need, sc.fixed_bytes);
    *base = sc.fixed;
    return BM25_OK;
  }
  if (need > sc.arena.bytes && sc.done) BM25_HIP(hipEventSynchronize(sc.done));
  BM25_RESERVE(sc.arena, need);
  *base = sc.arena.as<uint8_t>();
  return BM25_OK;
}

// Orders this call's use of the scratch after the previous call's: on the same stream the
// stream order does it; on another stream the call waits for the previous call's last launch.
static int scratch_begin(SearchScratch& sc, hipStream_t s) {
  if (sc.no_alloc) return BM25_OK;
  if (!sc.done) BM25_HIP(hipEventCreateWithFlags(&sc.done, hipEventDisableTiming));
  else if (sc.used && sc.last_stream != s) BM25_HIP(hipStreamWaitEvent(s, sc.done, 0));
  return BM25_OK;
}

static int scratch_end(SearchScratch& sc, hipStream_t s) {
  if (!sc.done) return BM25_OK;
  BM25_HIP(hipEventRecord(sc.done, s));
  sc.last_stream = s;
  sc.used = true;
  return BM25_OK;
}

// Copies the staged host plan into the arena's meta region.
static int upload_plan(SearchScratch& sc, hipStream_t s, int32_t n, const uint8_t* host,
                       uint8_t* meta) {
  const size_t bytes = batch_staging_bytes(n);
  BM25_HIP(hipMemcpyAsync(meta, host, bytes, hipMemcpyHostToDevice, s));
  if (!sc.host_fixed) BM25_HIP(hipEventRecord(sc.host_free, s));
  return BM25_OK;
}

static void stage_queries(const Staged& hs, const int64_t* q_off, const int32_t* k, int32_t n,
                          int32_t k_max) {
  std::memcpy(hs.q_off, q_off, ((size_t)n + 1) * 8);
  if (k) std::memcpy(hs.q_k, k, (size_t)n * 4);
  else for (int32_t i = 0; i < n; ++i) hs.q_k[i] = k_max;
}

static int timed_begin(bm25_index* idx, hipStream_t s, hipEvent_t* b) {
  *b = nullptr;
  if (!idx->timing) return BM25_OK;
  BM25_HIP(hipEventCreate(b));
  BM25_HIP(hipEventRecord(*b, s));
  return BM25_OK;
}

static int timed_end(bm25_index* idx, hipStream_t s, hipEvent_t b) {
  if (!b) return BM25_OK;
  hipEvent_t e;
  BM25_HIP(hipEventCreate(&e));
  BM25_HIP(hipEventRecord(e, s));
  idx->timing_events.emplace_back(b, e);
  return BM25_OK;
}

// Records the launches that `enqueue` issues into a HIP graph on the scratch's capture stream
// (capture only: nothing runs there) and launches the graph on `s`. The executable graphs are
// kept (two, used in turn); the next batch with the same launch configuration `cfg` (same
// kernels, grid and LDS sizes: only pointers and scalar arguments differ) updates one in place,
// any other is instantiated anew. A kept graph is updated or destroyed only after its own last
// launch has finished. The captured sequence holds kernel launches only, no memset or copy nodes.
template <typename F>
static int launch_as_graph(SearchScratch& sc, hipStream_t s, const std::array<int64_t, 10>& cfg,
                           F& enqueue) {
  if (!sc.cap_stream) BM25_HIP(hipStreamCreateWithFlags(&sc.cap_stream, hipStreamNonBlocking));
  const int slot = sc.graph_next;
  sc.graph_next ^= 1;
  if (!sc.graph_done[slot])
    BM25_HIP(hipEventCreateWithFlags(&sc.graph_done[slot], hipEventDisableTiming));
  BM25_HIP(hipStreamBeginCapture(sc.cap_stream, hipStreamCaptureModeThreadLocal));
  const int rc = enqueue(sc.cap_stream);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(sc.cap_stream, &g);
  if (rc != BM25_OK || ec != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    if (rc != BM25_OK) return rc;
    return set_error(BM25_E_HIP, "graph capture failed: %s", hipGetErrorString(ec));
  }
  hipGraphExec_t& ex = sc.graph_exec[slot];
  if (ex) BM25_HIP(hipEventSynchronize(sc.graph_done[slot]));
  bool updated = false;
  if (ex && sc.graph_cfg[slot] != cfg) {
    (void)hipGraphExecDestroy(ex);
    ex = nullptr;
  }
  if (ex) {
    hipGraphNode_t bad = nullptr;
    hipGraphExecUpdateResult res = hipGraphExecUpdateError;
    if (hipGraphExecUpdate(ex, g, &bad, &res) == hipSuccess && res == hipGraphExecUpdateSuccess) {
      updated = true;
      ++sc.graph_updates;
    } else {
      (void)hipGetLastError();  // a refused update is not an error of this call
      (void)hipGraphExecDestroy(ex);
      ex = nullptr;
    }
  }
  if (!updated) {
    const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
      ex = nullptr;
      (void)hipGraphDestroy(g);
      return set_error(BM25_E_HIP, "graph instantiation failed: %s", hipGetErrorString(ei));
    }
    ++sc.graph_builds;
    sc.graph_cfg[slot] = cfg;
  }
  (void)hipGraphDestroy(g);
  BM25_HIP(hipGraphLaunch(ex, s));
  BM25_HIP(hipEventRecord(sc.graph_done[slot], s));
  return BM25_OK;
}

TileShape batch_shape(const bm25_index* idx, int32_t n, int32_t max_qlen, int32_t k_max) {
  TileShape t;
  if (idx->plan_fixed) {
    t = idx->fixed_plan;
  } else {
    auto it = idx->tuned.find(shape_class(n, max_qlen, k_max));
    t = (it != idx->tuned.end()) ? it->second : choose_shape(idx, n, max_qlen, k_max);
  }
  if (!shape_ok(t, k_max)) {
    // a fixed or tuned plan made for smaller lists: keep its tile, shrink the query tile
    t.q_tile = fit_q_tile(t.q_tile, kpl_for(k_max), t.waves,
                          t.doc_tile / (64 * std::max(1, t.waves)));
  }
  return t;
}

// Tiling of a batch under shape t. Grouped order: the batch is permuted on the device so that
// queries holding the same frequent (dense-row) tokens share query tiles; tiles are then q_tile
// consecutive grouped queries, sized for the longest query. As given: tiles of up to q_tile
// consecutive queries and kTileMaxPositions positions. Writes the tile bounds when tile_q0 is
// not null (room for n + 1 tiles), else bounds n_tiles and ent from above.
struct Tiling {
  bool grouped = false;
  int32_t n_tiles = 0;
  int64_t ent = 0, ecap = 0, pcap = 0;
};

static Tiling tile_batch(const bm25_index* idx, const TileShape& t, const int64_t* q_off,
                         int32_t n, int32_t max_qlen, int64_t positions, int32_t* tile_q0,
                         int64_t* tile_e0) {
  Tiling r;
  const int W = t.waves, QT = t.q_tile;
  const bool dense = !t.sparse_only && idx->n_dense > 0;
  const int64_t grouped_pos = (int64_t)QT * max_qlen;
  r.grouped = t.query_order != 2 && dense && n > QT && grouped_pos <= kTileMaxPositions;
  if (r.grouped) {
    int32_t i = 0;
    for (int32_t q = 0; q < n; q += QT, ++i) {
      if (tile_q0) {
        tile_q0[i] = q;
        tile_e0[i] = r.ent;
      }
      r.ent += grouped_pos + W;
    }
    r.n_tiles = i;
    r.ecap = grouped_pos + W;
    r.pcap = grouped_pos;
  } else if (!tile_q0) {
    r.n_tiles = n;
    r.ent = positions + (int64_t)W * n;
    r.ecap = std::min<int64_t>(positions, kTileMaxPositions) + W;
    r.pcap = std::min<int64_t>(positions, kTileMaxPositions);
  } else {
    int32_t q = 0, i = 0;
    while (q < n) {
      tile_q0[i] = q;
      tile_e0[i] = r.ent;
      int64_t pos = 0;
      int cnt = 0;
      while (q < n && cnt < QT && pos + (q_off[q + 1] - q_off[q]) <= kTileMaxPositions) {
        pos += q_off[q + 1] - q_off[q];
        ++q;
        ++cnt;
      }
      r.ent += pos + W;
      r.ecap = std::max<int64_t>(r.ecap, pos + W);
      r.pcap = std::max<int64_t>(r.pcap, pos);
      ++i;
    }
    r.n_tiles = i;
  }
  if (tile_q0) {
    tile_q0[r.n_tiles] = n;
    tile_e0[r.n_tiles] = r.ent;
  }
  return r;
}

static ArenaNeed batch_need(const TileShape& t, const Tiling& tl, int32_t n, int64_t positions,
                            int32_t k_max) {
  ArenaNeed a;
  a.n = n;
  a.n_tiles = tl.n_tiles;
  a.waves = t.waves;
  a.ent = tl.ent;
  a.positions = positions;
  a.cand_keys = (int64_t)n * t.doc_groups * 64 * kpl_for(k_max);
  a.ordered = tl.n_tiles > 1 && tl.n_tiles <= kOrderMax;
  a.grouped = tl.grouped;
  return a;
}

size_t batch_arena_bytes(const bm25_index* idx, int32_t n, int64_t positions, int32_t max_qlen,
                         int32_t k_max) {
  const TileShape t = batch_shape(idx, n, max_qlen, k_max);
  const Tiling tl = tile_batch(idx, t, nullptr, n, max_qlen, positions, nullptr, nullptr);
  ArenaNeed a = batch_need(t, tl, n, positions, k_max);
  a.ordered = tl.n_tiles > 1;  // an upper bound: the as-given tiling may hold fewer tiles
  return arena_layout(a).total;
}

int search_batch_impl(bm25_index* idx, const int32_t* q_ids, const int64_t* q_off, int32_t n,
                      const int32_t* k, int32_t k_max, int32_t* out_ids, float* out_scores,
                      int32_t* out_count, hipStream_t s, SearchScratch& sc,
                      const TileShape* force) {
  BatchInfo info;
  int rc = check_batch(idx, q_ids, q_off, n, k, k_max, out_ids, out_scores, out_count, info);
  if (rc != BM25_OK || n == 0) return rc;
  const TileShape t = force ? *force : batch_shape(idx, n, info.max_qlen, k_max);
  if (!shape_ok(t, k_max)) return set_error(BM25_E_INVAL, "invalid launch shape");
  const int W = t.waves, QT = t.q_tile, R = t.doc_tile / (64 * t.waves);
  const int KPL = kpl_for(k_max);

  IndexView ix = index_view(idx, t.sparse_only != 0);
  uint8_t* host = nullptr;
  rc = acquire_staging(sc, n, &host);
  if (rc != BM25_OK) return rc;
  Staged hs;
  stage_layout(host, n, hs);
  stage_queries(hs, q_off, k, n, k_max);
  const Tiling tl = tile_batch(idx, t, q_off, n, info.max_qlen, info.positions, hs.tile_q0,
                               hs.tile_e0);
  const bool grouped = tl.grouped;
  const int32_t n_tiles = tl.n_tiles;

  const int64_t lds = gather_lds(t, tl.ecap, tl.pcap);
  if (lds > kMaxLdsBytes) return set_error(BM25_E_INVAL, "launch shape exceeds LDS");
  const int64_t G = t.doc_groups;
  const int64_t ntile_docs = std::max<int64_t>(1, (idx->n_docs + t.doc_tile - 1) / t.doc_tile);
  const int64_t group_docs = ((ntile_docs + G - 1) / G) * t.doc_tile;
  // longest tiles first when there is more than one round of workgroups to balance
  const ArenaNeed need = batch_need(t, tl, n, info.positions, k_max);
  const bool ordered = need.ordered;
  const ArenaLayout L = arena_layout(need);

  rc = scratch_begin(sc, s);
  if (rc != BM25_OK) return rc;
  uint8_t* base = nullptr;
  rc = acquire_arena(sc, L.total, &base);
  if (rc != BM25_OK) return rc;
  Staged dev;
  stage_layout(base + L.meta, n, dev);
  rc = upload_plan(sc, s, n, host, base + L.meta);
  if (rc != BM25_OK) return rc;

  if (grouped) {
    // the kernel takes more than the default 64 KB of LDS (setting it twice is harmless); set
    // before any capture begins
    static std::atomic<bool> reorder_lds{false};
    if (!reorder_lds.load(std::memory_order_acquire)) {
      BM25_HIP(hipFuncSetAttribute((const void*)k_reorder,
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)kReorderLds));
      reorder_lds.store(true, std::memory_order_release);
    }
  }
  const bool graph = idx->use_graphs && !sc.no_alloc;
  int32_t* const s_perm = reinterpret_cast<int32_t*>(base + L.perm);
  uint64_t* const s_cand = reinterpret_cast<uint64_t*>(base + L.cand);
  int32_t* const s_qstat = reinterpret_cast<int32_t*>(base + L.qstat);
  // Everything after the plan upload: grouping, planner, gather, merge. Enqueued on `q`, which
  // is the caller's stream, or the capture stream in graph mode.
  auto enqueue = [&](hipStream_t q) -> int {
    const int32_t* b_ids = q_ids;
    const int64_t* b_off = dev.q_off;
    const int32_t* b_k = dev.q_k;
    if (grouped) {
      ReorderArgs ra;
      ra.q_ids = q_ids;
      ra.q_off = dev.q_off;
      ra.q_k = dev.q_k;
      ra.dense_id = ix.dense_id;
      ra.dense_rank = ix.dense_rank;
      ra.vocab = idx->vocab;
      ra.n = n;
      ra.ids2 = reinterpret_cast<int32_t*>(base + L.ids2);
      ra.off2 = reinterpret_cast<int64_t*>(base + L.off2);
      ra.k2 = reinterpret_cast<int32_t*>(base + L.k2);
      ra.perm = s_perm;
      hipLaunchKernelGGL(k_reorder, dim3((unsigned)((n + kPlanSort - 1) / kPlanSort)),
                         dim3(kPlanThreads), kReorderLds, q, ra);
      BM25_HIP(hipGetLastError());
      b_ids = ra.ids2;
      b_off = ra.off2;
      b_k = ra.k2;
    }
    BatchView bv;
    bv.q_ids = b_ids;
    bv.q_off = b_off;
    bv.q_k = b_k;
    bv.q_stat = s_qstat;
    bv.tile_q0 = dev.tile_q0;
    bv.tile_e0 = dev.tile_e0;
    bv.wave_e0 = reinterpret_cast<int32_t*>(base + L.wave_e0);
    bv.entries = reinterpret_cast<Entry*>(base + L.entries);
    bv.members = reinterpret_cast<int32_t*>(base + L.members);
    bv.dense_ent = reinterpret_cast<DenseEntry*>(base + L.dense_ent);
    bv.dense_n = reinterpret_cast<int32_t*>(base + L.dense_n);
    bv.tile_cost = ordered ? reinterpret_cast<float*>(base + L.tile_cost) : nullptr;
    bv.n_queries = n;
    bv.n_tiles = n_tiles;
    bv.dense_mult_max = dense_mult_max(idx);

    hipLaunchKernelGGL(k_plan, dim3(n_tiles), dim3(kPlanThreads), 0, q, ix, bv, W);
    BM25_HIP(hipGetLastError());
    int32_t* const order = ordered ? reinterpret_cast<int32_t*>(base + L.order) : nullptr;
    if (ordered) {
      hipLaunchKernelGGL(k_order, dim3(1), dim3(kPlanThreads), 0, q, bv.tile_cost, n_tiles,
                         order);
      BM25_HIP(hipGetLastError());
    }

    GatherArgs ga;
    ga.ix = ix;
    ga.bv = bv;
    ga.order = order;
    ga.cand = s_cand;
    ga.group_docs = group_docs;
    ga.n_groups = (int32_t)G;
    ga.ecap = (int32_t)tl.ecap;
    ga.pcap = (int32_t)tl.pcap;
    hipEvent_t tb = nullptr;
    int r = (graph || sc.no_alloc) ? BM25_OK : timed_begin(idx, q, &tb);
    if (r != BM25_OK) return r;
    BM25_HIP(launch_gather(idx->params.store_dtype, W, QT, R, KPL,
                           dim3((unsigned)((int64_t)n_tiles * G)), (size_t)lds, q, ga));
    r = (graph || sc.no_alloc) ? BM25_OK : timed_end(idx, q, tb);
    if (r != BM25_OK) return r;

    MergeArgs ma;
    ma.cand = s_cand;
    ma.q_ids = b_ids;
    ma.q_off = b_off;
    ma.q_k = b_k;
    ma.q_stat = s_qstat;
    ma.theta32 = ix.theta32;
    ma.out_ids = out_ids;
    ma.out_scores = out_scores;
    ma.out_count = out_count;
    ma.perm = grouped ? s_perm : nullptr;
    ma.n_docs = idx->n_docs;
    ma.lists = (int32_t)G;
    ma.k_max = k_max;
    ma.q_first = 0;
    BM25_HIP(launch_merge(KPL, dim3(n), q, ma));
    return BM25_OK;
  };
  if (!graph) {
    rc = enqueue(s);
    if (rc != BM25_OK) return rc;
    return scratch_end(sc, s);
  }
  // graph mode: the timing events (if enabled) bracket the whole graph
  hipEvent_t tb = nullptr;
  rc = timed_begin(idx, s, &tb);
  if (rc != BM25_OK) return rc;
  // launch configuration: every grid size follows from n, n_tiles and G; the kernels and LDS
  // sizes from the shape, list size, store type and grouping
  const std::array<int64_t, 10> cfg = {(int64_t)n, (int64_t)n_tiles, G, lds, (int64_t)W,
                                        (int64_t)QT, (int64_t)R, (int64_t)KPL,
                                        (int64_t)idx->params.store_dtype, (int64_t)grouped};
  rc = launch_as_graph(sc, s, cfg, enqueue);
  if (rc != BM25_OK) return rc;
  rc = timed_end(idx, s, tb);
  if (rc != BM25_OK) return rc;
  return scratch_end(sc, s);
}

int search_plain_impl(bm25_index* idx, const int32_t* q_ids, const int64_t* q_off, int32_t n,
                      const int32_t* k, int32_t k_max, int32_t* out_ids, float* out_scores,
                      int32_t* out_count, hipStream_t s) {
  BatchInfo info;
  int rc = check_batch(idx, q_ids, q_off, n, k, k_max, out_ids, out_scores, out_count, info);
  if (rc != BM25_OK || n == 0) return rc;
  SearchScratch& sc = idx->plain_scratch;
  const int KPL = kpl_for(k_max), KP = 64 * KPL;
  const int W = 1;  // one-wave workgroups: a query's sweepers spread over every CU
  const int DT = 64 * 16;  // documents per wave tile (16 per lane)
  const int64_t ecap = (int64_t)info.max_qlen + 1;
  const int64_t pcap = std::max<int64_t>(info.max_qlen, 1);
  // the list merge at the end reuses the accumulator region
  const int64_t acc_bytes = std::max<int64_t>((int64_t)W * DT * 4, (int64_t)W * KP * 8);
  const int64_t lds =
      acc_bytes + ecap * (kEntryStaticBytes + (int64_t)W * kEntryDynBytes) + pcap * 4 + 64;
  if (lds > kMaxLdsBytes) return set_error(BM25_E_INVAL, "query too long for the per-query form");
  const int64_t nb = std::max<int64_t>(1, idx->n_blocks);
  const int64_t blocks_per_sweep = std::max<int64_t>(1, (nb + 2047) / 2048);
  const int64_t sweep_docs = blocks_per_sweep * kSkipBlock;
  const int64_t sweepers = (idx->n_docs + sweep_docs - 1) / sweep_docs;
  const int64_t G = (sweepers + W - 1) / W;

  uint8_t* host = nullptr;
  rc = acquire_staging(sc, n, &host);
  if (rc != BM25_OK) return rc;
  Staged hs;
  stage_layout(host, n, hs);
  stage_queries(hs, q_off, k, n, k_max);
  int64_t ent = 0;
  for (int32_t i = 0; i < n; ++i) {
    hs.tile_q0[i] = i;
    hs.tile_e0[i] = ent;
    ent += (q_off[i + 1] - q_off[i]) + 1;
  }
  hs.tile_q0[n] = n;
  hs.tile_e0[n] = ent;

  // candidate lists of up to kPlainMergeBatch queries (and at most kPlainCandBytes), merged by
  // one launch per batch
  const int64_t cand_per_query = G * KP * 8;
  const int32_t mb = (int32_t)std::max<int64_t>(
      1, std::min<int64_t>({(int64_t)n, (int64_t)kPlainMergeBatch, kPlainCandBytes / cand_per_query}));
  ArenaNeed need;
  need.n = n;
  need.n_tiles = n;
  need.waves = 1;
  need.ent = ent;
  need.positions = info.positions;
  need.cand_keys = (int64_t)mb * G * KP;
  const ArenaLayout L = arena_layout(need);
  rc = scratch_begin(sc, s);
  if (rc != BM25_OK) return rc;
  uint8_t* base = nullptr;
  rc = acquire_arena(sc, L.total, &base);
  if (rc != BM25_OK) return rc;
  Staged dev;
  stage_layout(base + L.meta, n, dev);
  rc = upload_plan(sc, s, n, host, base + L.meta);
  if (rc != BM25_OK) return rc;
  uint64_t* const s_cand = reinterpret_cast<uint64_t*>(base + L.cand);
  int32_t* const s_qstat = reinterpret_cast<int32_t*>(base + L.qstat);

  IndexView ix = index_view(idx, idx->plan_fixed && idx->fixed_plan.sparse_only != 0);
  BatchView bv;
  bv.q_ids = q_ids;
  bv.q_off = dev.q_off;
  bv.q_k = dev.q_k;
  bv.q_stat = s_qstat;
  bv.tile_q0 = dev.tile_q0;
  bv.tile_e0 = dev.tile_e0;
  bv.wave_e0 = reinterpret_cast<int32_t*>(base + L.wave_e0);
  bv.entries = reinterpret_cast<Entry*>(base + L.entries);
  bv.members = reinterpret_cast<int32_t*>(base + L.members);
  bv.dense_ent = reinterpret_cast<DenseEntry*>(base + L.dense_ent);
  bv.dense_n = reinterpret_cast<int32_t*>(base + L.dense_n);
  bv.n_queries = n;
  bv.n_tiles = n;
  hipLaunchKernelGGL(k_plan, dim3(n), dim3(kPlanThreads), 0, s, ix, bv, 1);
  BM25_HIP(hipGetLastError());

  SweepArgs sa;
  sa.ix = ix;
  sa.bv = bv;
  sa.cand = s_cand;
  sa.sweep_docs = sweep_docs;
  sa.n_groups = (int32_t)G;
  sa.acc_bytes = (int32_t)acc_bytes;
  sa.ecap = (int32_t)ecap;
  sa.pcap = (int32_t)pcap;
  MergeArgs ma;
  ma.cand = s_cand;
  ma.q_ids = q_ids;
  ma.q_off = dev.q_off;
  ma.q_k = dev.q_k;
  ma.q_stat = s_qstat;
  ma.theta32 = ix.theta32;
  ma.out_ids = out_ids;
  ma.out_scores = out_scores;
  ma.out_count = out_count;
  ma.perm = nullptr;
  ma.n_docs = idx->n_docs;
  ma.lists = (int32_t)G;
  ma.k_max = k_max;
  for (int32_t i0 = 0; i0 < n; i0 += mb) {
    const int32_t i1 = std::min<int32_t>(n, i0 + mb);
    for (int32_t i = i0; i < i1; ++i) {
      sa.query = i;
      sa.cand = s_cand + (size_t)(i - i0) * G * KP;
      hipEvent_t tb;
      rc = timed_begin(idx, s, &tb);
      if (rc != BM25_OK) return rc;
      BM25_HIP(
          launch_sweep(idx->params.store_dtype, W, KPL, dim3((unsigned)G), (size_t)lds, s, sa));
      rc = timed_end(idx, s, tb);
      if (rc != BM25_OK) return rc;
    }
    ma.q_first = i0;
    BM25_HIP(launch_merge(KPL, dim3((unsigned)(i1 - i0)), s, ma));
  }
  return scratch_end(sc, s);
}

// Scratch of bm25_search_batch_noalloc. In host code `scratch` only names the array: its device
// address comes from hipGetSymbolAddress, once per device (each device holds its own copy), and
// only that address is handed to kernels or copies.
static constexpr size_t kNoAllocScratchBytes = (size_t)BM25_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];
static constexpr int kNoAllocMaxDevices = 64;
static std::atomic<uint8_t*> g_scratch_ptr[kNoAllocMaxDevices];
static std::mutex g_scratch_mu;
// Host staging of the plan (pageable: hipMemcpyAsync has consumed it when it returns).
static uint8_t g_noalloc_staging[(size_t)BM25_NOALLOC_MAX_QUERIES * 24 + 4096];

static int noalloc_scratch(int device, uint8_t** ptr) {
  if (device < 0 || device >= kNoAllocMaxDevices)
    return set_error(BM25_E_INVAL, "device %d outside the %d devices served", device,
                     kNoAllocMaxDevices);
  uint8_t* p = g_scratch_ptr[device].load(std::memory_order_acquire);
  if (!p) {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    p = g_scratch_ptr[device].load(std::memory_order_acquire);
    if (!p) {
      void* a = nullptr;
      const hipError_t e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !a)
        return set_error(BM25_E_HIP, "hipGetSymbolAddress of the scratch array failed: %s",
                         hipGetErrorString(e));
      p = static_cast<uint8_t*>(a);
      g_scratch_ptr[device].store(p, std::memory_order_release);
    }
  }
  *ptr = p;
  return BM25_OK;
}

}  // namespace bm25

using namespace bm25;

extern "C" int bm25_search_batch_noalloc(const bm25_index* index, const int32_t* q_ids,
                                         const int64_t* q_offsets, int32_t n_queries,
                                         const int32_t* k, int32_t k_max, int32_t* out_ids,
                                         float* out_scores, int32_t* out_count, void* stream) {
  clear_error();
  if (!index) return set_error(BM25_E_INVAL, "index is NULL");
  if (n_queries > BM25_NOALLOC_MAX_QUERIES)
    return set_error(BM25_E_NOMEM, "%d queries exceed the %d this entry point plans without "
                     "allocating", n_queries, BM25_NOALLOC_MAX_QUERIES);
  int device = 0;
  BM25_HIP(hipGetDevice(&device));
  if (device != index->device)
    return set_error(BM25_E_INVAL, "the index lives on device %d, the current device is %d",
                     index->device, device);
  uint8_t* base = nullptr;
  int rc = noalloc_scratch(device, &base);
  if (rc != BM25_OK) return rc;
  bm25_index* idx = const_cast<bm25_index*>(index);
  std::lock_guard<std::mutex> g(idx->mu);
  SearchScratch sc;
  sc.fixed = base;
  sc.fixed_bytes = kNoAllocScratchBytes;
  sc.host_fixed = g_noalloc_staging;
  sc.host_fixed_bytes = sizeof(g_noalloc_staging);
  sc.no_alloc = true;
  return search_batch_impl(idx, q_ids, q_offsets, n_queries, k, k_max, out_ids, out_scores,
                           out_count, (hipStream_t)stream, sc, nullptr);
}

extern "C" int bm25_search_batch(const bm25_index* index, const int32_t* q_ids,
                                 const int64_t* q_offsets, int32_t n_queries, const int32_t* k,
                                 int32_t k_max, int32_t* out_ids, float* out_scores,
                                 int32_t* out_count, void* stream) {
  clear_error();
  if (!index) return set_error(BM25_E_INVAL, "index is NULL");
  bm25_index* idx = const_cast<bm25_index*>(index);
  std::lock_guard<std::mutex> g(idx->mu);
  idx->alloc.stream = (hipStream_t)stream;
  return search_batch_impl(idx, q_ids, q_offsets, n_queries, k, k_max, out_ids, out_scores,
                           out_count, (hipStream_t)stream, idx->batch_scratch, nullptr);
}

extern "C" int bm25_search_plain(const bm25_index* index, const int32_t* q_ids,
                                 const int64_t* q_offsets, int32_t n_queries, const int32_t* k,
                                 int32_t k_max, int32_t* out_ids, float* out_scores,
                                 int32_t* out_count, void* stream) {
  clear_error();
  if (!index) return set_error(BM25_E_INVAL, "index is NULL");
  bm25_index* idx = const_cast<bm25_index*>(index);
  std::lock_guard<std::mutex> g(idx->mu);
  idx->alloc.stream = (hipStream_t)stream;
  return search_plain_impl(idx, q_ids, q_offsets, n_queries, k, k_max, out_ids, out_scores,
                           out_count, (hipStream_t)stream);
}

extern "C" int bm25_search_set_plan(bm25_index* index, const bm25_tile_plan* plan) {
  clear_error();
  if (!index) return set_error(BM25_E_INVAL, "index is NULL");
  std::lock_guard<std::mutex> g(index->mu);
  if (!plan) {
    index->plan_fixed = false;
    return BM25_OK;
  }
  TileShape t;
  t.q_tile = plan->q_tile;
  t.waves = plan->waves;
  t.doc_tile = plan->doc_tile;
  t.doc_groups = plan->doc_groups;
  t.query_order = plan->query_order;
  t.sparse_only = plan->sparse_only;
  if (!shape_ok(t, 64)) return set_error(BM25_E_INVAL, "plan fields out of range");
  index->fixed_plan = t;
  index->plan_fixed = true;
  return BM25_OK;
}

extern "C" int bm25_search_get_plan(const bm25_index* index, int32_t n_queries,
                                    int32_t max_query_len, int32_t k_max, bm25_tile_plan* plan) {
  clear_error();
  if (!index || !plan) return set_error(BM25_E_INVAL, "NULL argument");
  bm25_index* idx = const_cast<bm25_index*>(index);
  std::lock_guard<std::mutex> g(idx->mu);
  const TileShape t = batch_shape(idx, n_queries, max_query_len, k_max);
  plan->q_tile = t.q_tile;
  plan->waves = t.waves;
  plan->doc_tile = t.doc_tile;
  plan->doc_groups = t.doc_groups;
  plan->query_order = t.query_order;
  plan->sparse_only = t.sparse_only;
  return BM25_OK;
}

extern "C" int bm25_search_set_graphs(bm25_index* index, int32_t enable) {
  clear_error();
  if (!index) return set_error(BM25_E_INVAL, "index is NULL");
  std::lock_guard<std::mutex> g(index->mu);
  index->use_graphs = enable != 0;
  return BM25_OK;
}

extern "C" int bm25_search_graph_stats(const bm25_index* index, int64_t* builds,
                                       int64_t* updates) {
  clear_error();
  if (!index || !builds || !updates) return set_error(BM25_E_INVAL, "NULL argument");
  bm25_index* idx = const_cast<bm25_index*>(index);
  std::lock_guard<std::mutex> g(idx->mu);
  *builds = idx->batch_scratch.graph_builds;
  *updates = idx->batch_scratch.graph_updates;
  return BM25_OK;
}

extern "C" int bm25_autotune(bm25_index* index, const int32_t* q_ids, const int64_t* q_offsets,
                             int32_t n_queries, const int32_t* k, int32_t k_max,
                             int32_t* out_ids, float* out_scores, int32_t* out_count,
                             void* stream, bm25_tile_plan* best) {
  clear_error();
  if (!index) return set_error(BM25_E_INVAL, "index is NULL");
  std::lock_guard<std::mutex> g(index->mu);
  BatchInfo info;
  int rc = check_batch(index, q_ids, q_offsets, n_queries, k, k_max, out_ids, out_scores,
                       out_count, info);
  if (rc != BM25_OK) return rc;
  if (n_queries == 0) return set_error(BM25_E_INVAL, "autotune needs at least one query");
  hipStream_t s = (hipStream_t)stream;
  index->alloc.stream = s;
  const TileShape base = choose_shape(index, n_queries, info.max_qlen, k_max);
  std::vector<TileShape> cands;
  const int kpl = kpl_for(k_max);
  const int wr[3][2] = {{8, 2}, {4, 4}, {8, 4}};
  for (const auto& shp : wr)
    for (int qt : {shp[0], 2 * shp[0], 4 * shp[0]})
      for (int gmul : {1, 2, 4}) {
        TileShape t = base;
        t.waves = shp[0];
        t.doc_tile = 64 * shp[0] * shp[1];
        t.q_tile = qt;
        if (!shape_ok(t, k_max)) continue;
        const int64_t ntiles = (n_queries + t.q_tile - 1) / t.q_tile;
        int64_t gg = (1024 * gmul + ntiles - 1) / ntiles;
        gg = ((gg + 7) / 8) * 8;
        gg = std::min<int64_t>(std::max<int64_t>(gg, 8), 1024);
        gg = std::min<int64_t>(gg, std::max<int64_t>(1, (index->n_docs + t.doc_tile - 1) /
                                                             t.doc_tile));
        t.doc_groups = (int)gg;
        const int64_t pc =
            std::min<int64_t>((int64_t)t.q_tile * info.max_qlen, kTileMaxPositions);
        if (gather_lds(t, pc + t.waves, pc) > 128 * 1024) continue;
        (void)kpl;
        cands.push_back(t);
      }
  hipEvent_t e0, e1;
  BM25_HIP(hipEventCreate(&e0));
  BM25_HIP(hipEventCreate(&e1));
  float best_ms = 1e30f;
  TileShape best_t = base;
  for (const TileShape& t : cands) {
    // one warm-up, then two timed runs
    rc = search_batch_impl(index, q_ids, q_offsets, n_queries, k, k_max, out_ids, out_scores,
                           out_count, s, index->batch_scratch, &t);
    if (rc != BM25_OK) continue;
    BM25_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < 2; ++r)
      (void)search_batch_impl(index, q_ids, q_offsets, n_queries, k, k_max, out_ids, out_scores,
                              out_count, s, index->batch_scratch, &t);
    BM25_HIP(hipEventRecord(e1, s));
    BM25_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    BM25_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best_ms) {
      best_ms = ms;
      best_t = t;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  index->tuned[shape_class(n_queries, info.max_qlen, k_max)] = best_t;
  if (best) {
    best->q_tile = best_t.q_tile;
    best->waves = best_t.waves;
    best->doc_tile = best_t.doc_tile;
    best->doc_groups = best_t.doc_groups;
    best->query_order = best_t.query_order;
    best->sparse_only = best_t.sparse_only;
  }
  clear_error();
  return BM25_OK;
}
