// Query-time kernels: planner, cursor search, batched gather + top-k, per-query sweep, merge.
//
// Query scoring follows Section 2 ("Assigning Query Scores"): the rows of the query's tokens are
// sliced from the token-major score matrix and summed, position by position, into one FP32
// accumulator per document; "Top-k selection" keeps the k best. Section 2.1's shift is added to
// the returned scores of shifted variants in the merge kernel.
//
// Layout of the work:
//   * a query tile is a run of consecutive queries of the batch; its planner entry table lists
//     the distinct tokens of the tile, each with the (query, multiplicity) pairs that use it.
//     A token whose posting volume times member count dominates the tile is split into several
//     entries over disjoint member subsets, and entries are dealt to the waves of the workgroup
//     in descending cost ("snake" order) so that waves carry similar loads;
//   * the documents are cut into doc groups (multiples of the skip block); a workgroup owns one
//     (query tile, doc group) pair and sweeps the group in LDS tiles of doc_tile documents,
//     keeping one FP32 accumulator row per query of the tile;
//   * each wave keeps, in registers, the best keys of the queries it owns (TopList) and filters
//     every tile against its current k-th key.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.hpp"

namespace bm25dev {

constexpr int kPlanThreads = 256;
constexpr int kTileMaxPositions = 4080;  // positions in one query tile (LDS sort capacity)
constexpr int kPlanSort = 4096;          // power-of-two sort capacity
constexpr int64_t kSkipBlockDev = 1024;  // must equal bm25::kSkipBlock

struct Entry {
  int64_t row_lo;   // first entry of the token's row
  int64_t row_hi;   // one past the last
  int32_t mem_off;  // first member in the member list
  int32_t mem_cnt;  // members (<= 64)
  int32_t long_id;  // row id in the skip table, or -1
  int32_t token;
};

struct IndexView {
  const int64_t* indptr;
  const int32_t* indices;
  const void* data;
  const int32_t* long_id;
  const uint32_t* skip;
  const float* theta32;  // nullptr for sparse variants
  int64_t n_docs;
  int64_t n_blocks;
  int32_t vocab;
};

struct BatchView {
  const int32_t* q_ids;    // device token ids of the batch
  const int64_t* q_off;    // device [n+1]
  const int32_t* q_k;      // device [n]
  int32_t* q_stat;         // device [n]: 1 if the query holds an id outside [0, V)
  const int32_t* tile_q0;  // [n_tiles+1]
  const int64_t* tile_e0;  // [n_tiles+1]: entry base of each tile
  int32_t* wave_e0;        // [n_tiles * (W+1)]: entry range of each wave inside the tile
  Entry* entries;
  int32_t* members;        // q_local | mult << 16
  int32_t n_queries;
  int32_t n_tiles;
};

// ------------------------------------------------------------------------------------------
// Planner: one workgroup per query tile.

template <typename T>
__device__ T block_scan_excl_256(T v, T* lds4, T& total) {
  const int l = lane();
  const int w = threadIdx.x >> 6;
  T x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    T y;
    if constexpr (sizeof(T) == 8)
      y = (T)bperm64((uint64_t)x, (l - o) & 63);
    else
      y = (T)bperm((uint32_t)x, (l - o) & 63);
    if (l >= o) x += y;
  }
  if (l == 63) lds4[w] = x;
  __syncthreads();
  T off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kPlanThreads / 64; ++i) {
    T t = lds4[i];
    if (i < w) off += t;
    tot += t;
  }
  __syncthreads();
  total = tot;
  return x - v + off;
}

// Exclusive scan of n (<= kPlanSort) uint32 values held in LDS, in place; returns the total.
static __device__ uint32_t lds_scan_u32(uint32_t* a, int n, uint32_t* lds4) {
  constexpr int per = kPlanSort / kPlanThreads;  // 16
  const int base = threadIdx.x * per;
  uint32_t v[per];
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < per; ++i) {
    v[i] = (base + i < n) ? a[base + i] : 0u;
    s += v[i];
  }
  uint32_t tot;
  uint32_t off = block_scan_excl_256<uint32_t>(s, lds4, tot);
#pragma unroll
  for (int i = 0; i < per; ++i) {
    if (base + i < n) a[base + i] = off;
    off += v[i];
  }
  __syncthreads();
  return tot;
}

// Ascending bitonic sort of n (power of two) uint64 keys in LDS.
static __device__ void lds_bitonic_sort(uint64_t* s, int n) {
  for (int k = 2; k <= n; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const uint64_t a = s[i], b = s[ixj];
          const bool asc = (i & k) == 0;
          if ((a > b) == asc) {
            s[i] = b;
            s[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
  }
}

struct PlanSmem {
  uint64_t key[kPlanSort];
  uint32_t pos_of_member[kPlanSort + 1];
  uint32_t first_member[kPlanSort + 1];  // per distinct token: first member index
  int32_t tok[kPlanSort];
  uint32_t parts[kPlanSort + 1];         // per distinct token: number of entries
  uint32_t tmp[kPlanSort + 1];
  int64_t qoff[65];
  uint32_t err[64];
  float cost_sum[4];
  uint32_t lds4[4];
  uint32_t counters[4];
};

#ifdef BM25_SEARCH_MAIN
// W: waves of the consuming gather kernel (entries are dealt to them); W == 1 disables splits.
__global__ __launch_bounds__(kPlanThreads) void k_plan(IndexView ix, BatchView bv, int W) {
  __shared__ PlanSmem sm;
  const int tile = blockIdx.x;
  const int tid = threadIdx.x;
  const int q0 = bv.tile_q0[tile], q1 = bv.tile_q0[tile + 1];
  const int nq = q1 - q0;
  const int64_t p0 = bv.q_off[q0];
  const int P = (int)(bv.q_off[q1] - p0);
  for (int i = tid; i <= nq; i += kPlanThreads) sm.qoff[i] = bv.q_off[q0 + i] - p0;
  for (int i = tid; i < nq; i += kPlanThreads) sm.err[i] = 0;
  __syncthreads();

  // 1. (token, query) keys; ids outside [0, V) mark the query and are dropped
  int npow = 1;
  while (npow < P) npow <<= 1;
  for (int i = tid; i < npow; i += kPlanThreads) {
    uint64_t key = ~0ull;
    if (i < P) {
      int lo = 0, hi = nq - 1;  // query holding position i
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sm.qoff[mid] <= i) lo = mid; else hi = mid - 1;
      }
      const int32_t t = bv.q_ids[p0 + i];
      if (t < 0 || t >= ix.vocab) {
        sm.err[lo] = 1;
      } else {
        key = ((uint64_t)(uint32_t)t << 32) | (uint32_t)lo;
      }
    }
    sm.key[i] = key;
  }
  __syncthreads();
  lds_bitonic_sort(sm.key, npow);

  // 2. members (distinct (token, query) pairs) and distinct tokens
  //    tmp[i] = 1 at the first position of each pair; parts[i] = 1 at the first of each token
  for (int i = tid; i < kPlanSort; i += kPlanThreads) {
    uint32_t ph = 0, th = 0;
    if (i < P) {
      const uint64_t k = sm.key[i];
      if (k != ~0ull) {
        const uint64_t prev = (i > 0) ? sm.key[i - 1] : ~0ull;
        ph = (i == 0 || k != prev) ? 1u : 0u;
        th = (i == 0 || (k >> 32) != (prev >> 32)) ? 1u : 0u;
      }
    }
    sm.tmp[i] = ph;
    sm.parts[i] = th;
  }
  __syncthreads();
  // flags -> exclusive ranks (keep a copy of the flags in first_member/pos_of_member first)
  for (int i = tid; i < kPlanSort; i += kPlanThreads) {
    sm.pos_of_member[i] = sm.tmp[i];
    sm.first_member[i] = sm.parts[i];
  }
  __syncthreads();
  const uint32_t n_mem = lds_scan_u32(sm.tmp, kPlanSort, sm.lds4);
  const uint32_t n_tok = lds_scan_u32(sm.parts, kPlanSort, sm.lds4);
  // scatter: pos_of_member[m] = i, tok[u] = token, first_member[u] = member rank
  uint32_t* mflag = sm.pos_of_member;  // reused below; read flags into registers first
  uint32_t fl_m[kPlanSort / kPlanThreads], fl_t[kPlanSort / kPlanThreads];
#pragma unroll
  for (int r = 0; r < kPlanSort / kPlanThreads; ++r) {
    const int i = tid + r * kPlanThreads;
    fl_m[r] = mflag[i];
    fl_t[r] = sm.first_member[i];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kPlanSort / kPlanThreads; ++r) {
    const int i = tid + r * kPlanThreads;
    if (fl_m[r]) sm.pos_of_member[sm.tmp[i]] = (uint32_t)i;
    if (fl_t[r]) {
      const uint32_t u = sm.parts[i];
      sm.tok[u] = (int32_t)(sm.key[i] >> 32);
      sm.first_member[u] = sm.tmp[i];
    }
  }
  if (tid == 0) {
    uint32_t valid = 0;  // number of valid positions = first invalid index
    // positions are sorted with invalid keys last
    int lo = 0, hi = P;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (sm.key[mid] != ~0ull) lo = mid + 1; else hi = mid;
    }
    valid = (uint32_t)lo;
    sm.pos_of_member[n_mem] = valid;
    sm.first_member[n_tok] = n_mem;
  }
  __syncthreads();

  // 3. member list: q_local | multiplicity << 16
  for (uint32_t m = tid; m < n_mem; m += kPlanThreads) {
    const uint32_t i = sm.pos_of_member[m];
    const uint32_t mult = sm.pos_of_member[m + 1] - i;
    const uint32_t ql = (uint32_t)(sm.key[i] & 0xFFFFu);
    bv.members[p0 + m] = (int32_t)(ql | (mult << 16));
  }

  // 4. cost of each token and number of entries it is split into
  float local = 0.f;
  for (uint32_t u = tid; u < n_tok; u += kPlanThreads) {
    const int32_t t = sm.tok[u];
    const float df = (float)(ix.indptr[t + 1] - ix.indptr[t]);
    const float mc = (float)(sm.first_member[u + 1] - sm.first_member[u]);
    local += df * mc;
  }
  // block sum of the cost
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) local += __shfl_xor(local, o);
  if (lane() == 0) sm.cost_sum[tid >> 6] = local;
  __syncthreads();
  const float total = sm.cost_sum[0] + sm.cost_sum[1] + sm.cost_sum[2] + sm.cost_sum[3];
  const float target = total / (float)W;
  for (int u = tid; u < kPlanSort; u += kPlanThreads) {
    uint32_t parts = 0;
    if ((uint32_t)u < n_tok) {
      const int32_t t = sm.tok[u];
      const int64_t df = ix.indptr[t + 1] - ix.indptr[t];
      const uint32_t mc = sm.first_member[u + 1] - sm.first_member[u];
      if (df > 0) {
        parts = 1;
        if (W > 1 && mc > 1 && target > 0.f) {
          const float c = (float)df * (float)mc;
          uint32_t want = (uint32_t)ceilf(c / target);
          if (want > mc) want = mc;
          if (want > (uint32_t)W) want = (uint32_t)W;
          if (want > 1) parts = want;
        }
      }
    }
    sm.parts[u] = parts;
  }
  __syncthreads();
  // entry ranks per token (parts[] becomes exclusive offsets); the tile has room for
  // n_tok + W entries, so if rounding produced more splits than that, split nothing
  for (int u = tid; u < kPlanSort; u += kPlanThreads) sm.tmp[u] = sm.parts[u];
  __syncthreads();
  uint32_t n_ent = lds_scan_u32(sm.parts, kPlanSort, sm.lds4);
  if (n_ent > n_tok + (uint32_t)W) {
    for (int u = tid; u < kPlanSort; u += kPlanThreads) {
      const uint32_t p1 = sm.tmp[u] > 0 ? 1u : 0u;
      sm.tmp[u] = p1;
      sm.parts[u] = p1;
    }
    __syncthreads();
    n_ent = lds_scan_u32(sm.parts, kPlanSort, sm.lds4);
  }
  // 5. sort entries by cost (descending); key = (~cost << 32) | (u << 8 | part)
  //    reuse key[] (positions are no longer needed)
  int epow = 1;
  while (epow < (int)n_ent) epow <<= 1;
  for (int i = tid; i < epow; i += kPlanThreads) sm.key[i] = ~0ull;
  __syncthreads();
  for (uint32_t u = tid; u < n_tok; u += kPlanThreads) {
    const uint32_t np = sm.tmp[u];
    if (np == 0) continue;
    const int32_t t = sm.tok[u];
    const int64_t df = ix.indptr[t + 1] - ix.indptr[t];
    const uint32_t mc = sm.first_member[u + 1] - sm.first_member[u];
    for (uint32_t j = 0; j < np; ++j) {
      const uint32_t cnt = mc / np + (j < mc % np ? 1u : 0u);
      uint64_t cost = (uint64_t)df * cnt;
      if (cost > 0xFFFFFFFFull) cost = 0xFFFFFFFFull;
      sm.key[sm.parts[u] + j] = ((uint64_t)(~(uint32_t)cost) << 32) | ((uint64_t)u << 8) | j;
    }
  }
  __syncthreads();
  lds_bitonic_sort(sm.key, epow);

  // 6. deal entries to waves in snake order; wave w receives ranks with w(r) == w
  const int64_t e_base = bv.tile_e0[tile];
  const int R = (int)n_ent / W, rem = (int)n_ent % W;
  if (tid == 0) {
    int32_t* we = bv.wave_e0 + (int64_t)tile * (W + 1);
    int acc = 0;
    for (int w = 0; w < W; ++w) {
      we[w] = acc;
      const bool extra = rem > 0 && ((R % 2 == 0) ? (w < rem) : (w >= W - rem));
      acc += R + (extra ? 1 : 0);
    }
    we[W] = acc;
  }
  __syncthreads();
  const int32_t* we = bv.wave_e0 + (int64_t)tile * (W + 1);
  for (uint32_t r = tid; r < n_ent; r += kPlanThreads) {
    const uint64_t k = sm.key[r];
    const uint32_t u = (uint32_t)((k >> 8) & 0xFFFFFFu);
    const uint32_t j = (uint32_t)(k & 0xFFu);
    const int32_t t = sm.tok[u];
    const uint32_t np = sm.tmp[u];
    const uint32_t mc = sm.first_member[u + 1] - sm.first_member[u];
    uint32_t start = 0;
    for (uint32_t jj = 0; jj < j; ++jj) start += mc / np + (jj < mc % np ? 1u : 0u);
    const uint32_t cnt = mc / np + (j < mc % np ? 1u : 0u);
    const int row = (int)r / W, col = (int)r % W;
    const int w = (row % 2 == 0) ? col : (W - 1 - col);
    Entry e;
    e.row_lo = ix.indptr[t];
    e.row_hi = ix.indptr[t + 1];
    e.mem_off = (int32_t)(p0 + sm.first_member[u] + start);
    e.mem_cnt = (int32_t)cnt;
    e.long_id = ix.long_id[t];
    e.token = t;
    bv.entries[e_base + we[w] + row] = e;
  }
  __syncthreads();
  // 7. per-query status (errors were recorded in step 1; err[] was not touched since)
  for (int i = tid; i < nq; i += kPlanThreads) bv.q_stat[q0 + i] = (int32_t)sm.err[i];
}
#endif  // BM25_SEARCH_MAIN

// ------------------------------------------------------------------------------------------
// Cursor search: offset inside the row of the first entry with document id >= d0.
// Long rows read the skip table (d0 is a multiple of the skip block). Other rows (fewer than
// 4096 entries) compare d0 against every 64th entry of the row, then scan one 64-entry chunk.
// Whole wave, uniform arguments.
__device__ __forceinline__ int64_t find_cursor(const IndexView& ix, const Entry& e, int64_t d0) {
  if (d0 <= 0) return 0;
  const int64_t len = e.row_hi - e.row_lo;
  if (len == 0) return 0;
  if (e.long_id >= 0) {
    const int64_t b = d0 / kSkipBlockDev;
    return (int64_t)ix.skip[(int64_t)e.long_id * (ix.n_blocks + 1) + b];
  }
  const int l = lane();
  // samples at absolute positions 64*j inside [row_lo, row_hi)
  const int64_t j0 = (e.row_lo + 63) >> 6;
  const int64_t j1 = (e.row_hi - 1) >> 6;  // inclusive
  const int64_t js = j0 + l;
  const bool has = js <= j1;
  const int32_t sv = has ? ix.indices[js << 6] : INT32_MAX;
  const int c_s = __popcll(ballot(has && sv < d0));
  // chunk to scan: before the first sample if c_s == 0, else from the last sample below d0
  const int64_t from = (c_s == 0) ? e.row_lo : ((j0 + c_s - 1) << 6);
  const int64_t p = from + l;
  const bool in = p < e.row_hi && p < from + 64;
  const int32_t v = in ? ix.indices[p] : INT32_MAX;
  const int c = __popcll(ballot(in && v < d0));
  return from + c - e.row_lo;
}

// ------------------------------------------------------------------------------------------
// Batched gather + top-k. Workgroup = (query tile, doc group); W waves; QPW queries per wave.

struct GatherArgs {
  IndexView ix;
  BatchView bv;
  uint64_t* cand;       // [n_queries][n_groups][KP]
  int64_t group_docs;   // multiple of the skip block
  int32_t n_groups;
  int32_t doc_tile;     // multiple of 256
  int32_t ecap;         // cursor slots per workgroup (>= entries of any tile)
};

__device__ __forceinline__ void map_block(int bid, int n_groups, int& tile, int& group) {
  if ((n_groups & 7) == 0) {
    // consecutive workgroup ids land on different XCDs (round-robin); give every XCD its own
    // doc groups so that the posting segments it reads stay in its L2
    const int xcd = bid & 7;
    const int j = bid >> 3;
    const int gpx = n_groups >> 3;
    group = xcd * gpx + (j % gpx);
    tile = j / gpx;
  } else {
    group = bid % n_groups;
    tile = bid / n_groups;
  }
}

template <int W, int QPW, int KPL, typename ST>
__global__ __launch_bounds__(W * 64) void k_gather(GatherArgs a) {
  constexpr int QT = W * QPW;
  constexpr int KP = KPL * 64;
  extern __shared__ __align__(16) uint8_t smem[];
  const int DT = a.doc_tile;
  float* acc = reinterpret_cast<float*>(smem);
  int32_t* cursor = reinterpret_cast<int32_t*>(smem + (size_t)QT * DT * 4);

  int tile, group;
  map_block(blockIdx.x, a.n_groups, tile, group);
  const int w = threadIdx.x >> 6;
  const int l = lane();
  const BatchView& bv = a.bv;
  const IndexView& ix = a.ix;
  const int q0 = bv.tile_q0[tile];
  const int nq = bv.tile_q0[tile + 1] - q0;
  const int64_t e_base = bv.tile_e0[tile];
  const int32_t* we = bv.wave_e0 + (int64_t)tile * (W + 1);
  const int e_lo = we[w], e_hi = we[w + 1];
  const int64_t d_lo = (int64_t)group * a.group_docs;
  const int64_t d_hi = (d_lo + a.group_docs < ix.n_docs) ? d_lo + a.group_docs : ix.n_docs;
  const typename ST::T* data = reinterpret_cast<const typename ST::T*>(ix.data);

  for (int e = e_lo; e < e_hi; ++e) {
    const Entry en = bv.entries[e_base + e];
    const int64_t c = (d_lo < d_hi) ? find_cursor(ix, en, d_lo) : 0;
    if (l == 0) cursor[e] = (int32_t)c;
  }
  {
    float4* a4 = reinterpret_cast<float4*>(acc);
    const int n4 = QT * DT / 4;
    for (int i = threadIdx.x; i < n4; i += W * 64) a4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  TopList<KPL> L[QPW];
  uint64_t thr[QPW];
  int cap[QPW];
#pragma unroll
  for (int j = 0; j < QPW; ++j) {
    L[j].clear();
    thr[j] = 0;
    const int ql = w * QPW + j;
    cap[j] = (ql < nq) ? bv.q_k[q0 + ql] : 1;
  }
  __syncthreads();

  for (int64_t t0 = d_lo; t0 < d_hi; t0 += DT) {
    const int64_t t1 = (t0 + DT < d_hi) ? t0 + DT : d_hi;
    const int32_t t1i = (int32_t)t1;
    // accumulate this wave's entries into the tile
    for (int e = e_lo; e < e_hi; ++e) {
      const Entry en = bv.entries[e_base + e];
      const int64_t len = en.row_hi - en.row_lo;
      int64_t c = cursor[e];
      const int32_t mem = (l < en.mem_cnt) ? bv.members[en.mem_off + l] : 0;
      while (true) {
        const int64_t off = c + l;
        const bool in_row = off < len;
        const int32_t d = in_row ? ix.indices[en.row_lo + off] : INT32_MAX;
        const bool v = d < t1i && d >= (int32_t)t0;
        const float s = v ? ST::load(data, en.row_lo + off) : 0.f;
        const int rel = d - (int32_t)t0;
        for (int m = 0; m < en.mem_cnt; ++m) {
          const uint32_t mm = readlane((uint32_t)mem, m);
          const int ql = (int)(mm & 0xFFFFu);
          const float mult = (float)(mm >> 16);
          if (v) atomicAdd(&acc[ql * DT + rel], s * mult);
        }
        const int n = __popcll(ballot(v));
        c += n;
        if (n < 64) break;
      }
      if (l == 0) cursor[e] = (int32_t)c;
    }
    __syncthreads();
    // select: filter each owned query's row against its k-th key, then clear it
#pragma unroll
    for (int j = 0; j < QPW; ++j) {
      const int ql = w * QPW + j;
      if (ql < nq) {
        float4* row = reinterpret_cast<float4*>(acc + ql * DT);
        for (int i = l; i < DT / 4; i += 64) {
          const float4 v4 = row[i];
          row[i] = make_float4(0.f, 0.f, 0.f, 0.f);
          const int64_t db = t0 + 4 * i;
          const float vs[4] = {v4.x, v4.y, v4.z, v4.w};
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const int64_t doc = db + c;
            const uint64_t key = (doc < t1) ? make_key(vs[c], (uint32_t)doc) : 0ull;
            L[j].offer(key, cap[j], thr[j]);
          }
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < QPW; ++j) {
    const int ql = w * QPW + j;
    if (ql < nq) {
      uint64_t* out = a.cand + ((int64_t)(q0 + ql) * a.n_groups + group) * KP;
#pragma unroll
      for (int i = 0; i < KPL; ++i) out[l + 64 * i] = L[j].e[i];
    }
  }
}

// ------------------------------------------------------------------------------------------
// Per-query sweep: one query; every wave of every workgroup sweeps its own document range with
// a private accumulator tile; the waves of a workgroup merge their lists at the end.

struct SweepArgs {
  IndexView ix;
  BatchView bv;       // entry table of one-query tiles (tile index = query index)
  uint64_t* cand;     // [n_groups][KP] for this query
  int32_t query;      // index of the query in the batch
  int64_t sweep_docs; // documents per wave, multiple of the skip block
  int32_t n_groups;   // workgroups
  int32_t doc_tile;
  int32_t ecap;       // cursor slots per wave
};

template <int W, int KPL, typename ST>
__global__ __launch_bounds__(W * 64) void k_sweep(SweepArgs a) {
  constexpr int KP = KPL * 64;
  extern __shared__ __align__(16) uint8_t smem[];
  const int DT = a.doc_tile;
  const int w = threadIdx.x >> 6;
  const int l = lane();
  float* acc = reinterpret_cast<float*>(smem) + (size_t)w * DT;
  int32_t* cursor = reinterpret_cast<int32_t*>(smem + (size_t)W * DT * 4) + (size_t)w * a.ecap;
  const IndexView& ix = a.ix;
  const BatchView& bv = a.bv;
  const typename ST::T* data = reinterpret_cast<const typename ST::T*>(ix.data);
  const int q = a.query;
  const int64_t e_base = bv.tile_e0[q];
  const int E = bv.wave_e0[(int64_t)q * 2 + 1];
  const int64_t sw = (int64_t)blockIdx.x * W + w;
  const int64_t d_lo = sw * a.sweep_docs;
  const int64_t d_hi = (d_lo + a.sweep_docs < ix.n_docs) ? d_lo + a.sweep_docs : ix.n_docs;
  const int cap = bv.q_k[q];

  for (int e = 0; e < E; ++e) {
    const Entry en = bv.entries[e_base + e];
    const int64_t c = (d_lo < d_hi) ? find_cursor(ix, en, d_lo) : 0;
    if (l == 0) cursor[e] = (int32_t)c;
  }
  for (int i = l; i < DT / 4; i += 64)
    reinterpret_cast<float4*>(acc)[i] = make_float4(0.f, 0.f, 0.f, 0.f);
  TopList<KPL> L;
  L.clear();
  uint64_t thr = 0;

  for (int64_t t0 = d_lo; t0 < d_hi; t0 += DT) {
    const int64_t t1 = (t0 + DT < d_hi) ? t0 + DT : d_hi;
    const int32_t t1i = (int32_t)t1;
    for (int e = 0; e < E; ++e) {
      const Entry en = bv.entries[e_base + e];
      const int64_t len = en.row_hi - en.row_lo;
      const float mult = (float)((uint32_t)bv.members[en.mem_off] >> 16);
      int64_t c = cursor[e];
      while (true) {
        const int64_t off = c + l;
        const bool in_row = off < len;
        const int32_t d = in_row ? ix.indices[en.row_lo + off] : INT32_MAX;
        const bool v = d < t1i && d >= (int32_t)t0;
        if (v) acc[d - (int32_t)t0] += ST::load(data, en.row_lo + off) * mult;
        const int n = __popcll(ballot(v));
        c += n;
        if (n < 64) break;
      }
      if (l == 0) cursor[e] = (int32_t)c;
    }
    float4* row = reinterpret_cast<float4*>(acc);
    for (int i = l; i < DT / 4; i += 64) {
      const float4 v4 = row[i];
      row[i] = make_float4(0.f, 0.f, 0.f, 0.f);
      const int64_t db = t0 + 4 * i;
      const float vs[4] = {v4.x, v4.y, v4.z, v4.w};
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int64_t doc = db + c;
        const uint64_t key = (doc < t1) ? make_key(vs[c], (uint32_t)doc) : 0ull;
        L.offer(key, cap, thr);
      }
    }
  }
  // merge the W lists of the workgroup (the accumulator region is reused)
  __syncthreads();
  uint64_t* sh = reinterpret_cast<uint64_t*>(smem);
#pragma unroll
  for (int i = 0; i < KPL; ++i) sh[(size_t)w * KP + l + 64 * i] = L.e[i];
  __syncthreads();
  if (w == 0) {
    for (int o = 1; o < W; ++o) {
#pragma unroll
      for (int i = 0; i < KPL; ++i) {
        const uint64_t x = sh[(size_t)o * KP + l + 64 * i];
        if (ballot(x > thr) == 0) break;
        L.offer(x, cap, thr);
      }
    }
    uint64_t* out = a.cand + (int64_t)blockIdx.x * KP;
#pragma unroll
    for (int i = 0; i < KPL; ++i) out[l + 64 * i] = L.e[i];
  }
}

// ------------------------------------------------------------------------------------------
// Merge: one workgroup per query; its waves filter strided 64-key chunks of the query's
// candidate lists, then wave 0 merges the wave lists and writes the final ranked rows.

struct MergeArgs {
  const uint64_t* cand;   // [n][lists][KP] (row stride lists*KP) starting at query q_first
  const int32_t* q_ids;
  const int64_t* q_off;
  const int32_t* q_k;
  const int32_t* q_stat;
  const float* theta32;   // nullptr for sparse variants
  int32_t* out_ids;
  float* out_scores;
  int32_t* out_count;
  int64_t n_docs;
  int32_t lists;
  int32_t k_max;
  int32_t q_first;        // first query handled by this launch (block b -> query q_first + b)
};

template <int KPL>
__global__ __launch_bounds__(256) void k_merge(MergeArgs a) {
  constexpr int KP = KPL * 64;
  constexpr int MW = 4;
  __shared__ uint64_t sh[MW - 1][KP];
  const int w = threadIdx.x >> 6;
  const int l = lane();
  const int q = a.q_first + blockIdx.x;
  const int cap = a.q_k[q];
  const uint64_t* base = a.cand + (int64_t)blockIdx.x * a.lists * KP;
  const int64_t chunks = (int64_t)a.lists * KPL;
  TopList<KPL> L;
  L.clear();
  uint64_t thr = 0;
  for (int64_t c = w; c < chunks; c += MW) {
    const uint64_t x = base[c * 64 + l];
    L.offer(x, cap, thr);
  }
  if (w > 0) {
#pragma unroll
    for (int i = 0; i < KPL; ++i) sh[w - 1][l + 64 * i] = L.e[i];
  }
  __syncthreads();
  if (w != 0) return;
  for (int o = 0; o < MW - 1; ++o) {
#pragma unroll
    for (int i = 0; i < KPL; ++i) {
      const uint64_t x = sh[o][l + 64 * i];
      if (ballot(x > thr) == 0) break;
      L.offer(x, cap, thr);
    }
  }
  // shift = sum of S_theta over the query's positions (Section 2.1)
  const bool bad = a.q_stat[q] != 0;
  float shift = 0.f;
  const int64_t p0 = a.q_off[q], p1 = a.q_off[q + 1];
  if (a.theta32 && !bad) {
    float part = 0.f;
    for (int64_t p = p0 + l; p < p1; p += 64) part += a.theta32[a.q_ids[p]];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
    shift = part;
  }
  const int64_t count = bad ? 0 : ((int64_t)cap < a.n_docs ? cap : a.n_docs);
  int32_t* oid = a.out_ids + (int64_t)q * a.k_max;
  float* osc = a.out_scores + (int64_t)q * a.k_max;
  for (int r0 = 0; r0 < a.k_max; r0 += 64) {
    const int r = r0 + l;
    const int i = r0 >> 6;
    uint64_t key = 0;
#pragma unroll
    for (int ii = 0; ii < KPL; ++ii)
      if (ii == i) key = L.e[ii];
    if (r < a.k_max) {
      if (r < count && key != 0) {
        oid[r] = (int32_t)key_doc(key);
        osc[r] = key_score(key) + shift;
      } else {
        oid[r] = -1;
        osc[r] = -INFINITY;
      }
    }
  }
  if (l == 0) a.out_count[q] = bad ? -2 : (int32_t)count;
}

}  // namespace bm25dev
