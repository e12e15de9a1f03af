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

#include <type_traits>

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
  const float* theta32;   // nullptr for sparse variants
  const int32_t* dense_id;  // dense row of each token or -1; nullptr: no dense rows used
  const int32_t* dense_rank;  // rank of each dense row by document frequency (0 = most)
  const void* dense;      // [n_dense][n_pad] stored scores
  int64_t n_docs;
  int64_t n_blocks;
  int64_t n_pad;
  int32_t vocab;
};

// A dense-row token of a query tile: its stored scores are added, times `mult`, to every query
// of the tile whose bit is set in `qmask` (one entry per distinct multiplicity).
struct DenseEntry {
  int32_t row;
  uint32_t qmask;
  float mult;
  int32_t token;
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
  DenseEntry* dense_ent;   // per tile, at the tile's first position
  int32_t* dense_n;        // [n_tiles]: dense entries of each tile
  float* tile_cost = nullptr;  // [n_tiles]: estimated gather work of each tile, if wanted
  int32_t n_queries;
  int32_t n_tiles;
  // largest multiplicity of one dense entry (larger ones are split over several entries): the
  // largest integer up to which the matrix-core operand of the stored type is exact
  int32_t dense_mult_max = INT32_MAX;
};

// Relative gather work of a tile, in units of one sparse posting added for one query, used only
// to order the launch. Timing the phases on the 8.8M-document batches gave about 218k postings
// per dense row and 127k per query's selection; weighting a dense row twice that ordered the
// launch best (its memory latency is exposed once per tile), and larger weights change nothing.
constexpr float kCostDenseRow = 436000.f;
constexpr float kCostQuery = 127000.f;

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
  uint32_t dcnt[kPlanSort + 1];          // per distinct token: dense entries
  int64_t qoff[65];
  uint32_t err[64];
  float cost_sum[4];
  uint32_t lds4[4];
  uint32_t counters[4];
};

#ifdef BM25_SEARCH_MAIN
// Query grouping: one workgroup per window of up to kPlanSort consecutive queries. A query's
// signature has one bit per dense row it holds (the least frequent row in the highest bit); the
// window is sorted by signature, descending, then by position, so that queries holding the same
// dense rows, the rarer ones deciding first, fall into the same query tile, and that tile reads
// each shared dense row once (the most frequent rows are in most tiles anyway). Writes the
// grouped batch (ids, offsets, k) and perm[grouped index] = caller's index.
struct ReorderArgs {
  const int32_t* q_ids;
  const int64_t* q_off;
  const int32_t* q_k;
  const int32_t* dense_id;
  const int32_t* dense_rank;
  int32_t vocab;
  int32_t n;
  int32_t* ids2;
  int64_t* off2;
  int32_t* k2;
  int32_t* perm;
};

// LDS: sort keys [kPlanSort] u64 | grouped offsets [kPlanSort + 1] u32 | caller's offsets
//      [kPlanSort + 1] u32 | scan scratch [4] u32 (all window-relative).
constexpr size_t kReorderLds = (size_t)kPlanSort * 8 + 2 * ((size_t)kPlanSort + 1) * 4 + 16;

__global__ __launch_bounds__(kPlanThreads) void k_reorder(ReorderArgs a) {
  constexpr int kSigBits = 52;  // rows ranked below this share no bit
  extern __shared__ __align__(16) uint8_t smem[];
  uint64_t* key = reinterpret_cast<uint64_t*>(smem);
  uint32_t* len = reinterpret_cast<uint32_t*>(key + kPlanSort);
  uint32_t* qoff = len + kPlanSort + 1;
  uint32_t* lds4 = qoff + kPlanSort + 1;
  const int tid = threadIdx.x;
  const int w0 = blockIdx.x * kPlanSort;
  const int m = (a.n - w0 < kPlanSort) ? a.n - w0 : kPlanSort;
  int npow = 1;
  while (npow < m) npow <<= 1;
  const int64_t base = a.q_off[w0];
  const int64_t P = a.q_off[w0 + m] - base;  // at most 4096 * BM25_MAX_QUERY_LEN
  for (int i = tid; i <= m; i += kPlanThreads) qoff[i] = (uint32_t)(a.q_off[w0 + i] - base);
  for (int i = tid; i < npow; i += kPlanThreads) key[i] = 0;
  __syncthreads();
  // signatures, one thread per position: the query holding position p is the last i with
  // qoff[i] <= p (empty queries hold none)
  for (int64_t p = tid; p < P; p += kPlanThreads) {
    const int32_t t = a.q_ids[base + p];
    if (t < 0 || t >= a.vocab) continue;
    const int32_t h = a.dense_id[t];
    if (h < 0) continue;
    const int32_t r = a.dense_rank[h];
    if (r >= kSigBits) continue;
    int lo = 0, hi = m - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (qoff[mid] <= (uint32_t)p) lo = mid; else hi = mid - 1;
    }
    atomicOr(reinterpret_cast<unsigned long long*>(key + lo),
             (unsigned long long)(1ull << r));
  }
  __syncthreads();
  // sort by signature descending, then position; padding sorts last (a real key has a zero
  // bit since i < m <= 4096)
  for (int i = tid; i < npow; i += kPlanThreads)
    key[i] = (i < m) ? (((~key[i] & ((1ull << kSigBits) - 1)) << 12) | (uint64_t)i) : ~0ull;
  __syncthreads();
  lds_bitonic_sort(key, npow);
  for (int i = tid; i < kPlanSort; i += kPlanThreads) {
    uint32_t n_i = 0;
    if (i < m) {
      const int src = (int)(key[i] & 0xFFFu);
      n_i = qoff[src + 1] - qoff[src];
      a.perm[w0 + i] = w0 + src;
      a.k2[w0 + i] = a.q_k[w0 + src];
    }
    len[i] = n_i;
  }
  __syncthreads();
  lds_scan_u32(len, kPlanSort, lds4);  // exclusive offsets of the grouped queries
  if (tid == 0) len[m] = (uint32_t)P;
  __syncthreads();
  for (int i = tid; i < m; i += kPlanThreads) a.off2[w0 + i] = base + len[i];
  if (w0 + m == a.n && tid == 0) a.off2[a.n] = a.q_off[a.n];
  // token ids, one thread per grouped position
  for (int64_t p = tid; p < P; p += kPlanThreads) {
    int lo = 0, hi = m - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (len[mid] <= (uint32_t)p) lo = mid; else hi = mid - 1;
    }
    const int src = (int)(key[lo] & 0xFFFu);
    a.ids2[base + p] = a.q_ids[base + qoff[src] + ((uint32_t)p - len[lo])];
  }
}

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

  // 3b. dense tokens: one entry per distinct multiplicity, with the mask of its queries; a
  //     multiplicity above bv.dense_mult_max is split over entries of the same row and mask whose
  //     multiplicities add up to it (at most one entry per query position, so they fit)
  auto is_dense = [&](uint32_t u) {
    return ix.dense_id != nullptr && ix.dense_id[sm.tok[u]] >= 0;
  };
  const uint32_t mmax = (uint32_t)bv.dense_mult_max;
  auto pieces = [&](uint32_t mult) { return (mult + mmax - 1) / mmax; };
  for (int u = tid; u < kPlanSort; u += kPlanThreads) {
    uint32_t cnt = 0;
    if ((uint32_t)u < n_tok && is_dense((uint32_t)u)) {
      const uint32_t m0 = sm.first_member[u], m1 = sm.first_member[u + 1];
      for (uint32_t m = m0; m < m1; ++m) {
        const uint32_t mult = sm.pos_of_member[m + 1] - sm.pos_of_member[m];
        bool seen = false;
        for (uint32_t mm = m0; mm < m; ++mm)
          seen |= (sm.pos_of_member[mm + 1] - sm.pos_of_member[mm]) == mult;
        cnt += seen ? 0u : pieces(mult);
      }
    }
    sm.dcnt[u] = cnt;
  }
  __syncthreads();
  const uint32_t n_dent = lds_scan_u32(sm.dcnt, kPlanSort, sm.lds4);
  for (uint32_t u = tid; u < n_tok; u += kPlanThreads) {
    if (!is_dense(u)) continue;
    const uint32_t m0 = sm.first_member[u], m1 = sm.first_member[u + 1];
    uint32_t o = sm.dcnt[u];
    for (uint32_t m = m0; m < m1; ++m) {
      const uint32_t mult = sm.pos_of_member[m + 1] - sm.pos_of_member[m];
      bool seen = false;
      for (uint32_t mm = m0; mm < m; ++mm)
        seen |= (sm.pos_of_member[mm + 1] - sm.pos_of_member[mm]) == mult;
      if (seen) continue;
      uint32_t mask = 0;
      for (uint32_t mm = m; mm < m1; ++mm)
        if (sm.pos_of_member[mm + 1] - sm.pos_of_member[mm] == mult)
          mask |= 1u << (uint32_t)(sm.key[sm.pos_of_member[mm]] & 31u);
      for (uint32_t rest = mult; rest > 0;) {
        const uint32_t take = rest < mmax ? rest : mmax;
        DenseEntry de;
        de.row = ix.dense_id[sm.tok[u]];
        de.qmask = mask;
        de.mult = (float)take;
        de.token = sm.tok[u];
        bv.dense_ent[p0 + o] = de;
        ++o;
        rest -= take;
      }
    }
  }
  if (tid == 0) bv.dense_n[tile] = (int32_t)n_dent;

  // 4. cost of each sparse token and number of entries it is split into
  float local = 0.f;
  for (uint32_t u = tid; u < n_tok; u += kPlanThreads) {
    if (is_dense(u)) continue;
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
  if (tid == 0 && bv.tile_cost)
    bv.tile_cost[tile] = total + kCostDenseRow * (float)n_dent + kCostQuery * (float)nq;
  for (int u = tid; u < kPlanSort; u += kPlanThreads) {
    uint32_t parts = 0;
    if ((uint32_t)u < n_tok && !is_dense((uint32_t)u)) {
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

// Tile order for the gather launch, longest first: workgroups are dispatched in block order, so
// the tiles with the most work start first and short ones fill the end of the launch. One
// workgroup; n_tiles <= kOrderMax. order[i] = tile with the i-th largest estimated cost (ties by
// tile index).
constexpr int kOrderMax = 4096;

__global__ __launch_bounds__(kPlanThreads) void k_order(const float* cost, int32_t n_tiles,
                                                          int32_t* order) {
  __shared__ uint64_t key[kOrderMax];
  int npow = 1;
  while (npow < n_tiles) npow <<= 1;
  for (int i = threadIdx.x; i < npow; i += kPlanThreads) {
    uint64_t k = ~0ull;
    if (i < n_tiles) {
      const float c = cost[i] > 0.f ? cost[i] : 0.f;
      const uint32_t cq = c < 4.0e9f ? (uint32_t)c : 0xFFFFFFFFu;
      k = ((uint64_t)(~cq) << 32) | (uint32_t)i;
    }
    key[i] = k;
  }
  __syncthreads();
  lds_bitonic_sort(key, npow);
  for (int i = threadIdx.x; i < n_tiles; i += kPlanThreads) order[i] = (int32_t)(uint32_t)key[i];
}
#endif  // BM25_SEARCH_MAIN

// ------------------------------------------------------------------------------------------
// Cursor search: offset inside the row of the first entry with document id >= d0.
// Long rows read the skip table (d0 is a multiple of the skip block). Other rows (fewer than
// 1024 entries; up to 4096 would do) compare d0 against every 64th entry of the row, one per
// lane, then scan one 64-entry chunk.
// Whole wave, uniform arguments.
__device__ __forceinline__ int32_t find_cursor(const IndexView& ix, int64_t row_lo, int32_t len,
                                               int32_t long_id, int64_t d0) {
  if (d0 <= 0 || len == 0) return 0;
  if (long_id >= 0)
    return (int32_t)ix.skip[(int64_t)long_id * (ix.n_blocks + 1) + d0 / kSkipBlockDev];
  const int l = lane();
  const int64_t row_hi = row_lo + len;
  // samples at absolute positions 64*j inside [row_lo, row_hi)
  const int64_t j0 = (row_lo + 63) >> 6;
  const int64_t j1 = (row_hi - 1) >> 6;  // inclusive
  const int64_t js = j0 + l;
  const bool has = js <= j1;
  const int32_t sv = has ? ix.indices[js << 6] : INT32_MAX;
  const int c_s = __popcll(ballot(has && sv < d0));
  // chunk to scan: before the first sample if c_s == 0, else from the last sample below d0
  const int64_t from = (c_s == 0) ? row_lo : ((j0 + c_s - 1) << 6);
  const int64_t p = from + l;
  const bool in = p < row_hi && p < from + 64;
  const int32_t v = in ? ix.indices[p] : INT32_MAX;
  const int c = __popcll(ballot(in && v < d0));
  return (int32_t)(from + c - row_lo);
}

// ------------------------------------------------------------------------------------------
// Sweep state of the entries (query tokens) a wave walks through, structure of arrays in LDS:
// static fields (row start, row length, skip-table row for placing the first cursor, members)
// and the dynamic cursor (offset of the next unconsumed entry of the row) plus the document id
// at the cursor (INT32_MAX past the end), so that a tile without postings of that row costs no
// memory access.
struct EntryState {
  int64_t* row_lo;
  int32_t* len;
  int32_t* lid;
  int32_t* mem;  // see kInlineMember
  int32_t* cur;
  int32_t* nd;
};

constexpr int kEntryStaticBytes = 8 + 4 + 4 + 4;

// Member field of an entry. Most entries have one member; its word (q_local | multiplicity
// << 16) is then kept inline with this flag set. Otherwise the field is the member offset in the
// LDS member copy | member count << 16.
constexpr uint32_t kInlineMember = 0x80000000u;

struct Members {
  uint32_t first;  // the first member word
  int count;
  uint32_t off;    // offset of the members in the LDS copy (count > 1)
};

__device__ __forceinline__ Members decode_members(uint32_t w, const int32_t* mem_lds) {
  Members m;
  if (w & kInlineMember) {
    m.first = w & ~kInlineMember;
    m.count = 1;
    m.off = 0;
  } else {
    m.count = (int)(w >> 16);
    m.off = w & 0xFFFFu;
    m.first = (m.count > 0) ? (uint32_t)mem_lds[m.off] : 0u;
  }
  return m;
}
constexpr int kEntryDynBytes = 4 + 4;

__device__ __forceinline__ EntryState carve_state(uint8_t* base, int cap, int dyn_copies,
                                                  int dyn_index) {
  EntryState st;
  st.row_lo = reinterpret_cast<int64_t*>(base);
  st.len = reinterpret_cast<int32_t*>(base + (size_t)cap * 8);
  st.lid = st.len + cap;
  st.mem = st.lid + cap;
  int32_t* dyn = st.mem + cap;
  st.cur = dyn + (size_t)dyn_index * 2 * cap;
  st.nd = st.cur + cap;
  (void)dyn_copies;
  return st;
}

// Loads static fields of entries [e_lo, e_hi) (lane-parallel) from the planner table and the
// member list.
__device__ __forceinline__ void load_static(const Entry* ents, const int32_t* members, int e_lo,
                                            int e_hi, int64_t mem_base, const EntryState& st) {
  for (int j = e_lo + lane(); j < e_hi; j += 64) {
    const Entry en = ents[j];
    st.row_lo[j] = en.row_lo;
    st.len[j] = (int32_t)(en.row_hi - en.row_lo);
    st.lid[j] = en.long_id;
    st.mem[j] = (en.mem_cnt == 1)
                    ? (int32_t)((uint32_t)members[en.mem_off] | kInlineMember)
                    : (int32_t)((en.mem_off - mem_base) | ((int64_t)en.mem_cnt << 16));
  }
}

// Cursor and next document at the sweep start d0 for entries [e_lo, e_hi) (whole wave).
__device__ __forceinline__ void init_cursors(const IndexView& ix, int e_lo, int e_hi, int64_t d0,
                                             const EntryState& st) {
  for (int j = e_lo; j < e_hi; ++j) {
    const int64_t row_lo = st.row_lo[j];
    const int32_t len = st.len[j];
    const int32_t c = find_cursor(ix, row_lo, len, st.lid[j], d0);
    if (lane() == 0) {
      st.cur[j] = c;
      st.nd[j] = (c < len) ? ix.indices[row_lo + c] : INT32_MAX;
    }
  }
}

// Runs group(integral_constant<int, n>, c0) for a run-time group size 1 <= n <= K, so that each
// size is a compile-time unrolled group.
template <int K, typename G>
__device__ __forceinline__ void run_group_of(int32_t n, int32_t c0, G& group) {
  if constexpr (K > 0) {
    if (n == K)
      group(std::integral_constant<int, K>{}, c0);
    else
      run_group_of<K - 1>(n, c0, group);
  }
}

// Adds the postings of entries [e_lo, e_hi) that fall in the document tile [t0, t1) into the
// accumulator rows acc[q * DT + (d - t0)] of their member queries. Every entry keeps its cursor
// and the document id at the cursor (nd), so the entries with a posting in [t0, t1) are those
// with nd < t1: no lookup per tile. Each of them takes one 64-posting chunk from its cursor; the
// chunks of the wave's entries are loaded U at a time, all loads of a group in flight together
// (addresses are clamped inside the row instead of predicated, so no load waits behind a
// branch), and a last group of fewer than U chunks issues only the loads it needs. The postings
// below t1 form a prefix of the chunk: they are added for every member query, the cursor moves
// past them and nd becomes the first document id >= t1 (read from the same chunk). An entry whose
// 64 postings were all below t1 takes another chunk in a further pass.
template <typename ST, int U>
__device__ __forceinline__ void accumulate_tile_stream(const EntryState& st, const IndexView& ix,
                                                       int e_lo, int e_hi,
                                                       const int32_t* mem_lds, float* acc,
                                                       int DT, int64_t t0, int64_t t1) {
  const int l = lane();
  const typename ST::T* data = reinterpret_cast<const typename ST::T*>(ix.data);
  const int32_t t0i = (int32_t)t0, t1i = (int32_t)t1;
  for (int g0 = e_lo; g0 < e_hi; g0 += 64) {
    const int j = g0 + l;
    const bool ve = j < e_hi;
    int32_t nd = ve ? st.nd[j] : INT32_MAX;
    uint64_t todo = ballot(nd < t1i);
    if (todo == 0) continue;
    int32_t cur = ve ? st.cur[j] : 0;
    const int32_t len = ve ? st.len[j] : 0;
    const int64_t rlo = ve ? st.row_lo[j] : 0;
    const int32_t mw = ve ? st.mem[j] : 0;
    uint64_t more = 0;  // entries whose chunk held only postings below t1
    auto group = [&](auto uu, int32_t) {
      constexpr int UU = decltype(uu)::value;
      int src[UU];
      int32_t dv[UU];
      float sv[UU];
      int32_t memw[UU];
      int32_t csv[UU];
      int32_t lnv[UU];
#pragma unroll
      for (int u = 0; u < UU; ++u) {
        src[u] = __builtin_ctzll(todo);
        todo &= todo - 1;
        const int64_t row = (int64_t)readlane64((uint64_t)rlo, src[u]);
        const int32_t cs = (int32_t)readlane((uint32_t)cur, src[u]);
        const int32_t ln = (int32_t)readlane((uint32_t)len, src[u]);
        memw[u] = (int32_t)readlane((uint32_t)mw, src[u]);
        csv[u] = cs;
        lnv[u] = ln;
        const int32_t p = cs + l;
        const bool in_row = p < ln;
        const int64_t off = row + (in_row ? p : cs);  // cs < ln: the entry has a posting
        const int32_t d = ix.indices[off];
        sv[u] = ST::load(data, off);
        dv[u] = in_row ? d : INT32_MAX;
      }
#pragma unroll
      for (int u = 0; u < UU; ++u) {
        const bool valid = dv[u] < t1i;
        const int32_t r = dv[u] - t0i;
        const int rel = (valid && r >= 0) ? r : -1;
        // a single member comes inline with the entry; more (rare) from the LDS member copy
        const Members ms = decode_members((uint32_t)memw[u], mem_lds);
        if (ms.count > 0 && rel >= 0)
          atomicAdd(acc + (int)(ms.first & 0xFFFFu) * DT + rel, sv[u] * (float)(ms.first >> 16));
        if (ms.count > 1) {
          const int32_t mem = (l < ms.count) ? mem_lds[ms.off + l] : 0;
          for (int m = 1; m < ms.count; ++m) {
            const uint32_t mm = readlane((uint32_t)mem, m);
            const float v = sv[u] * (float)(mm >> 16);
            if (rel >= 0) atomicAdd(acc + (int)(mm & 0xFFFFu) * DT + rel, v);
          }
        }
        // postings are sorted by document: the ones below t1 are lanes 0 .. n-1. After a full
        // chunk the entry either has postings left (another pass reads them and sets nd; until
        // then nd only has to stay below t1) or is exhausted.
        const int n = __popcll(ballot(valid));
        int32_t next;
        if (n < 64) {
          next = (int32_t)readlane((uint32_t)dv[u], n);
        } else if (csv[u] + 64 < lnv[u]) {
          next = t0i;
          more |= 1ull << src[u];
        } else {
          next = INT32_MAX;
        }
        if (l == src[u]) {
          cur = csv[u] + n;
          nd = next;
        }
      }
    };
    while (todo) {
      while (todo) {
        const int32_t cnt = __popcll(todo);
        if (cnt >= U)
          group(std::integral_constant<int, U>{}, 0);
        else
          run_group_of<U - 1>(cnt, 0, group);
      }
      todo = more;
      more = 0;
    }
    if (ve) {
      st.cur[j] = cur;
      st.nd[j] = nd;
    }
  }
}

// Loads R consecutive stored scores (R * sizeof(T) bytes, aligned) and widens them to FP32.
template <typename ST, int R>
__device__ __forceinline__ void load_dense(const typename ST::T* p, float* v) {
  constexpr int NW = R * (int)sizeof(typename ST::T) / 4;
  static_assert(NW >= 1 && (NW == 1 || NW % 2 == 0), "unsupported dense width");
  uint32_t w[NW];
  const uint32_t* q = reinterpret_cast<const uint32_t*>(p);
  if constexpr (NW % 4 == 0) {
#pragma unroll
    for (int i = 0; i < NW / 4; ++i) {
      const uint4 x = reinterpret_cast<const uint4*>(q)[i];
      w[4 * i] = x.x;
      w[4 * i + 1] = x.y;
      w[4 * i + 2] = x.z;
      w[4 * i + 3] = x.w;
    }
  } else if constexpr (NW == 2) {
    const uint2 x = reinterpret_cast<const uint2*>(q)[0];
    w[0] = x.x;
    w[1] = x.y;
  } else {
    w[0] = q[0];
  }
  if constexpr (sizeof(typename ST::T) == 4) {
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = __uint_as_float(w[i]);
  } else {
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      v[2 * i] = ST::widen_lo(w[i]);
      v[2 * i + 1] = ST::widen_hi(w[i]);
    }
  }
}

// Reads R consecutive floats of an LDS row and clears them.
template <int R>
__device__ __forceinline__ void take_lds(float* p, float* v) {
  if constexpr (R % 4 == 0) {
#pragma unroll
    for (int i = 0; i < R / 4; ++i) {
      const float4 x = reinterpret_cast<float4*>(p)[i];
      reinterpret_cast<float4*>(p)[i] = make_float4(0.f, 0.f, 0.f, 0.f);
      v[4 * i] = x.x;
      v[4 * i + 1] = x.y;
      v[4 * i + 2] = x.z;
      v[4 * i + 3] = x.w;
    }
  } else {
    static_assert(R == 2, "unsupported width");
    const float2 x = reinterpret_cast<float2*>(p)[0];
    reinterpret_cast<float2*>(p)[0] = make_float2(0.f, 0.f);
    v[0] = x.x;
    v[1] = x.y;
  }
}

// Adds the dense-row entries [0, n) to the register accumulators acc[q][r] of the lane's R
// documents starting at tile document `first`. Loads run U = max(2, 16 / R) entries at a time
// (16 values per lane) and the next group's loads are issued before the current group's
// additions.
// acc += a * (half in the low / high 16 bits of h2), one FMA rounding: v_fma_mix_f32 widens the
// FP16 operand inside the multiply-add, so no separate conversion is issued. `a` must be the same
// in every lane (it is read from a scalar register).
__device__ __forceinline__ void fma_mix_lo(float& acc, float a, uint32_t h2) {
  asm("v_fma_mix_f32 %0, %1, %2, %0 op_sel_hi:[0,1,0]" : "+v"(acc) : "s"(a), "v"(h2));
}
__device__ __forceinline__ void fma_mix_hi(float& acc, float a, uint32_t h2) {
  asm("v_fma_mix_f32 %0, %1, %2, %0 op_sel:[0,1,0] op_sel_hi:[0,1,0]"
      : "+v"(acc)
      : "s"(a), "v"(h2));
}

// accumulate_dense for FP16 rows: the stored halves stay packed in registers (R/2 words per
// entry) and enter the FMAs directly.
template <int QT, int R>
__device__ __forceinline__ void accumulate_dense_f16(const IndexView& ix, const DenseEntry* de,
                                                     int n, int64_t first,
                                                     float (&acc)[QT][R]) {
  static_assert(R % 2 == 0, "FP16 rows are read in pairs");
  constexpr int U = (16 / R) > 2 ? (16 / R) : 2;
  constexpr int NW = R / 2;
  const __half* dense = reinterpret_cast<const __half*>(ix.dense) + first;
  uint32_t w[2][U][NW];
  uint32_t mk[2][U];
  float mu[2][U];
  auto load_group = [&](int e0, uint32_t (&dst)[U][NW], uint32_t (&m)[U], float (&f)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = (e0 + u < n) ? e0 + u : n - 1;  // clamped: always a valid row
      const DenseEntry d = de[e];
      const uint32_t* q = reinterpret_cast<const uint32_t*>(dense + (int64_t)d.row * ix.n_pad);
      if constexpr (NW % 4 == 0) {
#pragma unroll
        for (int i = 0; i < NW / 4; ++i) {
          const uint4 x = reinterpret_cast<const uint4*>(q)[i];
          dst[u][4 * i] = x.x;
          dst[u][4 * i + 1] = x.y;
          dst[u][4 * i + 2] = x.z;
          dst[u][4 * i + 3] = x.w;
        }
      } else if constexpr (NW == 2) {
        const uint2 x = reinterpret_cast<const uint2*>(q)[0];
        dst[u][0] = x.x;
        dst[u][1] = x.y;
      } else {
        dst[u][0] = q[0];
      }
      m[u] = (e0 + u < n) ? d.qmask : 0u;
      f[u] = d.mult;
    }
  };
  if (n <= 0) return;
  load_group(0, w[0], mk[0], mu[0]);
  for (int e0 = 0; e0 < n; e0 += 2 * U) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int eg = e0 + h * U;
      if (eg >= n) break;
      if (eg + U < n) load_group(eg + U, w[h ^ 1], mk[h ^ 1], mu[h ^ 1]);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t mask = mk[h][u];
        const float mult = mu[h][u];
#pragma unroll
        for (int q = 0; q < QT; ++q) {
          if ((mask >> q) & 1u) {
#pragma unroll
            for (int i = 0; i < NW; ++i) {
              fma_mix_lo(acc[q][2 * i], mult, w[h][u][i]);
              fma_mix_hi(acc[q][2 * i + 1], mult, w[h][u][i]);
            }
          }
        }
      }
    }
  }
}

// Dense rows of 16-bit stored scores on the matrix cores. For a tile, the dense-row work is the
// product (queries x entries) . (entries x documents): A[q][e] = the multiplicity of entry e for
// query q (0 when q is not a member), B[e][d] = the stored score of entry e's row at document d.
// v_mfma_f32_4x4x4{f16,bf16_1k} runs 16 blocks of a 4x4x4 product; in block b, lane 4b + i
// supplies row i of A and lane 4b + j column j of B, and lane 4b + j receives column j of D, one
// query per register (the layout was checked on the device). So every lane supplies, as A, the
// multiplicities of query (lane & 3) (+ 4 per query group) for 4 entries, and as B the 4 entries'
// scores at one of its own documents, and gets back the 4 queries' sums for that document: one
// instruction per (query group, document of the lane) per 4 entries, with no per-query branch.
// Products of 16-bit values are exact in FP32, and the sums accumulate in FP32. The planner keeps
// every entry's multiplicity within the integers the operand type holds exactly (2^11 in FP16,
// 2^8 in BF16: dense_mult_max), splitting larger ones over several entries.
constexpr bool kDenseMfma = true;

typedef _Float16 mfma_h4 __attribute__((ext_vector_type(4)));
typedef short mfma_s4 __attribute__((ext_vector_type(4)));
typedef float mfma_f4 __attribute__((ext_vector_type(4)));
typedef uint32_t mfma_u2 __attribute__((ext_vector_type(2)));  // 4 packed 16-bit operands

template <typename ST>
__device__ __forceinline__ uint32_t mult_bits16(float m) {
  if constexpr (std::is_same<ST, F16>::value)
    return (uint32_t)__half_as_ushort(__float2half_rn(m));
  else
    return __float_as_uint(m) >> 16;  // exact for the integers this is used for
}

template <typename ST>
__device__ __forceinline__ mfma_f4 mfma_4x4x4(mfma_u2 a, mfma_u2 b, mfma_f4 c) {
  if constexpr (std::is_same<ST, F16>::value)
    return __builtin_amdgcn_mfma_f32_4x4x4f16(__builtin_bit_cast(mfma_h4, a),
                                              __builtin_bit_cast(mfma_h4, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(__builtin_bit_cast(mfma_s4, a),
                                                  __builtin_bit_cast(mfma_s4, b), c, 0, 0, 0);
}

// acc must be zero on entry (the gather stores and clears it every tile); it receives the sums.
template <typename ST, int QT, int R>
__device__ __forceinline__ void accumulate_dense_mfma(const IndexView& ix, const DenseEntry* de,
                                                      int n, int64_t first,
                                                      float (&acc)[QT][R]) {
  static_assert(QT % 4 == 0 && R % 2 == 0, "4-query groups, pairs of documents");
  constexpr int NW = R / 2;  // words of two 16-bit scores per entry and lane
  constexpr int QG = QT / 4;
  const uint16_t* dense = reinterpret_cast<const uint16_t*>(ix.dense) + first;
  const int qs = lane() & 3;
  uint32_t w[2][4][NW];
  uint32_t mk[2][4];
  float mu[2][4];
  auto load_group = [&](int e0, uint32_t (&dst)[4][NW], uint32_t (&m)[4], float (&f)[4]) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = (e0 + u < n) ? e0 + u : n - 1;  // clamped: always a valid row
      const DenseEntry d = de[e];
      const uint32_t* q = reinterpret_cast<const uint32_t*>(dense + (int64_t)d.row * ix.n_pad);
      if constexpr (NW % 4 == 0) {
#pragma unroll
        for (int i = 0; i < NW / 4; ++i) {
          const uint4 x = reinterpret_cast<const uint4*>(q)[i];
          dst[u][4 * i] = x.x;
          dst[u][4 * i + 1] = x.y;
          dst[u][4 * i + 2] = x.z;
          dst[u][4 * i + 3] = x.w;
        }
      } else if constexpr (NW == 2) {
        const uint2 x = reinterpret_cast<const uint2*>(q)[0];
        dst[u][0] = x.x;
        dst[u][1] = x.y;
      } else {
        dst[u][0] = q[0];
      }
      m[u] = (e0 + u < n) ? d.qmask : 0u;  // entries past the end add nothing
      f[u] = d.mult;
    }
  };
  if (n <= 0) return;
  // the sums as the instruction's columns: ca[g][j] = queries 4g..4g+3 at document j (acc is
  // zero on entry, so they start at zero and replace acc at the end)
  mfma_f4 ca[QG][R];
#pragma unroll
  for (int g = 0; g < QG; ++g)
#pragma unroll
    for (int j = 0; j < R; ++j) ca[g][j] = mfma_f4{0.f, 0.f, 0.f, 0.f};
  load_group(0, w[0], mk[0], mu[0]);
  for (int e0 = 0; e0 < n; e0 += 8) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int eg = e0 + 4 * h;
      if (eg >= n) break;
      if (eg + 4 < n) load_group(eg + 4, w[h ^ 1], mk[h ^ 1], mu[h ^ 1]);
      uint32_t mb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) mb[u] = mult_bits16<ST>(mu[h][u]);
#pragma unroll
      for (int g = 0; g < QG; ++g) {
        const int q = 4 * g + qs;
        uint32_t av[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) av[u] = ((mk[h][u] >> q) & 1u) ? mb[u] : 0u;
        const mfma_u2 a = {av[0] | (av[1] << 16), av[2] | (av[3] << 16)};
#pragma unroll
        for (int j = 0; j < R; ++j) {
          uint32_t bv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u)
            bv[u] = (j & 1) ? (w[h][u][j >> 1] >> 16) : (w[h][u][j >> 1] & 0xFFFFu);
          const mfma_u2 b = {bv[0] | (bv[1] << 16), bv[2] | (bv[3] << 16)};
          ca[g][j] = mfma_4x4x4<ST>(a, b, ca[g][j]);
        }
      }
    }
  }
#pragma unroll
  for (int g = 0; g < QG; ++g)
#pragma unroll
    for (int j = 0; j < R; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[4 * g + v][j] = ca[g][j][v];
}

template <typename ST, int QT, int R>
__device__ __forceinline__ void accumulate_dense(const IndexView& ix, const DenseEntry* de, int n,
                                                 int64_t first, float (&acc)[QT][R]) {
  if constexpr (kDenseMfma && sizeof(typename ST::T) == 2 && QT % 4 == 0 && R % 2 == 0) {
    // only the gather's tiles (QT >= 4) come here, with acc cleared by the previous tile's store
    accumulate_dense_mfma<ST, QT, R>(ix, de, n, first, acc);
    return;
  }
  if constexpr (std::is_same<ST, F16>::value) {
    accumulate_dense_f16<QT, R>(ix, de, n, first, acc);
    return;
  }
  constexpr int U = (16 / R) > 2 ? (16 / R) : 2;
  const typename ST::T* dense = reinterpret_cast<const typename ST::T*>(ix.dense) + first;
  // values and (query mask, multiplier) of two groups of U entries: one in use, one loading
  float v[2][U][R];
  uint32_t mk[2][U];
  float mu[2][U];
  auto load_group = [&](int e0, float (&dst)[U][R], uint32_t (&m)[U], float (&f)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = (e0 + u < n) ? e0 + u : n - 1;  // clamped: always a valid row
      const DenseEntry d = de[e];                   // one 16-byte scalar load
      load_dense<ST, R>(dense + (int64_t)d.row * ix.n_pad, dst[u]);
      m[u] = (e0 + u < n) ? d.qmask : 0u;           // entries past the end add nothing
      f[u] = d.mult;
    }
  };
  if (n <= 0) return;
  load_group(0, v[0], mk[0], mu[0]);
  for (int e0 = 0; e0 < n; e0 += 2 * U) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int eg = e0 + h * U;
      if (eg >= n) break;
      if (eg + U < n) load_group(eg + U, v[h ^ 1], mk[h ^ 1], mu[h ^ 1]);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t mask = mk[h][u];
        const float mult = mu[h][u];
#pragma unroll
        for (int q = 0; q < QT; ++q) {
          if ((mask >> q) & 1u) {
#pragma unroll
            for (int r = 0; r < R; ++r) acc[q][r] = fmaf(mult, v[h][u][r], acc[q][r]);
          }
        }
      }
    }
  }
}

// Filters one accumulator row of a tile against the wave's current k-th key and offers the
// survivors to the list. Each lane reads its NB float4 of a span together (the LDS reads are in
// flight at once); a plain FP32 comparison of each float4's maximum with the k-th score rejects
// most of them, and only float4 groups with a candidate build 64-bit keys. Every list sweeps
// its documents in increasing id order, so a document that only ties the k-th score has a
// larger id than the k-th key's and ranks below it: the comparison is strict (a list that holds
// fewer than k keys has no threshold and takes everything).
__device__ __forceinline__ float max4(const float4& v) {
  return fmaxf(fmaxf(v.x, v.y), fmaxf(v.z, v.w));
}

template <int DT>
struct RowSpan {
  static_assert(DT % 256 == 0, "rows are read 64 float4 at a time");
  static constexpr int NB = (DT / 256) < 2 ? (DT / 256) : 2;  // float4 per lane per span
  static_assert((DT / 256) % NB == 0, "spans must tile the row");
};

template <int KPL, int DT>
__device__ __forceinline__ void select_row(const float* rowp, int64_t t0, int64_t t1,
                                           TopList<KPL>& L, int cap, uint64_t& thr) {
  constexpr int NB = RowSpan<DT>::NB;
  const int l = lane();
  const float4* row = reinterpret_cast<const float4*>(rowp);
  float thr_s = (thr == 0) ? -INFINITY : key_score(thr);
  for (int s0 = 0; s0 < DT / 4; s0 += 64 * NB) {
    float4 v4[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) v4[b] = row[s0 + 64 * b + l];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      if (ballot(max4(v4[b]) > thr_s)) {
        const int64_t db = t0 + 4 * (s0 + 64 * b + l);
        const float vs[4] = {v4[b].x, v4[b].y, v4[b].z, v4[b].w};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int64_t doc = db + c;
          const uint64_t key = (doc < t1) ? make_key(vs[c], (uint32_t)doc) : 0ull;
          L.offer(key, cap, thr);
        }
        thr_s = (thr == 0) ? -INFINITY : key_score(thr);
      }
    }
  }
}

// The same filter feeding a staged list (long lists, where one insertion per key is costly).
template <int KPL, int DT>
__device__ __forceinline__ void select_row(const float* rowp, int64_t t0, int64_t t1,
                                           StagedTopList<KPL>& S) {
  constexpr int NB = RowSpan<DT>::NB;
  const int l = lane();
  const float4* row = reinterpret_cast<const float4*>(rowp);
  float thr_s = S.thr_score();
  for (int s0 = 0; s0 < DT / 4; s0 += 64 * NB) {
    float4 v4[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) v4[b] = row[s0 + 64 * b + l];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      if (ballot(max4(v4[b]) > thr_s)) {
        const int64_t db = t0 + 4 * (s0 + 64 * b + l);
        const float vs[4] = {v4[b].x, v4[b].y, v4[b].z, v4[b].w};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int64_t doc = db + c;
          S.offer((doc < t1 && vs[c] > thr_s) ? make_key(vs[c], (uint32_t)doc) : 0ull);
        }
        thr_s = S.thr_score();
      }
    }
  }
}

// Stores R register values into an LDS row (the lane owns these documents) and clears them.
template <int R>
__device__ __forceinline__ void put_lds(float* p, float* v) {
  if constexpr (R % 4 == 0) {
#pragma unroll
    for (int i = 0; i < R / 4; ++i)
      reinterpret_cast<float4*>(p)[i] = make_float4(v[4 * i], v[4 * i + 1], v[4 * i + 2], v[4 * i + 3]);
  } else {
    static_assert(R == 2, "unsupported width");
    reinterpret_cast<float2*>(p)[0] = make_float2(v[0], v[1]);
  }
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = 0.f;
}

// Offers the lane's R documents of one query (scores v, documents first..first+R-1, only those
// below t1) to the wave's list when any of them reaches the list's k-th score.
template <int KPL, int R>
__device__ __forceinline__ void select_regs(const float* v, int64_t first, int64_t t1,
                                            StagedTopList<KPL>& S, float& thr_s) {
  float mx = v[0];
#pragma unroll
  for (int r = 1; r < R; ++r) mx = fmaxf(mx, v[r]);
  if (ballot(mx > thr_s)) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t doc = first + r;
      S.offer((doc < t1 && v[r] > thr_s) ? make_key(v[r], (uint32_t)doc) : 0ull);
    }
    thr_s = S.thr_score();
  }
}

// ------------------------------------------------------------------------------------------
// Batched gather + top-k. Workgroup = (query tile of up to QT queries, doc group), W waves.
// A tile spans DT = W * 64 * R documents; lane l of wave w owns documents w*64*R + l*R .. +R-1
// of the tile for every query of the tile, with FP32 accumulators in registers. Once per tile:
// the dense-row tokens are added into the registers, which the lanes then store into an LDS
// accumulator row per query (each lane owns its documents: plain stores over the previous
// tile's values); the other tokens' postings are added on top with LDS atomics; and the wave
// owning a query filters its row against the query's k-th key (QPW = QT / W queries per wave,
// one list each).
//
// LDS: accumulator rows [QT][DT] | entry static fields [ecap] | cursors [ecap] |
//      member copy [pcap].

struct GatherArgs {
  IndexView ix;
  BatchView bv;
  const int32_t* order = nullptr;  // tile of each tile slot (longest first), or the identity
  uint64_t* cand;       // [n_queries][n_groups][KP]
  int64_t group_docs;   // multiple of the skip block and of DT
  int32_t n_groups;
  int32_t ecap;         // entry slots per workgroup (>= sparse entries of any tile)
  int32_t pcap;         // member slots per workgroup (>= positions of any tile)
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

// With 4 waves, 1024-key lists need about 143 VGPRs (3 waves per SIMD). The fp16 form is held
// to 128 (4 waves): the compiler spills about 10 registers, and the kernel is still 10-13%
// faster (top-1000 on 8.8M documents, 1024 to 4096 queries of up to 64 ids per batch). The bf16
// form spills more and was 8% slower so (top-1000 on 5M long documents, 30-200-id queries).
template <typename ST>
struct LongListFourWaves {
  static constexpr bool value = false;
};
template <>
struct LongListFourWaves<F16> {
  static constexpr bool value = true;
};

template <int W, int QT, int R, int KPL, typename ST>
__global__ __launch_bounds__(W * 64)
__attribute__((amdgpu_waves_per_eu((KPL >= 16 && W == 4 && LongListFourWaves<ST>::value) ? 4 : 1)))
void k_gather(GatherArgs a) {
  constexpr int DT = W * 64 * R;
  constexpr int KP = KPL * 64;
  constexpr int QPW = QT / W;
  static_assert(QT % W == 0, "queries must divide evenly over the waves");
  extern __shared__ __align__(16) uint8_t smem[];
  float* rows = reinterpret_cast<float*>(smem);
  uint8_t* sbase = smem + (size_t)QT * DT * 4;
  const EntryState st = carve_state(sbase, a.ecap, 1, 0);
  int32_t* mem_lds = reinterpret_cast<int32_t*>(sbase + (size_t)a.ecap *
                                                           (kEntryStaticBytes + kEntryDynBytes));

  int tile, group;
  map_block(blockIdx.x, a.n_groups, tile, group);
  if (a.order) tile = a.order[tile];
  const int w = threadIdx.x >> 6;
  const int l = lane();
  const BatchView& bv = a.bv;
  const IndexView& ix = a.ix;
  const int q0 = bv.tile_q0[tile];
  const int nq = bv.tile_q0[tile + 1] - q0;
  const int64_t p0 = bv.q_off[q0];
  const int P = (int)(bv.q_off[q0 + nq] - p0);
  const int64_t e_base = bv.tile_e0[tile];
  const int32_t* we = bv.wave_e0 + (int64_t)tile * (W + 1);
  const int e_lo = we[w], e_hi = we[w + 1];
  const DenseEntry* dent = bv.dense_ent + p0;
  const int n_dense = bv.dense_n[tile];
  const int64_t d_lo = (int64_t)group * a.group_docs;
  const int64_t d_hi = (d_lo + a.group_docs < ix.n_docs) ? d_lo + a.group_docs : ix.n_docs;

  for (int i = threadIdx.x; i < P; i += W * 64) mem_lds[i] = bv.members[p0 + i];
  load_static(bv.entries + e_base, bv.members, e_lo, e_hi, p0, st);
  if (d_lo < d_hi) init_cursors(ix, e_lo, e_hi, d_lo, st);
  float acc[QT][R];
#pragma unroll
  for (int q = 0; q < QT; ++q)
#pragma unroll
    for (int r = 0; r < R; ++r) acc[q][r] = 0.f;
  // lists of 256 keys and more take their candidates through a staging register
  constexpr bool kStaged = KPL >= 4;
  TopList<KPL> L[kStaged ? 1 : QPW];
  uint64_t thr[kStaged ? 1 : QPW];
  int cap[kStaged ? 1 : QPW];
  StagedTopList<KPL> S[kStaged ? QPW : 1];
#pragma unroll
  for (int j = 0; j < QPW; ++j) {
    const int ql = w * QPW + j;
    const int k = (ql < nq) ? bv.q_k[q0 + ql] : 1;
    if constexpr (kStaged) {
      S[j].init(k);
    } else {
      L[j].clear();
      thr[j] = 0;
      cap[j] = k;
    }
  }
  __syncthreads();
  const int first = w * 64 * R + l * R;

  for (int64_t t0 = d_lo; t0 < d_hi; t0 += DT) {
    const int64_t t1 = (t0 + DT < d_hi) ? t0 + DT : d_hi;
    // dense rows first, stored (not added) over the previous tile's slots, then the sparse rows
    // added on top: no slot is ever cleared. The dense rows go to registers while slower waves
    // still select from the previous tile; the barrier comes before the stores.
    accumulate_dense<ST, QT, R>(ix, dent, n_dense, t0 + first, acc);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < QT; ++q)
      if (q < nq) put_lds<R>(rows + q * DT + first, acc[q]);
    __syncthreads();
    accumulate_tile_stream<ST, (KPL <= 2 ? 8 : 4)>(st, ix, e_lo, e_hi, mem_lds, rows, DT, t0, t1);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < QPW; ++j) {
      const int ql = w * QPW + j;
      if (ql < nq) {
        if constexpr (kStaged)
          select_row<KPL, DT>(rows + ql * DT, t0, t1, S[j]);
        else
          select_row<KPL, DT>(rows + ql * DT, t0, t1, L[j], cap[j], thr[j]);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < QPW; ++j) {
    const int ql = w * QPW + j;
    if (ql < nq) {
      uint64_t* out = a.cand + ((int64_t)(q0 + ql) * a.n_groups + group) * KP;
      if constexpr (kStaged) {
        S[j].flush();
#pragma unroll
        for (int i = 0; i < KPL; ++i) out[l + 64 * i] = S[j].L.e[i];
      } else {
#pragma unroll
        for (int i = 0; i < KPL; ++i) out[l + 64 * i] = L[j].e[i];
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// Per-query sweep: one query; every wave of every workgroup sweeps its own document range in
// tiles of 64 * RS documents (RS per lane, in registers) with a private LDS accumulator for the
// sparse rows; the waves of a workgroup merge their lists at the end.
//
// LDS: max(sparse accumulators [W][64*RS], lists [W][KP]) | entry static fields [ecap] |
//      cursors [W][ecap] | members [pcap].

struct SweepArgs {
  IndexView ix;
  BatchView bv;       // entry table of one-query tiles (tile index = query index)
  uint64_t* cand;     // [n_groups][KP] for this query
  int32_t query;      // index of the query in the batch
  int64_t sweep_docs; // documents per wave, multiple of the skip block
  int32_t n_groups;   // workgroups
  int32_t acc_bytes;  // bytes of the first LDS region
  int32_t ecap;       // entry slots
  int32_t pcap;       // member slots
};

template <int W, int RS, int KPL, typename ST>
__global__ __launch_bounds__(W * 64) void k_sweep(SweepArgs a) {
  constexpr int KP = KPL * 64;
  constexpr int DT = 64 * RS;
  extern __shared__ __align__(16) uint8_t smem[];
  const int w = threadIdx.x >> 6;
  const int l = lane();
  float* acc_sp = reinterpret_cast<float*>(smem) + (size_t)w * DT;
  uint8_t* sbase = smem + a.acc_bytes;
  const EntryState st = carve_state(sbase, a.ecap, W, w);
  int32_t* mem_lds = reinterpret_cast<int32_t*>(
      sbase + (size_t)a.ecap * (kEntryStaticBytes + (size_t)W * kEntryDynBytes));
  const IndexView& ix = a.ix;
  const BatchView& bv = a.bv;
  const int q = a.query;
  const int64_t e_base = bv.tile_e0[q];
  const int E = bv.wave_e0[(int64_t)q * 2 + 1];
  const int64_t p0 = bv.q_off[q];
  const int P = (int)(bv.q_off[q + 1] - p0);
  const DenseEntry* dent = bv.dense_ent + p0;
  const int n_dense = bv.dense_n[q];
  const int64_t sw = (int64_t)blockIdx.x * W + w;
  const int64_t d_lo = sw * a.sweep_docs;
  const int64_t d_hi = (d_lo + a.sweep_docs < ix.n_docs) ? d_lo + a.sweep_docs : ix.n_docs;
  const int cap = bv.q_k[q];

  for (int i = threadIdx.x; i < P; i += W * 64) mem_lds[i] = bv.members[p0 + i];
  if (w == 0) load_static(bv.entries + e_base, bv.members, 0, E, p0, st);
  __syncthreads();
  if (d_lo < d_hi) init_cursors(ix, 0, E, d_lo, st);
  for (int i = l; i < DT / 4; i += 64)
    reinterpret_cast<float4*>(acc_sp)[i] = make_float4(0.f, 0.f, 0.f, 0.f);
  float acc[1][RS];
#pragma unroll
  for (int r = 0; r < RS; ++r) acc[0][r] = 0.f;
  StagedTopList<KPL> S;
  S.init(cap);
  float thr_s = -INFINITY;

  for (int64_t t0 = d_lo; t0 < d_hi; t0 += DT) {
    const int64_t t1 = (t0 + DT < d_hi) ? t0 + DT : d_hi;
    accumulate_tile_stream<ST, 4>(st, ix, 0, E, mem_lds, acc_sp, DT, t0, t1);
    accumulate_dense<ST, 1, RS>(ix, dent, n_dense, t0 + l * RS, acc);
    float v[RS];
    take_lds<RS>(acc_sp + l * RS, v);
#pragma unroll
    for (int r = 0; r < RS; ++r) {
      v[r] += acc[0][r];
      acc[0][r] = 0.f;
    }
    select_regs<KPL, RS>(v, t0 + l * RS, t1, S, thr_s);
  }
  S.flush();
  TopList<KPL>& L = S.L;
  uint64_t thr = S.thr;
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
  const int32_t* perm;    // output row of each query, or nullptr for the identity
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
  __shared__ uint64_t tau_w[MW];
  // Every list holds distinct documents sorted descending, so the largest k-th key of any one
  // list is a lower bound of the query's k-th key: keys below it are dropped before the merge.
  uint64_t tau = 0;
  for (int64_t j = threadIdx.x; j < a.lists; j += MW * 64) tau = umax64(tau, base[j * KP + cap - 1]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) tau = umax64(tau, bperm64(tau, l ^ o));
  if (l == 0) tau_w[w] = tau;
  __syncthreads();
  tau = umax64(umax64(tau_w[0], tau_w[1]), umax64(tau_w[2], tau_w[3]));
  TopList<KPL> L;
  L.clear();
  uint64_t thr = 0;
  // chunks are loaded kMergeAhead at a time so that their loads overlap (most are rejected by
  // one ballot)
  constexpr int kMergeAhead = KPL >= 8 ? 2 : 8;  // long lists leave few registers
  for (int64_t c0 = w; c0 < chunks; c0 += (int64_t)MW * kMergeAhead) {
    uint64_t x[kMergeAhead];
#pragma unroll
    for (int u = 0; u < kMergeAhead; ++u) {
      const int64_t c = c0 + (int64_t)u * MW;
      x[u] = (c < chunks) ? base[c * 64 + l] : 0ull;
    }
#pragma unroll
    for (int u = 0; u < kMergeAhead; ++u) L.offer(x[u] >= tau ? x[u] : 0ull, cap, thr);
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
  if (shift != 0.f) {
    // Returned scores are (sum of S_delta) + shift rounded to FP32, and the rounding can make
    // two different sums equal: re-rank by the returned value, then document id, the order the
    // results promise.
    // (the new keys go through the LDS buffer, free by now, so that one list is live at a time)
#pragma unroll
    for (int i = 0; i < KPL; ++i) {
      const uint64_t k0 = L.e[i];
      sh[0][l + 64 * i] = (k0 != 0) ? make_key(key_score(k0) + shift, key_doc(k0)) : 0ull;
    }
    L.clear();
#pragma unroll
    for (int i = 0; i < KPL; ++i) L.merge_chunk(sh[0][l + 64 * i]);
  }
  const int64_t count = bad ? 0 : ((int64_t)cap < a.n_docs ? cap : a.n_docs);
  const int64_t row = a.perm ? a.perm[q] : q;
  int32_t* oid = a.out_ids + row * a.k_max;
  float* osc = a.out_scores + row * a.k_max;
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
        osc[r] = key_score(key);
      } else {
        oid[r] = -1;
        osc[r] = -INFINITY;
      }
    }
  }
  if (l == 0) a.out_count[row] = bad ? -2 : (int32_t)count;
}

}  // namespace bm25dev
