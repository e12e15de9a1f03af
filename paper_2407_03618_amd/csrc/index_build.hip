// Index build: eager index-time scoring into a token-major sparse matrix.
//
// Steps (Section 2 "Calculation of BM25", "Eager index-time scoring", "Efficient Matrix
// Sparsity"; Section 2.1 for shifted variants):
//   1. validate the offsets on the device: |D| per document, sum |D| in int64, the longest
//      document, the document at every 1024th position;
//   2. one 64-bit key per token position, token | document | |D| (KeyLayout), with the first radix
//      histogram and the token id range check in the same pass;
//   3. stable LSD radix sort of the keys by the token bits (digits of at most 8 bits, each pass
//      ranked in LDS and written out as contiguous runs); positions arrive in document order, so
//      equal tokens stay ordered by document;
//   4. run-length encoding of equal keys: one stored pair per distinct (t, D), TF = run length,
//      and indptr from the first pair of every token;
//   5. DF = row length, IDF in FP64, long rows, dense-row candidates (chosen on the host: few);
//   6. per-pair score S(t, D) (or S - S_theta) in FP32, rounded to the storage type, with the
//      skip table of long rows (first entry at or after each document block) and the dense rows
//      written from the same pass.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <memory>
#include <utility>
#include <type_traits>
#include <vector>

#include "device.hpp"
#include "internal.hpp"
#include "scan.hpp"

using namespace bm25dev;

namespace bm25 {

// ------------------------------------------------------------------------------------------
// Device-wide exclusive scan.

constexpr int kScanThreads = 256;
constexpr int kScanPerThread = 16;
constexpr int64_t kScanChunk = kScanThreads * kScanPerThread;

template <typename T>
__device__ __forceinline__ T shfl_up_t(T v, int o) {
  const int src = (lane() - o) & 63;
  if constexpr (sizeof(T) == 8) {
    return (T)bperm64((uint64_t)v, src);
  } else {
    return (T)bperm((uint32_t)v, src);
  }
}

// Exclusive scan across a 256-thread block; returns the block total in `total`.
template <typename T>
__device__ T block_exclusive_scan(T v, T* lds, T& total) {
  const int l = lane();
  const int w = threadIdx.x >> 6;
  T x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    T y = shfl_up_t(x, o);
    if (l >= o) x += y;
  }
  if (l == 63) lds[w] = x;
  __syncthreads();
  T off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kScanThreads / 64; ++i) {
    T t = lds[i];
    if (i < w) off += t;
    tot += t;
  }
  __syncthreads();
  total = tot;
  return x - v + off;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const T* in, int64_t n, T* part) {
  __shared__ T lds[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPerThread;
  T s = 0;
#pragma unroll
  for (int i = 0; i < kScanPerThread; ++i) {
    int64_t j = base + i;
    if (j < n) s += in[j];
  }
  T tot;
  (void)block_exclusive_scan(s, lds, tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_top(T* part, int64_t nparts, T* total) {
  __shared__ T lds[kScanThreads / 64];
  T carry = 0;
  for (int64_t c = 0; c < nparts; c += kScanChunk) {
    const int64_t base = c + (int64_t)threadIdx.x * kScanPerThread;
    T v[kScanPerThread];
    T s = 0;
#pragma unroll
    for (int i = 0; i < kScanPerThread; ++i) {
      int64_t j = base + i;
      v[i] = (j < nparts) ? part[j] : (T)0;
      s += v[i];
    }
    T tot;
    T off = block_exclusive_scan(s, lds, tot) + carry;
#pragma unroll
    for (int i = 0; i < kScanPerThread; ++i) {
      int64_t j = base + i;
      if (j < nparts) part[j] = off;
      off += v[i];
    }
    carry += tot;
  }
  if (threadIdx.x == 0 && total != nullptr) *total = carry;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const T* in, T* out, int64_t n,
                                                             const T* part) {
  __shared__ T lds[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPerThread;
  T v[kScanPerThread];
  T s = 0;
#pragma unroll
  for (int i = 0; i < kScanPerThread; ++i) {
    int64_t j = base + i;
    v[i] = (j < n) ? in[j] : (T)0;
    s += v[i];
  }
  T tot;
  T off = block_exclusive_scan(s, lds, tot) + part[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanPerThread; ++i) {
    int64_t j = base + i;
    if (j < n) out[j] = off;
    off += v[i];
  }
}

int64_t scan_tmp_elems(int64_t n) { return (n + kScanChunk - 1) / kScanChunk + 1; }

template <typename T>
hipError_t scan_exclusive(const T* in, T* out, int64_t n, T* tmp, T* total, hipStream_t s) {
  if (n <= 0) {
    if (total) return hipMemsetAsync(total, 0, sizeof(T), s);
    return hipSuccess;
  }
  const int64_t nparts = (n + kScanChunk - 1) / kScanChunk;
  hipLaunchKernelGGL(k_scan_reduce<T>, dim3((unsigned)nparts), dim3(kScanThreads), 0, s, in, n,
                     tmp);
  hipLaunchKernelGGL(k_scan_top<T>, dim3(1), dim3(kScanThreads), 0, s, tmp, nparts, total);
  hipLaunchKernelGGL(k_scan_apply<T>, dim3((unsigned)nparts), dim3(kScanThreads), 0, s, in, out,
                     n, tmp);
  return hipGetLastError();
}

template hipError_t scan_exclusive<uint32_t>(const uint32_t*, uint32_t*, int64_t, uint32_t*,
                                             uint32_t*, hipStream_t);
template hipError_t scan_exclusive<int64_t>(const int64_t*, int64_t*, int64_t, int64_t*,
                                            int64_t*, hipStream_t);

// ------------------------------------------------------------------------------------------
// Build kernels.

struct BuildStatus {
  unsigned long long sum_len;
  unsigned int flags;  // 1: malformed offsets, 2: token id out of range, 4: document too long
  unsigned int max_len;  // longest document (clamped to 2^31 - 1)
};

// Layout of the 64-bit sort key of a token position, from the top: token | document | |D|.
// The document length rides in the low bits when the bits left over by the token and document
// ids hold the longest document (len_bits > 0); the score then reads it from the key instead of
// gathering doclen[d] for every stored pair. Equal (token, document) keys are equal keys either
// way, since |D| is a function of the document.
struct KeyLayout {
  int tok_shift;      // token = key >> tok_shift
  int doc_shift;      // document = (key >> doc_shift) & doc_mask
  uint64_t doc_mask;
  uint32_t len_mask;  // |D| = key & len_mask when len_bits > 0
  int len_bits;
};

__device__ __forceinline__ uint32_t key_token(uint64_t k, const KeyLayout& L) {
  return (uint32_t)(k >> L.tok_shift);
}
__device__ __forceinline__ uint32_t key_doc(uint64_t k, const KeyLayout& L) {
  return (uint32_t)((k >> L.doc_shift) & L.doc_mask);
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += bperm64(v, lane() ^ o);
  return v;
}

// Positions per entry of the granule table: gran_doc[g] = the document holding position
// g * kGranule (documents of valid offsets only).
constexpr int64_t kGranule = 1024;

__global__ __launch_bounds__(256) void k_validate(int64_t T, const int64_t* __restrict__ off,
                                                  int64_t N, int32_t* __restrict__ doclen,
                                                  int32_t* __restrict__ gran_doc,
                                                  BuildStatus* st) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  uint64_t local = 0;
  unsigned flags = 0;
  unsigned mx = 0;
  for (int64_t d = gid; d < N; d += stride) {
    const int64_t lo = off[d], hi = off[d + 1];
    const int64_t len = hi - lo;
    if (len < 0 || lo < 0 || hi > T) flags |= 1u;
    if (len > (int64_t)INT32_MAX) flags |= 4u;
    const int32_t lc = (int32_t)(len < 0 ? 0 : (len > INT32_MAX ? INT32_MAX : len));
    doclen[d] = lc;
    mx = mx > (unsigned)lc ? mx : (unsigned)lc;
    local += (uint64_t)(len > 0 ? len : 0);
    if (lo >= 0 && hi <= T && lo < hi)
      for (int64_t g = (lo + kGranule - 1) / kGranule; g * kGranule < hi; ++g)
        gran_doc[g] = (int32_t)d;
  }
  if (gid == 0 && (off[0] != 0 || off[N] != T)) flags |= 1u;
  // one atomic per block and quantity (same-address atomics from every wave serialize)
  __shared__ unsigned long long bsum[4];
  __shared__ unsigned bmax[4];
  local = wave_sum_u64(local);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned y = bperm(mx, lane() ^ o);
    mx = mx > y ? mx : y;
  }
  if (lane() == 0) {
    bsum[threadIdx.x >> 6] = local;
    bmax[threadIdx.x >> 6] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long sum = bsum[0] + bsum[1] + bsum[2] + bsum[3];
    const unsigned m01 = bmax[0] > bmax[1] ? bmax[0] : bmax[1];
    const unsigned m23 = bmax[2] > bmax[3] ? bmax[2] : bmax[3];
    const unsigned m = m01 > m23 ? m01 : m23;
    if (sum) atomicAdd(&st->sum_len, sum);
    if (m) atomicMax(&st->max_len, m);
  }
  if (flags) atomicOr(&st->flags, flags);
}

// Stable LSD radix sort by digits of the token (at most 8 bits each). A block owns
// kRadixBlockItems consecutive keys and each of its 4 waves a contiguous quarter, read 64 keys at a
// time, so the order (wave, round, lane) is the index order. The histogram holds one count per
// (digit, block), digit-major, so its exclusive scan gives every block the output start of each
// digit. The scatter ranks its block's keys by digit in LDS (stable), then writes each digit's
// keys as one contiguous run: consecutive lanes store to consecutive addresses.
constexpr int kRadixRounds = 16;
constexpr int kRadixWaveItems = 64 * kRadixRounds;
constexpr int kRadixBlockItems = 4 * kRadixWaveItems;
constexpr int kRadixBuckets = 256;

// Lanes whose digit equals this lane's (bits above the digit width are zero in every lane).
__device__ __forceinline__ uint64_t match_digit8(uint32_t d) {
  uint64_t m = ~0ull;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t x = ballot(bit);
    m &= bit ? x : ~x;
  }
  return m;
}

__global__ __launch_bounds__(256) void k_radix_hist(const uint64_t* __restrict__ keys, int64_t n,
                                                    int shift, uint32_t mask,
                                                    uint32_t* __restrict__ hist, int64_t nblk) {
  __shared__ uint32_t h[kRadixBuckets];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int w = threadIdx.x >> 6;
  const int l = lane();
  const int64_t base = (int64_t)blockIdx.x * kRadixBlockItems + (int64_t)w * kRadixWaveItems;
  uint64_t key[kRadixRounds];  // all loads in flight before the counting
#pragma unroll
  for (int r = 0; r < kRadixRounds; ++r) {
    const int64_t i = base + r * 64 + l;
    key[r] = (i < n) ? keys[i] : 0ull;
  }
#pragma unroll
  for (int r = 0; r < kRadixRounds; ++r) {
    const bool valid = base + r * 64 + l < n;
    const uint32_t d = (uint32_t)(key[r] >> shift) & mask;
    // the digits above the first are mostly zero (small token ids dominate under a Zipf law):
    // zeros are counted with one ballot, the other digits, spread out, with an LDS atomic each
    const uint64_t zeros = ballot(valid && d == 0u);
    if (valid && d != 0u) atomicAdd(&h[d], 1u);
    if (l == 0 && zeros) atomicAdd(&h[0], (uint32_t)__popcll(zeros));
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(256) void k_radix_scatter(const uint64_t* __restrict__ in,
                                                       uint64_t* __restrict__ out, int64_t n,
                                                       int shift, uint32_t mask,
                                                       const uint32_t* __restrict__ pos,
                                                       int64_t nblk) {
  __shared__ uint64_t sk[kRadixBlockItems];      // the block's keys in digit order
  __shared__ uint32_t cnt[4][kRadixBuckets];     // per wave: keys of each digit
  __shared__ uint32_t dstart[kRadixBuckets];     // block-local start of each digit
  __shared__ uint32_t gstart[kRadixBuckets];     // output start of each digit for this block
  __shared__ uint32_t scan4[4];
  const int t = threadIdx.x;
  const int w = t >> 6;
  const int l = lane();
#pragma unroll
  for (int ww = 0; ww < 4; ++ww) cnt[ww][t] = 0;
  gstart[t] = pos[(int64_t)t * nblk + blockIdx.x];
  const int64_t blk0 = (int64_t)blockIdx.x * kRadixBlockItems;
  const int64_t base = blk0 + (int64_t)w * kRadixWaveItems;
  uint64_t key[kRadixRounds];
#pragma unroll
  for (int r = 0; r < kRadixRounds; ++r) {
    const int64_t i = base + r * 64 + l;
    key[r] = (i < n) ? in[i] : 0ull;
  }
  __syncthreads();
  // rank of each key among the wave's keys of its digit, in index order
  const uint64_t lt = lanemask_lt();
  uint32_t rk[kRadixRounds];
#pragma unroll
  for (int r = 0; r < kRadixRounds; ++r) {
    const bool valid = base + r * 64 + l < n;
    const uint32_t d = (uint32_t)(key[r] >> shift) & mask;
    const uint64_t peers = match_digit8(d) & ballot(valid);
    const uint32_t c0 = cnt[w][d];
    rk[r] = c0 + (uint32_t)__popcll(peers & lt);
    if (valid && __builtin_ctzll(peers) == l) cnt[w][d] = c0 + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  // thread t = digit t: the waves' counts become exclusive prefixes, dstart the digit starts
  {
    uint32_t run = 0;
#pragma unroll
    for (int ww = 0; ww < 4; ++ww) {
      const uint32_t c = cnt[ww][t];
      cnt[ww][t] = run;
      run += c;
    }
    uint32_t tot;
    dstart[t] = block_exclusive_scan<uint32_t>(run, scan4, tot);
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRadixRounds; ++r) {
    if (base + r * 64 + l < n) {
      const uint32_t d = (uint32_t)(key[r] >> shift) & mask;
      sk[dstart[d] + cnt[w][d] + rk[r]] = key[r];
    }
  }
  __syncthreads();
  const int64_t nb = (n - blk0 < kRadixBlockItems) ? n - blk0 : kRadixBlockItems;
  for (int i = t; i < nb; i += 256) {
    const uint64_t k = sk[i];
    const uint32_t d = (uint32_t)(k >> shift) & mask;
    out[(int64_t)gstart[d] + (i - (int64_t)dstart[d])] = k;
  }
}

// One key per position (KeyLayout), with the histogram of the first radix pass (digit `mask0`
// of the token) for the same blocks the radix passes use, and the token range check (flag 2).
// The offsets are valid when this runs. Each wave walks its kRadixWaveItems positions 64 at a time
// and finds each position's document with a binary search over a window of 64 document starts
// held one per lane (s_i = off[base + 1 + i]): the document of p is base + #{i : s_i <= p}. A
// window serves until a round's last position lies past it. A round's first and last positions
// are searched once for the whole wave; the few documents starting between them decide each
// lane's document and give its length from the same window. A round in which more than 64
// documents start (empty documents) has every lane search the window, then further windows.
__global__ __launch_bounds__(256) void k_keys_hist(const int32_t* __restrict__ tok, int64_t T,
                                                   const int64_t* __restrict__ off, int64_t N,
                                                   int32_t V, const int32_t* __restrict__ doclen,
                                                   const int32_t* __restrict__ gran_doc,
                                                   KeyLayout L, uint32_t mask0,
                                                   uint64_t* __restrict__ keys,
                                                   uint32_t* __restrict__ hist, int64_t nblk,
                                                   BuildStatus* st) {
  __shared__ uint32_t h[kRadixBuckets];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int w = threadIdx.x >> 6;
  const int l = lane();
  const int64_t q0 = (int64_t)blockIdx.x * kRadixBlockItems + (int64_t)w * kRadixWaveItems;
  unsigned flags = 0;
  if (q0 < T) {
    // window of document starts: lane i holds off[base + 1 + i] (UINT32_MAX past the last)
    auto window = [&](int64_t b) -> uint32_t {
      const int64_t i = b + 1 + l;
      return (i <= N) ? (uint32_t)off[i] : UINT32_MAX;
    };
    // #{i < 64 : s_i <= p} for ascending s_i held by the lanes. Every lane runs the search (a
    // lane permute reads 0 from an inactive lane), so the call must be made by the whole wave.
    auto count_le = [&](uint32_t sv, uint32_t p) -> int {
      int pos = 0;
#pragma unroll
      for (int step = 32; step >= 1; step >>= 1) {
        const uint32_t v = bperm(sv, pos + step - 1);
        pos += (v <= p) ? step : 0;
      }
      return (readlane(sv, 63) <= p) ? 64 : pos;
    };
    // the same count for a position x held by every lane (a scalar search)
    auto count_le_u = [&](uint32_t sv, uint32_t x) -> int {
      if (readlane(sv, 63) <= x) return 64;
      int pos = 0;
#pragma unroll
      for (int step = 32; step >= 1; step >>= 1)
        if (readlane(sv, pos + step - 1) <= x) pos += step;
      return pos;
    };
    int64_t base = gran_doc[q0 / kGranule];
    uint32_t sv = window(base);
    uint32_t off_base = (uint32_t)off[base];
    int64_t dcur = base;
    for (int r = 0; r < kRadixRounds; ++r) {
      const int64_t p0 = q0 + r * 64;
      if (p0 >= T) break;
      const int64_t plast = (p0 + 63 < T) ? p0 + 63 : T - 1;
      if (readlane(sv, 63) <= (uint32_t)plast) {
        base = dcur;
        sv = window(base);
        off_base = (uint32_t)off[base];
      }
      const int64_t p = p0 + l;
      const bool valid = p < T;
      const int32_t t = valid ? tok[p] : 0;
      int64_t doc;
      uint32_t len;
      // documents starting inside this round: window entries [c0, c1)
      const int c0 = count_le_u(sv, (uint32_t)p0);
      const int c1 = count_le_u(sv, (uint32_t)plast);
      if (c1 < 64) {
        int cnt = c0;
        uint32_t lo = (c0 > 0) ? readlane(sv, c0 - 1) : off_base;
        uint32_t hi = readlane(sv, c0);
        for (int i = c0; i < c1; ++i) {
          const uint32_t si = readlane(sv, i);
          const uint32_t sn = readlane(sv, i + 1);
          if (si <= (uint32_t)p) {
            ++cnt;
            lo = si;
            hi = sn;
          }
        }
        doc = base + cnt;
        len = hi - lo;
      } else {
        // more than 64 documents start inside the round (empty documents): each lane searches
        // the window, then further windows
        const int cnt = count_le(sv, (uint32_t)p);
        doc = base + cnt;
        uint64_t more = ballot(valid && cnt == 64);
        for (int64_t b2 = base + 64; more != 0; b2 += 64) {
          const uint32_t s2 = window(b2);
          const int cc = count_le(s2, (uint32_t)p);
          if ((more >> l) & 1ull) doc = b2 + cc;
          more &= ballot(cc == 64);
        }
        len = valid ? (uint32_t)doclen[doc] : 0u;
      }
      if (valid && (t < 0 || t >= V)) flags |= 2u;
      if (valid)
        keys[p] = ((uint64_t)(uint32_t)t << L.tok_shift) | ((uint64_t)doc << L.doc_shift) |
                  (L.len_bits > 0 ? (uint64_t)len : 0ull);
      // the first digit is the token's low bits, spread enough that one LDS atomic per key costs
      // less than matching equal digits across the wave
      if (valid) atomicAdd(&h[(uint32_t)t & mask0], 1u);
      dcur = (int64_t)readlane((uint32_t)doc, 63);
    }
  }
  if (flags) atomicOr(&st->flags, flags);
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// Run-length encoding of equal keys. Each wave owns kRleWaveItems consecutive keys.
constexpr int kRleWaveItems = 64 * 32;
constexpr int kRleBlockItems = 4 * kRleWaveItems;

__global__ __launch_bounds__(256) void k_rle_count(const uint64_t* __restrict__ keys, int64_t n,
                                                   uint32_t* __restrict__ counts) {
  const int w = threadIdx.x >> 6;
  const int l = lane();
  const int64_t base = (int64_t)blockIdx.x * kRleBlockItems + (int64_t)w * kRleWaveItems;
  uint32_t c = 0;
  for (int r = 0; r < kRleWaveItems / 64; ++r) {
    const int64_t i = base + r * 64 + l;
    const bool head = i < n && (i == 0 || keys[i] != keys[i - 1]);
    c += (uint32_t)__popcll(ballot(head));
  }
  if (l == 0) counts[(int64_t)blockIdx.x * 4 + w] = c;
}

// Write side: the head of every run (a key that differs from the one before it) at position i
// becomes stored pair j, its rank among the heads: uniq[j] = key and tf[j] = the run length (the
// next head's position - i; the last run of a wave may end in the next wave's range, which the
// wave then reads until a different key). Where the token changes at a head, indptr[t] = j for the
// tokens t after the previous head's token up to this one; the wave holding the last position
// sets indptr[t] = nnz above the last token. Token ids are clamped to V here, so that ids out of
// range (reported at the next host sync) never index past indptr.
__global__ __launch_bounds__(256) void k_rle_write(const uint64_t* __restrict__ keys, int64_t n,
                                                   const uint32_t* __restrict__ bases,
                                                   KeyLayout L, int32_t V,
                                                   uint64_t* __restrict__ uniq,
                                                   int32_t* __restrict__ tf,
                                                   int64_t* __restrict__ indptr) {
  const int w = threadIdx.x >> 6;
  const int l = lane();
  const int64_t base = (int64_t)blockIdx.x * kRleBlockItems + (int64_t)w * kRleWaveItems;
  if (base >= n) return;
  uint32_t run = bases[(int64_t)blockIdx.x * 4 + w];
  const uint64_t lt = lanemask_lt();
  auto tok_of = [&](uint64_t k) -> int64_t {
    const uint32_t t = key_token(k, L);
    return t < (uint32_t)V ? (int64_t)t : (int64_t)V;
  };
  int64_t pend_i = -1;  // last head so far, whose run is still open, and its pair
  uint32_t pend_j = 0;
  for (int r = 0; r < kRleWaveItems / 64; ++r) {
    const int64_t i0 = base + r * 64;
    if (i0 >= n) break;
    const int64_t i = i0 + l;
    const bool valid = i < n;
    const uint64_t key = valid ? keys[i] : 0ull;
    const uint64_t prev = (valid && i > 0) ? keys[i - 1] : 0ull;
    const bool head = valid && (i == 0 || key != prev);
    const uint64_t m = ballot(head);
    if (head) {
      const uint32_t j = run + (uint32_t)__popcll(m & lt);
      uniq[j] = key;
      const uint64_t after = (l == 63) ? 0ull : (m >> (l + 1));
      if (after) tf[j] = (int32_t)(__builtin_ctzll(after) + 1);
      const int64_t t = tok_of(key);
      const int64_t pt = (i == 0) ? -1 : tok_of(prev);
      for (int64_t u = pt + 1; u <= t; ++u) indptr[u] = j;
    }
    if (m) {
      if (pend_i >= 0 && l == 0) tf[pend_j] = (int32_t)(i0 + __builtin_ctzll(m) - pend_i);
      pend_i = i0 + (63 - __builtin_clzll(m));
      pend_j = run + (uint32_t)__popcll(m) - 1;
    }
    run += (uint32_t)__popcll(m);
  }
  if (pend_i >= 0) {
    const uint64_t pk = keys[pend_i];
    int64_t end = n;
    for (int64_t q = base + kRleWaveItems; q < n; q += 64) {
      const uint64_t dm = ballot(q + l < n && keys[q + l] != pk);
      if (dm) {
        end = q + __builtin_ctzll(dm);
        break;
      }
    }
    if (l == 0) tf[pend_j] = (int32_t)(end - pend_i);
  }
  if (n - 1 < base + kRleWaveItems && l == 0) {
    const int64_t t_last = tok_of(keys[n - 1]);
    for (int64_t u = t_last + 1; u <= (int64_t)V; ++u) indptr[u] = run;
  }
}

// IDF(t, C) in FP64 per variant; the Lucene form is the IDF equation of Section 2.
__device__ double idf_of(int64_t df, double N, int variant) {
  if (df <= 0) return 0.0;
  const double d = (double)df;
  switch (variant) {
    case BM25_LUCENE: return log((N - d + 0.5) / (d + 0.5) + 1.0);
    case BM25_ROBERTSON: return log((N - d + 0.5) / (d + 0.5));
    case BM25_ATIRE: return log(N / d);
    case BM25_BM25L: return log((N + 1.0) / (d + 0.5));
    default: return log((N + 1.0) / d);  // BM25+, TF_ldp
  }
}

// S_theta(t) / IDF(t): the score at TF = 0 (Section 2.1); zero for sparse variants.
__device__ double theta_factor(int variant, double k1, double delta) {
  switch (variant) {
    case BM25_BM25PLUS: return delta;
    case BM25_BM25L: return (k1 + 1.0) * delta / (k1 + delta);
    case BM25_TFLDP: return 1.0 + log(1.0 + log(delta));
    default: return 0.0;
  }
}

__global__ __launch_bounds__(256) void k_df_idf(const int64_t* __restrict__ indptr, int32_t V,
                                                double N, int variant, double k1, double delta,
                                                int32_t* __restrict__ df,
                                                double* __restrict__ idf,
                                                double* __restrict__ theta,
                                                float* __restrict__ theta32,
                                                uint32_t* __restrict__ is_long,
                                                int64_t min_dense_df,
                                                uint32_t* __restrict__ is_dense) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= V) return;
  const int64_t d = indptr[t + 1] - indptr[t];
  df[t] = (int32_t)d;
  const double w = idf_of(d, N, variant);
  idf[t] = w;
  const double th = (d > 0) ? w * theta_factor(variant, k1, delta) : 0.0;
  theta[t] = th;
  theta32[t] = (float)th;
  is_long[t] = (d >= kLongRow) ? 1u : 0u;
  is_dense[t] = (d >= min_dense_df) ? 1u : 0u;
}

// Tokens flagged as dense-row candidates, compacted in token order with their document
// frequencies (the choice among them is made on the host: there are few).
__global__ void k_dense_candidates(const uint32_t* __restrict__ flag,
                                   const uint32_t* __restrict__ excl,
                                   const int32_t* __restrict__ df, int32_t V,
                                   int32_t* __restrict__ cand_tok, int32_t* __restrict__ cand_df) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= V || !flag[t]) return;
  cand_tok[excl[t]] = (int32_t)t;
  cand_df[excl[t]] = df[t];
}

// dense_id[tok[i]] = i for the chosen dense-row tokens (dense_id holds -1 elsewhere).
__global__ void k_set_dense_ids(const int32_t* __restrict__ tok, int32_t n,
                                int32_t* __restrict__ dense_id) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dense_id[tok[i]] = i;
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_long_id(const uint32_t* __restrict__ flag, const uint32_t* __restrict__ excl,
                          int32_t V, int32_t* __restrict__ long_id) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= V) return;
  long_id[t] = flag[t] ? (int32_t)excl[t] : -1;
}

struct ScoreParams {
  float k1, b, delta, inv_lavg, delta_log0;  // delta_log0 = 1 + ln(delta) (TF_ldp)
  int variant;
};

// Stored value per pair divided by IDF: S / IDF for sparse variants, (S - S_theta) / IDF for
// shifted ones, written in forms free of cancellation (Section 2.1: S_delta = S - S_theta).
__device__ __forceinline__ float stored_factor(float tf, float len, const ScoreParams& p) {
  const float norm = (1.0f - p.b) + p.b * (len * p.inv_lavg);
  switch (p.variant) {
    case BM25_LUCENE:
    case BM25_ROBERTSON: return tf / (tf + p.k1 * norm);
    case BM25_ATIRE: return (p.k1 + 1.0f) * tf / (tf + p.k1 * norm);
    case BM25_BM25PLUS: return (p.k1 + 1.0f) * tf / (p.k1 * norm + tf);
    case BM25_BM25L: {
      const float c = tf / norm;
      return (p.k1 + 1.0f) * p.k1 * c / ((p.k1 + c + p.delta) * (p.k1 + p.delta));
    }
    default: {  // TF_ldp: ln(1 + ln(c + delta)) - ln(1 + ln(delta))
      const float c = tf / norm;
      return logf((1.0f + logf(c + p.delta)) / p.delta_log0);
    }
  }
}

// Range class of a stored value v (the FP32 score x rounded to the storage type): bit 0 when v is
// subnormal in that type, bit 1 when x != 0 rounded to zero, bit 2 when finite x became infinite.
template <typename ST>
__device__ __forceinline__ uint32_t range_class(float x, typename ST::T v) {
  float back;
  float min_normal;
  if constexpr (sizeof(typename ST::T) == 4) {
    back = v;
    min_normal = 1.17549435e-38f;  // 2^-126
  } else if constexpr (std::is_same<ST, F16>::value) {
    back = __half2float(v);
    min_normal = 6.103515625e-05f;  // 2^-14
  } else {
    back = __uint_as_float((uint32_t)v << 16);
    min_normal = 1.17549435e-38f;
  }
  const float a = fabsf(back);
  uint32_t c = 0;
  if (a != 0.0f && a < min_normal) c |= 1u;
  if (back == 0.0f && x != 0.0f) c |= 2u;
  if (isinf(back) && !isinf(x)) c |= 4u;
  return c;
}

struct SkipOut {
  const int32_t* long_id;
  const int64_t* indptr;
  int64_t nblocks;
  uint32_t* skip;
};

template <typename T>
struct DenseOut {
  const int32_t* dense_id;  // dense row of each token or -1
  int64_t n_pad;
  T* dense;
};

// Per stored pair: document id, stored score and its range class; the pair's entries in the
// skip table (long rows) and its value in the dense rows (dense-row tokens).
template <typename ST>
__global__ __launch_bounds__(256) void k_score(const uint64_t* __restrict__ uniq,
                                               const int32_t* __restrict__ tf_in, int64_t nnz,
                                               const int32_t* __restrict__ doclen,
                                               const double* __restrict__ idf, ScoreParams p,
                                               KeyLayout L,
                                               int32_t* __restrict__ indices,
                                               typename ST::T* __restrict__ data,
                                               unsigned long long* __restrict__ range,
                                               SkipOut sko, DenseOut<typename ST::T> dno) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t cls = 0;
  if (j < nnz) {
    const uint64_t key = uniq[j];
    const uint32_t t = key_token(key, L);
    const uint32_t d = key_doc(key, L);
    const uint32_t tf = (uint32_t)tf_in[j];
    indices[j] = (int32_t)d;
    const float w = (float)idf[t];
    const uint32_t len = (L.len_bits > 0) ? (uint32_t)key & L.len_mask : (uint32_t)doclen[d];
    const float x = w * stored_factor((float)tf, (float)len, p);
    const typename ST::T v = ST::store(x);
    data[j] = v;
    cls = range_class<ST>(x, v);
    // skip table: skip[lid][b] = offset inside the row of the first entry whose document id is
    // >= b * kSkipBlock (the row length if none), for b in [0, nblocks]
    const int32_t lid = sko.long_id[t];
    if (lid >= 0) {
      const int64_t lo = sko.indptr[t], hi = sko.indptr[t + 1];
      uint32_t* row = sko.skip + (int64_t)lid * (sko.nblocks + 1);
      const int64_t blk = (int64_t)d / kSkipBlock;
      const int64_t prev = (j == lo) ? -1 : (int64_t)key_doc(uniq[j - 1], L) / kSkipBlock;
      for (int64_t b = prev + 1; b <= blk; ++b) row[b] = (uint32_t)(j - lo);
      if (j == hi - 1)
        for (int64_t b = blk + 1; b <= sko.nblocks; ++b) row[b] = (uint32_t)(hi - lo);
    }
    // dense rows: dense[h][d] = stored score of (t, d) for the dense tokens t
    const int32_t h = dno.dense_id[t];
    if (h >= 0) dno.dense[(int64_t)h * dno.n_pad + d] = v;
  }
  // one atomic per wave and class that occurs (almost never)
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const uint64_t m = ballot((cls >> c) & 1u);
    if (m != 0 && lane() == 0) atomicAdd(range + c, (unsigned long long)__popcll(m));
  }
}

static unsigned grid_for(int64_t n, int threads) {
  int64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  return (unsigned)g;
}

static int bits_needed(uint32_t x) {
  int b = 0;
  while (x) {
    ++b;
    x >>= 1;
  }
  return b;
}

size_t store_bytes(int dtype) { return dtype == BM25_F32 ? 4 : 2; }

}  // namespace bm25

using namespace bm25;

extern "C" int bm25_index_build(const int32_t* token_ids, int64_t n_tokens,
                                const int64_t* doc_offsets, int64_t n_docs, int32_t vocab_size,
                                const bm25_params* params, const bm25_allocator* allocator,
                                void* stream, bm25_index** out) {
  clear_error();
  if (!out) return set_error(BM25_E_INVAL, "out is NULL");
  *out = nullptr;
  if (!token_ids && n_tokens > 0) return set_error(BM25_E_INVAL, "token_ids is NULL");
  if (!doc_offsets || !params) return set_error(BM25_E_INVAL, "doc_offsets or params is NULL");
  if (n_docs < 1 || n_docs > INT32_MAX) return set_error(BM25_E_INVAL, "n_docs out of range");
  if (n_tokens < 0 || n_tokens >= (int64_t)UINT32_MAX)
    return set_error(BM25_E_INVAL, "n_tokens out of range");
  if (vocab_size < 1) return set_error(BM25_E_INVAL, "vocab_size must be >= 1");
  const bm25_params P = *params;
  if (!(P.k1 >= 0.0) || !(P.b >= 0.0 && P.b <= 1.0) || !(P.delta >= 0.0) ||
      !std::isfinite(P.k1) || !std::isfinite(P.delta))
    return set_error(BM25_E_INVAL, "k1, b or delta out of range");
  if (P.variant < BM25_LUCENE || P.variant > BM25_TFLDP)
    return set_error(BM25_E_INVAL, "unknown variant %d", P.variant);
  if (P.variant == BM25_TFLDP && !(P.delta > std::exp(-1.0)))
    return set_error(BM25_E_INVAL, "TF_ldp needs delta > 1/e");
  if (P.store_dtype < BM25_F32 || P.store_dtype > BM25_BF16)
    return set_error(BM25_E_INVAL, "unknown store dtype %d", P.store_dtype);
  if (n_tokens == 0) return set_error(BM25_E_INVAL, "sum of |D| is 0: L_avg is undefined");
  if (allocator && (!allocator->alloc || !allocator->free))
    return set_error(BM25_E_INVAL, "allocator callbacks are NULL");

  hipStream_t s = (hipStream_t)stream;
  std::unique_ptr<bm25_index> idx(new bm25_index());
  if (allocator) {
    idx->alloc.fn = *allocator;
    idx->alloc.custom = true;
  }
  idx->alloc.stream = s;
  idx->bind_alloc();
  const Alloc* al = &idx->alloc;
  BM25_HIP(hipGetDevice(&idx->device));
  idx->n_docs = n_docs;
  idx->n_tokens = n_tokens;
  idx->vocab = vocab_size;
  idx->params = P;
  const int64_t N = n_docs, T = n_tokens;
  const int32_t V = vocab_size;

#define BM25_ALLOC(buf, bytes)                                                          \
  do {                                                                                  \
    hipError_t e_ = (buf).reserve(bytes);                                               \
    if (e_ != hipSuccess)                                                               \
      return set_error(BM25_E_NOMEM, "device allocation of %lld bytes failed: %s",     \
                       (long long)(bytes), hipGetErrorString(e_));                      \
  } while (0)

  // 1. validation of the offsets, |D|, sum |D|, longest document, granule table (the token ids
  //    are checked with the keys, step 2)
  DevBuf st(al);
  BM25_ALLOC(st, sizeof(BuildStatus) + 4 * sizeof(unsigned long long));
  BM25_HIP(hipMemsetAsync(st.ptr, 0, sizeof(BuildStatus) + 4 * sizeof(unsigned long long), s));
  unsigned long long* range_dev = reinterpret_cast<unsigned long long*>(st.as<uint8_t>() +
                                                                         sizeof(BuildStatus));
  BM25_ALLOC(idx->doclen, (size_t)N * 4);
  DevBuf gran(al);
  BM25_ALLOC(gran, (size_t)((T + kGranule - 1) / kGranule) * 4);
  {
    unsigned g = (unsigned)std::min<int64_t>(grid_for(N, 256), 2048);
    hipLaunchKernelGGL(k_validate, dim3(g), dim3(256), 0, s, T, doc_offsets, N,
                       idx->doclen.as<int32_t>(), gran.as<int32_t>(), st.as<BuildStatus>());
    BM25_HIP(hipGetLastError());
  }
  BuildStatus hst{};
  BM25_HIP(hipMemcpyAsync(&hst, st.ptr, sizeof(hst), hipMemcpyDeviceToHost, s));
  BM25_HIP(hipStreamSynchronize(s));
  if (hst.flags & 1u) return set_error(BM25_E_RANGE, "document offsets are malformed");
  if (hst.flags & 4u) return set_error(BM25_E_RANGE, "a document holds more than 2^31-1 tokens");
  if (hst.sum_len == 0) return set_error(BM25_E_INVAL, "sum of |D| is 0: L_avg is undefined");
  idx->sum_len = (int64_t)hst.sum_len;
  idx->l_avg = (double)idx->sum_len / (double)N;

  // 2. keys with the first radix histogram and the token range check
  const int tbits = bits_needed((uint32_t)(V - 1));
  const int passes = (tbits + 7) / 8;
  const int dbits = passes > 0 ? (tbits + passes - 1) / passes : 0;  // digit width, <= 8
  const uint32_t dmask = (1u << dbits) - 1u;
  const int64_t nblk = (T + kRadixBlockItems - 1) / kRadixBlockItems;
  const int64_t hn = nblk * kRadixBuckets;
  KeyLayout kl;
  {
    const int dbits_doc = std::max(1, bits_needed((uint32_t)(N - 1)));
    const int lbits = std::max(1, bits_needed(hst.max_len));
    kl.len_bits = (tbits + dbits_doc + lbits <= 64) ? lbits : 0;
    kl.len_mask = kl.len_bits > 0 ? (uint32_t)((1ull << kl.len_bits) - 1) : 0u;
    kl.doc_shift = kl.len_bits;
    kl.doc_mask = (1ull << dbits_doc) - 1;
    kl.tok_shift = kl.len_bits + dbits_doc;
  }
  DevBuf ka(al), kb(al), hist(al), tmp(al);
  BM25_ALLOC(ka, (size_t)T * 8);
  BM25_ALLOC(kb, (size_t)T * 8);
  BM25_ALLOC(hist, (size_t)hn * 4);
  hipLaunchKernelGGL(k_keys_hist, dim3((unsigned)nblk), dim3(256), 0, s, token_ids, T,
                     doc_offsets, N, V, idx->doclen.as<int32_t>(), gran.as<int32_t>(), kl, dmask,
                     ka.as<uint64_t>(), hist.as<uint32_t>(), nblk, st.as<BuildStatus>());
  BM25_HIP(hipGetLastError());

  // 3. stable LSD radix sort by token digits (out-of-range ids, reported below, are sorted by
  //    their masked digits and never index anything)
  const int64_t nrb = (T + kRleBlockItems - 1) / kRleBlockItems;
  BM25_ALLOC(tmp, (size_t)std::max({scan_tmp_elems(hn), scan_tmp_elems(T), scan_tmp_elems(V),
                                    scan_tmp_elems(nrb * 4)}) * 8 + 64);
  uint64_t* src = ka.as<uint64_t>();
  uint64_t* dst = kb.as<uint64_t>();
  for (int pass = 0; pass < passes; ++pass) {
    const int shift = kl.tok_shift + dbits * pass;
    if (pass > 0) {  // the first pass's histogram came with the keys
      hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nblk), dim3(256), 0, s, src, T, shift,
                         dmask, hist.as<uint32_t>(), nblk);
      BM25_HIP(hipGetLastError());
    }
    BM25_HIP(scan_exclusive<uint32_t>(hist.as<uint32_t>(), hist.as<uint32_t>(), hn,
                                      tmp.as<uint32_t>(), nullptr, s));
    hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nblk), dim3(256), 0, s, src, dst, T, shift,
                       dmask, hist.as<uint32_t>(), nblk);
    BM25_HIP(hipGetLastError());
    std::swap(src, dst);
  }
  hist.release();

  // 4. run-length encoding: distinct (t, D) pairs and TF
  DevBuf counts(al), total(al);
  BM25_ALLOC(counts, (size_t)nrb * 4 * 4);
  BM25_ALLOC(total, 16);
  hipLaunchKernelGGL(k_rle_count, dim3((unsigned)nrb), dim3(256), 0, s, src, T,
                     counts.as<uint32_t>());
  BM25_HIP(hipGetLastError());
  BM25_HIP(scan_exclusive<uint32_t>(counts.as<uint32_t>(), counts.as<uint32_t>(), nrb * 4,
                                    tmp.as<uint32_t>(), total.as<uint32_t>(), s));
  uint32_t nnz32 = 0;
  BM25_HIP(hipMemcpyAsync(&nnz32, total.ptr, 4, hipMemcpyDeviceToHost, s));
  BM25_HIP(hipMemcpyAsync(&hst, st.ptr, sizeof(hst), hipMemcpyDeviceToHost, s));
  BM25_HIP(hipStreamSynchronize(s));
  if (hst.flags & 2u) return set_error(BM25_E_RANGE, "a token id lies outside [0, vocab_size)");
  const int64_t nnz = nnz32;
  idx->nnz = nnz;
  uint64_t* uniq = dst;  // the other sort buffer
  BM25_ALLOC(idx->tf, (size_t)std::max<int64_t>(nnz, 1) * 4);
  BM25_ALLOC(idx->indptr, ((size_t)V + 1) * 8);
  hipLaunchKernelGGL(k_rle_write, dim3((unsigned)nrb), dim3(256), 0, s, src, T,
                     counts.as<uint32_t>(), kl, V, uniq, idx->tf.as<int32_t>(),
                     idx->indptr.as<int64_t>());
  BM25_HIP(hipGetLastError());

  // 5. DF, IDF, S_theta, long rows, dense-row candidates
  BM25_ALLOC(idx->df, (size_t)V * 4);
  BM25_ALLOC(idx->idf, (size_t)V * 8);
  BM25_ALLOC(idx->theta, (size_t)V * 8);
  BM25_ALLOC(idx->theta32, (size_t)V * 4);
  BM25_ALLOC(idx->long_id, (size_t)V * 4);
  const int64_t min_dense_df = std::max<int64_t>(2, (N + kDenseFraction - 1) / kDenseFraction);
  DevBuf is_long(al), long_excl(al), is_dense(al), dense_excl(al);
  BM25_ALLOC(is_long, (size_t)V * 4);
  BM25_ALLOC(long_excl, (size_t)V * 4);
  BM25_ALLOC(is_dense, (size_t)V * 4);
  BM25_ALLOC(dense_excl, (size_t)V * 4);
  hipLaunchKernelGGL(k_df_idf, dim3(grid_for(V, 256)), dim3(256), 0, s,
                     idx->indptr.as<int64_t>(), V, (double)N, P.variant, P.k1, P.delta,
                     idx->df.as<int32_t>(), idx->idf.as<double>(), idx->theta.as<double>(),
                     idx->theta32.as<float>(), is_long.as<uint32_t>(), min_dense_df,
                     is_dense.as<uint32_t>());
  BM25_HIP(hipGetLastError());
  BM25_HIP(scan_exclusive<uint32_t>(is_long.as<uint32_t>(), long_excl.as<uint32_t>(), V,
                                    tmp.as<uint32_t>(), total.as<uint32_t>() + 1, s));
  hipLaunchKernelGGL(k_long_id, dim3(grid_for(V, 256)), dim3(256), 0, s, is_long.as<uint32_t>(),
                     long_excl.as<uint32_t>(), V, idx->long_id.as<int32_t>());
  BM25_HIP(hipGetLastError());
  BM25_HIP(scan_exclusive<uint32_t>(is_dense.as<uint32_t>(), dense_excl.as<uint32_t>(), V,
                                    tmp.as<uint32_t>(), total.as<uint32_t>() + 2, s));
  // candidate lists in the long-row scratch, which the long ids no longer need
  int32_t* cand_tok = reinterpret_cast<int32_t*>(is_long.ptr);
  int32_t* cand_df = reinterpret_cast<int32_t*>(long_excl.ptr);
  hipLaunchKernelGGL(k_dense_candidates, dim3(grid_for(V, 256)), dim3(256), 0, s,
                     is_dense.as<uint32_t>(), dense_excl.as<uint32_t>(), idx->df.as<int32_t>(), V,
                     cand_tok, cand_df);
  BM25_HIP(hipGetLastError());
  uint32_t counts_h[2] = {0, 0};  // long rows, dense-row candidates
  BM25_HIP(hipMemcpyAsync(counts_h, total.as<uint32_t>() + 1, 8, hipMemcpyDeviceToHost, s));
  BM25_HIP(hipStreamSynchronize(s));
  const uint32_t n_long = counts_h[0];
  const uint32_t n_cand = counts_h[1];

  // 6. dense rows of the most frequent tokens: the candidates are few (a token in at least 1/16
  //    of the documents), so the choice runs on the host. The rows are kept in token order, so
  //    that the layout does not depend on tie order.
  const int64_t sb = (int64_t)store_bytes(P.store_dtype);
  idx->n_pad = ((N + kDensePad - 1) / kDensePad) * kDensePad;
  {
    std::vector<int32_t> ct(n_cand), cd(n_cand);
    if (n_cand > 0) {
      BM25_HIP(hipMemcpyAsync(ct.data(), cand_tok, (size_t)n_cand * 4, hipMemcpyDeviceToHost, s));
      BM25_HIP(hipMemcpyAsync(cd.data(), cand_df, (size_t)n_cand * 4, hipMemcpyDeviceToHost, s));
      BM25_HIP(hipStreamSynchronize(s));
    }
    const int64_t h_max = kDenseBytes / (idx->n_pad * sb);
    std::vector<std::pair<int32_t, int32_t>> cand;  // (-df, token): most frequent first
    cand.reserve(n_cand);
    for (uint32_t i = 0; i < n_cand; ++i) cand.emplace_back(-cd[i], ct[i]);
    std::sort(cand.begin(), cand.end());
    if ((int64_t)cand.size() > h_max) cand.resize((size_t)std::max<int64_t>(h_max, 0));
    std::vector<int32_t> toks;
    for (auto& c : cand) toks.push_back(c.second);
    std::sort(toks.begin(), toks.end());
    idx->n_dense = (int64_t)toks.size();
    // rank of each row by document frequency, for grouping queries that share frequent rows
    std::vector<int32_t> rank(std::max<size_t>(toks.size(), 1), 0);
    for (size_t r = 0; r < cand.size(); ++r)
      rank[(size_t)(std::lower_bound(toks.begin(), toks.end(), cand[r].second) - toks.begin())] =
          (int32_t)r;
    BM25_ALLOC(idx->dense_rank, rank.size() * 4);
    BM25_HIP(hipMemcpyAsync(idx->dense_rank.ptr, rank.data(), rank.size() * 4,
                            hipMemcpyHostToDevice, s));
    BM25_ALLOC(idx->dense_id, (size_t)V * 4);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(V, 256)), dim3(256), 0, s,
                       idx->dense_id.as<int32_t>(), (int64_t)V, -1);
    BM25_HIP(hipGetLastError());
    if (!toks.empty()) {
      // the chosen tokens go through the (now free) candidate list
      BM25_HIP(hipMemcpyAsync(cand_tok, toks.data(), toks.size() * 4, hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_set_dense_ids, dim3(grid_for((int64_t)toks.size(), 256)), dim3(256),
                         0, s, cand_tok, (int32_t)toks.size(), idx->dense_id.as<int32_t>());
      BM25_HIP(hipGetLastError());
    }
    // the host vectors above are read by the copies in flight: wait before they go
    BM25_HIP(hipStreamSynchronize(s));
  }
  const size_t dbytes = (size_t)std::max<int64_t>(1, idx->n_dense) * idx->n_pad * sb;
  BM25_ALLOC(idx->dense, dbytes);
  if (idx->n_dense > 0) BM25_HIP(hipMemsetAsync(idx->dense.ptr, 0, dbytes, s));
  idx->n_long = n_long;
  idx->n_blocks = (N + kSkipBlock - 1) / kSkipBlock;
  BM25_ALLOC(idx->skip, (size_t)std::max<int64_t>(1, (int64_t)n_long * (idx->n_blocks + 1)) * 4);

  // 7. per-pair scores, with the skip table of long rows and the dense rows
  BM25_ALLOC(idx->indices, (size_t)std::max<int64_t>(nnz, 1) * 4);
  BM25_ALLOC(idx->data, (size_t)std::max<int64_t>(nnz, 1) * sb);
  ScoreParams sp;
  sp.k1 = (float)P.k1;
  sp.b = (float)P.b;
  sp.delta = (float)P.delta;
  sp.inv_lavg = (float)(1.0 / idx->l_avg);
  sp.delta_log0 = (P.variant == BM25_TFLDP) ? (float)(1.0 + std::log(P.delta)) : 1.0f;
  sp.variant = P.variant;
  SkipOut sko;
  sko.long_id = idx->long_id.as<int32_t>();
  sko.indptr = idx->indptr.as<int64_t>();
  sko.nblocks = idx->n_blocks;
  sko.skip = idx->skip.as<uint32_t>();
  if (nnz > 0) {
    const unsigned g = grid_for(nnz, 256);
    switch (P.store_dtype) {
      case BM25_F32: {
        DenseOut<float> dno{idx->dense_id.as<int32_t>(), idx->n_pad, idx->dense.as<float>()};
        hipLaunchKernelGGL(k_score<F32>, dim3(g), dim3(256), 0, s, uniq, idx->tf.as<int32_t>(),
                           nnz, idx->doclen.as<int32_t>(), idx->idf.as<double>(), sp, kl,
                           idx->indices.as<int32_t>(), idx->data.as<float>(), range_dev, sko,
                           dno);
        break;
      }
      case BM25_F16: {
        DenseOut<__half> dno{idx->dense_id.as<int32_t>(), idx->n_pad, idx->dense.as<__half>()};
        hipLaunchKernelGGL(k_score<F16>, dim3(g), dim3(256), 0, s, uniq, idx->tf.as<int32_t>(),
                           nnz, idx->doclen.as<int32_t>(), idx->idf.as<double>(), sp, kl,
                           idx->indices.as<int32_t>(), idx->data.as<__half>(), range_dev, sko,
                           dno);
        break;
      }
      default: {
        DenseOut<uint16_t> dno{idx->dense_id.as<int32_t>(), idx->n_pad,
                               idx->dense.as<uint16_t>()};
        hipLaunchKernelGGL(k_score<BF16>, dim3(g), dim3(256), 0, s, uniq, idx->tf.as<int32_t>(),
                           nnz, idx->doclen.as<int32_t>(), idx->idf.as<double>(), sp, kl,
                           idx->indices.as<int32_t>(), idx->data.as<uint16_t>(), range_dev, sko,
                           dno);
      }
    }
    BM25_HIP(hipGetLastError());
  }
  unsigned long long range_h[3] = {0, 0, 0};
  BM25_HIP(hipMemcpyAsync(range_h, range_dev, sizeof(range_h), hipMemcpyDeviceToHost, s));
  BM25_HIP(hipStreamSynchronize(s));
  idx->range_subnormal = (int64_t)range_h[0];
  idx->range_to_zero = (int64_t)range_h[1];
  idx->range_overflow = (int64_t)range_h[2];
#undef BM25_ALLOC
  idx->alloc.stream = nullptr;
  *out = idx.release();
  return BM25_OK;
}

extern "C" int bm25_index_range_stats(const bm25_index* index, int64_t* subnormal,
                                      int64_t* flushed_to_zero, int64_t* overflow) {
  clear_error();
  if (!index) return set_error(BM25_E_INVAL, "index is NULL");
  if (subnormal) *subnormal = index->range_subnormal;
  if (flushed_to_zero) *flushed_to_zero = index->range_to_zero;
  if (overflow) *overflow = index->range_overflow;
  return BM25_OK;
}

extern "C" int bm25_index_info(const bm25_index* index, int64_t* n_docs, int32_t* vocab_size,
                               int64_t* nnz, int64_t* sum_len, double* l_avg,
                               bm25_params* params) {
  clear_error();
  if (!index) return set_error(BM25_E_INVAL, "index is NULL");
  if (n_docs) *n_docs = index->n_docs;
  if (vocab_size) *vocab_size = index->vocab;
  if (nnz) *nnz = index->nnz;
  if (sum_len) *sum_len = index->sum_len;
  if (l_avg) *l_avg = index->l_avg;
  if (params) *params = index->params;
  return BM25_OK;
}

extern "C" int bm25_index_export(const bm25_index* index, int64_t* indptr, int32_t* indices,
                                 int32_t* tf, int32_t* df, double* idf, double* theta,
                                 void* data, void* stream) {
  clear_error();
  if (!index) return set_error(BM25_E_INVAL, "index is NULL");
  hipStream_t s = (hipStream_t)stream;
  const size_t V = (size_t)index->vocab, nnz = (size_t)index->nnz;
  auto cp = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    if (!dst || bytes == 0) return hipSuccess;
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s);
  };
  BM25_HIP(cp(indptr, index->indptr.ptr, (V + 1) * 8));
  BM25_HIP(cp(indices, index->indices.ptr, nnz * 4));
  BM25_HIP(cp(tf, index->tf.ptr, nnz * 4));
  BM25_HIP(cp(df, index->df.ptr, V * 4));
  BM25_HIP(cp(idf, index->idf.ptr, V * 8));
  BM25_HIP(cp(theta, index->theta.ptr, V * 8));
  BM25_HIP(cp(data, index->data.ptr, nnz * store_bytes(index->params.store_dtype)));
  return BM25_OK;
}

extern "C" int64_t bm25_index_device_bytes(const bm25_index* index) {
  if (!index) return 0;
  const bm25::DevBuf* bufs[] = {&index->indptr, &index->indices, &index->tf, &index->data,
                                &index->df, &index->idf, &index->theta, &index->theta32,
                                &index->doclen, &index->long_id, &index->skip,
                                &index->dense_id, &index->dense_rank, &index->dense};
  int64_t total = 0;
  for (auto* b : bufs) total += (int64_t)b->bytes;
  total += (int64_t)index->batch_scratch.arena.bytes + (int64_t)index->plain_scratch.arena.bytes;
  return total;
}

extern "C" void bm25_index_free(bm25_index* index) {
  if (!index) return;
  (void)hipDeviceSynchronize();
  index->alloc.stream = nullptr;
  for (auto& ev : index->timing_events) {
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  for (auto* sc : {&index->batch_scratch, &index->plain_scratch}) sc->release_handles();
  delete index;
}
