// Device-side helpers for gfx950 (wave64): lane utilities, ordered keys, score storage,
// wave-resident top-k lists.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>

namespace bm25dev {

constexpr int kWave = 64;

__device__ __forceinline__ int lane() { return (int)__lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return (uint64_t)__ballot(p ? 1 : 0); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  return (lane() == 0) ? 0ull : (~0ull >> (64 - lane()));
}

__device__ __forceinline__ uint32_t readlane(uint32_t v, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
  uint32_t lo = readlane((uint32_t)v, l);
  uint32_t hi = readlane((uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

// Value of lane `src` (0..63) for every lane, through the LDS crossbar (no memory traffic).
__device__ __forceinline__ uint32_t bperm(uint32_t v, int src) {
  return (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)v);
}

__device__ __forceinline__ uint64_t bperm64(uint64_t v, int src) {
  uint32_t lo = bperm((uint32_t)v, src);
  uint32_t hi = bperm((uint32_t)(v >> 32), src);
  return ((uint64_t)hi << 32) | lo;
}

// Monotone map of FP32 to uint32: a < b (as floats, -0 == +0 canonicalised) iff ord(a) < ord(b).
__device__ __forceinline__ uint32_t f32_ord(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float ord_f32(uint32_t o) {
  uint32_t u = (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
  return __uint_as_float(u);
}

// Selection key: larger key = better result. Score descending first, then document id
// ascending. Key 0 never occurs for a real document and marks an empty list slot.
__device__ __forceinline__ uint64_t make_key(float s, uint32_t doc) {
  if (s == 0.0f) s = 0.0f;  // canonical +0
  return ((uint64_t)f32_ord(s) << 32) | (uint64_t)(~doc);
}

__device__ __forceinline__ uint32_t key_doc(uint64_t k) { return ~(uint32_t)k; }
__device__ __forceinline__ float key_score(uint64_t k) { return ord_f32((uint32_t)(k >> 32)); }

// Stored score types.
struct F32 {
  using T = float;
  static __device__ __forceinline__ float load(const T* p, int64_t i) { return p[i]; }
  static __device__ __forceinline__ T store(float v) { return v; }
};
struct F16 {
  using T = __half;
  static __device__ __forceinline__ float load(const T* p, int64_t i) { return __half2float(p[i]); }
  static __device__ __forceinline__ T store(float v) { return __float2half_rn(v); }
  static __device__ __forceinline__ float widen_lo(uint32_t w) {
    return __half2float(__ushort_as_half((unsigned short)(w & 0xFFFFu)));
  }
  static __device__ __forceinline__ float widen_hi(uint32_t w) {
    return __half2float(__ushort_as_half((unsigned short)(w >> 16)));
  }
};
struct BF16 {
  using T = uint16_t;
  static __device__ __forceinline__ float load(const T* p, int64_t i) {
    return __uint_as_float((uint32_t)p[i] << 16);
  }
  static __device__ __forceinline__ float widen_lo(uint32_t w) { return __uint_as_float(w << 16); }
  static __device__ __forceinline__ float widen_hi(uint32_t w) {
    return __uint_as_float(w & 0xFFFF0000u);
  }
  // round to nearest even (inputs are finite)
  static __device__ __forceinline__ T store(float v) {
    uint32_t u = __float_as_uint(v);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (T)(u >> 16);
  }
};

__device__ __forceinline__ uint64_t umax64(uint64_t a, uint64_t b) { return a > b ? a : b; }
__device__ __forceinline__ uint64_t umin64(uint64_t a, uint64_t b) { return a < b ? a : b; }

// Descending bitonic sort of one uint64 per lane across the wave.
__device__ __forceinline__ uint64_t wave_sort_desc(uint64_t v) {
  const int l = lane();
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      uint64_t o = bperm64(v, l ^ j);
      bool desc = (l & k) == 0;
      bool lower = (l & j) == 0;
      v = (desc == lower) ? umax64(v, o) : umin64(v, o);
    }
  }
  return v;
}

// Wave-resident list of the best KPL*64 keys, sorted descending: entry p = lane + 64 * i lives
// in e[i] of lane p % 64. Every call must be made by the whole wave with uniform arguments.
template <int KPL>
struct TopList {
  uint64_t e[KPL];

  __device__ __forceinline__ void clear() {
#pragma unroll
    for (int i = 0; i < KPL; ++i) e[i] = 0;
  }

  // Key at position p (uniform 0 <= p < 64*KPL).
  __device__ __forceinline__ uint64_t at(int p) const {
    const int r = p >> 6;
    uint64_t v = 0;
#pragma unroll
    for (int i = 0; i < KPL; ++i)
      if (i == r) v = e[i];
    return readlane64(v, p & 63);
  }

  // Inserts one key x (uniform) that is larger than the current key at position cap-1.
  __device__ __forceinline__ void insert(uint64_t x) {
    const int l = lane();
    int pos = 0;
#pragma unroll
    for (int i = 0; i < KPL; ++i) pos += __popcll(ballot(e[i] > x));
    uint64_t prev[KPL];
#pragma unroll
    for (int i = 0; i < KPL; ++i) {
      uint64_t up = bperm64(e[i], (l + 63) & 63);
      uint64_t carry = (i > 0) ? readlane64(e[i - 1], 63) : 0ull;
      prev[i] = (l == 0) ? carry : up;
    }
#pragma unroll
    for (int i = 0; i < KPL; ++i) {
      const int p = l + 64 * i;
      e[i] = (p < pos) ? e[i] : ((p == pos) ? x : prev[i]);
    }
  }

  // Merges 64 new keys (one per lane; 0 = none) into the list, keeping the best 64*KPL.
  __device__ __forceinline__ void merge_chunk(uint64_t c) {
    const int l = lane();
    c = wave_sort_desc(c);
    // half-cleaner of (list descending) ++ (chunk ascending): only the last register meets
    // the chunk; the result holds the best 64*KPL keys as a bitonic sequence
    uint64_t rev = bperm64(c, 63 - l);
    e[KPL - 1] = umax64(e[KPL - 1], rev);
    // bitonic merge to descending order
#pragma unroll
    for (int s = 32 * KPL; s >= 64; s >>= 1) {
      const int sr = s >> 6;
#pragma unroll
      for (int i = 0; i < KPL; ++i) {
        if ((i & sr) == 0) {
          uint64_t a = e[i], b = e[i + sr];
          e[i] = umax64(a, b);
          e[i + sr] = umin64(a, b);
        }
      }
    }
#pragma unroll
    for (int j = 32; j > 0; j >>= 1) {
#pragma unroll
      for (int i = 0; i < KPL; ++i) {
        uint64_t o = bperm64(e[i], l ^ j);
        e[i] = ((l & j) == 0) ? umax64(e[i], o) : umin64(e[i], o);
      }
    }
  }

  // Offers 64 keys (one per lane) against threshold position cap-1; returns nothing.
  __device__ __forceinline__ void offer(uint64_t key, int cap, uint64_t& thr) {
    uint64_t m = ballot(key > thr);
    if (m == 0) return;
    if (__popcll(m) >= 8) {
      merge_chunk(key > thr ? key : 0ull);
      thr = at(cap - 1);
      return;
    }
    while (m) {
      const int src = __builtin_ctzll(m);
      m &= m - 1;
      const uint64_t x = readlane64(key, src);
      if (x > thr) {
        insert(x);
        thr = at(cap - 1);
      }
    }
  }
};

// A TopList fed through a staging register: keys above the list's threshold are compacted
// into one staged key per lane and merged 64 at a time, so a key that enters costs a few
// instructions instead of a full insertion. The threshold is refreshed at each merge; until
// then it may lag, which only lets more keys into the stage. Whole-wave, uniform calls.
template <int KPL>
struct StagedTopList {
  TopList<KPL> L;
  uint64_t b;    // this lane's staged key (lanes < n)
  int n;         // staged keys
  int cap;       // list positions that count (k)
  uint64_t thr;  // key at position cap-1 after the last merge (0 while fewer than cap keys)

  __device__ __forceinline__ void init(int k) {
    L.clear();
    b = 0;
    n = 0;
    cap = k;
    thr = 0;
  }

  __device__ __forceinline__ float thr_score() const {
    return (thr == 0) ? -INFINITY : key_score(thr);
  }

  __device__ __forceinline__ void flush() {
    if (n == 0) return;
    L.merge_chunk(lane() < n ? b : 0ull);
    n = 0;
    thr = L.at(cap - 1);
  }

  // Offers one key per lane (0: none).
  __device__ __forceinline__ void offer(uint64_t key) {
    bool p = key > thr;
    uint64_t m = ballot(p);
    if (m == 0) return;
    int c = __popcll(m);
    if (n + c > 64) {
      flush();
      p = key > thr;
      m = ballot(p);
      if (m == 0) return;
      c = __popcll(m);
    }
    const int l = lane();
    const int rp = __popcll(m & lanemask_lt());
    // passing lanes go to n.., the others fill the remaining lanes (a permutation of 0..63)
    const int dest = p ? (n + rp) : ((n + c + (l - rp)) & 63);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_permute(dest << 2, (int)(uint32_t)key);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_permute(dest << 2, (int)(uint32_t)(key >> 32));
    if (l >= n && l < n + c) b = ((uint64_t)hi << 32) | lo;
    n += c;
  }
};

}  // namespace bm25dev
