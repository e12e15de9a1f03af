// Tokenization and vocabulary mapping on the device: the step in front of the index build.
//
// Section 2 ("Tokenization"): the text is split with the pattern (?u)\b\w\w+\b (a token is a
// maximal run of at least two Unicode word characters), then a dictionary maps each distinct
// word to an integer index and the documents' words become indices.
//
// Steps, per document (documents never share a token):
//   1. every byte that starts a valid UTF-8 sequence is a character; bytes that do not (stray
//      continuation bytes, invalid leads, overlong, surrogate or out-of-range sequences) are
//      separators, as the replacement characters Python's decoder puts there would be;
//   2. a character is a word character when the generated table says so (Python's \w: isalnum()
//      or "_", over the whole code space); with lowercasing each code point first takes its
//      simple lowercase mapping, and U+0130 becomes "i" followed by U+0307 (not a word
//      character), so a run ends after it;
//   3. a run starts at a word character whose predecessor does not continue a run; the run
//      starts are compacted in byte order, then one thread per run walks it, counts its code
//      points and hashes them (64-bit FNV-1a with one round per
//      code point, finalised with the splitmix64 mixer); runs of two or more code points are the
//      tokens;
//   4. tokens go into an open-addressing hash table keyed by their hash; the table records each
//      word's first token; every token is then compared with its word's first token code point
//      by code point, so two words with the same 64-bit hash are detected (an error, not a merge);
//   5. ids follow the order of first occurrence (a scan over first-token flags), the corpus
//      becomes int32 ids with per-document offsets, and the words are written as UTF-8.
// Queries go through steps 1-3 and look their hashes up in the corpus table; words absent from
// it are dropped.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>

#include "device.hpp"
#include "internal.hpp"
#include "scan.hpp"
#include "unicode_tables.inc"

using namespace bm25dev;

namespace bm25 {
namespace tok {

constexpr int kThreads = 256;
constexpr uint64_t kEmpty = 0;

__device__ __forceinline__ bool uni_word(uint32_t cp) {
  if (cp >= 0x110000u) return false;
  const uint32_t b = kUniBlockIndex[cp >> 8];
  return (kUniBlockBits[b][(cp >> 5) & 7u] >> (cp & 31u)) & 1u;
}

__device__ __forceinline__ uint32_t uni_lower(uint32_t cp) {
  if (cp >= 0x110000u) return cp;
  const uint32_t b = kUniLowerIndex[cp >> 7];
  return b == 0 ? cp : (uint32_t)((int32_t)cp + kUniLowerDelta[b][cp & 127u]);
}

// Length (1..4) of the valid UTF-8 sequence starting at byte i of a document ending at `hi`, and
// its code point; 0 when none starts there.
__device__ __forceinline__ int decode(const uint8_t* t, int64_t i, int64_t hi, uint32_t& cp) {
  const uint32_t b0 = t[i];
  if (b0 < 0x80u) {
    cp = b0;
    return 1;
  }
  if (b0 < 0xC2u || b0 > 0xF4u) return 0;
  int n;
  uint32_t lo2 = 0x80u, hi2 = 0xBFu;
  if (b0 < 0xE0u) {
    n = 2;
    cp = b0 & 0x1Fu;
  } else if (b0 < 0xF0u) {
    n = 3;
    cp = b0 & 0x0Fu;
    if (b0 == 0xE0u) lo2 = 0xA0u;       // overlong
    else if (b0 == 0xEDu) hi2 = 0x9Fu;  // surrogates
  } else {
    n = 4;
    cp = b0 & 0x07u;
    if (b0 == 0xF0u) lo2 = 0x90u;       // overlong
    else if (b0 == 0xF4u) hi2 = 0x8Fu;  // above U+10FFFF
  }
  if (i + n > hi) return 0;
  const uint32_t b1 = t[i + 1];
  if (b1 < lo2 || b1 > hi2) return 0;
  cp = (cp << 6) | (b1 & 0x3Fu);
  for (int j = 2; j < n; ++j) {
    const uint32_t bj = t[i + j];
    if ((bj & 0xC0u) != 0x80u) return 0;
    cp = (cp << 6) | (bj & 0x3Fu);
  }
  return n;
}

// A character after case mapping: its code point, whether it is a word character, and whether a
// run continues past it (false for U+0130 when lowercasing: "i" then a non-word U+0307).
struct Char {
  int len;  // bytes; 0: not a character start
  uint32_t cp;
  bool word;
  bool joins;
};

__device__ __forceinline__ Char char_at(const uint8_t* t, int64_t i, int64_t hi, bool lower) {
  Char c;
  c.len = decode(t, i, hi, c.cp);
  c.word = false;
  c.joins = false;
  if (c.len == 0) return c;
  if (c.cp < 0x80u) {
    // ASCII, most of most text: the tables' answers, without their lookups (letters map A-Z to
    // a-z; word characters are letters, digits and the underscore)
    if (lower && c.cp - 'A' < 26u) c.cp += 32u;
    c.word = (c.cp - 'a' < 26u) || (c.cp - 'A' < 26u) || (c.cp - '0' < 10u) || c.cp == '_';
    c.joins = c.word;
    return c;
  }
  bool split_after = false;
  if (lower) {
    if (c.cp == 0x130u) {
      c.cp = 'i';
      split_after = true;
    } else {
      c.cp = uni_lower(c.cp);
    }
  }
  c.word = uni_word(c.cp);
  c.joins = c.word && !split_after;
  return c;
}

// Whether the character that ends just before byte i (i > lo) continues a run into i.
__device__ __forceinline__ bool prev_joins(const uint8_t* t, int64_t lo, int64_t i, bool lower) {
  for (int back = 1; back <= 4 && i - back >= lo; ++back) {
    const int64_t s = i - back;
    const Char c = char_at(t, s, i, lower);
    if (c.len == back) return c.joins;
    if ((t[s] & 0xC0u) != 0x80u) return false;  // a lead byte: nothing valid spans further back
  }
  return false;
}

__device__ __forceinline__ uint64_t hash_step(uint64_t h, uint32_t cp) {
  // one FNV-1a round per code point (the whole code point, not its bytes: one 64-bit multiply
  // per character); hash_final's mixer spreads the bits
  h ^= cp;
  h *= 0x100000001b3ull;
  return h;
}

__device__ __forceinline__ uint64_t hash_final(uint64_t h) {
  h ^= h >> 30;
  h *= 0xbf58476d1ce4e5b9ull;
  h ^= h >> 27;
  h *= 0x94d049bb133111ebull;
  h ^= h >> 31;
  return h == kEmpty ? 1ull : h;
}

struct TextView {
  const uint8_t* text;
  const int64_t* doc_off;  // [n_docs + 1] byte offsets
  int64_t n_docs;
  bool lower;
};

// 1. run starts: mark[i] = 1 where a run of word characters starts. One workgroup per document
//    at a time, its threads striding over the document's bytes.
__global__ __launch_bounds__(kThreads) void k_mark_runs(TextView tv, uint32_t* mark) {
  for (int64_t d = blockIdx.x; d < tv.n_docs; d += gridDim.x) {
    const int64_t lo = tv.doc_off[d], hi = tv.doc_off[d + 1];
    for (int64_t i = lo + threadIdx.x; i < hi; i += kThreads) {
      const Char c = char_at(tv.text, i, hi, tv.lower);
      uint32_t m = 0;
      if (c.len > 0 && c.word) m = (i == lo || !prev_joins(tv.text, lo, i, tv.lower)) ? 1u : 0u;
      mark[i] = m;
    }
  }
}

struct Run {
  uint32_t start, end;  // byte span
  uint32_t n_cp;        // code points
  int32_t doc;
  uint64_t hash;
};

// 2a. each run start's byte and document go to the run's slot (same document iteration as
//     k_mark_runs).
__global__ __launch_bounds__(kThreads) void k_run_starts(TextView tv, const uint32_t* mark,
                                                         const uint32_t* run_idx, Run* runs) {
  for (int64_t d = blockIdx.x; d < tv.n_docs; d += gridDim.x) {
    const int64_t lo = tv.doc_off[d], hi = tv.doc_off[d + 1];
    for (int64_t i = lo + threadIdx.x; i < hi; i += kThreads) {
      if (!mark[i]) continue;
      const uint32_t r = run_idx[i];
      runs[r].start = (uint32_t)i;
      runs[r].doc = (int32_t)d;
    }
  }
}

// 2b. one thread per run walks it: consecutive lanes take consecutive runs, so a wave walks 64
//     runs at once instead of the few that start in 64 consecutive bytes.
__global__ __launch_bounds__(kThreads) void k_walk_runs(TextView tv, Run* runs, uint32_t* keep,
                                                        int64_t n_runs) {
  const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (r >= n_runs) return;
  const int64_t i = runs[r].start;
  const int64_t hi = tv.doc_off[runs[r].doc + 1];
  uint64_t h = 0xcbf29ce484222325ull;
  uint32_t n = 0;
  int64_t j = i;
  while (j < hi) {
    const Char c = char_at(tv.text, j, hi, tv.lower);
    if (c.len == 0 || !c.word) break;
    h = hash_step(h, c.cp);
    ++n;
    j += c.len;
    if (!c.joins) break;
  }
  runs[r].end = (uint32_t)j;
  runs[r].n_cp = n;
  runs[r].hash = hash_final(h);
  keep[r] = n >= 2 ? 1u : 0u;
}

// 3. compaction of the tokens (runs of two or more code points).
__global__ __launch_bounds__(kThreads) void k_compact(const Run* runs, const uint32_t* keep,
                                                      const uint32_t* tok_idx, int64_t n_runs,
                                                      Run* toks) {
  const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (r < n_runs && keep[r]) toks[tok_idx[r]] = runs[r];
}

// Per-document token offsets: the first token of each document (tokens are in byte order).
__global__ __launch_bounds__(kThreads) void k_doc_offsets(const Run* toks, int64_t n_toks,
                                                          int64_t n_docs, int64_t* doc_tok) {
  const int64_t d = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (d > n_docs) return;
  if (d == n_docs) {
    doc_tok[d] = n_toks;
    return;
  }
  int64_t lo = 0, hi = n_toks;  // first token with doc >= d
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (toks[mid].doc < d) lo = mid + 1;
    else hi = mid;
  }
  doc_tok[d] = lo;
}

// Offsets must start at 0, never decrease and end at the text size; bad[0] != 0 otherwise.
__global__ __launch_bounds__(kThreads) void k_check_offsets(const int64_t* off, int64_t n,
                                                           int64_t n_bytes, unsigned int* bad) {
  const int64_t d = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (d > n) return;
  bool ok = true;
  if (d == 0) ok = off[0] == 0;
  if (d == n) ok = ok && off[n] == n_bytes;
  if (d < n) ok = ok && off[d] <= off[d + 1];
  if (!ok) atomicOr(bad, 1u);
}

__global__ __launch_bounds__(kThreads) void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ __launch_bounds__(kThreads) void k_fill_u64(uint64_t* p, int64_t n, uint64_t v) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) p[i] = v;
}

// 4. insertion: slot of each token's hash (linear probing); the slot keeps the word's first token.
//    status[0] counts occupied slots, status[1] flags a full table.
__global__ __launch_bounds__(kThreads) void k_insert(const Run* toks, int64_t n_toks,
                                                     unsigned long long* keys, uint32_t* first,
                                                     int64_t cap, uint32_t* tok_slot,
                                                     unsigned int* status) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= n_toks) return;
  const unsigned long long h = toks[t].hash;
  int64_t s = (int64_t)(h & (uint64_t)(cap - 1));
  for (int64_t probe = 0; probe < cap; ++probe) {
    // a plain read first: a frequent word's slot is found filled by almost all of its tokens,
    // which then skip the atomic (same-address atomics from millions of tokens serialize)
    unsigned long long k = __hip_atomic_load(keys + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (k == kEmpty) k = atomicCAS(keys + s, (unsigned long long)kEmpty, h);
    if (k == kEmpty || k == h) {
      if (k == kEmpty) atomicAdd(status, 1u);
      // first only decreases: a token at or after the value read needs no update
      if ((uint32_t)t < __hip_atomic_load(first + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMin(first + s, (uint32_t)t);
      tok_slot[t] = (uint32_t)s;
      return;
    }
    s = (s + 1) & (cap - 1);
  }
  atomicOr(status + 1, 1u);
  tok_slot[t] = 0xFFFFFFFFu;
}

// Code point by code point comparison of two tokens' words (after case mapping).
__device__ bool same_word(const uint8_t* text, const Run& a, const Run& b, bool lower) {
  if (a.n_cp != b.n_cp) return false;
  // most repeats are byte for byte the same text, which decodes and maps to the same code
  // points; only spans that differ (case, with lowercasing) are compared code point by code point
  const uint32_t len = a.end - a.start;
  if (b.end - b.start == len) {
    uint32_t x = 0;
    while (x < len && text[(int64_t)a.start + x] == text[(int64_t)b.start + x]) ++x;
    if (x == len) return true;
  }
  int64_t i = a.start, j = b.start;
  for (uint32_t n = 0; n < a.n_cp; ++n) {
    const Char ca = char_at(text, i, a.end, lower);
    const Char cb = char_at(text, j, b.end, lower);
    if (ca.len == 0 || cb.len == 0 || ca.cp != cb.cp) return false;
    i += ca.len;
    j += cb.len;
  }
  return true;
}

// 4b. every token against its word's first token; 5a. first-token flags for the id scan.
__global__ __launch_bounds__(kThreads) void k_verify(const uint8_t* text, const Run* toks,
                                                     int64_t n_toks, const uint32_t* tok_slot,
                                                     const uint32_t* first, bool lower,
                                                     uint32_t* lead, unsigned int* status) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= n_toks) return;
  const uint32_t f = first[tok_slot[t]];
  lead[t] = (f == (uint32_t)t) ? 1u : 0u;
  if (f != (uint32_t)t && !same_word(text, toks[t], toks[f], lower)) atomicOr(status + 2, 1u);
}

// 5b. ids: the slot of a word takes the rank of its first token among first tokens.
__global__ __launch_bounds__(kThreads) void k_slot_ids(const uint32_t* lead, const uint32_t* rank,
                                                       const uint32_t* tok_slot, int64_t n_toks,
                                                       int32_t* slot_id, uint32_t* leader) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= n_toks || !lead[t]) return;
  slot_id[tok_slot[t]] = (int32_t)rank[t];
  leader[rank[t]] = (uint32_t)t;
}

__global__ __launch_bounds__(kThreads) void k_token_ids(const uint32_t* tok_slot,
                                                        const int32_t* slot_id, int64_t n_toks,
                                                        int32_t* ids) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t < n_toks) ids[t] = slot_id[tok_slot[t]];
}

__device__ __forceinline__ int utf8_len(uint32_t cp) {
  return cp < 0x80u ? 1 : cp < 0x800u ? 2 : cp < 0x10000u ? 3 : 4;
}

// 5c. UTF-8 bytes of each word (after case mapping): sizes, then the bytes.
__global__ __launch_bounds__(kThreads) void k_word_sizes(const uint8_t* text, const Run* toks,
                                                         const uint32_t* leader, int64_t V,
                                                         bool lower, uint32_t* sizes) {
  const int64_t w = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (w >= V) return;
  const Run r = toks[leader[w]];
  uint32_t n = 0;
  for (int64_t i = r.start; i < r.end;) {
    const Char c = char_at(text, i, r.end, lower);
    n += (uint32_t)utf8_len(c.cp);
    i += c.len;
  }
  sizes[w] = n;
}

__global__ __launch_bounds__(kThreads) void k_word_bytes(const uint8_t* text, const Run* toks,
                                                         const uint32_t* leader, int64_t V,
                                                         bool lower, const uint32_t* off,
                                                         uint8_t* out) {
  const int64_t w = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (w >= V) return;
  const Run r = toks[leader[w]];
  uint8_t* o = out + off[w];
  for (int64_t i = r.start; i < r.end;) {
    const Char c = char_at(text, i, r.end, lower);
    const uint32_t cp = c.cp;
    const int n = utf8_len(cp);
    if (n == 1) {
      *o++ = (uint8_t)cp;
    } else if (n == 2) {
      *o++ = (uint8_t)(0xC0u | (cp >> 6));
      *o++ = (uint8_t)(0x80u | (cp & 0x3Fu));
    } else if (n == 3) {
      *o++ = (uint8_t)(0xE0u | (cp >> 12));
      *o++ = (uint8_t)(0x80u | ((cp >> 6) & 0x3Fu));
      *o++ = (uint8_t)(0x80u | (cp & 0x3Fu));
    } else {
      *o++ = (uint8_t)(0xF0u | (cp >> 18));
      *o++ = (uint8_t)(0x80u | ((cp >> 12) & 0x3Fu));
      *o++ = (uint8_t)(0x80u | ((cp >> 6) & 0x3Fu));
      *o++ = (uint8_t)(0x80u | (cp & 0x3Fu));
    }
    i += c.len;
  }
}

// Query side: id of each query token in the corpus table (-1 when absent), checked against the
// word's UTF-8 bytes.
__global__ __launch_bounds__(kThreads) void k_lookup(const uint8_t* text, const Run* toks,
                                                     int64_t n_toks, const unsigned long long* keys,
                                                     const int32_t* slot_id, int64_t cap,
                                                     const uint32_t* word_off,
                                                     const uint8_t* words, bool lower,
                                                     int32_t* ids, uint32_t* keep) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= n_toks) return;
  const Run r = toks[t];
  int64_t s = (int64_t)(r.hash & (uint64_t)(cap - 1));
  int32_t id = -1;
  for (int64_t probe = 0; probe < cap; ++probe) {
    const unsigned long long k = keys[s];
    if (k == kEmpty) break;
    if (k == r.hash) {
      id = slot_id[s];
      break;
    }
    s = (s + 1) & (cap - 1);
  }
  if (id >= 0) {
    // compare code points with the stored word
    const int64_t w0 = word_off[id], w1 = word_off[id + 1];
    int64_t i = r.start, j = w0;
    bool same = true;
    for (uint32_t n = 0; n < r.n_cp && same; ++n) {
      const Char c = char_at(text, i, r.end, lower);
      uint32_t wc = 0;
      const int wl = (j < w1) ? decode(words, j, w1, wc) : 0;
      same = c.len > 0 && wl > 0 && c.cp == wc;
      i += c.len;
      j += wl;
    }
    if (!same || j != w1) id = -1;
  }
  ids[t] = id;
  keep[t] = id >= 0 ? 1u : 0u;
}

__global__ __launch_bounds__(kThreads) void k_compact_ids(const int32_t* ids, const uint32_t* keep,
                                                          const uint32_t* pos, const Run* toks,
                                                          int64_t n_toks, int32_t* out,
                                                          int32_t* out_doc) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t < n_toks && keep[t]) {
    out[pos[t]] = ids[t];
    out_doc[pos[t]] = toks[t].doc;
  }
}

__global__ __launch_bounds__(kThreads) void k_doc_offsets_i32(const int32_t* doc_of, int64_t n,
                                                              int64_t n_docs, int64_t* off) {
  const int64_t d = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (d > n_docs) return;
  if (d == n_docs) {
    off[d] = n;
    return;
  }
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (doc_of[mid] < d) lo = mid + 1;
    else hi = mid;
  }
  off[d] = lo;
}

static unsigned blocks_for(int64_t n) {
  return (unsigned)std::max<int64_t>(1, (n + kThreads - 1) / kThreads);
}

static unsigned doc_blocks(int64_t n_docs) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(n_docs, 65536));
}

}  // namespace tok
}  // namespace bm25

struct bm25_vocab {
  bm25::Alloc alloc;  // declared first: outlives every buffer below
  int32_t flags = 0;
  int64_t n_docs = 0;
  int64_t n_tokens = 0;
  int64_t vocab = 0;
  int64_t cap = 0;
  int64_t word_bytes_total = 0;
  bm25::DevBuf keys, slot_id;        // hash table: u64 keys, int32 id per slot
  bm25::DevBuf word_off, word_bytes; // uint32[V+1], UTF-8 of the words
  bm25::DevBuf ids, doc_tok;         // corpus: int32[n_tokens], int64[n_docs+1]
  void bind() {
    bm25::DevBuf* b[] = {&keys, &slot_id, &word_off, &word_bytes, &ids, &doc_tok};
    for (auto* x : b) x->al = &alloc;
  }
};

namespace bm25 {
namespace tok {

#define BM25_TALLOC(buf, bytes)                                                         \
  do {                                                                                  \
    hipError_t e_ = (buf).reserve(bytes);                                               \
    if (e_ != hipSuccess)                                                               \
      return set_error(BM25_E_NOMEM, "device allocation of %lld bytes failed: %s",     \
                       (long long)(bytes), hipGetErrorString(e_));                      \
  } while (0)

// Steps 1-3 on a text: the token records and their count.
static int split_text(const Alloc* al, const TextView& tv, int64_t n_bytes, hipStream_t s,
                      DevBuf& toks_out, int64_t& n_toks) {
  DevBuf mark(al), run_idx(al), tmp(al), total(al);
  {
    BM25_TALLOC(total, 16);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(kThreads), 0, s, total.as<uint32_t>(),
                       (int64_t)4, 0u);
    hipLaunchKernelGGL(k_check_offsets, dim3(blocks_for(tv.n_docs + 1)), dim3(kThreads), 0, s,
                       tv.doc_off, tv.n_docs, n_bytes, total.as<unsigned int>());
    BM25_HIP(hipGetLastError());
    unsigned int bad = 0;
    BM25_HIP(hipMemcpyAsync(&bad, total.ptr, 4, hipMemcpyDeviceToHost, s));
    BM25_HIP(hipStreamSynchronize(s));
    if (bad) return set_error(BM25_E_RANGE, "text offsets are malformed");
  }
  BM25_TALLOC(mark, (size_t)std::max<int64_t>(n_bytes, 1) * 4);
  BM25_TALLOC(run_idx, (size_t)std::max<int64_t>(n_bytes, 1) * 4);
  BM25_TALLOC(tmp, (size_t)scan_tmp_elems(std::max<int64_t>(n_bytes, 1)) * 4 + 64);
  BM25_TALLOC(total, 16);
  if (n_bytes > 0) {
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n_bytes)), dim3(kThreads), 0, s,
                       mark.as<uint32_t>(), n_bytes, 0u);
    hipLaunchKernelGGL(k_mark_runs, dim3(doc_blocks(tv.n_docs)), dim3(kThreads), 0, s, tv,
                       mark.as<uint32_t>());
    BM25_HIP(hipGetLastError());
  }
  BM25_HIP(scan_exclusive<uint32_t>(mark.as<uint32_t>(), run_idx.as<uint32_t>(), n_bytes,
                                    tmp.as<uint32_t>(), total.as<uint32_t>(), s));
  uint32_t n_runs = 0;
  BM25_HIP(hipMemcpyAsync(&n_runs, total.ptr, 4, hipMemcpyDeviceToHost, s));
  BM25_HIP(hipStreamSynchronize(s));
  DevBuf runs(al), keep(al), tok_idx(al), tmp2(al);
  BM25_TALLOC(runs, (size_t)std::max<uint32_t>(n_runs, 1) * sizeof(Run));
  BM25_TALLOC(keep, (size_t)std::max<uint32_t>(n_runs, 1) * 4);
  BM25_TALLOC(tok_idx, (size_t)std::max<uint32_t>(n_runs, 1) * 4);
  BM25_TALLOC(tmp2, (size_t)scan_tmp_elems(std::max<uint32_t>(n_runs, 1)) * 4 + 64);
  if (n_runs > 0) {
    hipLaunchKernelGGL(k_run_starts, dim3(doc_blocks(tv.n_docs)), dim3(kThreads), 0, s, tv,
                       mark.as<uint32_t>(), run_idx.as<uint32_t>(), runs.as<Run>());
    BM25_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_walk_runs, dim3(blocks_for(n_runs)), dim3(kThreads), 0, s, tv,
                       runs.as<Run>(), keep.as<uint32_t>(), (int64_t)n_runs);
    BM25_HIP(hipGetLastError());
  }
  mark.release();
  run_idx.release();
  BM25_HIP(scan_exclusive<uint32_t>(keep.as<uint32_t>(), tok_idx.as<uint32_t>(), n_runs,
                                    tmp2.as<uint32_t>(), total.as<uint32_t>(), s));
  uint32_t nt = 0;
  BM25_HIP(hipMemcpyAsync(&nt, total.ptr, 4, hipMemcpyDeviceToHost, s));
  BM25_HIP(hipStreamSynchronize(s));
  n_toks = nt;
  BM25_TALLOC(toks_out, (size_t)std::max<int64_t>(n_toks, 1) * sizeof(Run));
  if (n_runs > 0) {
    hipLaunchKernelGGL(k_compact, dim3(blocks_for(n_runs)), dim3(kThreads), 0, s,
                       runs.as<Run>(), keep.as<uint32_t>(), tok_idx.as<uint32_t>(),
                       (int64_t)n_runs, toks_out.as<Run>());
    BM25_HIP(hipGetLastError());
  }
  BM25_HIP(hipStreamSynchronize(s));  // the run buffers are released on return
  return BM25_OK;
}

static int check_text(const uint8_t* text, int64_t n_bytes, const int64_t* offsets, int64_t n) {
  if (!offsets) return set_error(BM25_E_INVAL, "offsets are NULL");
  if (n < 1 || n >= INT32_MAX) return set_error(BM25_E_INVAL, "document count out of range");
  if (n_bytes < 0 || n_bytes >= (int64_t)UINT32_MAX)
    return set_error(BM25_E_INVAL, "text size must lie in [0, 2^32 - 1)");
  if (n_bytes > 0 && !text) return set_error(BM25_E_INVAL, "text is NULL");
  return BM25_OK;
}

}  // namespace tok
}  // namespace bm25

using namespace bm25;
using namespace bm25::tok;

extern "C" int bm25_tokenize_corpus(const uint8_t* text, int64_t n_bytes, const int64_t* doc_offsets,
                                    int64_t n_docs, int32_t flags,
                                    const bm25_allocator* allocator, void* stream,
                                    bm25_vocab** out, int64_t* n_tokens, int32_t* vocab_size) {
  clear_error();
  if (!out) return set_error(BM25_E_INVAL, "out is NULL");
  *out = nullptr;
  int rc = check_text(text, n_bytes, doc_offsets, n_docs);
  if (rc != BM25_OK) return rc;
  if (flags & ~BM25_TOK_LOWERCASE) return set_error(BM25_E_INVAL, "unknown flags 0x%x", flags);
  if (allocator && (!allocator->alloc || !allocator->free))
    return set_error(BM25_E_INVAL, "allocator callbacks are NULL");
  hipStream_t s = (hipStream_t)stream;
  std::unique_ptr<bm25_vocab> v(new bm25_vocab());
  if (allocator) {
    v->alloc.fn = *allocator;
    v->alloc.custom = true;
  }
  v->alloc.stream = s;
  v->bind();
  v->flags = flags;
  v->n_docs = n_docs;
  const Alloc* al = &v->alloc;
  TextView tv{text, doc_offsets, n_docs, (flags & BM25_TOK_LOWERCASE) != 0};

  DevBuf toks(al);
  int64_t T = 0;
  rc = split_text(al, tv, n_bytes, s, toks, T);
  if (rc != BM25_OK) return rc;
  v->n_tokens = T;
  if (T > (int64_t)UINT32_MAX / 2) return set_error(BM25_E_INVAL, "too many tokens");

  BM25_TALLOC(v->doc_tok, ((size_t)n_docs + 1) * 8);
  hipLaunchKernelGGL(k_doc_offsets, dim3(blocks_for(n_docs + 1)), dim3(kThreads), 0, s,
                     toks.as<Run>(), T, n_docs, v->doc_tok.as<int64_t>());
  BM25_HIP(hipGetLastError());

  // hash table: twice the distinct words at most; start from a guess and grow if it fills
  DevBuf first(al), tok_slot(al), status(al);
  BM25_TALLOC(tok_slot, (size_t)std::max<int64_t>(T, 1) * 4);
  BM25_TALLOC(status, 16);
  int64_t cap = 1024;
  while (cap < 2 * std::min<int64_t>(std::max<int64_t>(T, 1), 1 << 22)) cap <<= 1;
  unsigned int st[4] = {0, 0, 0, 0};
  for (;;) {
    BM25_TALLOC(v->keys, (size_t)cap * 8);
    BM25_TALLOC(first, (size_t)cap * 4);
    hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(cap)), dim3(kThreads), 0, s,
                       v->keys.as<uint64_t>(), cap, (uint64_t)kEmpty);
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(cap)), dim3(kThreads), 0, s,
                       first.as<uint32_t>(), cap, 0xFFFFFFFFu);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(kThreads), 0, s, status.as<uint32_t>(),
                       (int64_t)4, 0u);
    if (T > 0)
      hipLaunchKernelGGL(k_insert, dim3(blocks_for(T)), dim3(kThreads), 0, s, toks.as<Run>(), T,
                         v->keys.as<unsigned long long>(), first.as<uint32_t>(), cap,
                         tok_slot.as<uint32_t>(), status.as<unsigned int>());
    BM25_HIP(hipGetLastError());
    BM25_HIP(hipMemcpyAsync(st, status.ptr, 16, hipMemcpyDeviceToHost, s));
    BM25_HIP(hipStreamSynchronize(s));
    if (st[1] == 0 && (int64_t)st[0] * 2 <= cap) break;  // at most half full
    if (cap >= (int64_t)1 << 32) return set_error(BM25_E_NOMEM, "vocabulary table too large");
    v->keys.release();
    first.release();
    cap = std::max<int64_t>(cap * 2, (int64_t)st[0] * 4);
    int64_t c2 = 1024;
    while (c2 < cap) c2 <<= 1;
    cap = c2;
  }
  v->cap = cap;
  const int64_t V = st[0];
  v->vocab = V;
  if (V > INT32_MAX) return set_error(BM25_E_INVAL, "vocabulary larger than 2^31 - 1 words");

  // verify against each word's first token, then ids in first-occurrence order
  DevBuf lead(al), rank(al), tmp(al), total(al), leader(al);
  BM25_TALLOC(lead, (size_t)std::max<int64_t>(T, 1) * 4);
  BM25_TALLOC(rank, (size_t)std::max<int64_t>(T, 1) * 4);
  BM25_TALLOC(tmp, (size_t)scan_tmp_elems(std::max<int64_t>(T, std::max<int64_t>(V, 1) + 1)) * 4 + 64);
  BM25_TALLOC(total, 16);
  BM25_TALLOC(leader, (size_t)std::max<int64_t>(V, 1) * 4);
  BM25_TALLOC(v->slot_id, (size_t)cap * 4);
  if (T > 0) {
    hipLaunchKernelGGL(k_verify, dim3(blocks_for(T)), dim3(kThreads), 0, s, text, toks.as<Run>(),
                       T, tok_slot.as<uint32_t>(), first.as<uint32_t>(), tv.lower,
                       lead.as<uint32_t>(), status.as<unsigned int>());
    BM25_HIP(hipGetLastError());
  }
  BM25_HIP(scan_exclusive<uint32_t>(lead.as<uint32_t>(), rank.as<uint32_t>(), T,
                                    tmp.as<uint32_t>(), total.as<uint32_t>(), s));
  BM25_TALLOC(v->ids, (size_t)std::max<int64_t>(T, 1) * 4);
  if (T > 0) {
    hipLaunchKernelGGL(k_slot_ids, dim3(blocks_for(T)), dim3(kThreads), 0, s,
                       lead.as<uint32_t>(), rank.as<uint32_t>(), tok_slot.as<uint32_t>(), T,
                       v->slot_id.as<int32_t>(), leader.as<uint32_t>());
    hipLaunchKernelGGL(k_token_ids, dim3(blocks_for(T)), dim3(kThreads), 0, s,
                       tok_slot.as<uint32_t>(), v->slot_id.as<int32_t>(), T,
                       v->ids.as<int32_t>());
    BM25_HIP(hipGetLastError());
  }
  // words as UTF-8
  DevBuf sizes(al);
  BM25_TALLOC(sizes, ((size_t)V + 1) * 4);
  BM25_TALLOC(v->word_off, ((size_t)V + 1) * 4);
  if (V > 0) {
    hipLaunchKernelGGL(k_word_sizes, dim3(blocks_for(V)), dim3(kThreads), 0, s, text,
                       toks.as<Run>(), leader.as<uint32_t>(), V, tv.lower, sizes.as<uint32_t>());
    BM25_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(kThreads), 0, s, sizes.as<uint32_t>() + V,
                     (int64_t)1, 0u);
  BM25_HIP(scan_exclusive<uint32_t>(sizes.as<uint32_t>(), v->word_off.as<uint32_t>(), V + 1,
                                    tmp.as<uint32_t>(), total.as<uint32_t>(), s));
  uint32_t wb = 0;
  BM25_HIP(hipMemcpyAsync(&wb, v->word_off.as<uint32_t>() + V, 4, hipMemcpyDeviceToHost, s));
  BM25_HIP(hipMemcpyAsync(st, status.ptr, 16, hipMemcpyDeviceToHost, s));
  BM25_HIP(hipStreamSynchronize(s));
  if (st[2] != 0)
    return set_error(BM25_E_STATE, "two distinct words share a 64-bit hash; the vocabulary is "
                     "not built");
  v->word_bytes_total = wb;
  BM25_TALLOC(v->word_bytes, (size_t)std::max<uint32_t>(wb, 1));
  if (V > 0) {
    hipLaunchKernelGGL(k_word_bytes, dim3(blocks_for(V)), dim3(kThreads), 0, s, text,
                       toks.as<Run>(), leader.as<uint32_t>(), V, tv.lower,
                       v->word_off.as<uint32_t>(), v->word_bytes.as<uint8_t>());
    BM25_HIP(hipGetLastError());
  }
  BM25_HIP(hipStreamSynchronize(s));
  if (n_tokens) *n_tokens = T;
  if (vocab_size) *vocab_size = (int32_t)V;
  v->alloc.stream = nullptr;
  *out = v.release();
  return BM25_OK;
}

extern "C" int bm25_vocab_info(const bm25_vocab* v, int64_t* n_docs, int64_t* n_tokens,
                               int32_t* vocab_size, int64_t* word_bytes, int32_t* flags) {
  clear_error();
  if (!v) return set_error(BM25_E_INVAL, "vocabulary is NULL");
  if (n_docs) *n_docs = v->n_docs;
  if (n_tokens) *n_tokens = v->n_tokens;
  if (vocab_size) *vocab_size = (int32_t)v->vocab;
  if (word_bytes) *word_bytes = v->word_bytes_total;
  if (flags) *flags = v->flags;
  return BM25_OK;
}

extern "C" int bm25_vocab_corpus(const bm25_vocab* v, int32_t* token_ids,
                                 int64_t* doc_token_offsets, void* stream) {
  clear_error();
  if (!v) return set_error(BM25_E_INVAL, "vocabulary is NULL");
  hipStream_t s = (hipStream_t)stream;
  if (token_ids && v->n_tokens > 0)
    BM25_HIP(hipMemcpyAsync(token_ids, v->ids.ptr, (size_t)v->n_tokens * 4,
                            hipMemcpyDeviceToDevice, s));
  if (doc_token_offsets)
    BM25_HIP(hipMemcpyAsync(doc_token_offsets, v->doc_tok.ptr, ((size_t)v->n_docs + 1) * 8,
                            hipMemcpyDeviceToDevice, s));
  return BM25_OK;
}

extern "C" int bm25_vocab_words(const bm25_vocab* v, uint32_t* word_offsets, uint8_t* word_bytes,
                                void* stream) {
  clear_error();
  if (!v) return set_error(BM25_E_INVAL, "vocabulary is NULL");
  hipStream_t s = (hipStream_t)stream;
  if (word_offsets)
    BM25_HIP(hipMemcpyAsync(word_offsets, v->word_off.ptr, ((size_t)v->vocab + 1) * 4,
                            hipMemcpyDeviceToDevice, s));
  if (word_bytes && v->word_bytes_total > 0)
    BM25_HIP(hipMemcpyAsync(word_bytes, v->word_bytes.ptr, (size_t)v->word_bytes_total,
                            hipMemcpyDeviceToDevice, s));
  return BM25_OK;
}

extern "C" int bm25_vocab_map(const bm25_vocab* vc, const uint8_t* text, int64_t n_bytes,
                              const int64_t* offsets, int64_t n_texts, int32_t* ids,
                              int64_t ids_capacity, int64_t* id_offsets, int64_t* n_ids,
                              void* stream) {
  clear_error();
  if (!vc || !id_offsets || !n_ids) return set_error(BM25_E_INVAL, "NULL argument");
  int rc = check_text(text, n_bytes, offsets, n_texts);
  if (rc != BM25_OK) return rc;
  bm25_vocab* v = const_cast<bm25_vocab*>(vc);
  hipStream_t s = (hipStream_t)stream;
  v->alloc.stream = s;
  const Alloc* al = &v->alloc;
  TextView tv{text, offsets, n_texts, (v->flags & BM25_TOK_LOWERCASE) != 0};
  DevBuf toks(al);
  int64_t T = 0;
  rc = split_text(al, tv, n_bytes, s, toks, T);
  if (rc != BM25_OK) return rc;
  DevBuf tid(al), keep(al), pos(al), tmp(al), total(al), doc_of(al);
  BM25_TALLOC(tid, (size_t)std::max<int64_t>(T, 1) * 4);
  BM25_TALLOC(keep, (size_t)std::max<int64_t>(T, 1) * 4);
  BM25_TALLOC(pos, (size_t)std::max<int64_t>(T, 1) * 4);
  BM25_TALLOC(tmp, (size_t)scan_tmp_elems(std::max<int64_t>(T, 1)) * 4 + 64);
  BM25_TALLOC(total, 16);
  BM25_TALLOC(doc_of, (size_t)std::max<int64_t>(T, 1) * 4);
  if (T > 0) {
    hipLaunchKernelGGL(k_lookup, dim3(blocks_for(T)), dim3(kThreads), 0, s, text,
                       toks.as<Run>(), T, v->keys.as<unsigned long long>(),
                       v->slot_id.as<int32_t>(), v->cap, v->word_off.as<uint32_t>(),
                       v->word_bytes.as<uint8_t>(), tv.lower, tid.as<int32_t>(),
                       keep.as<uint32_t>());
    BM25_HIP(hipGetLastError());
  }
  BM25_HIP(scan_exclusive<uint32_t>(keep.as<uint32_t>(), pos.as<uint32_t>(), T,
                                    tmp.as<uint32_t>(), total.as<uint32_t>(), s));
  uint32_t kept = 0;
  BM25_HIP(hipMemcpyAsync(&kept, total.ptr, 4, hipMemcpyDeviceToHost, s));
  BM25_HIP(hipStreamSynchronize(s));
  *n_ids = kept;
  if ((int64_t)kept > ids_capacity || (kept > 0 && !ids)) {
    v->alloc.stream = nullptr;
    return set_error(BM25_E_RANGE, "the texts hold %u known words; ids has room for %lld",
                     kept, (long long)ids_capacity);
  }
  if (T > 0) {
    hipLaunchKernelGGL(k_compact_ids, dim3(blocks_for(T)), dim3(kThreads), 0, s,
                       tid.as<int32_t>(), keep.as<uint32_t>(), pos.as<uint32_t>(),
                       toks.as<Run>(), T, ids, doc_of.as<int32_t>());
    BM25_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_doc_offsets_i32, dim3(blocks_for(n_texts + 1)), dim3(kThreads), 0, s,
                     doc_of.as<int32_t>(), (int64_t)kept, n_texts, id_offsets);
  BM25_HIP(hipGetLastError());
  BM25_HIP(hipStreamSynchronize(s));
  v->alloc.stream = nullptr;
  return BM25_OK;
}

extern "C" void bm25_vocab_free(bm25_vocab* v) {
  if (!v) return;
  (void)hipDeviceSynchronize();
  delete v;
}
