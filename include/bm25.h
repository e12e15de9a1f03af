/*
 * bm25.h -- C ABI of an MI355X (gfx950) implementation of BM25S eager sparse scoring
 * (arXiv 2407.03618).
 *
 * What the library computes (all section references are to the paper):
 *   Index time ("Eager index-time scoring", Section 2): for a corpus C of N documents given as
 *   pre-tokenized integer ids, every pair (t, D) with TF(t, D) > 0 is scored once,
 *       S(t, D) = IDF(t) * TF(t, D) / (TF(t, D) + k1 * (1 - b + b * |D| / L_avg))   (Lucene),
 *   with IDF(t) = ln((N - DF(t) + 0.5) / (DF(t) + 0.5) + 1) ("Calculation of BM25"), and stored in
 *   a token-major sparse matrix: one contiguous segment of (document id, score) per token, document
 *   ids ascending ("Efficient Matrix Sparsity"; the paper calls it CSC). Variants whose score is
 *   non-zero at TF = 0 (BM25+, BM25L, TF_ldp) store S - S_theta(t) and keep S_theta per token
 *   (Section 2.1, non-occurrence adjustment).
 *   Query time ("Assigning Query Scores"): the rows of the query's token ids are sliced and summed
 *   into one FP32 accumulator per document; every query position counts, so a repeated token is
 *   summed once per occurrence. For shifted variants sum_i S_theta(q_i) is added to the returned
 *   scores. The k best documents are returned ("Top-k selection"), ordered by score descending and,
 *   for equal scores, by document id ascending.
 *
 * Conventions:
 *   - "device" pointers are HIP device memory on the current device; "host" pointers are ordinary
 *     host memory. Every stream argument is a hipStream_t passed as void* (NULL = null stream).
 *   - The caller owns every buffer it passes. The library owns what it allocates (index arrays,
 *     scratch, server queues) and frees it in the matching *_free / *_destroy call. Device memory
 *     comes from the caller's bm25_allocator when one is given to bm25_index_build (for example
 *     PyTorch's caching allocator), else from hipMalloc.
 *   - Every int-returning call returns BM25_OK (0) on success or a negative bm25_status code; no
 *     C++ exception crosses the ABI. bm25_last_error() returns a thread-local message for the last
 *     failing call on the calling thread.
 *   - Calls on one index from several threads must be serialised by the caller, except the
 *     bm25_serve_* calls, which are thread-safe.
 */
#ifndef BM25_MI355X_H
#define BM25_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bm25_index bm25_index;   /* opaque; owns its device arrays */
typedef struct bm25_server bm25_server; /* opaque continuous-batching server */

/* Scoring variants. Lucene is printed in Section 2; the others are named in Section 2
 * ("Alternative BM25 implementations"), Section 2.1 and Table 3, with formulas from the variant
 * study the paper follows. BM25L, BM25+ and TF_ldp are stored shifted (Section 2.1). */
enum bm25_variant {
  BM25_LUCENE = 0,
  BM25_BM25L = 1,
  BM25_BM25PLUS = 2,
  BM25_ROBERTSON = 3,
  BM25_ATIRE = 4,
  BM25_TFLDP = 5
};

/* Storage type of the stored scores; accumulation is always FP32. */
enum bm25_dtype { BM25_F32 = 0, BM25_F16 = 1, BM25_BF16 = 2 };

enum bm25_status {
  BM25_OK = 0,
  BM25_E_INVAL = -1,   /* bad argument: NULL pointer, size <= 0, parameter out of range */
  BM25_E_RANGE = -2,   /* token id outside [0, vocab_size), or malformed document offsets */
  BM25_E_NOMEM = -3,   /* device or host allocation failed, or a request exceeds the budget */
  BM25_E_BUSY = -4,    /* server slot table full (bm25_serve_submit) */
  BM25_E_HIP = -5,     /* a HIP runtime call failed */
  BM25_E_STATE = -6,   /* call not valid in the object's current state */
  BM25_E_TIMEOUT = -7  /* bm25_serve_poll waited timeout_us without a completion */
};

#define BM25_MAX_K 1024            /* largest k accepted by the search calls */
#define BM25_MAX_QUERY_LEN 2048    /* most positions (token ids) in one query */

/* Scoring parameters. k1 >= 0; 0 <= b <= 1; delta >= 0 (BM25+ and BM25L), delta > 1/e (TF_ldp). */
typedef struct {
  double k1;
  double b;
  double delta;
  int32_t variant;      /* enum bm25_variant */
  int32_t store_dtype;  /* enum bm25_dtype */
} bm25_params;

/* Device memory provider. alloc returns a device pointer of at least `bytes` bytes, aligned to 256
 * bytes, usable on the current device, or NULL on failure (the library then returns
 * BM25_E_NOMEM); free releases a pointer alloc returned. `stream` is the stream of the library
 * call that allocates or frees (NULL = null stream): memory is used on that stream first, and the
 * library synchronises with its own work on a buffer before handing it to free. ctx is passed
 * through unchanged. Both callbacks may be called from the thread of any library call on the
 * index or on a server over it, never from a library thread, and never concurrently for one
 * index. */
typedef struct {
  void* (*alloc)(size_t bytes, void* stream, void* ctx);
  void (*free)(void* ptr, void* stream, void* ctx);
  void* ctx;
} bm25_allocator;

/* ---------------------------------------------------------------------------------------------
 * Index build (Section 2: "Calculation of BM25", "Eager index-time scoring",
 * "Efficient Matrix Sparsity"; Section 2.1 for shifted variants).
 *
 * token_ids   device int32[n_tokens]: the documents' token ids back to back.
 * doc_offsets device int64[n_docs + 1]: document d holds token_ids[doc_offsets[d] ..
 *             doc_offsets[d+1]); doc_offsets[0] = 0, non-decreasing, doc_offsets[n_docs] =
 *             n_tokens. |D| is the number of ids of D, repeats included. Empty documents are
 *             allowed and count in N and in L_avg.
 * vocab_size  V: every id must lie in [0, V). A token with DF = 0 contributes 0 everywhere.
 * allocator   device memory provider of the index: its arrays, the build's transient buffers
 *             and the search scratch (grown on demand) all come from it, and bm25_index_free
 *             returns them to it. NULL: hipMalloc / hipFree. The allocator struct is copied; its
 *             ctx must stay valid until the index is freed.
 * stream      the build's kernels run on it; the call is synchronous (returns after the index is
 *             complete) because the number of stored pairs sizes the index arrays.
 * out         receives a new index that stays resident in device memory until bm25_index_free.
 * Errors: BM25_E_INVAL for NULL pointers, n_docs < 1, n_tokens < 0 or >= 2^32, V < 1, a bad
 * parameter, or sum |D| = 0 (L_avg undefined); BM25_E_RANGE for an id outside [0, V) or
 * malformed offsets (checked on the device before any index array is written); BM25_E_NOMEM and
 * BM25_E_HIP as above. On error *out is left NULL and nothing is leaked.
 */
int bm25_index_build(const int32_t* token_ids, int64_t n_tokens, const int64_t* doc_offsets,
                     int64_t n_docs, int32_t vocab_size, const bm25_params* params,
                     const bm25_allocator* allocator, void* stream, bm25_index** out);

/* Sizes and corpus statistics of a built index; any output pointer may be NULL. sum_len is the
 * exact sum of |D| (int64) and l_avg = sum_len / n_docs (FP64). */
int bm25_index_info(const bm25_index* index, int64_t* n_docs, int32_t* vocab_size, int64_t* nnz,
                    int64_t* sum_len, double* l_avg, bm25_params* params);

/* Copies the index arrays into caller-owned device buffers (stream-ordered; any pointer may be
 * NULL to skip that array):
 *   indptr  int64[V+1]  token t owns entries [indptr[t], indptr[t+1])
 *   indices int32[nnz]  document ids, strictly ascending inside each token's segment
 *   tf      int32[nnz]  TF(t, D) of each entry
 *   df      int32[V]    DF(t) = indptr[t+1] - indptr[t]
 *   idf     double[V]   IDF(t) in FP64 (0 where DF = 0)
 *   theta   double[V]   S_theta(t) in FP64 (0 for sparse variants and where DF = 0)
 *   data    nnz values of the index's store_dtype (float, half or bfloat16 bits): S(t, D), or
 *           S(t, D) - S_theta(t) for shifted variants, computed in FP32 and rounded to nearest
 *           even. */
int bm25_index_export(const bm25_index* index, int64_t* indptr, int32_t* indices, int32_t* tf,
                      int32_t* df, double* idf, double* theta, void* data, void* stream);

/* Device bytes held by the index (its arrays plus search scratch currently allocated). */
int64_t bm25_index_device_bytes(const bm25_index* index);

/* Range of the stored scores (fp16 / bf16 storage keeps fewer exponent bits than the FP32 value
 * it rounds): counts, over all stored pairs, of values rounded to a subnormal of the storage
 * type, of non-zero values rounded to zero, and of finite values rounded to infinity. All three
 * are zero for FP32 storage unless the FP32 value itself is subnormal. Any pointer may be NULL. */
int bm25_index_range_stats(const bm25_index* index, int64_t* subnormal, int64_t* flushed_to_zero,
                           int64_t* overflow);

/* Frees the index and everything it allocated. NULL is a no-op. Waits for work issued by the
 * library on the index's streams. */
void bm25_index_free(bm25_index* index);

/* ---------------------------------------------------------------------------------------------
 * Search (Section 2: "Assigning Query Scores", "Top-k selection", "Multi-threading";
 * Section 2.1 for the shift).
 *
 * q_ids       device int32[q_offsets[n_queries]]: the queries' token ids back to back.
 * q_offsets   HOST int64[n_queries + 1]: query i is q_ids[q_offsets[i] .. q_offsets[i+1]);
 *             q_offsets[0] = 0, non-decreasing, each query at most BM25_MAX_QUERY_LEN ids. An
 *             empty query scores every document 0 (+ nothing), so its top-k is ids 0..k-1.
 *             The offsets are read on the host to plan the launch; the caller may reuse the
 *             buffer when the call returns.
 * k           HOST int32[n_queries] (1 <= k[i] <= k_max) or NULL for k_max everywhere.
 * k_max       1..BM25_MAX_K; the row stride of the outputs.
 * out_ids     device int32[n_queries * k_max]: row i holds query i's document ids, best first;
 *             ties in score are ordered by ascending id.
 * out_scores  device float[n_queries * k_max]: the matching B(Q, D) in FP32 (shift included).
 * out_count   device int32[n_queries]: min(k[i], N), or BM25_E_RANGE for a query holding an id
 *             outside [0, V) (its row is then all -1 / -inf). Slots past the count hold id -1
 *             and score -inf.
 * stream      all work is stream-ordered on it; the call returns once the work is enqueued.
 *             Outputs must not be read before the stream reaches that point.
 * Errors (returned synchronously, nothing enqueued): BM25_E_INVAL for NULL pointers,
 * n_queries < 0, k out of range, malformed q_offsets or a query longer than the limit.
 *
 * bm25_search_batch runs the batched form: queries are grouped into tiles that share posting
 * reads, accumulated in LDS-resident FP32 tiles and reduced to per-(query, document range)
 * top-k lists inside one gather kernel per batch (launch shape from the autotuner or
 * bm25_search_set_plan), then merged per query. With graph mode on (bm25_search_set_graphs) the
 * batch's launches after the plan upload run as one HIP graph launch.
 * bm25_search_plain runs the per-query form: each query is one launch that sweeps all
 * documents for that query alone (about 2048 one-wave workgroups, each over a contiguous range
 * of whole 1024-document blocks); one small merge launch per up to 256 queries then ranks each
 * query's candidate lists.
 */
int bm25_search_batch(const bm25_index* index, const int32_t* q_ids, const int64_t* q_offsets,
                      int32_t n_queries, const int32_t* k, int32_t k_max, int32_t* out_ids,
                      float* out_scores, int32_t* out_count, void* stream);

int bm25_search_plain(const bm25_index* index, const int32_t* q_ids, const int64_t* q_offsets,
                      int32_t n_queries, const int32_t* k, int32_t k_max, int32_t* out_ids,
                      float* out_scores, int32_t* out_count, void* stream);

/* bm25_search_batch without any allocation, for callers that cannot allocate: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation. Same arguments, results
 * and errors as bm25_search_batch (eager launches only: graph mode and kernel timing do not
 * apply). Its scratch is a fixed device array of BM25_NOALLOC_SCRATCH_BYTES bytes inside the
 * library (one per device, held until the process ends) and its host plan a fixed host array of
 * room for BM25_NOALLOC_MAX_QUERIES queries; nothing is allocated through hipMalloc, the index's
 * allocator or the host heap. A batch whose scratch does not fit (more queries, longer queries
 * or larger k than the array holds; about 4096 queries of 30 ids at k = 100 fit) or that holds
 * more than BM25_NOALLOC_MAX_QUERIES queries is refused with BM25_E_NOMEM before any device
 * work. The index must live on the current device (else BM25_E_INVAL). Every call on one device
 * shares that device's arrays and leaves its contents behind: calls that overlap on one device
 * (several threads, or several streams whose work overlaps) race, so the caller serialises them
 * (stream order on one stream does). */
#define BM25_NOALLOC_SCRATCH_BYTES (64 << 20)
#define BM25_NOALLOC_MAX_QUERIES 65536
int bm25_search_batch_noalloc(const bm25_index* index, const int32_t* q_ids,
                              const int64_t* q_offsets, int32_t n_queries, const int32_t* k,
                              int32_t k_max, int32_t* out_ids, float* out_scores,
                              int32_t* out_count, void* stream);

/* Launch shape of the batched form. Zero fields mean "choose automatically".
 *   q_tile      queries sharing one workgroup's accumulators (1..64)
 *   waves       wavefronts per workgroup (1..16)
 *   doc_tile    documents per LDS accumulator tile (multiple of 256)
 *   doc_groups  document ranges the corpus is split into; a workgroup owns one (tile, range)
 *   query_order 0: automatic (grouped when the index has dense rows and q_tile times the
 *               longest query fits one tile's position capacity of 4080); 1: grouped, under
 *               the same conditions; 2: as given. Grouped: the batch is permuted on the
 *               device so that queries holding the same frequent tokens share query tiles;
 *               results are still written in the caller's order
 *   sparse_only 1: read every token from the sparse rows, ignoring the dense copies of the most
 *               frequent tokens' rows (same results within rounding; for testing)
 * Built shapes: waves 8 with doc_tile 1024 (2 documents per lane) or 2048 (4 per lane), waves 4
 * with doc_tile 1024 (4 per lane). q_tile is waves times 1, 2 or 4 queries per wave; with L list
 * registers per query (k_max / 64 rounded up to a power of two): 1 query per wave for any L,
 * 2 for L <= 4, 4 for L <= 2 with waves * documents per lane <= 16. Plans outside these are
 * rejected; a fixed plan whose q_tile is too large for a batch's k_max is narrowed. */
typedef struct {
  int32_t q_tile;
  int32_t waves;
  int32_t doc_tile;
  int32_t doc_groups;
  int32_t query_order;
  int32_t sparse_only;
} bm25_tile_plan;

/* Fixes the batched form's launch shape for this index (NULL restores automatic choice).
 * BM25_E_INVAL if a field is out of range or the shape does not fit in LDS. */
int bm25_search_set_plan(bm25_index* index, const bm25_tile_plan* plan);

/* Reads the plan the batched form would use for a batch of the given shape. */
int bm25_search_get_plan(const bm25_index* index, int32_t n_queries, int32_t max_query_len,
                         int32_t k_max, bm25_tile_plan* plan);

/* Graph mode for the batched form (Section 2, "Multi-threading": many queries per submission,
 * carried to one device submission per batch). enable != 0: every later bm25_search_batch on
 * this index, and every micro-batch of a server over it, records its launches (grouping,
 * planner, gather, merge; kernels only, no memset or copy nodes) into a HIP graph on a private
 * capture stream and launches that graph on the caller's stream as one submission. The plan
 * upload stays an ordinary copy on the caller's stream ahead of the graph. The executable graph
 * is kept per scratch area and updated in place when the next batch has the same launch
 * topology (arguments and grid sizes may change), else instantiated anew. Results are those of
 * the eager path. With kernel timing enabled, the timing events bracket the whole graph.
 * enable == 0 (the default) returns to eager launches. BM25_E_INVAL for a NULL index. */
int bm25_search_set_graphs(bm25_index* index, int32_t enable);

/* Graph-mode counters of bm25_search_batch on this index: graph instantiations (*builds) and
 * in-place updates (*updates) since the index was built. BM25_E_INVAL for NULL arguments. */
int bm25_search_graph_stats(const bm25_index* index, int64_t* builds, int64_t* updates);

/* Autotuner: times candidate launch shapes of the batched form on the given batch (same
 * arguments as bm25_search_batch; results are written to the outputs by every candidate), keeps
 * the fastest for batches of this shape class, and returns it in *best. Synchronous. */
int bm25_autotune(bm25_index* index, const int32_t* q_ids, const int64_t* q_offsets,
                  int32_t n_queries, const int32_t* k, int32_t k_max, int32_t* out_ids,
                  float* out_scores, int32_t* out_count, void* stream, bm25_tile_plan* best);

/* Kernel timing for profiling: when enabled, the library brackets each launch of its main
 * gather kernel with HIP events on the launch stream; bm25_kernel_time_read synchronises,
 * returns the summed kernel milliseconds and launch count since the last reset, and resets. */
int bm25_kernel_timing(bm25_index* index, int32_t enable);
int bm25_kernel_time_read(bm25_index* index, double* total_ms, int64_t* launches);

/* ---------------------------------------------------------------------------------------------
 * Serving: continuous batching (Section 2, "Multi-threading", carried to a GPU request loop).
 *
 * The server keeps the index resident and runs a scheduler thread. Submitted queries wait in a
 * host queue; whenever one of the n_streams lanes is idle, the scheduler admits the waiting
 * requests that fit the lane into the next micro-batch and launches it on the lane's stream, so
 * micro-batches overlap on the device while later requests keep arriving. A micro-batch holds
 * one list-size class (k rounded up to a power of two, at least 64): the oldest waiting
 * request's, with the waiting requests of that class behind it.
 *
 * Memory: bm25_serve_create reserves the whole device budget at once, through the index's
 * allocator, split evenly over the lanes; each lane's share holds its micro-batch's query ids,
 * result rows and search scratch (planner tables, accumulator candidate lists). A request joins
 * a micro-batch only while the scratch of the enlarged batch, computed for the launch shape the
 * batch will run with, fits the lane's share, so nothing is allocated on the device after
 * create. Pinned host staging is reserved at create too. Results are copied to pinned host
 * memory and handed out by bm25_serve_poll.
 *
 * config: hbm_budget_bytes  device bytes reserved for the lanes (> 0); a lane's share must hold
 *                           at least one request of the longest query and the largest k
 *         max_slots         requests in flight (queued + on the device), 1..1<<20
 *         max_batch         most requests in one micro-batch, 1..65536
 *         max_k             largest k a request may ask for, 1..BM25_MAX_K
 *         n_streams         lanes: concurrent micro-batches on the device, 1..8
 * BM25_E_NOMEM if the budget cannot be reserved or a lane's share is too small.
 */
typedef struct {
  int64_t hbm_budget_bytes;
  int32_t max_slots;
  int32_t max_batch;
  int32_t max_k;
  int32_t n_streams;
} bm25_serve_config;

int bm25_serve_create(const bm25_index* index, const bm25_serve_config* config,
                      bm25_server** out);

/* Copies the query (host int32[q_len], 0 <= q_len <= BM25_MAX_QUERY_LEN) and returns at once with
 * a ticket. BM25_E_RANGE for an id outside [0, V); BM25_E_INVAL for k outside 1..max_k;
 * BM25_E_BUSY if max_slots requests are in flight; BM25_E_NOMEM if the request alone does not fit
 * a lane's share of the budget. */
int bm25_serve_submit(bm25_server* server, const int32_t* q_ids, int32_t q_len, int32_t k,
                      uint64_t* ticket);

/* Hands out up to max_results completed requests (host buffers): tickets[r], counts[r] =
 * min(k, N), ids/scores rows of stride k_stride (>= the request's k; padded with -1 / -inf).
 * Waits up to timeout_us for the first completion (0 = do not wait). Returns the number handed
 * out (>= 0), BM25_E_TIMEOUT if none completed in time, or another error. */
int bm25_serve_poll(bm25_server* server, uint64_t* tickets, int32_t* ids, float* scores,
                    int32_t* counts, int32_t max_results, int32_t k_stride, int64_t timeout_us);

/* Server counters since create. lane_busy_s sums, over lanes, the seconds each lane held a
 * micro-batch (from launch to the reaping of its results); divided by the wall time it is the
 * mean number of lanes in use. */
typedef struct {
  int64_t submitted;        /* requests accepted by bm25_serve_submit */
  int64_t completed;        /* requests handed to the done queue */
  int64_t batches;          /* micro-batches launched */
  int64_t rejected_busy;    /* submits refused with BM25_E_BUSY (slot table full) */
  int64_t rejected_nomem;   /* submits refused with BM25_E_NOMEM (request larger than a lane) */
  int32_t max_batch_seen;   /* largest micro-batch */
  int32_t waiting;          /* requests waiting for admission now */
  int32_t lanes_busy;       /* lanes holding a micro-batch now */
  int32_t max_lanes_busy;   /* most lanes busy at once */
  double lane_busy_s;
} bm25_serve_counters;

int bm25_serve_stats(bm25_server* server, bm25_serve_counters* out);

/* Open-loop load generator for latency measurement: a native thread submits request i (host
 * ids q_ids[q_offsets[i] .. q_offsets[i+1]), k[i]) at arrival_us[i] microseconds after the call
 * starts, while the calling thread polls. lat_us[i] receives completion time minus scheduled
 * arrival time (a request that waits for a free slot is charged from its scheduled arrival);
 * queue_us[i] (optional) the part of it spent before admission into a micro-batch, so that
 * lat_us[i] - queue_us[i] is the request's service time (device work, copies and hand-out).
 * Optional result rows (stride k_stride) and counts are stored per request. Tickets of this
 * replay must be consecutive: no other thread may submit to the server meanwhile. Returns the
 * number of completed requests or an error. */
int bm25_serve_replay(bm25_server* server, const int32_t* q_ids, const int64_t* q_offsets,
                      const int32_t* k, const double* arrival_us, int32_t n, double* lat_us,
                      double* queue_us, int32_t* out_ids, float* out_scores, int32_t* out_count,
                      int32_t k_stride);

/* Stops the scheduler after the in-flight work drains and frees the server. Results not yet
 * polled are dropped. NULL is a no-op returning BM25_OK. */
int bm25_serve_destroy(bm25_server* server);

/* ---------------------------------------------------------------------------------------------
 * Tokenization and vocabulary mapping (Section 2, "Tokenization"): the step in front of the index
 * build, for callers that hold text rather than token ids.
 *
 * A document is UTF-8 text. Its words are the matches of the pattern (?u)\b\w\w+\b: maximal runs
 * of at least two word characters, where a word character is one that Python's \w matches
 * (str.isalnum() or "_"), over the whole code space of the Unicode version the library was built
 * with. Bytes that do not form valid UTF-8 (stray continuation bytes, invalid or truncated
 * sequences, overlong forms, surrogates, code points above U+10FFFF) separate words. With
 * BM25_TOK_LOWERCASE each code point first takes its lowercase form as Python's str.lower()
 * gives it (U+0130 becomes "i" followed by U+0307, which ends the word). A dictionary maps each
 * distinct word to an id, in order of first occurrence in the corpus (documents in order, words in
 * order inside a document). Stemming and stopword removal are not applied.
 */
typedef struct bm25_vocab bm25_vocab;  /* opaque: the dictionary and the tokenized corpus */
#define BM25_TOK_LOWERCASE 1

/* Tokenizes a corpus and builds its dictionary. Synchronous.
 * text        device uint8[n_bytes], the documents back to back (n_bytes < 2^32 - 1)
 * doc_offsets device int64[n_docs + 1]: document d is text[doc_offsets[d] .. doc_offsets[d+1]);
 *             doc_offsets[0] = 0, non-decreasing, doc_offsets[n_docs] = n_bytes
 * flags       0 or BM25_TOK_LOWERCASE
 * allocator   device memory provider (NULL: hipMalloc), as for bm25_index_build
 * out         receives the vocabulary; *n_tokens and *vocab_size (either may be NULL) receive
 *             the corpus's word count and the number of distinct words.
 * Errors: BM25_E_INVAL for NULL pointers, sizes out of range or unknown flags; BM25_E_RANGE for
 * malformed offsets; BM25_E_STATE if two distinct words share a 64-bit hash (detected by comparing
 * every word with its dictionary entry; nothing is built); BM25_E_NOMEM, BM25_E_HIP. */
int bm25_tokenize_corpus(const uint8_t* text, int64_t n_bytes, const int64_t* doc_offsets,
                         int64_t n_docs, int32_t flags, const bm25_allocator* allocator,
                         void* stream, bm25_vocab** out, int64_t* n_tokens, int32_t* vocab_size);

/* Sizes of a vocabulary: documents, corpus words, distinct words, bytes of the words' UTF-8 and
 * the flags it was built with. Any pointer may be NULL. */
int bm25_vocab_info(const bm25_vocab* vocab, int64_t* n_docs, int64_t* n_tokens,
                    int32_t* vocab_size, int64_t* word_bytes, int32_t* flags);

/* Copies the tokenized corpus, ready for bm25_index_build with vocab_size as V: token_ids
 * (device int32[n_tokens]) and doc_token_offsets (device int64[n_docs + 1]). Stream-ordered;
 * either pointer may be NULL. */
int bm25_vocab_corpus(const bm25_vocab* vocab, int32_t* token_ids, int64_t* doc_token_offsets,
                      void* stream);

/* Copies the words: word_offsets (device uint32[vocab_size + 1]) and word_bytes (device
 * uint8[word_bytes]): word i is word_bytes[word_offsets[i] .. word_offsets[i+1]) in UTF-8, after
 * lowercasing when the vocabulary was built with it. Stream-ordered; either pointer may be NULL. */
int bm25_vocab_words(const bm25_vocab* vocab, uint32_t* word_offsets, uint8_t* word_bytes,
                     void* stream);

/* Maps texts (queries) to ids of the vocabulary with the same splitting and case rule; words not
 * in the vocabulary are dropped. Synchronous.
 * text, offsets  as for bm25_tokenize_corpus (n_texts texts)
 * ids            device int32[ids_capacity]: the ids, text after text
 * id_offsets     device int64[n_texts + 1]: text i holds ids[id_offsets[i] .. id_offsets[i+1])
 * n_ids          host: receives the number of ids, also when ids is too small, in which case
 *                BM25_E_RANGE is returned and nothing is written to ids. */
int bm25_vocab_map(const bm25_vocab* vocab, const uint8_t* text, int64_t n_bytes,
                   const int64_t* offsets, int64_t n_texts, int32_t* ids, int64_t ids_capacity,
                   int64_t* id_offsets, int64_t* n_ids, void* stream);

/* Frees the vocabulary. NULL is a no-op. */
void bm25_vocab_free(bm25_vocab* vocab);

/* ---------------------------------------------------------------------------------------------
 * Utilities. */

/* Plain device-to-device copy kernel of n bytes (both pointers 16-byte aligned), stream-ordered.
 * Used to calibrate hardware byte counters against a kernel with known traffic. */
int bm25_copy_bytes(void* dst, const void* src, int64_t n_bytes, void* stream);

/* Thread-local message of the last failing call on this thread ("" if none). */
const char* bm25_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BM25_MI355X_H */
