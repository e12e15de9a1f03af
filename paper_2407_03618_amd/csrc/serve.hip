// Continuous-batching server over a resident index.
//
// The paper spreads queries over a thread pool ("Multi-threading", Section 2). Here a scheduler
// thread turns a stream of single-query requests into micro-batches: whenever one of the
// server's device streams is idle, every waiting request that fits the in-flight slot count and
// the device-memory budget is admitted into the next micro-batch, which runs the batched search
// kernels on that stream. Several micro-batches are in flight on different streams at once, so
// requests that arrive while others are on the device start as soon as a stream frees up.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <thread>
#include <vector>

#include "internal.hpp"

namespace bm25 {

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t ticket;
  int32_t k;
  std::vector<int32_t> ids;
};

struct Done {
  uint64_t ticket;
  int32_t k;
  int32_t count;
  int64_t admit_ns;  // steady-clock time of admission into a micro-batch
  std::vector<int32_t> ids;
  std::vector<float> scores;
};

// One lane: a stream and its share of the budget, reserved at create as one device slab that
// holds the micro-batch's query ids, result rows and search arena, plus pinned host staging.
struct Lane {
  hipStream_t stream = nullptr;
  SearchScratch scratch;
  DevBuf slab;
  int32_t* q_ids = nullptr;      // [pos_cap]
  int32_t* out_ids = nullptr;    // [max_batch * max_k]
  float* out_scores = nullptr;   // [max_batch * max_k]
  int32_t* out_count = nullptr;  // [max_batch]
  PinnedBuf h_ids, h_out_ids, h_out_scores, h_out_count;
  std::vector<Request> batch;
  std::vector<int64_t> q_off;
  std::vector<int32_t> ks;
  int32_t k_max = 0;
  int64_t admit_ns = 0;
  Clock::time_point busy_since{};
  bool busy = false;
  std::atomic<bool> finished{false};
};

static int64_t kp_for(int k) {
  int64_t kp = 64;
  while (kp < k) kp *= 2;
  return kp;
}

static int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now().time_since_epoch())
      .count();
}

}  // namespace bm25

struct bm25_server {
  bm25_index* idx = nullptr;
  bm25_serve_config cfg{};
  std::mutex mu;
  std::condition_variable cv_work;
  std::condition_variable cv_done;
  std::deque<bm25::Request> waiting;
  std::deque<bm25::Done> done;
  std::vector<std::unique_ptr<bm25::Lane>> lanes;
  std::thread sched;
  bool stop = false;
  int64_t in_flight = 0;   // admitted or waiting, not yet handed to done
  uint64_t next_ticket = 1;
  int64_t submitted = 0, completed = 0, batches = 0, rejected_busy = 0, rejected_nomem = 0;
  int32_t max_batch_seen = 0;
  int32_t lanes_busy = 0, max_lanes_busy = 0;
  double lane_busy_s = 0.0;
  int64_t pos_cap = 0;     // query ids a lane holds
  size_t arena_cap = 0;    // search arena bytes of a lane
};

namespace bm25 {

// Device bytes of a lane's slab outside the search arena: query ids, result rows, counts.
static size_t lane_io_bytes(int64_t pos_cap, int32_t max_batch, int32_t max_k) {
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  return up((size_t)pos_cap * 4) + 2 * up((size_t)max_batch * max_k * 4) +
         up((size_t)max_batch * 4);
}

// Whether a micro-batch of n requests holding `positions` ids (the longest max_qlen) with lists
// for k_max fits a lane.
static bool fits_lane(const bm25_server* sv, int32_t n, int64_t positions, int32_t max_qlen,
                      int32_t k_max) {
  if (n > sv->cfg.max_batch || positions > sv->pos_cap) return false;
  std::lock_guard<std::mutex> g(sv->idx->mu);  // the launch shape reads the index's plans
  return batch_arena_bytes(sv->idx, n, positions, max_qlen, k_max) <= sv->arena_cap;
}

static void host_done(void* p) {
  Lane* lane = static_cast<Lane*>(p);
  lane->finished.store(true, std::memory_order_release);
}

// Launches the lane's micro-batch. Called by the scheduler with the server lock released.
// Every buffer was reserved at create; admission guaranteed that the batch fits them.
static int launch_lane(bm25_server* sv, Lane& ln) {
  const int32_t n = (int32_t)ln.batch.size();
  ln.q_off.assign((size_t)n + 1, 0);
  ln.ks.resize(n);
  ln.k_max = 1;
  for (int32_t i = 0; i < n; ++i) {
    ln.q_off[i + 1] = ln.q_off[i] + (int64_t)ln.batch[i].ids.size();
    ln.ks[i] = ln.batch[i].k;
    ln.k_max = std::max(ln.k_max, ln.batch[i].k);
  }
  const int64_t P = ln.q_off[n];
  if (P > sv->pos_cap || n > sv->cfg.max_batch || ln.k_max > sv->cfg.max_k)
    return set_error(BM25_E_STATE, "micro-batch exceeds the lane's reserved capacity");
  const size_t rows = (size_t)n * ln.k_max;
  int32_t* hid = ln.h_ids.as<int32_t>();
  for (int32_t i = 0; i < n; ++i)
    if (!ln.batch[i].ids.empty())
      std::memcpy(hid + ln.q_off[i], ln.batch[i].ids.data(), ln.batch[i].ids.size() * 4);
  if (P > 0)
    BM25_HIP(hipMemcpyAsync(ln.q_ids, hid, (size_t)P * 4, hipMemcpyHostToDevice, ln.stream));
  int rc;
  {
    std::lock_guard<std::mutex> g(sv->idx->mu);
    rc = search_batch_impl(sv->idx, ln.q_ids, ln.q_off.data(), n, ln.ks.data(), ln.k_max,
                           ln.out_ids, ln.out_scores, ln.out_count, ln.stream, ln.scratch,
                           nullptr);
  }
  if (rc != BM25_OK) return rc;
  BM25_HIP(hipMemcpyAsync(ln.h_out_ids.ptr, ln.out_ids, rows * 4, hipMemcpyDeviceToHost,
                          ln.stream));
  BM25_HIP(hipMemcpyAsync(ln.h_out_scores.ptr, ln.out_scores, rows * 4, hipMemcpyDeviceToHost,
                          ln.stream));
  BM25_HIP(hipMemcpyAsync(ln.h_out_count.ptr, ln.out_count, (size_t)n * 4,
                          hipMemcpyDeviceToHost, ln.stream));
  ln.finished.store(false, std::memory_order_relaxed);
  BM25_HIP(hipLaunchHostFunc(ln.stream, host_done, &ln));
  return BM25_OK;
}

static void lane_idle(bm25_server* sv, Lane& ln) {
  sv->lane_busy_s += std::chrono::duration<double>(Clock::now() - ln.busy_since).count();
  sv->lanes_busy -= 1;
  ln.batch.clear();
  ln.busy = false;
}

// Moves a finished lane's results to the done queue. Server lock held.
static void reap_lane(bm25_server* sv, Lane& ln) {
  const int32_t n = (int32_t)ln.batch.size();
  const int32_t* ids = ln.h_out_ids.as<int32_t>();
  const float* sc = ln.h_out_scores.as<float>();
  const int32_t* cnt = ln.h_out_count.as<int32_t>();
  for (int32_t i = 0; i < n; ++i) {
    Done d;
    d.ticket = ln.batch[i].ticket;
    d.k = ln.batch[i].k;
    d.count = cnt[i];
    d.admit_ns = ln.admit_ns;
    d.ids.assign(ids + (size_t)i * ln.k_max, ids + (size_t)i * ln.k_max + d.k);
    d.scores.assign(sc + (size_t)i * ln.k_max, sc + (size_t)i * ln.k_max + d.k);
    sv->done.push_back(std::move(d));
  }
  sv->completed += n;
  sv->in_flight -= n;
  lane_idle(sv, ln);
}

static void fail_lane(bm25_server* sv, Lane& ln, int code) {
  for (auto& r : ln.batch) {
    Done d;
    d.ticket = r.ticket;
    d.k = r.k;
    d.count = code;
    d.admit_ns = ln.admit_ns;
    d.ids.assign(r.k, -1);
    d.scores.assign(r.k, -INFINITY);
    sv->done.push_back(std::move(d));
  }
  sv->completed += (int64_t)ln.batch.size();
  sv->in_flight -= (int64_t)ln.batch.size();
  lane_idle(sv, ln);
}

static void scheduler(bm25_server* sv) {
  (void)hipSetDevice(sv->idx->device);
  std::unique_lock<std::mutex> lk(sv->mu);
  while (true) {
    bool progressed = false;
    for (auto& lp : sv->lanes) {
      Lane& ln = *lp;
      if (ln.busy && ln.finished.load(std::memory_order_acquire)) {
        reap_lane(sv, ln);
        progressed = true;
      }
    }
    if (progressed) sv->cv_done.notify_all();
    bool any_busy = false;
    for (auto& lp : sv->lanes) any_busy |= lp->busy;
    if (sv->stop && !any_busy) break;
    // admit waiting requests into idle lanes
    if (!sv->stop) {
      for (auto& lp : sv->lanes) {
        Lane& ln = *lp;
        if (ln.busy || sv->waiting.empty()) continue;
        // one list-size class per micro-batch (the oldest request's), so that short lists do
        // not run with the list registers of the longest k; later requests of other classes
        // keep their order for the next micro-batch. A request joins while the enlarged batch
        // still fits the lane.
        const int64_t cls = kp_for(sv->waiting.front().k);
        const size_t window = (size_t)sv->cfg.max_batch * 4;
        size_t scanned = 0;
        int64_t P = 0;
        int32_t max_qlen = 0, k_max = 1;
        auto it = sv->waiting.begin();
        while (it != sv->waiting.end() && scanned < window &&
               (int32_t)ln.batch.size() < sv->cfg.max_batch) {
          ++scanned;
          if (kp_for(it->k) != cls) {
            ++it;
            continue;
          }
          const int64_t len = (int64_t)it->ids.size();
          const int32_t ql = std::max<int32_t>(max_qlen, (int32_t)len);
          const int32_t km = std::max<int32_t>(k_max, it->k);
          if (!fits_lane(sv, (int32_t)ln.batch.size() + 1, P + len, ql, km)) break;
          P += len;
          max_qlen = ql;
          k_max = km;
          ln.batch.push_back(std::move(*it));
          it = sv->waiting.erase(it);
        }
        if (ln.batch.empty()) break;  // cannot happen: a lone request always fits (submit)
        ln.busy = true;
        ln.admit_ns = now_ns();
        ln.busy_since = Clock::now();
        sv->lanes_busy += 1;
        sv->max_lanes_busy = std::max(sv->max_lanes_busy, sv->lanes_busy);
        sv->batches += 1;
        sv->max_batch_seen = std::max<int32_t>(sv->max_batch_seen, (int32_t)ln.batch.size());
        lk.unlock();
        const int rc = launch_lane(sv, ln);
        lk.lock();
        if (rc != BM25_OK) {
          fail_lane(sv, ln, rc);
          sv->cv_done.notify_all();
        }
        progressed = true;
      }
    }
    if (!progressed) {
      any_busy = false;
      for (auto& lp : sv->lanes) any_busy |= lp->busy;
      if (any_busy)
        sv->cv_work.wait_for(lk, std::chrono::microseconds(20));
      else
        sv->cv_work.wait_for(lk, std::chrono::milliseconds(5));
    }
  }
}

}  // namespace bm25

using namespace bm25;

extern "C" int bm25_serve_create(const bm25_index* index, const bm25_serve_config* config,
                                 bm25_server** out) {
  clear_error();
  if (!index || !config || !out) return set_error(BM25_E_INVAL, "NULL argument");
  *out = nullptr;
  const bm25_serve_config c = *config;
  if (c.hbm_budget_bytes <= 0) return set_error(BM25_E_INVAL, "hbm_budget_bytes must be > 0");
  if (c.max_slots < 1 || c.max_slots > (1 << 20)) return set_error(BM25_E_INVAL, "max_slots");
  if (c.max_batch < 1 || c.max_batch > 65536) return set_error(BM25_E_INVAL, "max_batch");
  if (c.max_k < 1 || c.max_k > BM25_MAX_K) return set_error(BM25_E_INVAL, "max_k");
  if (c.n_streams < 1 || c.n_streams > 8) return set_error(BM25_E_INVAL, "n_streams");
  bm25_index* idx = const_cast<bm25_index*>(index);
  std::unique_ptr<bm25_server> sv(new bm25_server());
  sv->idx = idx;
  sv->cfg = c;
  BM25_HIP(hipSetDevice(index->device));
  // each lane's share of the budget: query ids (room for every request at the mean length the
  // share can plan, at least one longest query), result rows, and the rest as search arena
  const int64_t share = c.hbm_budget_bytes / c.n_streams;
  sv->pos_cap = std::max<int64_t>(BM25_MAX_QUERY_LEN, (int64_t)c.max_batch * 64);
  const size_t io = lane_io_bytes(sv->pos_cap, c.max_batch, c.max_k);
  if ((int64_t)io >= share)
    return set_error(BM25_E_NOMEM, "a lane's share of the budget (%lld bytes) does not hold its "
                     "result rows (%zu bytes)", (long long)share, io);
  sv->arena_cap = (size_t)share - io;
  if (!fits_lane(sv.get(), 1, BM25_MAX_QUERY_LEN, BM25_MAX_QUERY_LEN, c.max_k))
    return set_error(BM25_E_NOMEM, "a lane's share of the budget (%lld bytes) does not hold one "
                     "request of %d ids and k = %d", (long long)share, BM25_MAX_QUERY_LEN,
                     c.max_k);
  std::lock_guard<std::mutex> g(idx->mu);
  idx->alloc.stream = nullptr;
  for (int i = 0; i < c.n_streams; ++i) {
    std::unique_ptr<Lane> ln(new Lane());
    ln->slab.al = &idx->alloc;
    hipError_t e = ln->slab.reserve((size_t)share);
    if (e != hipSuccess)
      return set_error(BM25_E_NOMEM, "reserving %lld bytes for lane %d failed: %s",
                       (long long)share, i, hipGetErrorString(e));
    uint8_t* p = ln->slab.as<uint8_t>();
    auto take = [&](size_t bytes) {
      uint8_t* r = p;
      p += (bytes + 255) & ~(size_t)255;
      return r;
    };
    const size_t rows = (size_t)c.max_batch * c.max_k;
    ln->q_ids = reinterpret_cast<int32_t*>(take((size_t)sv->pos_cap * 4));
    ln->out_ids = reinterpret_cast<int32_t*>(take(rows * 4));
    ln->out_scores = reinterpret_cast<float*>(take(rows * 4));
    ln->out_count = reinterpret_cast<int32_t*>(take((size_t)c.max_batch * 4));
    ln->scratch.fixed = p;
    ln->scratch.fixed_bytes = sv->arena_cap;
    auto pin = [&](PinnedBuf& b, size_t bytes) -> int {
      hipError_t pe = b.reserve(bytes);
      return pe == hipSuccess ? BM25_OK
                              : set_error(BM25_E_NOMEM, "pinned host allocation failed: %s",
                                          hipGetErrorString(pe));
    };
    int rc;
    if ((rc = pin(ln->h_ids, (size_t)sv->pos_cap * 4))) return rc;
    if ((rc = pin(ln->h_out_ids, rows * 4))) return rc;
    if ((rc = pin(ln->h_out_scores, rows * 4))) return rc;
    if ((rc = pin(ln->h_out_count, (size_t)c.max_batch * 4))) return rc;
    if ((rc = pin(ln->scratch.host, batch_staging_bytes(c.max_batch)))) return rc;
    BM25_HIP(hipEventCreateWithFlags(&ln->scratch.host_free, hipEventDisableTiming));
    BM25_HIP(hipEventCreateWithFlags(&ln->scratch.done, hipEventDisableTiming));
    BM25_HIP(hipStreamCreateWithFlags(&ln->stream, hipStreamNonBlocking));
    sv->lanes.push_back(std::move(ln));
  }
  sv->sched = std::thread(scheduler, sv.get());
  *out = sv.release();
  return BM25_OK;
}

extern "C" int bm25_serve_submit(bm25_server* sv, const int32_t* q_ids, int32_t q_len, int32_t k,
                                 uint64_t* ticket) {
  clear_error();
  if (!sv || !ticket) return set_error(BM25_E_INVAL, "NULL argument");
  if (q_len < 0 || q_len > BM25_MAX_QUERY_LEN) return set_error(BM25_E_INVAL, "q_len");
  if (q_len > 0 && !q_ids) return set_error(BM25_E_INVAL, "q_ids is NULL");
  if (k < 1 || k > sv->cfg.max_k) return set_error(BM25_E_INVAL, "k outside [1, max_k]");
  const int32_t V = sv->idx->vocab;
  for (int32_t i = 0; i < q_len; ++i)
    if (q_ids[i] < 0 || q_ids[i] >= V)
      return set_error(BM25_E_RANGE, "token id %d outside [0, %d)", q_ids[i], V);
  if (!fits_lane(sv, 1, q_len, q_len, k)) {
    std::lock_guard<std::mutex> g(sv->mu);
    sv->rejected_nomem += 1;
    return set_error(BM25_E_NOMEM, "the request does not fit a lane's share of the budget");
  }
  Request r;
  r.k = k;
  r.ids.assign(q_ids, q_ids + q_len);
  {
    std::lock_guard<std::mutex> g(sv->mu);
    if (sv->stop) return set_error(BM25_E_STATE, "server is stopping");
    if (sv->in_flight >= sv->cfg.max_slots) {
      sv->rejected_busy += 1;
      return set_error(BM25_E_BUSY, "all slots in use");
    }
    r.ticket = sv->next_ticket++;
    *ticket = r.ticket;
    sv->waiting.push_back(std::move(r));
    sv->in_flight += 1;
    sv->submitted += 1;
  }
  sv->cv_work.notify_one();
  return BM25_OK;
}

namespace bm25 {

// bm25_serve_poll, also handing out each request's admission time when admit_ns is not null.
static int poll_impl(bm25_server* sv, uint64_t* tickets, int32_t* ids, float* scores,
                     int32_t* counts, int64_t* admit_ns, int32_t max_results, int32_t k_stride,
                     int64_t timeout_us) {
  if (!sv || !tickets || !counts || max_results < 1 || k_stride < 1)
    return set_error(BM25_E_INVAL, "bad poll arguments");
  std::unique_lock<std::mutex> lk(sv->mu);
  if (sv->done.empty() && timeout_us > 0)
    sv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us),
                         [&] { return !sv->done.empty(); });
  if (sv->done.empty()) return BM25_E_TIMEOUT;
  int32_t r = 0;
  while (r < max_results && !sv->done.empty()) {
    const Done& d = sv->done.front();
    if (d.k > k_stride) {
      if (r == 0) return set_error(BM25_E_INVAL, "k_stride %d < request k %d", k_stride, d.k);
      break;
    }
    tickets[r] = d.ticket;
    counts[r] = d.count;
    if (admit_ns) admit_ns[r] = d.admit_ns;
    if (ids) {
      int32_t* row = ids + (size_t)r * k_stride;
      std::copy(d.ids.begin(), d.ids.end(), row);
      std::fill(row + d.k, row + k_stride, -1);
    }
    if (scores) {
      float* row = scores + (size_t)r * k_stride;
      std::copy(d.scores.begin(), d.scores.end(), row);
      std::fill(row + d.k, row + k_stride, -INFINITY);
    }
    sv->done.pop_front();
    ++r;
  }
  return r;
}

}  // namespace bm25

extern "C" int bm25_serve_poll(bm25_server* sv, uint64_t* tickets, int32_t* ids, float* scores,
                               int32_t* counts, int32_t max_results, int32_t k_stride,
                               int64_t timeout_us) {
  clear_error();
  return poll_impl(sv, tickets, ids, scores, counts, nullptr, max_results, k_stride, timeout_us);
}

extern "C" int bm25_serve_stats(bm25_server* sv, bm25_serve_counters* out) {
  clear_error();
  if (!sv || !out) return set_error(BM25_E_INVAL, "NULL argument");
  std::lock_guard<std::mutex> g(sv->mu);
  bm25_serve_counters c{};
  c.submitted = sv->submitted;
  c.completed = sv->completed;
  c.batches = sv->batches;
  c.rejected_busy = sv->rejected_busy;
  c.rejected_nomem = sv->rejected_nomem;
  c.max_batch_seen = sv->max_batch_seen;
  c.waiting = (int32_t)sv->waiting.size();
  c.lanes_busy = sv->lanes_busy;
  c.max_lanes_busy = sv->max_lanes_busy;
  double busy = sv->lane_busy_s;
  const auto now = Clock::now();
  for (auto& lp : sv->lanes)
    if (lp->busy) busy += std::chrono::duration<double>(now - lp->busy_since).count();
  c.lane_busy_s = busy;
  *out = c;
  return BM25_OK;
}

extern "C" int bm25_serve_destroy(bm25_server* sv) {
  clear_error();
  if (!sv) return BM25_OK;
  {
    std::lock_guard<std::mutex> g(sv->mu);
    sv->stop = true;
    sv->in_flight -= (int64_t)sv->waiting.size();
    sv->waiting.clear();
  }
  sv->cv_work.notify_all();
  if (sv->sched.joinable()) sv->sched.join();
  for (auto& lp : sv->lanes) {
    if (lp->stream) {
      (void)hipStreamSynchronize(lp->stream);
      (void)hipStreamDestroy(lp->stream);
    }
    lp->scratch.release_handles();
  }
  {
    std::lock_guard<std::mutex> g(sv->idx->mu);
    sv->idx->alloc.stream = nullptr;
    sv->lanes.clear();  // slabs go back to the index's allocator
  }
  delete sv;
  return BM25_OK;
}

// Open-loop load generator: submits request i at start + arrival_us[i] from a native thread while
// another thread polls; lat_us[i] = completion observed - scheduled arrival (no coordinated
// omission: a late submission still counts from its scheduled time). Returns the number of
// requests that completed, or an error. Requests rejected with BM25_E_BUSY are retried until
// admitted; their wait counts in their latency.
extern "C" int bm25_serve_replay(bm25_server* sv, const int32_t* q_ids, const int64_t* q_offsets,
                                 const int32_t* k, const double* arrival_us, int32_t n,
                                 double* lat_us, double* queue_us, int32_t* out_ids,
                                 float* out_scores, int32_t* out_count, int32_t k_stride) {
  clear_error();
  if (!sv || !q_offsets || !k || !arrival_us || !lat_us || n < 0 || k_stride < 1)
    return set_error(BM25_E_INVAL, "bad replay arguments");
  std::vector<uint64_t> tick(n, 0);
  std::vector<int64_t> ticket_to_i;
  std::atomic<int> submitted{0};
  std::atomic<int> submit_rc{BM25_OK};
  const auto t0 = Clock::now();
  std::thread sub([&] {
    for (int32_t i = 0; i < n; ++i) {
      const auto at = t0 + std::chrono::nanoseconds((int64_t)(arrival_us[i] * 1000.0));
      while (Clock::now() < at) {
      }
      uint64_t t = 0;
      int rc;
      while ((rc = bm25_serve_submit(sv, q_ids + q_offsets[i],
                                     (int32_t)(q_offsets[i + 1] - q_offsets[i]), k[i], &t)) ==
             BM25_E_BUSY) {
        std::this_thread::yield();
      }
      if (rc != BM25_OK) {
        submit_rc.store(rc);
        break;
      }
      tick[i] = t;
      submitted.store(i + 1, std::memory_order_release);
    }
  });
  // tickets are issued in submission order starting from the first ticket of this replay
  int32_t got = 0;
  std::vector<uint64_t> tb(256);
  std::vector<int32_t> cb(256), ib((size_t)256 * k_stride);
  std::vector<float> sb((size_t)256 * k_stride);
  std::vector<int64_t> ab(256);
  const int64_t t0_ns = std::chrono::duration_cast<std::chrono::nanoseconds>(
                            t0.time_since_epoch()).count();
  uint64_t first_ticket = 0;
  while (got < n) {
    const int r = poll_impl(sv, tb.data(), out_ids ? ib.data() : nullptr,
                            out_scores ? sb.data() : nullptr, cb.data(), ab.data(), 256, k_stride,
                            2000);
    const auto now = Clock::now();
    if (r == BM25_E_TIMEOUT) {
      if (submit_rc.load() != BM25_OK) break;
      continue;
    }
    if (r < 0) {
      sub.join();
      return r;
    }
    if (first_ticket == 0) {
      while (submitted.load(std::memory_order_acquire) == 0) {
      }
      first_ticket = tick[0];
    }
    for (int j = 0; j < r; ++j) {
      const int64_t i = (int64_t)(tb[j] - first_ticket);
      if (i < 0 || i >= n) continue;
      const double done_us =
          std::chrono::duration<double, std::micro>(now - t0).count();
      lat_us[i] = done_us - arrival_us[i];
      if (queue_us) queue_us[i] = (double)(ab[j] - t0_ns) / 1000.0 - arrival_us[i];
      if (out_count) out_count[i] = cb[j];
      if (out_ids)
        std::copy(ib.begin() + (size_t)j * k_stride, ib.begin() + (size_t)(j + 1) * k_stride,
                  out_ids + (size_t)i * k_stride);
      if (out_scores)
        std::copy(sb.begin() + (size_t)j * k_stride, sb.begin() + (size_t)(j + 1) * k_stride,
                  out_scores + (size_t)i * k_stride);
      ++got;
    }
  }
  sub.join();
  if (submit_rc.load() != BM25_OK) return submit_rc.load();
  return got;
}
