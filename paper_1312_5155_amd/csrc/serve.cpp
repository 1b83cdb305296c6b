// Continuous-batching serving engine: HBM-budget admission, a device output
// pool, S streams of overlapping batches, latency accounting, and a trace
// replayer that injects requests at their arrival times.
#include <hip/hip_runtime_api.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/rs_poly.h"
#include "gf.h"
#include "rs_internal.h"
#include "runtime.h"

namespace rsp {
namespace {

using Clock = std::chrono::steady_clock;

double us_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::micro>(b - a).count();
}

// Ring allocator over one device allocation, 256-byte granularity.
// Outputs are allocated in admission order and freed roughly in completion
// order, so allocation takes the space after the newest live block and a
// free advances the tail over blocks already released: O(1) amortized, with
// no free-list scans under the engine lock.
class DevicePool {
 public:
  int init(size_t bytes) {
    size_ = (bytes + 255) / 256 * 256;
    if (hipMalloc(reinterpret_cast<void **>(&base_), size_) != hipSuccess) return RS_ENOMEM;
    return RS_OK;
  }
  ~DevicePool() {
    if (base_) (void)hipFree(base_);
  }
  // Returns the offset, or SIZE_MAX if the ring has no room now; *slot
  // receives the block's bookkeeping entry, which release() takes back
  // (entries never move: the deque only grows at the back and shrinks at
  // the front, which keeps references to the other entries valid).
  size_t alloc(size_t bytes, void **slot) {
    bytes = (bytes + 255) / 256 * 256;
    if (bytes > size_) return SIZE_MAX;
    size_t off;
    if (live_.empty()) {
      head_ = tail_ = 0;
      off = 0;
    } else if (head_ >= tail_) {
      // free space: [head, size) and [0, tail)
      if (size_ - head_ >= bytes)
        off = head_;
      else if (tail_ > bytes)   // wrap; strict so head never meets tail
        off = 0;
      else
        return SIZE_MAX;
    } else {
      if (tail_ - head_ > bytes)
        off = head_;
      else
        return SIZE_MAX;
    }
    head_ = off + bytes;
    live_.push_back({off, bytes, false});
    *slot = &live_.back();
    return off;
  }
  // Marks the block of `slot` free and advances the tail over the freed
  // blocks at the front: O(1) amortized.
  void release(void *slot) {
    static_cast<Block *>(slot)->freed = true;
    while (!live_.empty() && live_.front().freed) live_.pop_front();
    if (!live_.empty()) tail_ = live_.front().off;
  }
  uint8_t *base() const { return base_; }

 private:
  struct Block {
    size_t off, bytes;
    bool freed;
  };
  uint8_t *base_ = nullptr;
  size_t size_ = 0;
  size_t head_ = 0, tail_ = 0;   // next allocation / oldest live block
  std::deque<Block> live_;       // in allocation order
};

struct Request {
  uint64_t ticket = 0;
  rs_serve_request_t req{};
  std::vector<uint8_t *> blocks;     // copy of the caller's pointer array
  std::vector<int> erasures;         // sorted
  size_t charge = 0;
  size_t out_bytes = 0;              // pool bytes of the outputs
  size_t out_off = SIZE_MAX;
  void *out_slot = nullptr;          // the pool's entry for the outputs
  int n_out = 0;
  int status = RS_OK;
  Clock::time_point submitted, launched, done;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t start = nullptr;   // timing: before the batch's first command
  hipEvent_t done = nullptr;
  rs_poly_batch_t *batch = nullptr;
  std::vector<Request *> reqs;
  bool busy = false;
};

}  // namespace
}  // namespace rsp

using namespace rsp;

struct rs_serve {
  rs_serve_config_t cfg{};
  int device = 0;
  DevicePool pool;
  std::vector<Slot> slots;

  std::mutex mu;                       // guards everything below
  std::condition_variable cv_work;     // new submissions / shutdown
  std::condition_variable cv_done;     // new completions
  std::deque<Request *> pending;       // submitted, not admitted
  std::deque<Request *> admitted;      // outputs allocated, not launched
  std::deque<Request *> completed;     // finished, not polled
  std::unordered_map<uint64_t, Request *> held;   // polled, not released
  uint64_t next_ticket = 1;
  size_t in_use = 0;
  rs_serve_stats_t stats{};
  bool stopping = false;
  int inflight = 0;
  std::thread scheduler;
  std::vector<std::thread> replayers;

  ~rs_serve();
  int validate(const rs_serve_request_t &r, Request *q);
  int enqueue(const rs_serve_request_t &r, uint64_t *ticket);
  void run();
  bool reap();
  void admit();
  bool launch();
  void finish(Request *q);
  void free_outputs(Request *q);
};

int rs_serve::validate(const rs_serve_request_t &r, Request *q) {
  if (!r.code || !r.blocks) return RS_ENULL;
  if (r.op != RS_POLY_OP_ENCODE && r.op != RS_POLY_OP_DECODE) return RS_EINVAL;
  if (r.block_bytes == 0) return RS_EINVAL;
  if (cfg.max_block_bytes && r.block_bytes > cfg.max_block_bytes) return RS_EINVAL;
  Code &c = r.code->code;
  const int k = c.k(), m = c.m(), n = c.n();
  auto aligned = [](const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  q->req = r;
  q->blocks.assign(r.blocks, r.blocks + n);
  if (r.op == RS_POLY_OP_ENCODE) {
    for (int j = 0; j < k; ++j) {
      if (!r.blocks[j]) return RS_ENULL;
      if (!aligned(r.blocks[j])) return RS_EINVAL;
    }
    q->n_out = m;
    q->charge = (size_t)(k + m) * r.block_bytes;
  } else {
    int sorted[kMaxM];
    const int rc = validate_erasures(c, r.erasures, r.n_erasures, r.flags, sorted);
    if (rc != RS_OK) return rc;
    if (r.n_erasures < 1) return RS_EINVAL;
    q->erasures.assign(sorted, sorted + r.n_erasures);
    auto plan = c.plan(sorted, r.n_erasures, r.flags);
    for (int b : plan->read) {
      if (!r.blocks[b]) return RS_ENULL;
      if (!aligned(r.blocks[b])) return RS_EINVAL;
    }
    q->n_out = r.n_erasures;
    q->charge = (size_t)(k + r.n_erasures) * r.block_bytes;
  }
  q->req.blocks = nullptr;      // the copies above are used from here on
  q->req.erasures = nullptr;
  // each output block padded to 256 bytes so every one is aligned
  q->out_bytes = (size_t)q->n_out * ((r.block_bytes + 255) / 256 * 256);
  if (q->charge > cfg.hbm_budget_bytes || q->out_bytes > cfg.hbm_budget_bytes) return RS_EINVAL;
  return RS_OK;
}

int rs_serve::enqueue(const rs_serve_request_t &r, uint64_t *ticket) {
  std::unique_ptr<Request> q(new (std::nothrow) Request);
  if (!q) return RS_ENOMEM;
  const int rc = validate(r, q.get());
  if (rc != RS_OK) return rc;
  q->submitted = Clock::now();
  {
    std::lock_guard<std::mutex> lock(mu);
    if (stopping) return RS_EBUSY;
    q->ticket = next_ticket++;
    if (ticket) *ticket = q->ticket;
    ++stats.submitted;
    pending.push_back(q.release());
  }
  cv_work.notify_one();
  return RS_OK;
}

void rs_serve::free_outputs(Request *q) {
  if (q->out_off != SIZE_MAX) pool.release(q->out_slot);
  q->out_off = SIZE_MAX;
  q->out_slot = nullptr;
  in_use -= q->charge;
}

// Completed batch slots hand their requests to the completion queue.
bool rs_serve::reap() {
  bool any = false;
  for (Slot &s : slots) {
    if (!s.busy) continue;
    const hipError_t e = hipEventQuery(s.done);
    if (e == hipErrorNotReady) continue;
    const Clock::time_point now = Clock::now();
    float dev_ms = 0;
    if (e == hipSuccess && hipEventElapsedTime(&dev_ms, s.start, s.done) != hipSuccess) dev_ms = 0;
    std::lock_guard<std::mutex> lock(mu);
    stats.batch_device_us += 1e3 * dev_ms;
    for (Request *q : s.reqs) {
      q->done = now;
      if (e != hipSuccess) q->status = RS_EDEVICE;
      ++stats.completed;
      stats.user_bytes += (uint64_t)q->req.code->code.k() * q->req.block_bytes;
      if (cfg.auto_release) free_outputs(q);
      completed.push_back(q);
    }
    s.reqs.clear();
    s.busy = false;
    --inflight;
    any = true;
  }
  if (any) cv_done.notify_all();
  return any;
}

// Admits pending requests in arrival order while budget and pool allow.
void rs_serve::admit() {
  std::lock_guard<std::mutex> lock(mu);
  while (!pending.empty()) {
    Request *q = pending.front();
    if (in_use + q->charge > cfg.hbm_budget_bytes) break;
    void *slot = nullptr;
    const size_t off = pool.alloc(q->out_bytes, &slot);
    if (off == SIZE_MAX) break;
    q->out_off = off;
    q->out_slot = slot;
    in_use += q->charge;
    stats.budget_peak = std::max(stats.budget_peak, in_use);
    pending.pop_front();
    admitted.push_back(q);
  }
}

// Launches one batch of admitted requests on a free slot.
bool rs_serve::launch() {
  Slot *slot = nullptr;
  for (Slot &s : slots)
    if (!s.busy) {
      slot = &s;
      break;
    }
  if (!slot) return false;
  std::vector<Request *> batch;
  {
    std::lock_guard<std::mutex> lock(mu);
    while (!admitted.empty() && (int)batch.size() < cfg.max_batch) {
      batch.push_back(admitted.front());
      admitted.pop_front();
    }
  }
  if (batch.empty()) return false;

  // Stripe arrays: outputs point into the pool.
  std::vector<rs_poly_stripe_t> enc, dec;
  std::vector<std::vector<uint8_t *>> ptrs(batch.size());
  for (size_t i = 0; i < batch.size(); ++i) {
    Request *q = batch[i];
    const Code &c = q->req.code->code;
    const size_t stride = (q->req.block_bytes + 255) / 256 * 256;
    uint8_t *out = pool.base() + q->out_off;
    ptrs[i] = q->blocks;
    rs_poly_stripe_t st{};
    st.code = q->req.code;
    st.block_bytes = q->req.block_bytes;
    if (q->req.op == RS_POLY_OP_ENCODE) {
      for (int p = 0; p < c.m(); ++p) ptrs[i][c.k() + p] = out + p * stride;
      st.blocks = ptrs[i].data();
      enc.push_back(st);
    } else {
      for (int r = 0; r < q->n_out; ++r) ptrs[i][q->erasures[r]] = out + r * stride;
      st.blocks = ptrs[i].data();
      st.erasures = q->erasures.data();
      st.n_erasures = q->n_out;
      st.flags = q->req.flags;
      dec.push_back(st);
    }
  }
  const Clock::time_point now = Clock::now();
  int rc = RS_OK;
  if (hipEventRecord(slot->start, slot->stream) != hipSuccess) rc = RS_EDEVICE;
  if (rc == RS_OK && !enc.empty())
    rc = rs_poly_batch_encode(slot->batch, enc.data(), (int)enc.size(), slot->stream);
  if (rc == RS_OK && !dec.empty())
    rc = rs_poly_batch_decode(slot->batch, dec.data(), (int)dec.size(), slot->stream);
  if (rc == RS_OK && hipEventRecord(slot->done, slot->stream) != hipSuccess) rc = RS_EDEVICE;
  for (Request *q : batch) {
    q->launched = now;
    if (rc != RS_OK) q->status = rc;
  }
  slot->reqs = std::move(batch);
  slot->busy = true;
  std::lock_guard<std::mutex> lock(mu);
  stats.launch_host_us += us_between(now, Clock::now());
  ++inflight;
  ++stats.batches;
  stats.peak_inflight_batches = std::max(stats.peak_inflight_batches, inflight);
  if (rc != RS_OK) {
    // Nothing of this batch ran (or its state is unknown): report it done
    // with the error once the event (if recorded) completes.
    (void)hipEventRecord(slot->done, slot->stream);
  }
  return true;
}

void rs_serve::run() {
  (void)hipSetDevice(device);
  for (;;) {
    const Clock::time_point t0 = Clock::now();
    bool progress = reap();
    admit();
    const Clock::time_point t1 = Clock::now();
    while (launch()) progress = true;
    bool all_busy = true, any_busy = false;
    for (Slot &sl : slots) {
      all_busy = all_busy && sl.busy;
      any_busy = any_busy || sl.busy;
    }
    bool work_waiting;
    {
      std::unique_lock<std::mutex> lock(mu);
      stats.admit_host_us += us_between(t0, t1);
      const bool idle = pending.empty() && admitted.empty() && inflight == 0;
      if (stopping && idle) break;
      work_waiting = !pending.empty() || !admitted.empty();
      if (!progress && !any_busy) {
        // Nothing in flight: sleep until a submission arrives.
        cv_work.wait_for(lock, std::chrono::milliseconds(5));
        continue;
      }
    }
    if (!progress && (all_busy || work_waiting)) {
      // Every slot is busy, or admission waits for budget: nothing can
      // happen before some batch finishes.  Poll every busy slot (reap()
      // queries each one's event) rather than blocking on one of them, so
      // that whichever batch finishes first is seen, and stamped, when it
      // finishes.
      std::this_thread::yield();
    } else if (!progress) {
      // Slots free, nothing queued, batches in flight: keep polling them;
      // a submission is picked up on the next pass.
      std::this_thread::yield();
    }
  }
}

rs_serve::~rs_serve() {
  for (Slot &s : slots) {
    if (s.batch) rs_poly_batch_free(s.batch);
    if (s.start) (void)hipEventDestroy(s.start);
    if (s.done) (void)hipEventDestroy(s.done);
    if (s.stream) (void)hipStreamDestroy(s.stream);
  }
  for (Request *q : pending) delete q;
  for (Request *q : admitted) delete q;
  for (Request *q : completed) delete q;
  for (auto &kv : held) delete kv.second;
}

extern "C" {

int rs_serve_create(const rs_serve_config_t *cfg, rs_serve_t **out) {
  if (!cfg || !out) return RS_ENULL;
  *out = nullptr;
  if (cfg->hbm_budget_bytes == 0 || cfg->streams < 1 || cfg->streams > 8 || cfg->max_batch < 1)
    return RS_EINVAL;
  rs_serve_t *s = new (std::nothrow) rs_serve_t;
  if (!s) return RS_ENOMEM;
  s->cfg = *cfg;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return RS_EDEVICE;
  }
  int rc = s->pool.init(cfg->hbm_budget_bytes);
  s->slots.resize(cfg->streams);
  for (Slot &sl : s->slots) {
    if (rc != RS_OK) break;
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&sl.start) != hipSuccess || hipEventCreate(&sl.done) != hipSuccess)
      rc = RS_EDEVICE;
    else
      rc = rs_poly_batch_create(&sl.batch);
    if (rc == RS_OK && cfg->max_block_bytes)
      rc = rs_poly_batch_reserve(sl.batch, cfg->max_batch, cfg->max_block_bytes);
  }
  if (rc != RS_OK) {
    delete s;
    return rc;
  }
  s->scheduler = std::thread([s] { s->run(); });
  *out = s;
  return RS_OK;
}

int rs_serve_submit(rs_serve_t *s, const rs_serve_request_t *req, uint64_t *ticket) {
  if (!s || !req) return RS_ENULL;
  return s->enqueue(*req, ticket);
}

int rs_serve_replay(rs_serve_t *s, const rs_serve_request_t *reqs, const double *arrival_us,
                    int count) {
  if (!s) return RS_ENULL;
  if (count < 0) return RS_EINVAL;
  if (count == 0) return RS_OK;
  if (!reqs || !arrival_us) return RS_ENULL;
  for (int i = 1; i < count; ++i)
    if (arrival_us[i] < arrival_us[i - 1]) return RS_EINVAL;
  // Validate up front so the trace is all-or-nothing; copies are enqueued
  // by the arrival thread.
  std::vector<std::unique_ptr<Request>> qs(count);
  for (int i = 0; i < count; ++i) {
    qs[i].reset(new (std::nothrow) Request);
    if (!qs[i]) return RS_ENOMEM;
    const int rc = s->validate(reqs[i], qs[i].get());
    if (rc != RS_OK) return rc;
  }
  std::vector<double> times(arrival_us, arrival_us + count);
  auto *moved = new std::vector<std::unique_ptr<Request>>(std::move(qs));
  std::lock_guard<std::mutex> lock(s->mu);
  if (s->stopping) {
    delete moved;
    return RS_EBUSY;
  }
  s->replayers.emplace_back([s, moved, times] {
    const Clock::time_point t0 = Clock::now();
    for (size_t i = 0; i < moved->size(); ++i) {
      const auto at = t0 + std::chrono::duration_cast<Clock::duration>(
                               std::chrono::duration<double, std::micro>(times[i]));
      // Sleep through long gaps; yield (rather than spin) through short
      // ones so the scheduler and runtime threads keep their cores.
      for (Clock::time_point now = Clock::now(); now < at; now = Clock::now()) {
        if (at - now > std::chrono::microseconds(150))
          std::this_thread::sleep_for(at - now - std::chrono::microseconds(100));
        else
          std::this_thread::yield();
      }
      Request *q = (*moved)[i].release();
      q->submitted = Clock::now();
      {
        std::lock_guard<std::mutex> l2(s->mu);
        q->ticket = s->next_ticket++;
        ++s->stats.submitted;
        s->pending.push_back(q);
      }
      s->cv_work.notify_one();
    }
    delete moved;
  });
  return RS_OK;
}

int rs_serve_poll(rs_serve_t *s, rs_serve_completion_t *out, int max, int *n_done,
                  int timeout_us) {
  if (!s || !n_done || (max > 0 && !out)) return RS_ENULL;
  *n_done = 0;
  std::unique_lock<std::mutex> lock(s->mu);
  if (s->completed.empty() && timeout_us > 0)
    s->cv_done.wait_for(lock, std::chrono::microseconds(timeout_us),
                        [s] { return !s->completed.empty(); });
  int n = 0;
  while (n < max && !s->completed.empty()) {
    Request *q = s->completed.front();
    s->completed.pop_front();
    rs_serve_completion_t &c = out[n++];
    memset(&c, 0, sizeof(c));
    c.ticket = q->ticket;
    c.user_tag = q->req.user_tag;
    c.status = q->status;
    c.n_out = q->n_out;
    c.charge_bytes = q->charge;
    c.queue_us = us_between(q->submitted, q->launched);
    c.latency_us = us_between(q->submitted, q->done);
    const Code &code = q->req.code->code;
    const size_t stride = (q->req.block_bytes + 255) / 256 * 256;
    for (int r = 0; r < q->n_out; ++r) {
      c.out_index[r] = q->req.op == RS_POLY_OP_ENCODE ? code.k() + r : q->erasures[r];
      c.out[r] = q->out_off == SIZE_MAX ? nullptr : s->pool.base() + q->out_off + r * stride;
    }
    if (s->cfg.auto_release)
      delete q;
    else
      s->held[q->ticket] = q;
  }
  *n_done = n;
  return RS_OK;
}

int rs_serve_release(rs_serve_t *s, uint64_t ticket) {
  if (!s) return RS_ENULL;
  std::lock_guard<std::mutex> lock(s->mu);
  if (s->cfg.auto_release) return RS_OK;
  auto it = s->held.find(ticket);
  if (it == s->held.end()) return RS_ERANGE;
  s->free_outputs(it->second);
  delete it->second;
  s->held.erase(it);
  s->cv_work.notify_one();
  return RS_OK;
}

int rs_serve_stats(rs_serve_t *s, rs_serve_stats_t *out) {
  if (!s || !out) return RS_ENULL;
  std::lock_guard<std::mutex> lock(s->mu);
  *out = s->stats;
  out->budget_in_use = s->in_use;
  out->pending = (int)s->pending.size();
  return RS_OK;
}

void rs_serve_destroy(rs_serve_t *s) {
  if (!s) return;
  std::vector<std::thread> reps;
  {
    std::lock_guard<std::mutex> lock(s->mu);
    reps.swap(s->replayers);
  }
  for (auto &t : reps) t.join();
  {
    std::lock_guard<std::mutex> lock(s->mu);
    s->stopping = true;
  }
  s->cv_work.notify_all();
  if (s->scheduler.joinable()) s->scheduler.join();
  delete s;
}

}  // extern "C"
