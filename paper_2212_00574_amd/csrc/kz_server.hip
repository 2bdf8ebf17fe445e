// Serving (host code): admission by slot, arena scratch and resident bytes;
// continuous batching inside a running launch of the batched path's job
// runtime (its session mode); and a second lane for requests that do not
// suit the batched path.
//
// Session lane.  The arena starts with the runtime's device state (queue
// counters, the board of shared passes, one job state per slot); the rest is
// a first-fit heap of request scratch.  Pinned host memory holds, per slot,
// the request's descriptor, buffer table, ticket, result and done flag, and
// a ring of slot numbers with a published count.  A request is published
// (its slot written, then the ring entry, then the count) once an event
// recorded on the caller's stream after its submission has fired, so inputs
// written there before kz_server_submit are complete.  Workgroups of a
// running launch take published requests as they free up; a launch ends by
// itself once it has had nothing to do for idle_us, and the host starts one
// whenever published requests stay untaken with no launch running (or,
// behind a running one, once they have waited kRelaunchUs).  Completion is
// the slot's done flag reaching the request's ticket.
//
// Single-graph lane.  Requests with at least split_n vertices, or beyond
// the batched path's class and row-word limits, go to `workers` worker
// threads (at most kMaxWorkers): each runs them one at a time through
// kz_kernelize on a stream of its own, after waiting for an event recorded on the caller's stream at
// admission.  The runtime's tiles restage rows for every pair of blocks, a
// cost that grows with the cube of the row words, so large graphs go here.
//
// Sharing the device.  A session workgroup of 16 waves takes all of a
// compute unit's registers, so a launch of session_cus workgroups leaves
// the other units to this lane's kernels.  Each workgroup also takes no new
// request once lease_us has passed since it started, so a launch ends
// within about lease_us under load and whatever waits behind it on a shared
// hardware queue runs; the host then starts the next.  Both lanes share the
// request table and the arena heap under one mutex.
#include <string.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "kz.h"
#include "kz_internal.h"

namespace {

constexpr size_t kSrvAlign = 256;
constexpr int kSrvMaxSlots = 4096;
constexpr int kSrvMaxWorkgroups = 1024;
constexpr int kMaxWorkers = 8;     // single-graph lane: requests in flight at once (each its own context and stream)
constexpr int kDefaultWorkers = 6;
constexpr int kMaxFences = 16;     // input-ready events in flight
constexpr double kRelaunchUs = 500;  // untaken requests behind a running launch: queue another
constexpr int kSlicePasses = 2;    // single-graph lane: passes a request runs before the next one's turn
constexpr size_t kOutBytes = 256;  // its kz_out, after its workspace
static_assert(sizeof(kz_out) <= kOutBytes, "a request's kz_out fits its slot");
constexpr int kDefaultSplitN = 2048;
constexpr int kDefaultIdleUs = 20000;
constexpr int kDefaultLeaseUs = 10000;

// Session lane's share of the compute units by default: the batched
// runtime is the better path only for the smallest requests, which are a
// small part of a mixed stream's work.
int default_session_cus(int cus) { return std::max(1, cus * 3 / 16); }

size_t up(size_t x) { return (x + kSrvAlign - 1) / kSrvAlign * kSrvAlign; }

// Byte layout of the runtime's device state at the start of the arena.
struct FixedLayout {
  size_t ctl, board, jobs, total;
};
constexpr size_t kLine = 128;  // each control word on a cache line of its own

// The session's board has an entry per slot (a power of two, at least
// kBatchBoard): shared passes of jobs in different slots never hide one
// another.
int board_size(int slots) {
  int b = kzi::kBatchBoard;
  while (b < slots) b *= 2;
  return b;
}

FixedLayout fixed_layout(int slots) {
  FixedLayout L{};
  size_t o = 0;
  auto take = [&o](size_t b) {
    const size_t at = o;
    o += up(b);
    return at;
  };
  L.ctl = take(3 * kLine);  // queue, count copy, poll time
  L.board = take(sizeof(int) * (size_t)board_size(slots));
  L.jobs = take(sizeof(kzi::BatchJob) * (size_t)slots);
  L.total = o;
  return L;
}

// Byte layout of the pinned host tables.
struct HostLayout {
  size_t ring, head, graphs, ptrs, tickets, res, done, total;
};

HostLayout host_layout(int slots, int cap) {
  HostLayout L{};
  size_t o = 0;
  auto take = [&o](size_t b) {
    const size_t at = o;
    o += up(b);
    return at;
  };
  L.ring = take(sizeof(unsigned) * (size_t)cap);
  L.head = take(sizeof(unsigned long long));
  L.graphs = take(sizeof(kz_batch_graph) * (size_t)slots);
  L.ptrs = take(sizeof(kzi::BatchPtrs) * (size_t)slots);
  L.tickets = take(sizeof(unsigned long long) * (size_t)slots);
  L.res = take(sizeof(kz_result) * (size_t)slots);
  L.done = take(sizeof(unsigned long long) * (size_t)slots);
  L.total = o;
  return L;
}

// First-fit heap over [base, base + bytes) with coalescing on free.
class Heap {
 public:
  void init(size_t base, size_t bytes) {
    free_.clear();
    if (bytes) free_[base] = bytes;
  }
  bool take(size_t bytes, size_t *at) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *at = it->first;
      const size_t rest = it->second - bytes, next = it->first + bytes;
      free_.erase(it);
      if (rest) free_[next] = rest;
      return true;
    }
    return false;
  }
  void give(size_t at, size_t bytes) {
    auto it = free_.emplace(at, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;
};

struct Req {
  kz_request r;
  size_t at, bytes;  // scratch in the arena
  size_t resident;   // the caller's buffers: rows, colours, masks
  int state;         // 0 admitted, 1 published / taken by a worker, 2 done
  bool big;          // single-graph lane
  int slot;          // session lane
  int next_pass;     // single-graph lane: the next pass to run (0: not started)
  hipEvent_t ready;  // single-graph lane: inputs complete on the caller's stream
  kz_result res;
};

struct Fence {
  hipEvent_t ev;
  size_t count;  // pending requests it covers
};

using Clock = std::chrono::steady_clock;

}  // namespace

struct kz_server {
  kz_ctx *ctx;
  hipStream_t stream;   // the caller's
  hipStream_t sstream;  // session launches
  char *arena;
  size_t arena_bytes;
  int slots, cap;
  FixedLayout F;
  HostLayout H;
  char *host;      // pinned tables (host address)
  char *host_dev;  // the same, as the device sees them
  unsigned *ring;
  unsigned long long *head;
  kz_batch_graph *hgraphs;
  kzi::BatchPtrs *hptrs;
  unsigned long long *htickets;
  kz_result *hres;
  unsigned long long *hdone;
  std::vector<int> free_slots;
  std::vector<uint64_t> slot_ticket;  // published request in each slot (0: none)
  std::vector<int> running;           // slots published and not yet seen done
  Heap heap;
  std::deque<uint64_t> pending;  // session lane, admitted, not yet published (in order)
  size_t covered, ready;         // of pending (from the front): under a fence / fence fired
  std::deque<Fence> fences;
  std::vector<hipEvent_t> evpool;
  uint64_t published;
  std::deque<hipEvent_t> launches;  // session launches in flight on sstream
  bool untaken_seen;
  Clock::time_point untaken_since;
  std::unordered_map<uint64_t, Req> reqs;
  uint64_t next_ticket;
  int admitted;  // requests admitted and not yet retired by a poll
  // configuration
  int split_n, idle_us, lease_us, session_cus;
  int partition;  // 1: the lanes' streams carry complementary compute-unit masks
  int clock_khz;  // the device's constant-rate clock (wall_clock64)
  size_t resident_limit, resident;
  // single-graph lane
  int workers;                // running
  kz_ctx *wctx[kMaxWorkers];  // each worker's context (its own readback buffer)
  hipStream_t wstream[kMaxWorkers];
  std::thread worker[kMaxWorkers];
  std::mutex mu;  // everything above that both lanes touch
  std::condition_variable cv;
  std::deque<uint64_t> big;
  std::deque<uint64_t> finished;  // done, in completion order, not yet retired
  bool stop;
};

namespace {

hipEvent_t take_event(kz_server *s) {
  hipEvent_t e = nullptr;
  if (!s->evpool.empty()) {
    e = s->evpool.back();
    s->evpool.pop_back();
  } else if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
    e = nullptr;
  }
  return e;
}

void release(kz_server *s) {
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  for (std::thread &w : s->worker)
    if (w.joinable()) w.join();
  for (auto &kv : s->reqs)
    if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
  for (Fence &f : s->fences) (void)hipEventDestroy(f.ev);
  for (hipEvent_t e : s->launches) (void)hipEventDestroy(e);
  for (hipEvent_t e : s->evpool) (void)hipEventDestroy(e);
  for (int i = 0; i < kMaxWorkers; ++i) {
    if (s->wstream[i]) (void)hipStreamDestroy(s->wstream[i]);
    if (s->wctx[i]) kz_destroy(s->wctx[i]);
  }
  if (s->sstream) (void)hipStreamDestroy(s->sstream);
  if (s->host) (void)hipHostFree(s->host);
  delete s;
}

// The single-graph lane: worker `id` takes the request at the front of the
// lane's queue and runs up to kSlicePasses of its passes (the asynchronous
// call, continued from the request's own workspace); a request not yet at
// its fixpoint goes to the back of the queue, so a long cascade shares the
// workers with the requests behind it instead of holding one to its end.
void work(kz_server *s, int id) {
  kz_ctx *ctx = s->wctx[id];
  hipStream_t stream = s->wstream[id];
  (void)hipSetDevice(s->ctx->device);
  for (;;) {
    uint64_t t = 0;
    Req q{};
    {
      std::unique_lock<std::mutex> g(s->mu);
      s->cv.wait(g, [s, id] { return s->stop || id >= s->workers || !s->big.empty(); });
      if (s->stop || id >= s->workers) return;
      t = s->big.front();
      s->big.pop_front();
      Req &r = s->reqs[t];
      r.state = 1;
      q = r;
    }
    const int first = q.next_pass > 0 ? q.next_pass : 1;
    kz_out o{};
    o.result.status = KZ_EHIP;
    o.converged = 1;
    // the first slice waits for the inputs; later ones follow a slice that
    // was waited for on the host
    if (first > 1 || hipStreamWaitEvent(stream, q.ready, 0) == hipSuccess) {
      kz_graph gr{};
      gr.format = KZ_BITSET_U64;
      gr.n = q.r.n;
      gr.rows = q.r.rows;
      gr.row_words = q.r.row_words;
      kz_out *dout = (kz_out *)(s->arena + q.at + q.bytes - kOutBytes);
      const int st = kz_kernelize_async(ctx, &gr, q.r.colour, q.r.k, s->arena + q.at, q.bytes - kOutBytes,
                                        q.r.vmask, q.r.emask, first, kSlicePasses, stream, dout);
      if (st != KZ_OK) {
        o.result.status = st;
      } else if (hipMemcpyAsync(ctx->pinned, dout, sizeof(kz_out), hipMemcpyDeviceToHost, stream) == hipSuccess &&
                 hipStreamSynchronize(stream) == hipSuccess) {
        o = *(const kz_out *)ctx->pinned;
      }
    }
    std::lock_guard<std::mutex> g(s->mu);
    Req &r = s->reqs[t];
    if (!o.converged) {
      r.next_pass = first + kSlicePasses;
      s->big.push_back(t);
      s->cv.notify_one();
      continue;
    }
    r.res = o.result;
    r.state = 2;
    s->finished.push_back(t);
    (void)hipEventDestroy(r.ready);
    r.ready = nullptr;
    if (r.bytes) s->heap.give(r.at, r.bytes);
    r.bytes = 0;
    s->resident -= r.resident;
  }
}

// A lane's stream: with partition on, the session lane's on the first
// session_cus compute units (in the mask's bit order) and the other lane's
// on the rest; else a plain stream.  Masked streams are blocking streams
// (work on the legacy null stream waits for theirs), so a caller that
// partitions passes the server a stream of its own.
hipError_t make_stream(kz_server *s, bool session, hipStream_t *out) {
  const int cus = s->ctx->cus;
  if (!s->partition || s->session_cus >= cus) return hipStreamCreateWithFlags(out, hipStreamNonBlocking);
  std::vector<uint32_t> mask((size_t)(cus + 31) / 32, 0u);
  for (int c = 0; c < cus; ++c)
    if ((c < s->session_cus) == session) mask[(size_t)c / 32] |= 1u << (c % 32);
  return hipExtStreamCreateWithCUMask(out, (uint32_t)mask.size(), mask.data());
}

// Runs n workers (caller does not hold mu; no request is admitted): stops
// those beyond n, and makes contexts, streams and threads up to n.
int set_workers(kz_server *s, int n) {
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->workers = std::min(s->workers, n);
  }
  s->cv.notify_all();
  for (int i = n; i < kMaxWorkers; ++i)
    if (s->worker[i].joinable()) s->worker[i].join();
  for (int i = 0; i < n; ++i) {
    if (!s->wctx[i]) {
      if (kz_create(&s->wctx[i], s->ctx->device) != KZ_OK) return KZ_EHIP;
      s->wctx[i]->edge_path = s->ctx->edge_path;
    }
    if (!s->wstream[i] && make_stream(s, false, &s->wstream[i]) != hipSuccess) return KZ_EHIP;
  }
  std::lock_guard<std::mutex> g(s->mu);
  s->workers = n;
  for (int i = 0; i < n; ++i)
    if (!s->worker[i].joinable()) s->worker[i] = std::thread(work, s, i);
  return KZ_OK;
}

// Covers the pending requests no fence covers yet with an event on the
// caller's stream (caller holds mu).
int cover(kz_server *s) {
  if (s->pending.size() <= s->covered || (int)s->fences.size() >= kMaxFences) return KZ_OK;
  Fence f{take_event(s), s->pending.size() - s->covered};
  if (!f.ev) return KZ_EHIP;
  if (hipEventRecord(f.ev, s->stream) != hipSuccess) {
    s->evpool.push_back(f.ev);
    return KZ_EHIP;
  }
  s->fences.push_back(f);
  s->covered = s->pending.size();
  return KZ_OK;
}

// Writes request t into its slot and the ring, then bumps the count.
void publish(kz_server *s, uint64_t t) {
  Req &q = s->reqs[t];
  const int slot = q.slot;
  kz_batch_graph &g = s->hgraphs[slot];
  g.n = q.r.n;
  g.k = q.r.k;
  g.row_words = q.r.row_words;
  g.clique = q.r.clique;
  g.row_offset = 0;
  g.vertex_offset = 0;
  kzi::BatchPtrs &p = s->hptrs[slot];
  const size_t words = (size_t)q.r.n * (size_t)q.r.row_words;
  p.rows = q.r.rows;
  p.colour = q.r.colour;
  p.vmask = q.r.vmask;
  p.emask = q.r.emask;
  p.next = (uint64_t *)(s->arena + q.at);
  p.lists = (int *)(s->arena + q.at + up(words * sizeof(uint64_t)));
  p.items = (int *)(s->arena + q.at + up(words * sizeof(uint64_t)) + up(2 * words * sizeof(int)));
  s->htickets[slot] = t;
  s->hdone[slot] = 0;
  s->slot_ticket[slot] = t;
  __atomic_store_n(&s->ring[s->published % (uint64_t)s->cap], (unsigned)slot, __ATOMIC_RELEASE);
  ++s->published;
  __atomic_store_n(s->head, (unsigned long long)s->published, __ATOMIC_RELEASE);
  q.state = 1;
  s->running.push_back(slot);
}

int launch_session(kz_server *s) {
  hipEvent_t e = take_event(s);
  if (!e) return KZ_EHIP;
  kzi::BatchArgs a{};
  char *ctl = s->arena + s->F.ctl;
  a.session = 1;
  a.G = s->slots;
  a.share = s->ctx->batch_cfg.share;
  a.board = (int *)(s->arena + s->F.board);
  a.board_mask = board_size(s->slots) - 1;
  a.jobs = (kzi::BatchJob *)(s->arena + s->F.jobs);
  a.squeue = (unsigned long long *)ctl;
  a.dhead = (unsigned long long *)(ctl + kLine);
  a.hpoll = (unsigned long long *)(ctl + 2 * kLine);
  a.cap = s->cap;
  a.ring = (unsigned *)(s->host_dev + s->H.ring);
  a.head = (const unsigned long long *)(s->host_dev + s->H.head);
  a.hgraphs = (const kz_batch_graph *)(s->host_dev + s->H.graphs);
  a.hptrs = (const kzi::BatchPtrs *)(s->host_dev + s->H.ptrs);
  a.htickets = (const unsigned long long *)(s->host_dev + s->H.tickets);
  a.hres = (kz_result *)(s->host_dev + s->H.res);
  a.hdone = (unsigned long long *)(s->host_dev + s->H.done);
  a.idle_ticks = (unsigned long long)s->idle_us * (unsigned long long)s->clock_khz / 1000ull;
  a.lease_ticks = (unsigned long long)s->lease_us * (unsigned long long)s->clock_khz / 1000ull;
  kzi::BatchConfig c = s->ctx->batch_cfg;
  c.workgroups = s->session_cus * (16 / c.waves);
  if (c.workgroups > kSrvMaxWorkgroups) c.workgroups = kSrvMaxWorkgroups;
  kzi::launch_batch(a, c, s->sstream);
  if (hipGetLastError() != hipSuccess || hipEventRecord(e, s->sstream) != hipSuccess) {
    s->evpool.push_back(e);
    return KZ_EHIP;
  }
  s->launches.push_back(e);
  return KZ_OK;
}

// One step of the session lane (caller holds mu).
int step(kz_server *s) {
  // completions
  for (size_t i = 0; i < s->running.size();) {
    const int slot = s->running[i];
    const uint64_t t = s->slot_ticket[slot];
    if (__atomic_load_n(&s->hdone[slot], __ATOMIC_ACQUIRE) != t) {
      ++i;
      continue;
    }
    Req &q = s->reqs[t];
    q.res = s->hres[slot];
    q.state = 2;
    s->finished.push_back(t);
    if (q.bytes) s->heap.give(q.at, q.bytes);
    q.bytes = 0;
    s->resident -= q.resident;
    s->slot_ticket[slot] = 0;
    s->free_slots.push_back(slot);
    s->running[i] = s->running.back();
    s->running.pop_back();
  }
  // inputs ready: publish in order while the ring has room
  while (!s->fences.empty()) {
    const hipError_t e = hipEventQuery(s->fences.front().ev);
    if (e == hipErrorNotReady) break;
    if (e != hipSuccess) return KZ_EHIP;
    s->ready += s->fences.front().count;
    s->evpool.push_back(s->fences.front().ev);
    s->fences.pop_front();
  }
  while (s->ready > 0 &&
         __atomic_load_n(&s->ring[s->published % (uint64_t)s->cap], __ATOMIC_ACQUIRE) == kzi::kRingFree) {
    const uint64_t t = s->pending.front();
    s->pending.pop_front();
    --s->ready;
    --s->covered;
    publish(s, t);
  }
  int st = cover(s);
  if (st != KZ_OK) return st;
  // launches
  while (!s->launches.empty()) {
    const hipError_t e = hipEventQuery(s->launches.front());
    if (e == hipErrorNotReady) break;
    if (e != hipSuccess) return KZ_EHIP;
    s->evpool.push_back(s->launches.front());
    s->launches.pop_front();
  }
  const bool untaken =
      s->published > 0 &&
      __atomic_load_n(&s->ring[(s->published - 1) % (uint64_t)s->cap], __ATOMIC_ACQUIRE) != kzi::kRingFree;
  if (!untaken) {
    s->untaken_seen = false;
    return KZ_OK;
  }
  if (s->launches.empty()) {
    s->untaken_seen = false;
    return launch_session(s);
  }
  const Clock::time_point now = Clock::now();
  if (!s->untaken_seen) {
    s->untaken_seen = true;
    s->untaken_since = now;
  } else if (s->launches.size() < 2 &&
             std::chrono::duration<double, std::micro>(now - s->untaken_since).count() > kRelaunchUs) {
    // the running launch may be ending, or busy: queue one behind it
    s->untaken_seen = false;
    return launch_session(s);
  }
  return KZ_OK;
}

// Scratch of the session lane: next-state words, changed-tile and item lists.
size_t batch_bytes(const kz_request &r) {
  const size_t words = (size_t)r.n * (size_t)r.row_words;
  return up(words * sizeof(uint64_t)) + 2 * up(2 * words * sizeof(int));
}

// The caller's buffers of a request: rows, colours, vmask, emask.
size_t resident_bytes(const kz_request &r) {
  const size_t words = (size_t)r.n * (size_t)r.row_words;
  return 2 * words * sizeof(uint64_t) + (size_t)r.n * (sizeof(int32_t) + 1);
}

// Scratch of the single-graph lane: kz_kernelize's workspace.
int single_bytes(kz_ctx *ctx, const kz_request &r, size_t *bytes) {
  kz_graph gr{};
  gr.format = KZ_BITSET_U64;
  gr.n = r.n;
  gr.rows = r.rows;
  gr.row_words = r.row_words;
  const int st = kz_workspace_bytes(ctx, &gr, r.k, bytes);
  *bytes = up(*bytes) + kOutBytes;  // and the result the device writes after every pass
  return st;
}

bool fits_batch(const kz_request &r) {
  return r.k <= kzi::kBatchK && r.row_words <= kzi::kBatchR && r.n <= kzi::kBatchN;
}

// Lane of a valid request: true = single-graph.
bool takes_big(const kz_server *s, const kz_request &r) {
  const bool below = r.clique > 0 && r.clique < r.k;  // only the session lane takes a smaller clique size
  return !below && (r.n >= s->split_n || !fits_batch(r));
}

}  // namespace

extern "C" {

size_t kz_server_fixed_bytes(int32_t max_slots) {
  if (max_slots < 1 || max_slots > kSrvMaxSlots) return 0;
  return fixed_layout(max_slots).total;
}

size_t kz_server_request_bytes(const kz_server *s, const kz_request *req) {
  if (!s || !req || req->n < 0 || req->k < 1 || req->row_words < 0) return 0;
  if (!takes_big(s, *req)) return batch_bytes(*req);
  size_t b = 0;
  return single_bytes(s->wctx[0], *req, &b) == KZ_OK ? b : 0;
}

int kz_server_create(kz_ctx *ctx, void *arena, size_t arena_bytes, int32_t max_slots, void *stream,
                     kz_server **out) {
  if (!out) return KZ_EINVAL;
  *out = nullptr;
  if (!ctx || !arena || (uintptr_t)arena % kSrvAlign || max_slots < 1 || max_slots > kSrvMaxSlots)
    return KZ_EINVAL;
  const FixedLayout F = fixed_layout(max_slots);
  if (arena_bytes <= F.total) return KZ_EWORKSPACE;
  kz_server *s = new (std::nothrow) kz_server();
  if (!s) return KZ_ENOMEM;
  s->ctx = ctx;
  s->stream = (hipStream_t)stream;
  s->sstream = nullptr;
  s->arena = (char *)arena;
  s->arena_bytes = arena_bytes;
  s->slots = max_slots;
  s->cap = 2 * max_slots;
  s->F = F;
  s->H = host_layout(max_slots, s->cap);
  s->host = nullptr;
  s->covered = s->ready = 0;
  s->published = 0;
  s->untaken_seen = false;
  s->next_ticket = 1;
  s->admitted = 0;
  s->split_n = kDefaultSplitN;
  s->idle_us = kDefaultIdleUs;
  s->lease_us = kDefaultLeaseUs;
  s->session_cus = default_session_cus(ctx->cus);
  s->partition = 0;
  s->resident_limit = 0;
  s->resident = 0;
  s->stop = false;
  s->heap.init(F.total, arena_bytes - F.total);
  s->workers = 0;
  for (int i = 0; i < kMaxWorkers; ++i) {
    s->wctx[i] = nullptr;
    s->wstream[i] = nullptr;
  }
  if (hipSetDevice(ctx->device) != hipSuccess ||
      hipDeviceGetAttribute(&s->clock_khz, hipDeviceAttributeWallClockRate, ctx->device) != hipSuccess ||
      s->clock_khz <= 0) {
    release(s);
    return KZ_EHIP;
  }
  // host tables the device reads and writes while a launch runs: fine-grained
  if (hipHostMalloc((void **)&s->host, s->H.total, hipHostMallocCoherent) != hipSuccess) {
    s->host = nullptr;
    release(s);
    return KZ_EHIP;
  }
  if (hipHostGetDevicePointer((void **)&s->host_dev, s->host, 0) != hipSuccess) {
    release(s);
    return KZ_EHIP;
  }
  memset(s->host, 0, s->H.total);
  s->ring = (unsigned *)(s->host + s->H.ring);
  s->head = (unsigned long long *)(s->host + s->H.head);
  s->hgraphs = (kz_batch_graph *)(s->host + s->H.graphs);
  s->hptrs = (kzi::BatchPtrs *)(s->host + s->H.ptrs);
  s->htickets = (unsigned long long *)(s->host + s->H.tickets);
  s->hres = (kz_result *)(s->host + s->H.res);
  s->hdone = (unsigned long long *)(s->host + s->H.done);
  for (int i = 0; i < s->cap; ++i) s->ring[i] = kzi::kRingFree;
  s->slot_ticket.assign((size_t)max_slots, 0);
  for (int i = max_slots - 1; i >= 0; --i) s->free_slots.push_back(i);
  s->running.reserve((size_t)max_slots);
  // device state: counters zero, job states zero (first pass numbers start
  // at 1), board empty
  if (make_stream(s, true, &s->sstream) != hipSuccess ||
      hipMemsetAsync(s->arena, 0, F.total, s->sstream) != hipSuccess ||
      hipMemsetAsync(s->arena + F.board, 0xff, sizeof(int) * (size_t)board_size(max_slots), s->sstream) !=
          hipSuccess ||
      hipStreamSynchronize(s->sstream) != hipSuccess) {
    release(s);
    return KZ_EHIP;
  }
  if (set_workers(s, kDefaultWorkers) != KZ_OK) {
    release(s);
    return KZ_EHIP;
  }
  *out = s;
  return KZ_OK;
}

int kz_server_configure(kz_server *s, const kz_server_config *cfg) {
  if (!s || !cfg || cfg->split_n < 0 || cfg->idle_us < 0 || cfg->idle_us > 1000000 || cfg->lease_us < 0 ||
      cfg->lease_us > 1000000 || cfg->session_cus < 0 || cfg->session_cus > s->ctx->cus || cfg->workers < 0 ||
      cfg->workers > kMaxWorkers || cfg->partition < 0 || cfg->partition > 1 ||
      (cfg->partition && cfg->session_cus >= s->ctx->cus))
    return KZ_EINVAL;
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->admitted > 0) return KZ_EAGAIN;
  }
  // nothing is admitted, so every worker waits idle
  if (hipSetDevice(s->ctx->device) != hipSuccess) return KZ_EHIP;
  const int cus = cfg->session_cus > 0 ? cfg->session_cus : default_session_cus(s->ctx->cus);
  if (cfg->partition != s->partition || (cfg->partition && cus != s->session_cus)) {
    // new streams: wait for what the old ones run, then replace them
    for (hipEvent_t e : s->launches) (void)hipEventSynchronize(e);
    if (set_workers(s, 0) != KZ_OK || hipStreamSynchronize(s->sstream) != hipSuccess) return KZ_EHIP;
    s->partition = cfg->partition != 0;
    s->session_cus = cus;
    for (int i = 0; i < kMaxWorkers; ++i) {
      if (s->wstream[i]) (void)hipStreamDestroy(s->wstream[i]);
      s->wstream[i] = nullptr;
    }
    (void)hipStreamDestroy(s->sstream);
    s->sstream = nullptr;
    if (make_stream(s, true, &s->sstream) != hipSuccess) return KZ_EHIP;
  }
  const int st = set_workers(s, cfg->workers > 0 ? cfg->workers : kDefaultWorkers);
  if (st != KZ_OK) return st;
  std::lock_guard<std::mutex> g(s->mu);
  s->split_n = cfg->split_n > 0 ? cfg->split_n : kDefaultSplitN;
  s->idle_us = cfg->idle_us > 0 ? cfg->idle_us : kDefaultIdleUs;
  s->lease_us = cfg->lease_us > 0 ? cfg->lease_us : kDefaultLeaseUs;
  s->session_cus = cus;
  s->resident_limit = cfg->resident_limit;
  return KZ_OK;
}

int kz_server_submit(kz_server *s, const kz_request *req, uint64_t *ticket) {
  if (!s || !req || !ticket) return KZ_EINVAL;
  const kz_request &r = *req;
  if (r.n < 0 || r.k < 1 || r.row_words < 0 || (r.n > 0 && (!r.rows || !r.colour || !r.vmask || !r.emask)))
    return KZ_EINVAL;
  // the session lane's outputs must not share a 128-byte line with other data
  if ((uintptr_t)r.vmask % 128 || (uintptr_t)r.emask % 128) return KZ_EINVAL;
  if (r.clique < 0 || r.clique > r.k) return KZ_EINVAL;
  const bool below = r.clique > 0 && r.clique < r.k;
  if (below && !fits_batch(r)) return KZ_EINVAL;
  const bool big = takes_big(s, r);
  size_t bytes = batch_bytes(r);
  if (big && single_bytes(s->wctx[0], r, &bytes) != KZ_OK) return KZ_EINVAL;
  const size_t resident = resident_bytes(r);
  std::lock_guard<std::mutex> g(s->mu);
  if (s->resident_limit && resident > s->resident_limit) return KZ_EINVAL;  // could never be admitted
  if (s->admitted >= s->slots || (!big && s->free_slots.empty())) return KZ_EAGAIN;
  if (s->resident_limit && s->resident + resident > s->resident_limit) return KZ_EAGAIN;
  size_t at = 0;
  if (bytes && !s->heap.take(bytes, &at)) return KZ_EAGAIN;
  Req q{};
  q.r = r;
  q.at = at;
  q.bytes = bytes;
  q.resident = resident;
  q.state = 0;
  q.big = big;
  q.slot = -1;
  q.next_pass = 0;
  q.ready = nullptr;
  if (big && (hipEventCreateWithFlags(&q.ready, hipEventDisableTiming) != hipSuccess ||
              hipEventRecord(q.ready, s->stream) != hipSuccess)) {
    if (q.ready) (void)hipEventDestroy(q.ready);
    if (bytes) s->heap.give(at, bytes);
    return KZ_EHIP;
  }
  const uint64_t t = s->next_ticket++;
  if (!big) {
    q.slot = s->free_slots.back();
    s->free_slots.pop_back();
  }
  s->reqs.emplace(t, q);
  s->resident += resident;
  ++s->admitted;
  *ticket = t;
  if (big) {
    s->big.push_back(t);
    s->cv.notify_one();
    return KZ_OK;
  }
  s->pending.push_back(t);
  // an input-ready event right away (kz_server_progress covers the rest)
  (void)cover(s);
  return KZ_OK;
}

int kz_server_progress(kz_server *s) {
  if (!s) return KZ_EINVAL;
  if (hipSetDevice(s->ctx->device) != hipSuccess) return KZ_EHIP;
  std::lock_guard<std::mutex> g(s->mu);
  const int st = step(s);
  return st != KZ_OK ? st : s->admitted;
}

int kz_server_done(kz_server *s, uint64_t *tickets, kz_result *res, int32_t max) {
  if (!s || max < 0 || (max > 0 && !tickets)) return KZ_EINVAL;
  if (hipSetDevice(s->ctx->device) != hipSuccess) return KZ_EHIP;
  std::lock_guard<std::mutex> g(s->mu);
  const int st = step(s);
  if (st != KZ_OK) return st;
  int got = 0;
  while (got < max && !s->finished.empty()) {
    const uint64_t t = s->finished.front();
    s->finished.pop_front();
    auto it = s->reqs.find(t);
    if (it == s->reqs.end()) continue;  // retired by kz_server_poll meanwhile
    tickets[got] = t;
    if (res) res[got] = it->second.res;
    s->reqs.erase(it);
    --s->admitted;
    ++got;
  }
  return got;
}

int kz_server_poll(kz_server *s, uint64_t ticket, kz_result *res) {
  if (!s) return KZ_EINVAL;
  const int st = kz_server_progress(s);
  if (st < 0) return st;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return KZ_EINVAL;
  if (it->second.state != 2) return 0;
  if (res) *res = it->second.res;
  s->reqs.erase(it);
  --s->admitted;
  return 1;
}

void kz_server_destroy(kz_server *s) {
  if (!s) return;
  (void)hipSetDevice(s->ctx->device);
  {
    // workers finish what they hold and take nothing new; requests not yet
    // published are dropped
    std::unique_lock<std::mutex> g(s->mu);
    s->big.clear();
  }
  // session launches end once idle (published requests they took first)
  for (hipEvent_t e : s->launches) (void)hipEventSynchronize(e);
  release(s);
}

}  // extern "C"
