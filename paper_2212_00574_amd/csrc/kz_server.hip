// Serving (host code): admission by slot and arena scratch, continuous
// batching at launch granularity on top of the batched path's job runtime,
// and a second lane for large requests.
//
// The arena starts with two launch records (descriptors, pointer tables,
// job states, results, queue counters), each able to carry max_slots
// requests; the rest is a first-fit heap of request scratch.  A launch takes
// the waiting requests in arrival order, fills a free record's pinned host
// tables, copies them to the device, runs the batched kernels and copies
// the results back, all on the server's stream, and records an event;
// kz_server_progress retires launches whose event has fired.
//
// Requests with at least kSplitN vertices (or beyond the batched path's
// class and row-word limits) go to kWorkers worker threads instead: each
// runs them one at a time through the single-graph path (kz_kernelize,
// whose multi-workgroup passes suit large graphs) on a stream of its own,
// after waiting for an event recorded on the server's stream when the
// request was admitted (so inputs written there first are complete).  Both
// lanes overlap on the device.  The two threads share the request table and
// the arena heap under one mutex.
#include <string.h>

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
constexpr int kSplitN = 4096;  // vertices from which a request takes the single-graph lane
constexpr int kWorkers = 2;    // large requests in flight at once (each its own context and stream)

size_t up(size_t x) { return (x + kSrvAlign - 1) / kSrvAlign * kSrvAlign; }

// Byte layout of one launch record in the arena.
struct RecLayout {
  size_t graphs, ptrs, order, counters, board, jobs, results, total;
};

RecLayout rec_layout(int slots) {
  RecLayout L{};
  size_t o = 0;
  auto take = [&o](size_t b) {
    const size_t at = o;
    o += up(b);
    return at;
  };
  L.graphs = take(sizeof(kz_batch_graph) * (size_t)slots);
  L.ptrs = take(sizeof(kzi::BatchPtrs) * (size_t)slots);
  L.order = take(sizeof(int) * (size_t)slots);
  L.counters = take(2 * sizeof(int));
  L.board = take(sizeof(int) * kzi::kBatchBoard);
  L.jobs = take(sizeof(kzi::BatchJob) * (size_t)slots);
  L.results = take(sizeof(kz_result) * (size_t)slots);
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
  int state;         // 0 waiting, 1 launched, 2 done
  bool big;          // single-graph lane
  hipEvent_t ready;  // big: inputs complete on the server's stream
  kz_result res;
};

struct Record {
  char *dev;                    // in the arena
  kz_batch_graph *graphs_host;  // pinned
  kzi::BatchPtrs *ptrs_host;    // pinned
  kz_result *results_host;      // pinned
  hipEvent_t done;
  bool busy;
  std::vector<uint64_t> tickets;
};

}  // namespace

struct kz_server {
  kz_ctx *ctx;
  hipStream_t stream;
  char *arena;
  size_t arena_bytes;
  int slots;
  RecLayout L;
  Record rec[2];
  Heap heap;
  std::deque<uint64_t> waiting;
  std::unordered_map<uint64_t, Req> reqs;
  uint64_t next_ticket;
  int admitted;  // requests admitted and not yet retired by a poll
  // single-graph lane
  kz_ctx *wctx[kWorkers];  // each worker's context (its own readback buffer)
  hipStream_t wstream[kWorkers];
  std::thread worker[kWorkers];
  std::mutex mu;  // reqs, heap, big, stop, admitted
  std::condition_variable cv;
  std::deque<uint64_t> big;
  bool stop;
};

namespace {

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
  for (int i = 0; i < kWorkers; ++i) {
    if (s->wstream[i]) (void)hipStreamDestroy(s->wstream[i]);
    if (s->wctx[i]) kz_destroy(s->wctx[i]);
  }
  for (Record &r : s->rec) {
    if (r.done) (void)hipEventDestroy(r.done);
    if (r.graphs_host) (void)hipHostFree(r.graphs_host);
    if (r.ptrs_host) (void)hipHostFree(r.ptrs_host);
    if (r.results_host) (void)hipHostFree(r.results_host);
  }
  delete s;
}

// The single-graph lane: worker `id` runs one large request at a time.
void work(kz_server *s, int id) {
  kz_ctx *ctx = s->wctx[id];
  hipStream_t stream = s->wstream[id];
  (void)hipSetDevice(s->ctx->device);
  for (;;) {
    uint64_t t = 0;
    Req q{};
    {
      std::unique_lock<std::mutex> g(s->mu);
      s->cv.wait(g, [s] { return s->stop || !s->big.empty(); });
      if (s->stop) return;
      t = s->big.front();
      s->big.pop_front();
      Req &r = s->reqs[t];
      r.state = 1;
      q = r;
    }
    kz_result res{};
    res.status = KZ_EHIP;
    if (hipStreamWaitEvent(stream, q.ready, 0) == hipSuccess) {
      kz_graph gr{};
      gr.format = KZ_BITSET_U64;
      gr.n = q.r.n;
      gr.rows = q.r.rows;
      gr.row_words = q.r.row_words;
      (void)kz_kernelize(ctx, &gr, q.r.colour, q.r.k, s->arena + q.at, q.bytes, q.r.vmask, q.r.emask, stream,
                         &res);
      if (hipStreamSynchronize(stream) != hipSuccess) res.status = KZ_EHIP;
    }
    std::lock_guard<std::mutex> g(s->mu);
    Req &r = s->reqs[t];
    r.res = res;
    r.state = 2;
    (void)hipEventDestroy(r.ready);
    r.ready = nullptr;
    if (r.bytes) s->heap.give(r.at, r.bytes);
    r.bytes = 0;
  }
}

int launch(kz_server *s, Record &rec) {
  const int G = (int)std::min<size_t>(s->waiting.size(), (size_t)s->slots);
  if (G == 0) return KZ_OK;
  rec.tickets.clear();
  for (int i = 0; i < G; ++i) {
    const uint64_t t = s->waiting.front();
    s->waiting.pop_front();
    Req &q = s->reqs[t];
    q.state = 1;
    rec.tickets.push_back(t);
    kz_batch_graph &g = rec.graphs_host[i];
    g.n = q.r.n;
    g.k = q.r.k;
    g.row_words = q.r.row_words;
    g.clique = q.r.clique;
    g.row_offset = 0;
    g.vertex_offset = 0;
    kzi::BatchPtrs &p = rec.ptrs_host[i];
    const size_t words = (size_t)q.r.n * (size_t)q.r.row_words;
    p.rows = q.r.rows;
    p.colour = q.r.colour;
    p.vmask = q.r.vmask;
    p.emask = q.r.emask;
    p.next = (uint64_t *)(s->arena + q.at);
    p.lists = (int *)(s->arena + q.at + up(words * sizeof(uint64_t)));
    p.items = (int *)(s->arena + q.at + up(words * sizeof(uint64_t)) + up(2 * words * sizeof(int)));
  }
  kzi::BatchArgs a{};
  a.graphs = (const kz_batch_graph *)(rec.dev + s->L.graphs);
  a.ptrs = (const kzi::BatchPtrs *)(rec.dev + s->L.ptrs);
  a.G = G;
  a.share = s->ctx->batch_cfg.share;
  a.order = (int *)(rec.dev + s->L.order);
  a.queue = (int *)(rec.dev + s->L.counters);
  a.finished = a.queue + 1;
  a.board = (int *)(rec.dev + s->L.board);
  a.jobs = (kzi::BatchJob *)(rec.dev + s->L.jobs);
  a.results = (kz_result *)(rec.dev + s->L.results);
  kzi::BatchConfig c = s->ctx->batch_cfg;
  c.workgroups = c.workgroups > 0 ? c.workgroups : s->ctx->cus * (16 / c.waves);
  if (c.workgroups > kSrvMaxWorkgroups) c.workgroups = kSrvMaxWorkgroups;
  if (hipMemcpyAsync((void *)a.graphs, rec.graphs_host, sizeof(kz_batch_graph) * G, hipMemcpyHostToDevice,
                     s->stream) != hipSuccess ||
      hipMemcpyAsync((void *)a.ptrs, rec.ptrs_host, sizeof(kzi::BatchPtrs) * G, hipMemcpyHostToDevice,
                     s->stream) != hipSuccess)
    return KZ_EHIP;
  kzi::launch_batch(a, c, s->stream);
  if (hipGetLastError() != hipSuccess) return KZ_EHIP;
  if (hipMemcpyAsync(rec.results_host, a.results, sizeof(kz_result) * G, hipMemcpyDeviceToHost, s->stream) !=
          hipSuccess ||
      hipEventRecord(rec.done, s->stream) != hipSuccess)
    return KZ_EHIP;
  rec.busy = true;
  return KZ_OK;
}

}  // namespace

extern "C" {

size_t kz_server_fixed_bytes(int32_t max_slots) {
  if (max_slots < 1 || max_slots > kSrvMaxSlots) return 0;
  return 2 * rec_layout(max_slots).total;
}

namespace {

// Scratch of the batch lane: next-state words, changed-tile and item lists.
size_t batch_bytes(const kz_request &r) {
  const size_t words = (size_t)r.n * (size_t)r.row_words;
  return up(words * sizeof(uint64_t)) + 2 * up(2 * words * sizeof(int));
}

// Scratch of the single-graph lane: kz_kernelize's workspace.
int single_bytes(kz_ctx *ctx, const kz_request &r, size_t *bytes) {
  kz_graph gr{};
  gr.format = KZ_BITSET_U64;
  gr.n = r.n;
  gr.rows = r.rows;
  gr.row_words = r.row_words;
  const int st = kz_workspace_bytes(ctx, &gr, r.k, bytes);
  *bytes = up(*bytes);
  return st;
}

}  // namespace

size_t kz_server_request_bytes(const kz_server *s, const kz_request *req) {
  if (!s || !req || req->n < 0 || req->k < 1 || req->row_words < 0) return 0;
  if (req->n < kSplitN && req->k <= kzi::kBatchK && req->row_words <= kzi::kBatchR) return batch_bytes(*req);
  size_t b = 0;
  return single_bytes(s->wctx[0], *req, &b) == KZ_OK ? b : 0;
}

int kz_server_create(kz_ctx *ctx, void *arena, size_t arena_bytes, int32_t max_slots, void *stream,
                     kz_server **out) {
  if (!out) return KZ_EINVAL;
  *out = nullptr;
  if (!ctx || !arena || (uintptr_t)arena % kSrvAlign || max_slots < 1 || max_slots > kSrvMaxSlots)
    return KZ_EINVAL;
  const RecLayout L = rec_layout(max_slots);
  if (arena_bytes <= 2 * L.total) return KZ_EWORKSPACE;
  kz_server *s = new (std::nothrow) kz_server();
  if (!s) return KZ_ENOMEM;
  s->ctx = ctx;
  s->stream = (hipStream_t)stream;
  s->arena = (char *)arena;
  s->arena_bytes = arena_bytes;
  s->slots = max_slots;
  s->L = L;
  s->next_ticket = 1;
  s->admitted = 0;
  s->heap.init(2 * L.total, arena_bytes - 2 * L.total);
  for (int i = 0; i < kWorkers; ++i) {
    s->wctx[i] = nullptr;
    s->wstream[i] = nullptr;
  }
  s->stop = false;
  for (int i = 0; i < 2; ++i) {
    Record &r = s->rec[i];
    r.dev = s->arena + i * L.total;
    r.graphs_host = nullptr;
    r.ptrs_host = nullptr;
    r.results_host = nullptr;
    r.done = nullptr;
    r.busy = false;
  }
  if (hipSetDevice(ctx->device) != hipSuccess) {
    release(s);
    return KZ_EHIP;
  }
  for (Record &r : s->rec) {
    if (hipHostMalloc((void **)&r.graphs_host, sizeof(kz_batch_graph) * max_slots, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc((void **)&r.ptrs_host, sizeof(kzi::BatchPtrs) * max_slots, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc((void **)&r.results_host, sizeof(kz_result) * max_slots, hipHostMallocDefault) !=
            hipSuccess ||
        hipEventCreateWithFlags(&r.done, hipEventDisableTiming) != hipSuccess) {
      release(s);
      return KZ_EHIP;
    }
  }
  for (int i = 0; i < kWorkers; ++i) {
    if (kz_create(&s->wctx[i], ctx->device) != KZ_OK || hipStreamCreate(&s->wstream[i]) != hipSuccess) {
      release(s);
      return KZ_EHIP;
    }
    s->wctx[i]->edge_path = ctx->edge_path;
  }
  for (int i = 0; i < kWorkers; ++i) s->worker[i] = std::thread(work, s, i);
  *out = s;
  return KZ_OK;
}

int kz_server_submit(kz_server *s, const kz_request *req, uint64_t *ticket) {
  if (!s || !req || !ticket) return KZ_EINVAL;
  const kz_request &r = *req;
  if (r.n < 0 || r.k < 1 || r.row_words < 0 || (r.n > 0 && (!r.rows || !r.colour || !r.vmask || !r.emask)))
    return KZ_EINVAL;
  // the batch lane's outputs must not share a 128-byte line with other data
  if ((uintptr_t)r.vmask % 128 || (uintptr_t)r.emask % 128) return KZ_EINVAL;
  if (r.clique < 0 || r.clique > r.k) return KZ_EINVAL;
  const bool fits_batch = r.k <= kzi::kBatchK && r.row_words <= kzi::kBatchR && r.n <= kzi::kBatchN;
  const bool below = r.clique > 0 && r.clique < r.k;  // only the batched lane takes a smaller clique size
  if (below && !fits_batch) return KZ_EINVAL;
  const bool big = !below && (r.n >= kSplitN || !fits_batch);
  size_t bytes = batch_bytes(r);
  if (big && single_bytes(s->wctx[0], r, &bytes) != KZ_OK) return KZ_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  if (s->admitted >= s->slots) return KZ_EAGAIN;
  size_t at = 0;
  if (bytes && !s->heap.take(bytes, &at)) return KZ_EAGAIN;
  Req q{};
  q.r = r;
  q.at = at;
  q.bytes = bytes;
  q.state = 0;
  q.big = big;
  q.ready = nullptr;
  if (big && (hipEventCreateWithFlags(&q.ready, hipEventDisableTiming) != hipSuccess ||
              hipEventRecord(q.ready, s->stream) != hipSuccess)) {
    if (q.ready) (void)hipEventDestroy(q.ready);
    if (bytes) s->heap.give(at, bytes);
    return KZ_EHIP;
  }
  const uint64_t t = s->next_ticket++;
  s->reqs.emplace(t, q);
  if (big) s->big.push_back(t);
  else s->waiting.push_back(t);
  ++s->admitted;
  *ticket = t;
  if (big) s->cv.notify_one();
  return KZ_OK;
}

int kz_server_progress(kz_server *s) {
  if (!s) return KZ_EINVAL;
  if (hipSetDevice(s->ctx->device) != hipSuccess) return KZ_EHIP;
  std::lock_guard<std::mutex> g(s->mu);
  for (Record &rec : s->rec) {
    if (!rec.busy) continue;
    const hipError_t e = hipEventQuery(rec.done);
    if (e == hipErrorNotReady) continue;
    if (e != hipSuccess) return KZ_EHIP;
    for (size_t i = 0; i < rec.tickets.size(); ++i) {
      Req &q = s->reqs[rec.tickets[i]];
      q.res = rec.results_host[i];
      q.state = 2;
      if (q.bytes) s->heap.give(q.at, q.bytes);
      q.bytes = 0;
    }
    rec.tickets.clear();
    rec.busy = false;
  }
  // launch what waits, into a free record (the first in flight runs, a
  // second queues behind it on the stream)
  for (Record &rec : s->rec) {
    if (s->waiting.empty()) break;
    if (rec.busy) continue;
    const int st = launch(s, rec);
    if (st != KZ_OK) return st;
  }
  return s->admitted;
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
    // let the worker finish what it holds; it takes nothing new once stopped
    std::unique_lock<std::mutex> g(s->mu);
    s->big.clear();
  }
  for (Record &rec : s->rec)
    if (rec.busy) (void)hipEventSynchronize(rec.done);
  release(s);
}

}  // extern "C"
