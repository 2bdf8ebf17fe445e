// Host driver and C ABI of the colour-index kernelizer (see include/kz.h).
//
// One call: stage-1 checks and layout run on the device (no host round trip
// before the first pass); then synchronous passes -- vertex test, edge test
// and, from pass 2 on, apply -- each followed by one small device-to-host
// read of the pass counters, until a pass removes nothing.
#include <string.h>

#include <algorithm>
#include <climits>

#include <mutex>
#include <new>
#include <vector>

#include "kz.h"
#include "kz_internal.h"

// Workspace of kz_kernelize_noalloc: one copy per GPU, held until the process
// ends.  Host code never uses this name as a device address; it uses the
// address hipGetSymbolAddress returned on that device (scratch_ptr below).
static __device__ __align__(256) unsigned char kz_scratch[KZ_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];  // device address of kz_scratch on each device, once looked up

// Looks up kz_scratch's address on `device` (which must be current) the
// first time; KZ_EHIP if the runtime cannot give it.
int scratch_lookup(int device, void **out) {
  if (device < 0 || device >= kMaxDevices) return KZ_EHIP;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(kz_scratch)) != hipSuccess || !p) return KZ_EHIP;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return KZ_OK;
}

hipEvent_t take_event(kz_ctx *c) {
  hipEvent_t e = nullptr;
  if (!c->pool.empty()) {
    e = c->pool.back();
    c->pool.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    e = nullptr;
  }
  return e;
}

// Brackets one kernel launch with events on the launch stream when timing is on.
struct ProfScope {
  kz_ctx *c;
  int kind;
  hipStream_t s;
  hipEvent_t a = nullptr;
  ProfScope(kz_ctx *c_, int kind_, hipStream_t s_) : c(c_), kind(kind_), s(s_) {
    if (c->prof && (a = take_event(c))) (void)hipEventRecord(a, s);
  }
  ~ProfScope() {
    if (!a) return;
    hipEvent_t b = take_event(c);
    if (b && hipEventRecord(b, s) == hipSuccess) {
      c->pending.push_back({a, b, kind});
    } else {
      c->pool.push_back(a);
      if (b) c->pool.push_back(b);
    }
  }
};

// Call after the stream has been synchronised.
void prof_collect(kz_ctx *c) {
  for (auto &p : c->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      c->total_ms[p.kind] += ms;
      c->launches[p.kind] += 1;
    }
    c->pool.push_back(p.a);
    c->pool.push_back(p.b);
  }
  c->pending.clear();
}

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool shape_ok(const kz_graph *g, int32_t k) {
  if (!g || k < 1 || g->n < 0) return false;
  if (g->format == KZ_DENSE_U8) return g->n <= 65536;
  if (g->format == KZ_BITSET_U64) return g->row_words >= 0 && g->row_words <= 65535;
  if (g->format == KZ_CSR) return g->nnz >= 0 && k <= 1024 && g->n < 0x7fffffff;
  return false;
}

kzi::WsSizes plan_sizes_csr(const kz_graph *g, int32_t k) {
  kzi::WsSizes z{};
  const size_t n = (size_t)g->n, nnz = (size_t)g->nnz;
  size_t o = align_up(sizeof(kzi::Hdr));
  auto take = [&o](size_t bytes) {
    size_t at = o;
    o += align_up(bytes);
    return at;
  };
  z.off_counts = take(sizeof(int) * (size_t)k);
  z.off_coff = take(sizeof(int) * ((size_t)k + 1));
  z.off_soff = take(sizeof(int) * ((size_t)k + 1));
  z.off_touched0 = take(n);
  z.off_touched1 = take(n);
  z.off_src = take(sizeof(int32_t) * nnz);
  z.off_efail = take(nnz);
  z.off_pm = take(sizeof(uint64_t) * n * ((size_t)kzi::csr_words(k) + 1));  // presence mask + colour
  z.total = o;
  return z;
}

kzi::WsSizes plan_sizes(const kz_graph *g, int32_t k, bool mfma) {
  if (g->format == KZ_CSR) return plan_sizes_csr(g, k);
  kzi::WsSizes z{};
  const long long n = g->n;
  const bool dense = g->format == KZ_DENSE_U8;
  long long Rmax;
  if (dense) {
    Rmax = (n + 63) / 64 + k;
    if (Rmax > n) Rmax = n;
  } else {
    Rmax = g->row_words;
  }
  z.Rmax = (int)Rmax;
  z.Tmax = Rmax > 1 ? Rmax * (Rmax - 1) / 2 : 0;
  z.nchunks = (int)((n + kzi::kRankChunk - 1) / kzi::kRankChunk);
  size_t o = align_up(sizeof(kzi::Hdr));
  auto take = [&o](size_t bytes) {
    size_t at = o;
    o += align_up(bytes);
    return at;
  };
  z.off_counts = take(sizeof(int) * (size_t)k);
  z.off_coff = take(sizeof(int) * ((size_t)k + 1));
  z.off_soff = take(sizeof(int) * ((size_t)k + 1));
  z.off_bcls = take(sizeof(int) * (size_t)Rmax);
  z.off_bstart = take(sizeof(int) * (size_t)Rmax);
  z.off_blen = take(sizeof(int) * (size_t)Rmax);
  z.off_hist = take(dense ? sizeof(int) * (size_t)z.nchunks * (size_t)k : 0);
  z.off_perm = take(dense ? sizeof(int) * (size_t)n : 0);
  z.off_inv = take(dense ? sizeof(int) * (size_t)n : 0);
  z.off_scls = take(dense ? sizeof(int) * (size_t)n : 0);
  z.off_valive = take(dense ? (size_t)n : 0);
  z.off_touched0 = take((size_t)n);
  z.off_touched1 = take((size_t)n);
  z.off_bt0 = take((size_t)Rmax);
  z.off_bt1 = take((size_t)Rmax);
  z.off_tiles = take(sizeof(int2) * (size_t)z.Tmax);
  z.off_packed = take(dense ? sizeof(uint64_t) * (size_t)n * (size_t)Rmax : 0);
  z.off_spare = take(sizeof(uint64_t) * (size_t)n * (size_t)Rmax);
  z.off_fb = take(mfma ? sizeof(uint64_t) * (size_t)n * (size_t)Rmax : 0);
  z.off_F = take(sizeof(uint64_t) * (size_t)n * (size_t)kzi::f_stride(k));
  z.off_S = take(sizeof(uint64_t) * (size_t)n * (size_t)kzi::f_stride(k));
  z.total = o;
  return z;
}

int finish(kz_result *res, const kz_result &r) {
  if (res) *res = r;
  return r.status;
}

// ---- batched path
constexpr int kBatchMaxWorkgroups = 1024;

struct BatchWs {
  size_t off_queue, off_finished, off_board, off_order, off_jobs, off_next, off_lists, off_items, total;
};

// Every graph's ranges start on a 128-byte line (no line holds two graphs'
// data, see the batch kernel's notes on cache lines).
constexpr long long kLineWords = 16, kLineVertices = 128;

bool batch_fits(const kz_batch_graph &g) {
  return g.n >= 0 && g.k >= 1 && g.row_words >= 0 && g.row_offset >= 0 && g.vertex_offset >= 0 &&
         g.k <= kzi::kBatchK && g.row_words <= kzi::kBatchR && g.n <= kzi::kBatchN;
}

// Arenas indexed like rows: the next-state words (one word per row word), the
// changed-tile lists and the item lists (two ints per row word each).
BatchWs batch_ws(const kz_batch_graph *graphs, int32_t G) {
  BatchWs w{};
  long long extent = 0;
  for (int32_t i = 0; i < G; ++i) {
    const kz_batch_graph &g = graphs[i];
    if (!batch_fits(g)) continue;
    const long long end = g.row_offset + (long long)g.n * g.row_words;
    if (end > extent) extent = end;
  }
  size_t o = 0;
  auto take = [&o](size_t bytes) {
    size_t at = o;
    o += align_up(bytes);
    return at;
  };
  w.off_queue = take(sizeof(int));
  w.off_finished = take(sizeof(int));
  w.off_board = take(sizeof(int) * kzi::kBatchBoard);
  w.off_order = take(sizeof(int) * (size_t)G);
  w.off_jobs = take(sizeof(kzi::BatchJob) * (size_t)G);
  w.off_next = take(sizeof(uint64_t) * (size_t)extent);
  w.off_lists = take(2 * sizeof(int) * (size_t)extent);
  w.off_items = take(2 * sizeof(int) * (size_t)extent);
  w.total = o;
  return w;
}

// Persistent workgroups: as many as fit on the device at once (also for
// small batches: workgroups without a graph help with the running ones).
int batch_workgroups(const kz_ctx *ctx, const kzi::BatchConfig &cfg) {
  int wg = cfg.workgroups > 0 ? cfg.workgroups : ctx->cus * (16 / cfg.waves);
  if (wg > kBatchMaxWorkgroups) wg = kBatchMaxWorkgroups;
  return wg < 1 ? 1 : wg;
}

bool batch_cfg_ok(const kzi::BatchConfig &c) {
  return (c.waves == 4 || c.waves == 8 || c.waves == 16) && (c.chunk == 4 || c.chunk == 8) &&
         !(c.waves == 16 && c.chunk == 8) && (c.lpt == 0 || c.lpt == 1) && c.workgroups >= 0 &&
         c.workgroups <= kBatchMaxWorkgroups && c.share >= 0 && c.share <= 2;
}

int batch_launch(kz_ctx *ctx, const kzi::BatchConfig &cfg, const kz_batch_graph *graphs_host,
                 const kz_batch_graph *graphs_dev, int32_t G, const uint64_t *rows, const int32_t *colour,
                 void *ws, size_t ws_bytes, uint8_t *vmask, uint64_t *emask, kz_result *results,
                 hipStream_t s) {
  if (!ctx || G < 0 || (G > 0 && (!graphs_host || !graphs_dev || !rows || !colour || !ws || !vmask ||
                                  !emask || !results)))
    return KZ_EINVAL;
  if (G == 0) return KZ_OK;
  if ((uintptr_t)ws % kAlign) return KZ_EINVAL;
  if ((uintptr_t)rows % 128 || (uintptr_t)colour % 128 || (uintptr_t)vmask % 128 || (uintptr_t)emask % 128)
    return KZ_EINVAL;
  for (int32_t i = 0; i < G; ++i)
    if (graphs_host[i].row_offset % kLineWords || graphs_host[i].vertex_offset % kLineVertices) return KZ_EINVAL;
  const BatchWs w = batch_ws(graphs_host, G);
  if (ws_bytes < w.total) return KZ_EWORKSPACE;
  if (hipSetDevice(ctx->device) != hipSuccess) return KZ_EHIP;
  char *base = (char *)ws;
  kzi::BatchArgs a{};
  a.graphs = graphs_dev;
  a.G = G;
  a.share = cfg.share;
  a.order = (int *)(base + w.off_order);
  a.queue = (int *)(base + w.off_queue);
  a.finished = (int *)(base + w.off_finished);
  a.board = (int *)(base + w.off_board);
  a.jobs = (kzi::BatchJob *)(base + w.off_jobs);
  a.rows = rows;
  a.colour = colour;
  a.emask = emask;
  a.vmask = vmask;
  a.results = results;
  a.next = (uint64_t *)(base + w.off_next);
  a.lists = (int *)(base + w.off_lists);
  a.items = (int *)(base + w.off_items);
  kzi::BatchConfig c = cfg;
  c.workgroups = batch_workgroups(ctx, cfg);
  kzi::launch_batch(a, c, s);
  return hipGetLastError() == hipSuccess ? KZ_OK : KZ_EHIP;
}

// Sparse path: state in place in vmask / emask; every pass is vertex test,
// edge test, apply, then the device-side pass end.  Enqueues setup and the
// validating first sweep when first_pass is 1, then passes [first_pass,
// first_pass + npasses); no host synchronisation.
int enqueue_csr(kz_ctx *ctx, const kz_graph *g, const int32_t *colour, int32_t k, char *base,
                const kzi::WsSizes &z, uint8_t *vmask, uint8_t *emask, int first_pass, int npasses,
                hipStream_t s, kz_out *out) {
  kzi::Plan p{};
  p.hdr = (kzi::Hdr *)base;
  p.counts = (int *)(base + z.off_counts);
  p.coff = (int *)(base + z.off_coff);
  p.soff = (int *)(base + z.off_soff);
  p.touched[0] = (uint8_t *)(base + z.off_touched0);
  p.touched[1] = (uint8_t *)(base + z.off_touched1);
  p.src = (int32_t *)(base + z.off_src);
  p.efail = (uint8_t *)(base + z.off_efail);
  p.pm = (uint64_t *)(base + z.off_pm);
  p.n = g->n;
  p.k = k;
  const int64_t *rp = g->row_ptr;
  const int32_t *ci = g->col_idx;
  const long long nnz = g->nnz;
  if (first_pass == 1) {
    {
      ProfScope t(ctx, KZ_KERNEL_SETUP, s);
      kzi::launch_setup(p, colour, 0, kzi::SETUP_CSR, s);
    }
    // validation and pass 1's vertex test share one sweep over the rows
    ProfScope t(ctx, KZ_KERNEL_VERTEX, s);
    kzi::launch_csr_first(p, rp, ci, nnz, colour, vmask, emask, s);
  }
  for (int pass = first_pass; pass < first_pass + npasses; ++pass) {
    const bool first = pass == 1;
    if (!first) {
      ProfScope t(ctx, KZ_KERNEL_VERTEX, s);
      kzi::launch_csr_vertex(p, rp, ci, colour, vmask, emask, pass, s);
    }
    {
      ProfScope t(ctx, KZ_KERNEL_EDGE, s);
      kzi::launch_csr_edge(p, rp, ci, nnz, colour, emask, pass, first, s);
    }
    {
      ProfScope t(ctx, KZ_KERNEL_APPLY, s);
      kzi::launch_csr_apply(p, nnz, emask, s);
    }
    kzi::launch_pass_end(p, pass, true, out, s);
  }
  return hipGetLastError() == hipSuccess ? KZ_OK : KZ_EHIP;
}

constexpr int kMaxChunk = 16;      // passes the blocking call enqueues between two looks at the result
constexpr int kSinglePasses = 8;   // ... one at a time up to this pass

// Host-checkable errors of a single-graph call (nothing is enqueued when
// one is found); the workspace plan and the edge path otherwise.
int check_call(kz_ctx *ctx, const kz_graph *g, const int32_t *colour, int32_t k, void *ws, size_t ws_bytes,
               uint8_t *vmask, void *emask, kzi::WsSizes *z, bool *mfma) {
  if (!ctx || !shape_ok(g, k)) return KZ_EINVAL;
  const int n = g->n;
  const bool dense = g->format == KZ_DENSE_U8;
  const bool csr = g->format == KZ_CSR;
  if (n == 0) return KZ_OK;
  if (!colour || !vmask || !ws) return KZ_EINVAL;
  if (!emask && !(csr && g->nnz == 0)) return KZ_EINVAL;
  if (dense && !g->adj) return KZ_EINVAL;
  if (g->format == KZ_BITSET_U64 && !g->rows) return KZ_EINVAL;
  if (csr && (!g->row_ptr || (g->nnz > 0 && !g->col_idx))) return KZ_EINVAL;
  if ((uintptr_t)ws % kAlign) return KZ_EINVAL;
  *mfma = ctx->edge_path == KZ_EDGE_MFMA_I8 && !csr;
  *z = plan_sizes(g, k, *mfma);
  if (*mfma && z->Rmax > kzi::kMfMaxWords) return KZ_ETOOLARGE;
  if (ws_bytes < z->total) return KZ_EWORKSPACE;
  if (z->Tmax > 0x7fffffffLL) return KZ_EINVAL;
  return KZ_OK;
}

// Enqueues setup (first_pass == 1) and passes [first_pass, first_pass +
// npasses) of the single-graph path, each ended on the device by
// k_pass_end, then (dense input) the output unpack, which writes only at
// the fixpoint.  No host synchronisation: the whole call can be captured.
int enqueue_passes(kz_ctx *ctx, const kz_graph *g, const int32_t *colour, int32_t k, char *base,
                   const kzi::WsSizes &z, bool mfma, uint8_t *vmask, void *emask, int first_pass, int npasses,
                   bool unpack, hipStream_t s, kz_out *out) {
  if (g->format == KZ_CSR)
    return enqueue_csr(ctx, g, colour, k, base, z, vmask, (uint8_t *)emask, first_pass, npasses, s, out);
  const int n = g->n;
  const bool dense = g->format == KZ_DENSE_U8;
  kzi::Plan p{};
  p.hdr = (kzi::Hdr *)base;
  p.counts = (int *)(base + z.off_counts);
  p.coff = (int *)(base + z.off_coff);
  p.soff = (int *)(base + z.off_soff);
  p.bcls = (int *)(base + z.off_bcls);
  p.bstart = (int *)(base + z.off_bstart);
  p.blen = (int *)(base + z.off_blen);
  p.hist = (int *)(base + z.off_hist);
  p.perm = (int *)(base + z.off_perm);
  p.inv = (int *)(base + z.off_inv);
  p.scls = (int *)(base + z.off_scls);
  p.valive = dense ? (uint8_t *)(base + z.off_valive) : vmask;
  p.touched[0] = (uint8_t *)(base + z.off_touched0);
  p.touched[1] = (uint8_t *)(base + z.off_touched1);
  p.btouched[0] = (uint8_t *)(base + z.off_bt0);
  p.btouched[1] = (uint8_t *)(base + z.off_bt1);
  p.tiles = (int2 *)(base + z.off_tiles);
  p.packed = (uint64_t *)(base + z.off_packed);
  p.spare = (uint64_t *)(base + z.off_spare);
  p.F = (uint64_t *)(base + z.off_F);
  p.S = (uint64_t *)(base + z.off_S);
  p.fb = (uint64_t *)(base + z.off_fb);
  p.n = n;
  p.k = k;
  p.Rmax = z.Rmax;
  p.nchunks = z.nchunks;
  p.kF = kzi::f_stride(k);
  p.Tmax = z.Tmax;

  // Pass 1 reads the input rows (bitset: the caller's; dense: packed here)
  // and writes the whole state after round 1 into `cur`; later passes work
  // in place on `cur`, staging changed tiles in `scratch`.
  const uint64_t *in_rows = dense ? p.packed : g->rows;
  uint64_t *cur = dense ? p.spare : (uint64_t *)emask;
  uint64_t *scratch = dense ? p.packed : p.spare;
  if (first_pass == 1) {
    {
      ProfScope t(ctx, KZ_KERNEL_SETUP, s);
      kzi::launch_setup(p, colour, g->row_words, dense ? kzi::SETUP_DENSE : kzi::SETUP_BITSET, s);
    }
    if (dense) {
      {
        ProfScope t(ctx, KZ_KERNEL_SETUP, s);
        kzi::launch_rank(p, colour, s);
      }
      ProfScope t(ctx, KZ_KERNEL_PACK, s);
      kzi::launch_pack_dense(p, g->adj, colour, p.packed, s);
    }
  }
  const int *scls = dense ? p.scls : colour;
  for (int pass = first_pass; pass < first_pass + npasses; ++pass) {
    const bool first = pass == 1;
    const uint64_t *src = first ? in_rows : cur;
    {
      ProfScope t(ctx, KZ_KERNEL_VERTEX, s);
      kzi::launch_vertex_pass(p, scls, src, cur, pass, first, dense ? 0 : g->row_words, s);
    }
    {
      ProfScope t(ctx, KZ_KERNEL_EDGE, s);
      if (mfma) kzi::launch_edge_pass_mfma(p, src, first ? cur : scratch, p.fb, pass, first, s);
      else kzi::launch_edge_pass(p, src, first ? cur : scratch, pass, first, s);
    }
    if (!first) {
      ProfScope t(ctx, KZ_KERNEL_APPLY, s);
      kzi::launch_apply(p, scratch, cur, s);
    }
    kzi::launch_pass_end(p, pass, false, out, s);
  }
  if (dense && unpack) {
    ProfScope t(ctx, KZ_KERNEL_UNPACK, s);
    kzi::launch_unpack_dense(p, colour, cur, vmask, (uint8_t *)emask, s);
  }
  return hipGetLastError() == hipSuccess ? KZ_OK : KZ_EHIP;
}

}  // namespace

extern "C" {

int kz_create(kz_ctx **out, int device) {
  if (!out) return KZ_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return KZ_EHIP;
  kz_ctx *c = new (std::nothrow) kz_ctx();
  if (!c) return KZ_ENOMEM;
  c->device = device;
  c->pinned = nullptr;
  c->scratch = nullptr;
  c->prof = false;
  c->batch_cfg_set = false;
  c->batch_cfg = kzi::BatchConfig{16, 4, 1, 0, 0};
  c->edge_path = KZ_EDGE_BITSET;
  c->cus = 256;
  for (int i = 0; i < KZ_KERNEL_COUNT; ++i) {
    c->total_ms[i] = 0.0;
    c->launches[i] = 0;
  }
  if (hipSetDevice(device) != hipSuccess ||
      hipHostMalloc((void **)&c->pinned, sizeof(kzi::Hdr), hipHostMallocDefault) != hipSuccess) {
    delete c;
    return KZ_EHIP;
  }

  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
    c->cus = cus;
  // the device's copy of the no-allocation workspace, looked up while the
  // device is current
  if (scratch_lookup(device, &c->scratch) != KZ_OK) {
    kz_destroy(c);
    return KZ_EHIP;
  }
  *out = c;
  return KZ_OK;
}

void kz_destroy(kz_ctx *ctx) {
  if (!ctx) return;
  if (!ctx->pending.empty()) (void)hipDeviceSynchronize();
  for (auto &p : ctx->pending) {
    ctx->pool.push_back(p.a);
    ctx->pool.push_back(p.b);
  }
  for (hipEvent_t e : ctx->pool) (void)hipEventDestroy(e);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  delete ctx;
}

int kz_batch_workspace_bytes(const kz_ctx *ctx, const kz_batch_graph *graphs, int32_t G, size_t *bytes) {
  if (!ctx || !bytes || G < 0 || (G > 0 && !graphs)) return KZ_EINVAL;
  *bytes = batch_ws(graphs, G).total;
  return KZ_OK;
}

int kz_kernelize_batch(kz_ctx *ctx, const kz_batch_graph *graphs_host, const kz_batch_graph *graphs_dev,
                       int32_t G, const uint64_t *rows, const int32_t *colour, void *ws, size_t ws_bytes,
                       uint8_t *vmask, uint64_t *emask, kz_result *results, void *stream) {
  if (!ctx) return KZ_EINVAL;
  return batch_launch(ctx, ctx->batch_cfg, graphs_host, graphs_dev, G, rows, colour, ws, ws_bytes, vmask, emask,
                      results, (hipStream_t)stream);
}

int kz_batch_set_config(kz_ctx *ctx, const kz_batch_config *cfg) {
  if (!ctx || !cfg) return KZ_EINVAL;
  const kzi::BatchConfig c{cfg->waves, cfg->chunk, cfg->lpt, cfg->workgroups, cfg->share};
  if (!batch_cfg_ok(c)) return KZ_EINVAL;
  ctx->batch_cfg = c;
  ctx->batch_cfg_set = true;
  return KZ_OK;
}

int kz_batch_get_config(const kz_ctx *ctx, kz_batch_config *cfg) {
  if (!ctx || !cfg) return KZ_EINVAL;
  cfg->waves = ctx->batch_cfg.waves;
  cfg->chunk = ctx->batch_cfg.chunk;
  cfg->lpt = ctx->batch_cfg.lpt;
  cfg->workgroups = ctx->batch_cfg.workgroups;
  cfg->share = ctx->batch_cfg.share;
  return KZ_OK;
}

int kz_batch_autotune(kz_ctx *ctx, const kz_batch_graph *graphs_host, const kz_batch_graph *graphs_dev,
                      int32_t G, const uint64_t *rows, const int32_t *colour, void *ws, size_t ws_bytes,
                      uint8_t *vmask, uint64_t *emask, kz_result *results, void *stream,
                      kz_batch_config *best) {
  if (!ctx || !best) return KZ_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  static const kzi::BatchConfig cands[] = {{4, 4, 1, 0, 0}, {4, 8, 1, 0, 0}, {8, 4, 1, 0, 0},
                                           {8, 8, 1, 0, 0}, {16, 4, 1, 0, 0}, {8, 4, 0, 0, 0}};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return KZ_EHIP;
  int st = KZ_OK;
  float best_ms = 0.f;
  kzi::BatchConfig pick = ctx->batch_cfg;
  for (const kzi::BatchConfig &c : cands) {
    st = batch_launch(ctx, c, graphs_host, graphs_dev, G, rows, colour, ws, ws_bytes, vmask, emask, results, s);
    if (st != KZ_OK) break;
    float ms = 0.f;
    if (hipEventRecord(e0, s) != hipSuccess) { st = KZ_EHIP; break; }
    for (int rep = 0; rep < 2 && st == KZ_OK; ++rep)
      st = batch_launch(ctx, c, graphs_host, graphs_dev, G, rows, colour, ws, ws_bytes, vmask, emask, results, s);
    if (st != KZ_OK) break;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      st = KZ_EHIP;
      break;
    }
    if (best_ms == 0.f || ms < best_ms) {
      best_ms = ms;
      pick = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != KZ_OK) return st;
  ctx->batch_cfg = pick;
  ctx->batch_cfg_set = true;
  best->waves = pick.waves;
  best->chunk = pick.chunk;
  best->lpt = pick.lpt;
  best->workgroups = pick.workgroups;
  best->share = pick.share;
  return KZ_OK;
}

int kz_gen_bitset(kz_ctx *ctx, int32_t k, const int32_t *sizes, double p, uint32_t seed, uint32_t gid,
                  const int32_t *planted, uint64_t *rows, int32_t row_words, int32_t *colour, void *stream) {
  if (!ctx || k < 1 || k > kzi::kGenK || !sizes || !(p >= 0.0 && p <= 1.0)) return KZ_EINVAL;
  kzi::GenArgs g{};
  g.k = k;
  long long n = 0, R = 0;
  for (int c = 0; c < k; ++c) {
    if (sizes[c] < 0) return KZ_EINVAL;
    g.coff[c] = (int)n;
    g.soff[c] = (int)R;
    n += sizes[c];
    R += (sizes[c] + 63) / 64;
    if (n > INT32_MAX / 2) return KZ_EINVAL;
  }
  g.coff[k] = (int)n;
  g.soff[k] = (int)R;
  if (R != row_words || (n > 0 && !rows)) return KZ_EINVAL;
  g.n = (int)n;
  g.R = (int)R;
  g.planted = planted != nullptr;
  for (int c = 0; planted && c < k; ++c) {
    if (planted[c] < g.coff[c] || planted[c] >= g.coff[c + 1]) return KZ_EINVAL;
    g.pl[c] = planted[c];
  }
  // floor(p * 2^64) from the exact binary value of p
  if (p <= 0.0) {
    g.thr = 0;
  } else if (p >= 1.0) {
    g.thr = ~0ull;
  } else {
    int ex = 0;
    const double f = frexp(p, &ex);  // p = f * 2^ex, f in [0.5, 1)
    const unsigned long long mant = (unsigned long long)ldexp(f, 53);  // exact
    const int sh = ex + 11;          // p * 2^64 = mant * 2^(ex + 11)
    g.thr = sh >= 0 ? mant << sh : (-sh >= 64 ? 0ull : mant >> -sh);
  }
  auto mix = [](unsigned long long z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  g.base = mix(((unsigned long long)seed << 32) | gid);
  if (hipSetDevice(ctx->device) != hipSuccess) return KZ_EHIP;
  kzi::launch_gen_rows(g, rows, colour, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? KZ_OK : KZ_EHIP;
}

int kz_set_edge_path(kz_ctx *ctx, int32_t path) {
  if (!ctx || (path != KZ_EDGE_BITSET && path != KZ_EDGE_MFMA_I8)) return KZ_EINVAL;
  ctx->edge_path = path;
  return KZ_OK;
}

int kz_profile_enable(kz_ctx *ctx, int on) {
  if (!ctx) return KZ_EINVAL;
  ctx->prof = on != 0;
  for (int i = 0; i < KZ_KERNEL_COUNT; ++i) {
    ctx->total_ms[i] = 0.0;
    ctx->launches[i] = 0;
  }
  return KZ_OK;
}

int kz_profile_read(const kz_ctx *ctx, int kernel, double *total_ms, int64_t *launches) {
  if (!ctx || kernel < 0 || kernel >= KZ_KERNEL_COUNT || !total_ms || !launches) return KZ_EINVAL;
  *total_ms = ctx->total_ms[kernel];
  *launches = ctx->launches[kernel];
  return KZ_OK;
}

const char *kz_strerror(int status) {
  switch (status) {
    case KZ_OK: return "ok";
    case KZ_EINVAL: return "invalid argument or malformed input";
    case KZ_ECOLOUR: return "colour outside [0, k)";
    case KZ_EILLEGAL: return "edge inside a colour class (colouring not legal)";
    case KZ_EASYM: return "adjacency not symmetric";
    case KZ_ESELFLOOP: return "self-loop";
    case KZ_EWORKSPACE: return "workspace too small";
    case KZ_ENOMEM: return "host allocation failed";
    case KZ_EHIP: return "HIP runtime error";
    case KZ_EAGAIN: return "try again";
    default: return "unknown status";
  }
}

int kz_workspace_bytes(const kz_ctx *ctx, const kz_graph *g, int32_t k, size_t *bytes) {
  if (!ctx || !bytes || !shape_ok(g, k)) return KZ_EINVAL;
  *bytes = plan_sizes(g, k, ctx->edge_path == KZ_EDGE_MFMA_I8).total;
  return KZ_OK;
}

int kz_kernelize(kz_ctx *ctx, const kz_graph *g, const int32_t *colour, int32_t k, void *ws,
                 size_t ws_bytes, uint8_t *vmask, void *emask, void *stream, kz_result *res) {
  kz_result r{};
  kzi::WsSizes z{};
  bool mfma = false;
  r.status = check_call(ctx, g, colour, k, ws, ws_bytes, vmask, emask, &z, &mfma);
  if (r.status != KZ_OK || g->n == 0) {
    if (r.status == KZ_OK) r.equals_input = 1;
    return finish(res, r);
  }
  r.status = KZ_EHIP;
  if (hipSetDevice(ctx->device) != hipSuccess) return finish(res, r);
  hipStream_t s = (hipStream_t)stream;
  // The asynchronous passes in chunks, with one look at the device's result
  // per chunk: one pass at a time for the first kSinglePasses passes (most
  // runs end there, and a surplus pass still dispatches its grids), then
  // doubling chunks through the tail of a long cascade.  The dense output
  // is unpacked once, after the fixpoint.
  const kzi::Hdr *hdr = (const kzi::Hdr *)ws;
  int next = 1, chunk = 1;
  for (;;) {
    if (enqueue_passes(ctx, g, colour, k, (char *)ws, z, mfma, vmask, emask, next, chunk, false, s, nullptr) !=
        KZ_OK)
      return finish(res, r);
    if (hipMemcpyAsync(ctx->pinned, hdr, sizeof(kzi::Hdr), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return finish(res, r);
    prof_collect(ctx);
    const kz_out &o = ctx->pinned->out;
    if (o.converged) {
      r = o.result;
      break;
    }
    next += chunk;
    // every productive pass removes something: a run cannot outlast n + m + 1 passes
    if (next > (long long)g->n + o.result.input_edges + 2) return finish(res, r);
    chunk = next > kSinglePasses ? std::min(2 * chunk, kMaxChunk) : 1;
  }
  if (g->format == KZ_DENSE_U8 && r.status == KZ_OK &&
      enqueue_passes(ctx, g, colour, k, (char *)ws, z, mfma, vmask, emask, next + chunk, 0, true, s, nullptr) !=
          KZ_OK) {
    r.status = KZ_EHIP;
    return finish(res, r);
  }
  if (!ctx->pending.empty()) {
    // timing enabled: the unpack's events are read before returning
    if (hipStreamSynchronize(s) != hipSuccess) r.status = KZ_EHIP;
    prof_collect(ctx);
  }
  return finish(res, r);
}

int kz_kernelize_async(kz_ctx *ctx, const kz_graph *g, const int32_t *colour, int32_t k, void *ws,
                       size_t ws_bytes, uint8_t *vmask, void *emask, int32_t first_pass, int32_t npasses,
                       void *stream, kz_out *out) {
  kzi::WsSizes z{};
  bool mfma = false;
  const int st = check_call(ctx, g, colour, k, ws, ws_bytes, vmask, emask, &z, &mfma);
  if (st != KZ_OK) return st;
  if (first_pass < 1 || npasses < 1 || first_pass > INT32_MAX - npasses) return KZ_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return KZ_EHIP;
  hipStream_t s = (hipStream_t)stream;
  if (g->n == 0) {
    if (!out) return KZ_OK;
    kz_out o{};
    o.result.equals_input = 1;
    o.converged = 1;
    kzi::launch_write_out(out, o, s);
    return hipGetLastError() == hipSuccess ? KZ_OK : KZ_EHIP;
  }
  return enqueue_passes(ctx, g, colour, k, (char *)ws, z, mfma, vmask, emask, first_pass, npasses, true, s, out);
}

}  // extern "C"

extern "C" int kz_kernelize_noalloc(kz_ctx *ctx, const kz_graph *g, const int32_t *colour, int32_t k,
                                    uint8_t *vmask, void *emask, void *stream, kz_result *res) {
  kz_result r{};
  r.status = KZ_EINVAL;
  if (!ctx || !ctx->scratch || !shape_ok(g, k)) return finish(res, r);
  const bool mfma = ctx->edge_path == KZ_EDGE_MFMA_I8 && g->format != KZ_CSR;
  if (plan_sizes(g, k, mfma).total > (size_t)KZ_NOALLOC_SCRATCH_BYTES) {
    r.status = KZ_EWORKSPACE;
    return finish(res, r);
  }
  // every kernel of the path initialises what it reads from the workspace,
  // so the previous call's contents need no clearing
  return kz_kernelize(ctx, g, colour, k, ctx->scratch, (size_t)KZ_NOALLOC_SCRATCH_BYTES, vmask, emask, stream, res);
}
