// Batched kernelization (gfx950): many graphs in one persistent launch.
//
// Each graph is a job: a sequence of synchronous passes (Definition 4.2.1's
// vertex and edge colour-index tests, applied to a snapshot), and each pass
// is a list of items: 128-vertex chunks for the vertex test and 64x64 block
// tiles (X < Y) for the edge test.  A workgroup takes the next graph from an
// atomic queue, sets it up and lists its first pass; its waves split the
// items.  The workgroup that finishes the last item of a pass carries the
// job on: it applies the tiles that changed and either ends the job or lists
// the next pass.
//
// A pass normally belongs to the workgroup that listed it ("solo": no other
// workgroup touches the job, so no cross-workgroup fences are needed).  A
// pass with more items than the workgroup has waves is "shared" once the
// queue is empty, or earlier when it is very large: it is published on a
// board, and workgroups claim runs of its
// items with a compare-and-swap on the job's claim word (a workgroup looking
// for work prefers a well-stocked shared pass to a new graph), keep their
// counts and touched bits in LDS, and merge them into the job's state in HBM
// before they report the run finished.  The run that completes the pass makes its workgroup the
// carrier.  Nobody waits for anybody: a pass is continued by whoever
// finishes it, so the launch cannot deadlock, and a workgroup with nothing
// to do leaves once every graph is finished (or after a few milliseconds
// without finding work).
//
// Graph g's rows follow the bit-row layout of the single-graph path
// (class-major slots; class c's segment has ceil(s_c/64) words) and sit at
// word offset row_offset[g] of the rows arena; its colours and vertex mask at
// vertex_offset[g].  The state is kept in the emask arena (same layout); the
// changed words of a pass go to the next-state arena (same layout); the
// changed-tile list and the item list sit at int offset 2*row_offset[g] of
// two list arenas of their own.
//
// Cache lines.  The L2 of each XCD is a write-back cache, and an invalidate
// (the acquire half of a fence) keeps lines that hold dirty bytes.  A line
// that a workgroup reads while another workgroup on the same XCD writes
// other bytes of it can therefore survive a fence with stale bytes.  So no
// 128-byte line is shared between two graphs (the host requires every
// graph's ranges to start on a line, and the list arenas are laid out per
// row word), and within a pass every line that is read is written by at
// most the item that reads it: a vertex item owns 128 vertices (one line of
// the vertex mask), and the item list starts on a line of its own, away
// from the changed-tile list that tiles append to during the pass.  Lines
// that several items write in one pass (next-state words, the changed-tile
// list) are read only by the carrier, after every writer has released them.  Graphs too large for this path (k > kBatchK, row words >
// kBatchR, or n > kBatchN) get status KZ_ETOOLARGE in their result and are
// left to the single-graph path.
#include "kz_internal.h"

namespace kzi {

namespace {

constexpr int kVertexItem = 1 << 30;                 // item = kVertexItem | chunk, else X | Y << kYShift
constexpr int kVChunk = 128;                         // vertices of a vertex item: one line of the vertex mask
constexpr int kYShift = 9, kXMask = (1 << kYShift) - 1;
constexpr unsigned long long kIdleTicks = 2000000;   // 20 ms of the 100 MHz wall clock
constexpr unsigned long long kHostPoll = 200;        // 2 us: session mode's look at the host's count
// Claim word: pass (24 bits) | items (20 bits) | next unclaimed item (20 bits).
constexpr int kItemBits = 20;
constexpr unsigned kItemMask = (1u << kItemBits) - 1;
// A pass is shared once the queue is empty, or early when it is very large.
constexpr int kShareBig = 2048;   // items

__device__ __forceinline__ unsigned long long bcast64(unsigned long long x, int lane) {
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)x, lane);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(x >> 32), lane);
  return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ int bsum(int x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
  return x;
}

__device__ __forceinline__ bool tbit(const unsigned *b, int i) { return (b[i >> 5] >> (i & 31)) & 1u; }

__device__ __forceinline__ unsigned long long lanes_below(int lane) {
  return lane ? (~0ull >> (64 - lane)) : 0ull;
}

// Agent-scope relaxed accesses to the job's shared words.
template <typename T>
__device__ __forceinline__ T ald(T *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void ast(T *p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Release and acquire at agent scope, each with its wait.  A release writes
// this XCD's L2 back (buffer_wbl2) and must not let the atomic that
// publishes become visible before that write-back has landed; the sequence
// the compiler emits for a release atomic on gfx950 issues the atomic right
// after buffer_wbl2 with no wait in between, and a workgroup on another XCD
// can then see the published word while the words it guards (a counter
// reset, next-state words, list entries) are still on their way.  So the
// release is a fence followed by an explicit wait for every outstanding
// memory operation (the write-back included), and the publishing atomic is
// relaxed.  The acquire writes back first (the invalidate keeps dirty
// lines, stale bytes and all, so a line must be clean when it arrives),
// then invalidates, and waits for both before the workgroup's barrier lets
// other waves load.
__device__ __forceinline__ void release_agent() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __builtin_amdgcn_s_waitcnt(0);
}
// Release to the host (system scope), with its wait, for results that the
// host reads from pinned memory.
__device__ __forceinline__ void release_system() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
  __builtin_amdgcn_s_waitcnt(0);
}
__device__ __forceinline__ void acquire_system() {
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
  __builtin_amdgcn_s_waitcnt(0);
}
__device__ __forceinline__ void acquire_agent() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  __builtin_amdgcn_s_waitcnt(0);
}

// What a workgroup keeps in LDS about the job it works on.
struct BatchLds {
  int coff[kBatchK + 1], soff[kBatchK + 1];
  short bcls[kBatchR];
  unsigned short bstart[kBatchR];
  unsigned char blen[kBatchR];
  unsigned tc[kBatchN / 32], tn[kBatchN / 32];    // vertices touched in the previous / this pass
  unsigned btc[kBatchR / 32], btn[kBatchR / 32];  // blocks touched in the previous / this pass
  int job, pass;       // the job and pass the copies above belong to
  int pass0;           // the job's first pass
  int shared;          // the pass is shared
  int got, base, cnt, nitems, next_item, last, reload;
  int prio, nchanged;  // this run (solo: this pass)
  unsigned long long removed_v, removed_e, tests;
  int gi, queue_empty, bad_colour, bad_layout, pick, quit, end, status;
  unsigned long long ticket;  // session mode: the ticket of the job being started
};

struct GView {
  int g, n, k, R;
  int slack;  // classes a test may find without a witness: k - clique size
  const uint64_t *rows;
  uint64_t *cur, *nxt;
  const int *colour;
  uint8_t *valive;
  int *changed, *items;  // each starts on a 128-byte line
  BatchJob *J;
};

// A job's descriptor: the batch's, or in session mode the copy its starter
// made of the host slot.
__device__ __forceinline__ kz_batch_graph job_desc(const BatchArgs &a, int g) {
  return a.session ? a.jobs[g].sdesc : a.graphs[g];
}

__device__ __forceinline__ GView gview(const BatchArgs &a, int g) {
  const kz_batch_graph G = job_desc(a, g);
  GView v;
  v.g = g;
  v.n = G.n;
  v.k = G.k;
  v.R = G.row_words;
  v.slack = G.clique > 0 && G.clique < G.k ? G.k - G.clique : 0;
  const long long T = (long long)v.R * (v.R - 1) / 2;
  if (a.ptrs || a.session) {
    const BatchPtrs P = a.session ? a.jobs[g].sptrs : a.ptrs[g];
    v.rows = P.rows;
    v.cur = P.emask;
    v.nxt = P.next;
    v.colour = P.colour;
    v.valive = P.vmask;
    v.changed = P.lists;
    v.items = P.items;
  } else {
    v.rows = a.rows + G.row_offset;
    v.cur = a.emask + G.row_offset;
    v.nxt = a.next + G.row_offset;
    v.colour = a.colour + G.vertex_offset;
    v.valive = a.vmask + G.vertex_offset;
    v.changed = a.lists + 2 * G.row_offset;
    v.items = a.items + 2 * G.row_offset;
  }
  (void)T;
  v.J = a.jobs + g;
  return v;
}

// ---- vertex test on 64 vertices (one wave): vertex v fails when some other
// class holds none of its neighbours; pass 1 also validates the rows.
__device__ void vertex_chunk(const GView &V, BatchLds &S, int v0, bool first, int lane) {
  const int n = V.n, k = V.k, R = V.R;
  const uint64_t *src = V.cur;
  const int v = v0 + lane;
  const bool act = v < n && (first || (V.valive[v] && tbit(S.tc, v)));
  if (!__ballot(act)) return;
  const uint64_t *row = src + (long long)(act ? v : v0) * R;
  const int cv = act ? V.colour[v] : -1;
  int miss = 0;  // other classes without a neighbour
  int pr = 0;
  for (int c = 0; c < k; ++c) {
    const int w0 = S.soff[c], w1 = S.soff[c + 1];
    const int s = S.coff[c + 1] - S.coff[c];
    if (!act) continue;
    if (w1 == w0) {
      miss += c != cv;
      continue;
    }
    if (first && (s & 63) && (row[w1 - 1] >> (s & 63))) pr = max(pr, P_EINVAL);
    if (c == cv) {
      if (!first) continue;
      const int jv = v - S.coff[c];
      for (int w = w0; w < w1; ++w) {
        unsigned long long y = row[w];
        if (w == w1 - 1 && (s & 63)) y &= (1ull << (s & 63)) - 1;
        while (y) {
          const int b = __builtin_ctzll(y);
          y &= y - 1;
          const int t = S.coff[c] + (w - w0) * 64 + b;
          if (t == v) pr = max(pr, P_ESELFLOOP);
          else
            pr = max(pr, ((src[(long long)t * R + w0 + (jv >> 6)] >> (jv & 63)) & 1ull) ? (int)P_EILLEGAL
                                                                                         : (int)P_EASYM);
        }
      }
      continue;
    }
    bool nz = false;
    for (int w = w0; w < w1 && !nz; ++w) nz = row[w] != 0;
    miss += !nz;
  }
  if (pr) atomicMax(&S.prio, pr);
  const bool fail = act && miss > V.slack;
  if (act) {
    if (first) V.valive[v] = fail ? 0 : 1;
    else if (fail) V.valive[v] = 0;
  }
  const int nf = bsum(fail ? 1 : 0);
  if (lane == 0 && nf) atomicAdd(&S.removed_v, (unsigned long long)nf);
}

// ---- edge test on tile (X, Y) (one wave): edge (u, v) fails when some third
// class holds no common neighbour.  Only pairs with a touched endpoint are
// tested again after pass 1; the others keep their outcome.
template <int CH>
__device__ void tile(const GView &V, BatchLds &S, int X, int Y, bool first, int lane,
                     unsigned long long (*sU)[kBlk], unsigned long long (*sU2)[kBlk]) {
  const int R = V.R;
  const uint64_t *src = V.cur;
  const int cx = S.bcls[X], cy = S.bcls[Y];
  const int xs = S.bstart[X], xl = S.blen[X], ys = S.bstart[Y], yl = S.blen[Y];
  const unsigned long long ymask = yl == 64 ? ~0ull : ((1ull << yl) - 1);
  const unsigned long long xmask = xl == 64 ? ~0ull : ((1ull << xl) - 1);
  const uint64_t *rowu_l = src + (long long)(xs + (lane < xl ? lane : 0)) * R;  // lane as row u
  const uint64_t *rowv = src + (long long)(ys + (lane < yl ? lane : 0)) * R;    // lane as row v
  const unsigned long long Eu = lane < xl ? (rowu_l[Y] & ymask) : 0ull;          // E(u) of row u = lane
  const unsigned long long ET = lane < yl ? rowv[X] : 0ull;
  const unsigned long long TU = first ? ~0ull : __ballot(lane < xl && tbit(S.tc, xs + lane));
  const unsigned long long TV = first ? ~0ull : __ballot(lane < yl && tbit(S.tc, ys + lane));
  unsigned long long myP = Eu;  // P of the row this lane stands for
  const int nthird = V.slack > 0 ? 0 : V.k - 2;
  if (V.slack > 0) {
    // more classes than the clique size: an edge fails when more than slack
    // third classes hold no common neighbour; lane v counts its misses
    for (int u = 0; u < xl; ++u) {
      unsigned long long P = bcast64(myP, u);
      const unsigned long long Pt = P & (((TU >> u) & 1ull) ? ~0ull : TV);
      if (!Pt) continue;
      const uint64_t *rowu = src + (long long)(xs + u) * R;
      const bool tested = (Pt >> lane) & 1ull;
      int miss = 0;
      for (int c = 0; c < V.k; ++c) {
        if (c == cx || c == cy) continue;
        bool wit = false;
        for (int w = S.soff[c]; w < S.soff[c + 1]; ++w) {
          const uint64_t xu = rowu[w];
          if (!xu) continue;
          const uint64_t yv = tested && !wit ? rowv[w] : 0ull;
          wit |= (xu & yv) != 0ull;
          if (!(Pt & ~__ballot(wit))) break;  // every tested lane has its witness
        }
        miss += !wit;
      }
      P &= ~(Pt & __ballot(tested && miss > V.slack));
      if (lane == u) myP = P;
    }
  }
  for (int q = 0; q < nthird; q += CH) {
    // stage the first two words of each third-class segment: row u's in LDS
    // (read as broadcasts), row v's in registers
    unsigned long long vv[CH], vv2[CH];
    int w2[CH];
    bool any2 = false, any3 = false;  // some segment of the chunk has a second / third word
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const int i = q + j;
      if (i < nthird) {
        int c = i;
        if (c >= cx) ++c;
        if (c >= cy) ++c;
        const int w0 = S.soff[c], w1 = S.soff[c + 1];
        const bool has = w1 > w0, two = w1 > w0 + 1;
        any2 |= two;
        any3 |= w0 + 2 < w1;
        sU[j][lane] = (has && lane < xl) ? rowu_l[w0] : 0ull;
        sU2[j][lane] = (two && lane < xl) ? rowu_l[w0 + 1] : 0ull;
        vv[j] = (has && lane < yl) ? rowv[w0] : 0ull;
        vv2[j] = (two && lane < yl) ? rowv[w0 + 1] : 0ull;
        w2[j] = w0 + 2 < w1 ? w0 + 2 : -1;
      } else {
        sU[j][lane] = ~0ull;
        sU2[j][lane] = 0ull;
        vv[j] = ~0ull;
        vv2[j] = 0ull;
        w2[j] = -1;
      }
    }
    __builtin_amdgcn_wave_barrier();
    for (int u = 0; u < xl; ++u) {
      unsigned long long P = bcast64(myP, u);
      const unsigned long long Pt = P & (((TU >> u) & 1ull) ? ~0ull : TV);
      if (!Pt) continue;
      unsigned long long all = ~0ull;
#pragma unroll
      for (int j = 0; j < CH; ++j) all &= __ballot((sU[j][u] & vv[j]) != 0ull);
      if (!(Pt & ~all)) continue;
      // level 2: the first two words (nothing new when no segment has two)
      if (any2) {
        all = ~0ull;
#pragma unroll
        for (int j = 0; j < CH; ++j) all &= __ballot(((sU[j][u] & vv[j]) | (sU2[j][u] & vv2[j])) != 0ull);
        if (!(Pt & ~all)) continue;
      }
      if (!any3) {
        // the first two words are the whole segments: a lane missing a
        // witness in some class loses its edge
        P &= ~(Pt & ~all);
        if (lane == u) myP = P;
        continue;
      }
      // level 3: scan the rest of the segment in memory
      const uint64_t *rowu = src + (long long)(xs + u) * R;
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        unsigned long long miss = Pt & ~__ballot(((sU[j][u] & vv[j]) | (sU2[j][u] & vv2[j])) != 0ull);
        if (!miss) continue;
        if (w2[j] >= 0) {
          int c = q + j;
          if (c >= cx) ++c;
          if (c >= cy) ++c;
          for (int w = w2[j]; w < S.soff[c + 1] && miss; ++w) {
            const unsigned long long x = rowu[w];
            const unsigned long long y = ((miss >> lane) & 1ull) ? rowv[w] : 0ull;
            miss &= ~__ballot((x & y) != 0ull);
          }
        }
        P &= ~miss;
      }
      if (lane == u) myP = P;
    }
    __builtin_amdgcn_wave_barrier();
  }
  const unsigned long long Pu = myP;
  // transposes: lane v gets bit v of every P(u) (rows u >= xl hold zero) and,
  // in pass 1, of every E(u), to check that the rows are symmetric
  const unsigned long long newET = wave_transpose64(Pu, lane);
  if (first) {
    const unsigned long long trE = wave_transpose64(Eu, lane);
    if (lane < yl && ((trE ^ ET) & xmask)) atomicMax(&S.prio, P_EASYM);
  }
  const bool chU = lane < xl && Eu != Pu;
  const bool chV = lane < yl && (ET & xmask) != newET;
  const unsigned long long bu = __ballot(chU), bv = __ballot(chV);
  if (bu | bv) {
    if (lane < xl) V.nxt[(long long)(xs + lane) * R + Y] = Pu;
    if (lane < yl) V.nxt[(long long)(ys + lane) * R + X] = newET;
    if (chU) atomicOr(&S.tn[(xs + lane) >> 5], 1u << ((xs + lane) & 31));
    if (chV) atomicOr(&S.tn[(ys + lane) >> 5], 1u << ((ys + lane) & 31));
    const int rem = bsum(lane < xl ? __popcll(Eu & ~Pu) : 0);
    if (lane == 0) {
      if (bu) atomicOr(&S.btn[X >> 5], 1u << (X & 31));
      if (bv) atomicOr(&S.btn[Y >> 5], 1u << (Y & 31));
      const int at = S.shared ? atomicAdd(&V.J->nchanged, 1) : atomicAdd(&S.nchanged, 1);
      V.changed[at] = X | (Y << kYShift);
      atomicAdd(&S.removed_e, (unsigned long long)rem);
    }
  }
  const int cnt = bsum(lane < xl ? __popcll(Eu & (((TU >> lane) & 1ull) ? ~0ull : TV)) : 0);
  if (lane == 0 && cnt) atomicAdd(&S.tests, (unsigned long long)cnt);
}

// The waves of the workgroup take the items of the claimed run one by one.
template <int NW, int CH>
__device__ void run_items(const GView &V, BatchLds &S, unsigned long long (*sU)[CH][kBlk],
                          unsigned long long (*sU2)[CH][kBlk]) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const bool first = S.pass == S.pass0;
  const int cnt = S.cnt, base = S.base;
  for (;;) {
    int i = 0;
    if (lane == 0) i = atomicAdd(&S.next_item, 1);
    i = __builtin_amdgcn_readfirstlane(i);
    if (i >= cnt) break;
    const int it = V.items[base + i];
    if (it & kVertexItem) {
      // both halves of the item's line of the vertex mask, by this wave
      const int v0 = (it & 0xffff) * kVChunk;
      vertex_chunk(V, S, v0, first, lane);
      vertex_chunk(V, S, v0 + kWave, first, lane);
    }
    else tile<CH>(V, S, it & kXMask, (it >> kYShift) & kXMask, first, lane, sU[wid], sU2[wid]);
  }
  __syncthreads();
}

__device__ void write_result(const BatchArgs &a, int g, const kz_result &r) {
  if (a.session) {
    // the outputs and the result reach memory before the done flag
    a.hres[g] = r;
    release_system();
    __hip_atomic_store(&a.hdone[g], a.jobs[g].ticket, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    return;
  }
  a.results[g] = r;
  atomicAdd(a.finished, 1);
}

// Ends job g with an input error (thread 0).
__device__ void fail_job(const BatchArgs &a, int g, int status) {
  kz_result r{};
  r.status = status;
  write_result(a, g, r);
}

// Ends job g after `passes` passes (thread 0).
__device__ void end_job(const BatchArgs &a, const GView &V, int passes) {
  BatchJob *J = V.J;
  const int rounds = ald(&J->rounds);
  const long long m = ald(&J->m);
  kz_result r{};
  r.status = 0;
  r.rounds = rounds;
  r.equals_input = rounds == 0;
  r.passes = passes;
  r.surviving_vertices = V.n - ald(&J->tot_removed_v);
  r.surviving_edges = m - ald(&J->tot_removed_e);
  r.input_edges = m;
  r.edge_tests = ald(&J->tot_tests);
  write_result(a, V.g, r);
}

// Lists the items of pass S.pass (the touched sets are in S.tc / S.btc) and
// opens it: solo (the whole list is this workgroup's run) or shared
// (published, this workgroup's first run taken).  Returns false when the
// pass has nothing to test: the job is then finished.
template <int NW>
__device__ bool open_pass(const BatchArgs &a, const GView &V, BatchLds &S) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int n = V.n, R = V.R, p = S.pass;
  const int nw = (n + 31) >> 5, nbw = (R + 31) >> 5;
  if (tid == 0) {
    S.nitems = 0;
    // every pass number this job uses, the final empty one included: the
    // workgroup that ends the job keeps it in S.pass, and the slot's next
    // job must number its passes above it
    ast(&V.J->lastpass, p);
  }
  __syncthreads();
  // vertex chunks (128 vertices, four touched words) holding a touched vertex
  const int nvc = (n + kVChunk - 1) / kVChunk;
  for (int c0 = wid * kWave; c0 < nvc; c0 += NW * kWave) {
    const int c = c0 + lane;
    bool want = false;
    if (c < nvc) {
      unsigned t = 0;
#pragma unroll
      for (int j = 0; j < kVChunk / 32; ++j) t |= 4 * c + j < nw ? S.tc[4 * c + j] : 0u;
      want = t != 0u;
    }
    const unsigned long long b = __ballot(want);
    int at = 0;
    if (lane == 0 && b) at = atomicAdd(&S.nitems, __popcll(b));
    at = __builtin_amdgcn_readfirstlane(at);
    if (want) V.items[at + __popcll(b & lanes_below(lane))] = kVertexItem | c;
  }
  // tiles of two classes with a touched block: a wave per row X, lanes over Y
  for (int X = wid; X < R; X += NW) {
    const int cx = S.bcls[X];
    const bool tx = tbit(S.btc, X);
    for (int y0 = X + 1; y0 < R; y0 += kWave) {
      const int Y = y0 + lane;
      const bool want = Y < R && S.bcls[Y] != cx && (tx || tbit(S.btc, Y));
      const unsigned long long b = __ballot(want);
      int at = 0;
      if (lane == 0 && b) at = atomicAdd(&S.nitems, __popcll(b));
      at = __builtin_amdgcn_readfirstlane(at);
      if (want) V.items[at + __popcll(b & lanes_below(lane))] = X | (Y << kYShift);
    }
  }
  __syncthreads();
  const int ni = S.nitems;
  if (ni == 0) {
    if (tid == 0) end_job(a, V, p - S.pass0 + 1);
    __syncthreads();
    return false;
  }
  if (tid == 0) {
    bool shared = a.share == 1;
    if (a.share == 0 && ni > NW)
      shared = ni >= kShareBig ||
               (a.session ? ald(a.squeue) >= ald(a.dhead) : ald(a.queue) >= a.G);
    S.shared = shared;
    S.base = 0;
    S.cnt = shared ? min(ni, NW) : ni;
    S.next_item = 0;
    S.nchanged = 0;
    S.got = 1;
    if (shared) {
      BatchJob *J = V.J;
      ast(&J->removed_v, 0ull);
      ast(&J->removed_e, 0ull);
      ast(&J->tests, 0ull);
      ast(&J->prio, 0);
      ast(&J->nchanged, 0);
      ast(&J->done, 0u);
    }
  }
  __syncthreads();
  if (S.shared) {
    BatchJob *J = V.J;
    for (int i = tid; i < nw; i += NW * kWave) {
      ast(&J->touched[p & 1][i], S.tc[i]);
      ast(&J->touched[(p + 1) & 1][i], 0u);
    }
    for (int i = tid; i < nbw; i += NW * kWave) {
      ast(&J->btouched[p & 1][i], S.btc[i]);
      ast(&J->btouched[(p + 1) & 1][i], 0u);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) {
      const unsigned long long cw = ((unsigned long long)p << (2 * kItemBits)) |
                                    ((unsigned long long)ni << kItemBits) | (unsigned long long)S.cnt;
      release_agent();
      __hip_atomic_exchange(&J->claim, cw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&a.board[V.g & a.board_mask], V.g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  return true;
}

// Sets up graph g (validation, layout, state) and opens its first pass.
// Returns false when the graph needs no pass (error, empty graph).
template <int NW>
__device__ bool start_job(const BatchArgs &a, BatchLds &S, int g) {
  const int tid = threadIdx.x;
  if (a.session) {
    if (tid == 0) {
      BatchJob *J = a.jobs + g;
      J->sdesc = a.hgraphs[g];
      J->sptrs = a.hptrs[g];
      J->ticket = S.ticket;
    }
    __syncthreads();
  }
  const kz_batch_graph G = job_desc(a, g);
  const int n = G.n, k = G.k, R = G.row_words;
  int st = 0;
  if (n < 0 || k < 1 || R < 0 || G.clique < 0 || G.clique > k ||
      (!a.ptrs && !a.session && (G.row_offset < 0 || G.vertex_offset < 0)))
    st = KZ_EINVAL;
  else if (k > kBatchK || R > kBatchR || n > kBatchN) st = kBatchTooLarge;
  if (st != 0 || n == 0) {
    if (tid == 0) {
      if (st) {
        fail_job(a, g, st);
      } else {
        kz_result r{};
        r.equals_input = 1;
        write_result(a, g, r);
      }
    }
    return false;
  }
  const GView V = gview(a, g);
  // layout: colours are sorted class by class; class c starts at the first
  // vertex whose colour is >= c (binary search)
  // the layout copies in LDS are about to be overwritten: they no longer
  // belong to the job named in S.job (a later claim must reload them)
  if (tid == 0) {
    S.bad_colour = 0;
    S.bad_layout = 0;
    S.job = -1;
  }
  __syncthreads();
  for (int v = tid; v < n; v += NW * kWave) {
    const int c = V.colour[v];
    if (c < 0 || c >= k) S.bad_colour = 1;
    else if (v > 0 && V.colour[v - 1] > c) S.bad_layout = 1;
  }
  __syncthreads();
  if (S.bad_colour | S.bad_layout) {
    if (tid == 0) fail_job(a, g, S.bad_colour ? KZ_ECOLOUR : KZ_EINVAL);
    __syncthreads();
    return false;
  }
  for (int c = tid; c <= k; c += NW * kWave) {
    int lo = 0, hi = n;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (V.colour[mid] < c) lo = mid + 1;
      else hi = mid;
    }
    S.coff[c] = lo;
  }
  __syncthreads();
  if (tid == 0) {
    int w = 0;
    for (int c = 0; c < k; ++c) {
      S.soff[c] = w;
      const int s = S.coff[c + 1] - S.coff[c];
      for (int b = 0; 64 * b < s && w + b < kBatchR; ++b) {
        S.bcls[w + b] = (short)c;
        S.bstart[w + b] = (unsigned short)(S.coff[c] + 64 * b);
        S.blen[w + b] = (unsigned char)min(64, s - 64 * b);
      }
      w += (s + 63) / 64;
    }
    S.soff[k] = w;
    if (w != R) S.bad_layout = 1;
  }
  __syncthreads();
  if (S.bad_layout) {
    if (tid == 0) fail_job(a, g, KZ_EINVAL);
    __syncthreads();
    return false;
  }
  // the layout goes to the job too (helpers load it from there)
  BatchJob *J = V.J;
  for (int c = tid; c <= k; c += NW * kWave) {
    J->coff[c] = S.coff[c];
    J->soff[c] = S.soff[c];
  }
  for (int b = tid; b < R; b += NW * kWave) {
    J->bcls[b] = S.bcls[b];
    J->bstart[b] = S.bstart[b];
    J->blen[b] = S.blen[b];
  }
  // state: the rows, every vertex and block touched
  for (long long i = tid; i < (long long)n * R; i += NW * kWave) V.cur[i] = V.rows[i];
  for (int i = tid; i < kBatchN / 32; i += NW * kWave) {
    S.tc[i] = ~0u;
    S.tn[i] = 0;
  }
  for (int i = tid; i < kBatchR / 32; i += NW * kWave) {
    S.btc[i] = ~0u;
    S.btn[i] = 0;
  }
  if (tid == 0) {
    ast(&J->rounds, 0);
    ast(&J->tot_removed_v, 0ll);
    ast(&J->tot_removed_e, 0ll);
    ast(&J->tot_tests, 0ll);
    ast(&J->m, 0ll);
    int p0 = 1;
    if (a.session) {
      // above every pass number a workgroup may still hold for this slot
      // (after the wrap, numbers from over 2^23 passes ago: a launch ends
      // within its lease, and with it every copy in LDS, long before that)
      p0 = ald(&J->lastpass) + 1;
      if (p0 >= (1 << 23)) p0 = 1;
    }
    ast(&J->pass0, p0);
    ast(&J->lastpass, p0);
    S.job = g;
    S.pass = p0;
    S.pass0 = p0;
    S.prio = 0;
    S.removed_v = 0;
    S.removed_e = 0;
    S.tests = 0;
  }
  __syncthreads();
  return open_pass<NW>(a, V, S);
}

// Claims a run of unclaimed items of job g (thread 0; S.got = 0: none left).
// A workgroup joining a pass it did not list loads the job's layout and
// touched sets after an acquire fence.
template <int NW>
__device__ void claim(const BatchArgs &a, BatchLds &S, int g) {
  const int tid = threadIdx.x;
  BatchJob *J = a.jobs + g;
  // Every wave enters on S.got == 0, read after the previous barrier; thread
  // 0 rewrites S.got below, so it waits until each wave has made that read
  // (a late wave would otherwise see the new value, skip this function and
  // its barriers, and stay one barrier out of step with the others).
  __syncthreads();
  if (tid == 0) {
    unsigned long long old = __hip_atomic_load(&J->claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int got = 0, cp = 0;
    for (int tries = 0; tries < 64; ++tries) {
      const unsigned ni = (unsigned)(old >> kItemBits) & kItemMask, nx = (unsigned)old & kItemMask;
      if (nx >= ni) break;
      // guided run length: a share of what is left, between NW and 8*NW items
      const unsigned rem = ni - nx;
      const unsigned c = min(rem, max((unsigned)NW, min(8u * NW, rem / (2u * gridDim.x))));
      if (__hip_atomic_compare_exchange_strong(&J->claim, &old, old + c, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT)) {
        got = 1;
        cp = (int)(old >> (2 * kItemBits));
        S.base = (int)nx;
        S.cnt = (int)c;
        S.nitems = (int)ni;
        break;
      }
    }
    S.reload = 0;
    if (got) {
      if (!(S.job == g && S.pass == cp)) {
        acquire_agent();  // the pass was listed by another workgroup
        // a new job in the slot has another first pass: its layout differs
        const int p0 = ald(&J->pass0);
        S.reload = S.job != g || S.pass0 != p0 ? 2 : 1;
        S.pass0 = p0;
        S.job = g;
        S.pass = cp;
        S.shared = 1;
      }
      S.next_item = 0;
    }
    S.got = got;
  }
  __syncthreads();
  if (S.got && S.reload) {
    const kz_batch_graph G = job_desc(a, g);
    const int p = S.pass, nw = (G.n + 31) >> 5, nbw = (G.row_words + 31) >> 5;
    if (S.reload == 2) {
      for (int c = tid; c <= G.k; c += NW * kWave) {
        S.coff[c] = J->coff[c];
        S.soff[c] = J->soff[c];
      }
      for (int b = tid; b < G.row_words; b += NW * kWave) {
        S.bcls[b] = J->bcls[b];
        S.bstart[b] = J->bstart[b];
        S.blen[b] = J->blen[b];
      }
    }
    for (int i = tid; i < nw; i += NW * kWave) {
      S.tc[i] = ald(&J->touched[p & 1][i]);
      S.tn[i] = 0;
    }
    for (int i = tid; i < nbw; i += NW * kWave) {
      S.btc[i] = ald(&J->btouched[p & 1][i]);
      S.btn[i] = 0;
    }
    if (tid == 0) {
      S.prio = 0;
      S.removed_v = 0;
      S.removed_e = 0;
      S.tests = 0;
    }
    __syncthreads();
  }
}

// Reports a finished run.  Solo: the run was the pass.  Shared: merge the
// run's counts and touched bits into the job, then count the run's items
// done; the run that completes the pass returns true, after an acquire
// fence.
__device__ bool retire(const GView &V, BatchLds &S) {
  const int tid = threadIdx.x;
  if (!S.shared) {
    if (tid == 0) S.got = 0;
    __syncthreads();
    return true;
  }
  BatchJob *J = V.J;
  const int tnx = (S.pass + 1) & 1;
  const int nw = (V.n + 31) >> 5, nbw = (V.R + 31) >> 5;
  for (int i = tid; i < nw; i += blockDim.x) {
    const unsigned x = S.tn[i];
    if (x) {
      atomicOr(&J->touched[tnx][i], x);
      S.tn[i] = 0;
    }
  }
  for (int i = tid; i < nbw; i += blockDim.x) {
    const unsigned x = S.btn[i];
    if (x) {
      atomicOr(&J->btouched[tnx][i], x);
      S.btn[i] = 0;
    }
  }
  if (tid == 0) {
    if (S.removed_v) atomicAdd(&J->removed_v, S.removed_v);
    if (S.removed_e) atomicAdd(&J->removed_e, S.removed_e);
    if (S.tests) atomicAdd(&J->tests, S.tests);
    if (S.prio) atomicMax(&J->prio, S.prio);
    S.removed_v = 0;
    S.removed_e = 0;
    S.tests = 0;
    S.prio = 0;
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (tid == 0) {
    const unsigned add = (unsigned)S.cnt;
    release_agent();
    const unsigned now = __hip_atomic_fetch_add(&J->done, add, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + add;
    S.last = (int)now == S.nitems;
    // acquire what the other workgroups wrote (and drop this CU's cached
    // copies of the job's merged state)
    if (S.last) acquire_agent();
    S.got = 0;
  }
  __syncthreads();
  return S.last;
}

// The carrier: applies the changed tiles, closes the pass, and ends the job
// or opens the next pass.  Returns true when a next pass is open.
template <int NW>
__device__ bool carry(const BatchArgs &a, const GView &V, BatchLds &S) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  BatchJob *J = V.J;
  const int p = S.pass, R = V.R;
  const int nw = (V.n + 31) >> 5, nbw = (R + 31) >> 5;
  if (S.shared) {
    const int tnx = (p + 1) & 1;
    for (int i = tid; i < nw; i += NW * kWave) S.tn[i] = ald(&J->touched[tnx][i]);
    for (int i = tid; i < nbw; i += NW * kWave) S.btn[i] = ald(&J->btouched[tnx][i]);
    if (tid == 0) {
      S.removed_v = ald(&J->removed_v);
      S.removed_e = ald(&J->removed_e);
      S.tests = ald(&J->tests);
      S.prio = ald(&J->prio);
      S.nchanged = ald(&J->nchanged);
    }
    __syncthreads();
  }
  // apply: copy the changed tiles into the state
  const int nch = S.nchanged;
  for (int i = wid; i < nch; i += NW) {
    const int it = V.changed[i];
    const int X = it & kXMask, Y = (it >> kYShift) & kXMask;
    const int xs = S.bstart[X], xl = S.blen[X], ys = S.bstart[Y], yl = S.blen[Y];
    if (lane < xl) V.cur[(long long)(xs + lane) * R + Y] = V.nxt[(long long)(xs + lane) * R + Y];
    if (lane < yl) V.cur[(long long)(ys + lane) * R + X] = V.nxt[(long long)(ys + lane) * R + X];
  }
  if (tid == 0) {
    const long long rv = (long long)S.removed_v, re = (long long)S.removed_e;
    S.status = 0;
    if (p == 1 && S.prio)
      S.status = S.prio == P_EINVAL      ? KZ_EINVAL
                 : S.prio == P_ESELFLOOP ? KZ_ESELFLOOP
                 : S.prio == P_EASYM     ? KZ_EASYM
                                         : KZ_EILLEGAL;
    if (p == S.pass0) ast(&J->m, (long long)S.tests);
    ast(&J->tot_tests, ald(&J->tot_tests) + (long long)S.tests);
    ast(&J->tot_removed_v, ald(&J->tot_removed_v) + rv);
    ast(&J->tot_removed_e, ald(&J->tot_removed_e) + re);
    if (!S.status && rv + re > 0) ast(&J->rounds, ald(&J->rounds) + 1);
    S.end = S.status != 0 || rv + re == 0;
  }
  __syncthreads();
  if (S.end) {
    if (tid == 0) {
      if (S.status) fail_job(a, V.g, S.status);
      else end_job(a, V, p - S.pass0 + 1);
    }
    __syncthreads();
    return false;
  }
  // next pass: what this pass touched is what the next one tests
  for (int i = tid; i < kBatchN / 32; i += NW * kWave) {
    S.tc[i] = i < nw ? S.tn[i] : 0u;
    S.tn[i] = 0;
  }
  for (int i = tid; i < kBatchR / 32; i += NW * kWave) {
    S.btc[i] = i < nbw ? S.btn[i] : 0u;
    S.btn[i] = 0;
  }
  if (tid == 0) {
    S.pass = p + 1;
    S.prio = 0;
    S.removed_v = 0;
    S.removed_e = 0;
    S.tests = 0;
  }
  __syncthreads();
  return open_pass<NW>(a, V, S);
}

// Looks on the board for the shared pass with the most unclaimed items, if
// it has at least `least` of them; -1 otherwise.
__device__ int find_job(const BatchArgs &a, BatchLds &S, unsigned least) {
  const int tid = threadIdx.x;
  if (tid < kWave) {
    unsigned long long key = 0;
    // kBatchBoard entries per step: their loads, then their claim words', in flight together
    for (int base = 0; base <= a.board_mask; base += kBatchBoard) {
      int gs[kBatchBoard / kWave];
#pragma unroll
      for (int j = 0; j < kBatchBoard / kWave; ++j)
        gs[j] = __hip_atomic_load(&a.board[base + j * kWave + tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
      for (int j = 0; j < kBatchBoard / kWave; ++j) {
        if (gs[j] < 0) continue;
        const unsigned long long cw =
            __hip_atomic_load(&a.jobs[gs[j]].claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned ni = (unsigned)(cw >> kItemBits) & kItemMask, nx = (unsigned)cw & kItemMask;
        if (nx < ni && ni - nx >= least)
          key = max(key, ((unsigned long long)(ni - nx) << 32) | (unsigned)(gs[j] + 1));
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const unsigned long long o = (unsigned long long)__shfl_xor((long long)key, off, kWave);
      key = max(key, o);
    }
    if (tid == 0) S.pick = key ? (int)(key & 0xffffffffu) - 1 : -1;
  }
  __syncthreads();
  return S.pick;
}

// Session mode (thread 0): refreshes the device's copy of the host's
// request count.  The count lives in pinned host memory; one workgroup at a
// time reads it, at most every kHostPoll ticks.
__device__ void poll_host(const BatchArgs &a) {
  const unsigned long long now = wall_clock64();
  unsigned long long last = ald(a.hpoll);
  if (now - last < kHostPoll || !__hip_atomic_compare_exchange_strong(a.hpoll, &last, now, __ATOMIC_RELAXED,
                                                                      __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
    return;
  const unsigned long long hh = __hip_atomic_load(a.head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  // the copy is written after the count's load has returned (it is the
  // operand); a taker's own acquire orders its reads of the host tables
  if (hh > ald(a.dhead)) __hip_atomic_fetch_max(a.dhead, hh, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Session mode (thread 0): takes the next published request, if any, and
// returns its slot (S.ticket: its ticket), else -1.
__device__ int take_request(const BatchArgs &a, BatchLds &S) {
  poll_host(a);
  unsigned long long h = ald(a.dhead), q = ald(a.squeue);
  while (q < h) {
    if (__hip_atomic_compare_exchange_strong(a.squeue, &q, q + 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT)) {
      acquire_system();
      unsigned *e = a.ring + q % (unsigned long long)a.cap;
      unsigned slot = __hip_atomic_load(e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      // the host wrote the entry before the count; should the entry still
      // read as free, look again for a while rather than take a bad slot
      for (int i = 0; i < 4096 && slot >= (unsigned)a.G; ++i) {
        __builtin_amdgcn_s_sleep(8);
        acquire_system();
        slot = __hip_atomic_load(e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      }
      if (slot >= (unsigned)a.G) return -1;  // never observed: the request stays untaken for good
      S.ticket = __hip_atomic_load(a.htickets + slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      // the host may write the entry again once it sees it read
      __hip_atomic_store(e, kRingFree, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      return (int)slot;
    }
  }
  return -1;
}

template <int NW, int CH>
__global__ void __launch_bounds__(NW * 64) k_batch(BatchArgs a) {
  __shared__ BatchLds S;
  __shared__ unsigned long long sU[NW][CH][kBlk];
  __shared__ unsigned long long sU2[NW][CH][kBlk];
  const int tid = threadIdx.x;
  if (tid == 0) {
    S.job = -1;
    S.pass = 0;
    S.pass0 = 0;
    S.got = 0;
    S.queue_empty = 0;
  }
  __syncthreads();
  int job = -1;
  const unsigned long long born = wall_clock64();  // session mode: the lease runs from here
  unsigned long long idle0 = 0;  // thread 0: when this workgroup ran out of work
  int backoff = 1;                // idle polls sleep 1, 2, 4 or 8 times between looks
  for (;;) {
    if (job >= 0) {
      if (!S.got) claim<NW>(a, S, job);
      if (S.got) {
        const GView V = gview(a, job);
        run_items<NW, CH>(V, S, sU, sU2);
        if (retire(V, S) && !carry<NW>(a, V, S)) job = -1;
        continue;
      }
      job = -1;
    }
    // a shared pass with plenty of unclaimed items comes before a new graph
    if (!S.queue_empty) {
      job = find_job(a, S, 2u * NW);
      if (job >= 0) continue;
      __syncthreads();
      if (tid == 0) {
        if (a.session) {
          // past its lease a workgroup takes no new request, so the launch
          // ends and kernels queued behind it on the same hardware queue run
          const bool leased = a.lease_ticks && wall_clock64() - born > a.lease_ticks;
          S.gi = leased ? -1 : take_request(a, S);
        } else {
          const int t = atomicAdd(a.queue, 1);
          S.gi = t < a.G ? a.order[t] : -1;
          if (t >= a.G) S.queue_empty = 1;
        }
      }
      __syncthreads();
      const int g = S.gi;
      if (g >= 0) {
        if (start_job<NW>(a, S, g)) job = g;
        idle0 = 0;
        backoff = 1;
        continue;
      }
    }
    job = find_job(a, S, 1u);
    if (job >= 0) {
      idle0 = 0;
      backoff = 1;
      continue;
    }
    if (tid == 0) {
      const unsigned long long now = wall_clock64();
      if (!idle0) idle0 = now;
      // a session's workgroups stay for new requests until idle for idle_ticks
      S.quit = a.session ? now - idle0 > a.idle_ticks || (a.lease_ticks && now - born > a.lease_ticks)
                         : __hip_atomic_load(a.finished, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= a.G ||
                               now - idle0 > kIdleTicks;
    }
    __syncthreads();
    if (S.quit) break;
    // back off while idle: every look at the board is a few KiB of loads
    // that bypass the caches, and hundreds of idle workgroups looking at
    // once slow down the ones still working
    for (int i = 0; i < backoff; ++i) __builtin_amdgcn_s_sleep(32);
    backoff = backoff < 8 ? 2 * backoff : 8;
  }
}

// Orders the graphs by an estimate of their work, largest first (so the
// persistent workgroups finish together), or keeps the given order; resets
// the queue, the finished count and the board.  One workgroup, bitonic sort
// in LDS for up to kBatchSortMax graphs.
__global__ void __launch_bounds__(1024) k_batch_order(BatchArgs a, int lpt) {
  __shared__ unsigned long long key[kBatchSortMax];
  const int t = threadIdx.x, G = a.G;
  if (t == 0) {
    *a.queue = 0;
    *a.finished = 0;
  }
  for (int i = t; i <= a.board_mask; i += 1024) a.board[i] = -1;
  if (!lpt || G > kBatchSortMax) {
    for (int i = t; i < G; i += 1024) a.order[i] = i;
    return;
  }
  int P = 1;
  while (P < G) P <<= 1;
  for (int i = t; i < P; i += 1024) {
    unsigned long long cost = 0;
    if (i < G) {
      const kz_batch_graph gg = a.graphs[i];
      const long long R = gg.row_words > 0 ? gg.row_words : 0;
      cost = (unsigned long long)(R * R * 64LL * (gg.k > 2 ? gg.k : 1) + gg.n);
      if (cost > 0xffffffffull) cost = 0xffffffffull;
      key[i] = (~cost << 32) | (unsigned)i;  // ascending key = descending cost
    } else {
      key[i] = ~0ull;
    }
  }
  __syncthreads();
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = t; i < P; i += 1024) {
        const int j = i ^ stride;
        if (j > i) {
          const bool up = (i & size) == 0;
          const unsigned long long x = key[i], y = key[j];
          if ((x > y) == up) {
            key[i] = y;
            key[j] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = t; i < G; i += 1024) a.order[i] = (int)(key[i] & 0xffffffffu);
}

}  // namespace

void launch_batch(const BatchArgs &args, const BatchConfig &cfg, hipStream_t s) {
  BatchArgs a = args;
  if (a.board_mask <= 0) a.board_mask = kBatchBoard - 1;
  // a session's queue and board are set up once, when its server is made
  if (!a.session) hipLaunchKernelGGL(k_batch_order, dim3(1), dim3(1024), 0, s, a, cfg.lpt);
  const dim3 grid(cfg.workgroups);
#define KZ_B(NW, CH) hipLaunchKernelGGL((k_batch<NW, CH>), grid, dim3(NW * 64), 0, s, a)
  if (cfg.waves == 4) {
    if (cfg.chunk == 4) KZ_B(4, 4);
    else KZ_B(4, 8);
  } else if (cfg.waves == 8) {
    if (cfg.chunk == 4) KZ_B(8, 4);
    else KZ_B(8, 8);
  } else {
    KZ_B(16, 4);  // 16 waves with 8-class chunks would exceed the LDS and register budget
  }
#undef KZ_B
}

}  // namespace kzi
