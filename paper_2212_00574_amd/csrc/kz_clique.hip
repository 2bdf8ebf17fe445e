// k-clique search on a (kernelized) legally k-coloured graph (gfx950): the
// search the kernel is handed to.  A k-clique holds one vertex of every
// class; the search returns the lexicographically smallest one (class 0's
// vertex first, then class 1's, ...) among the live vertices, or none.
//
// Roots are the pairs (v0, v1) of class 0 x class 1 in lexicographic order,
// handed out one at a time from an atomic counter.  The children of a root
// are its class-2 vertices j, each searched depth first over classes 3, 4,
// ... in index order.  The wave that took a root searches its children in
// order itself; once it has extended kClqShareAfter picks below the root it
// opens the remaining children on its share word, and from then on any wave
// -- its own, or a helper (a wave of the first kClqHelperBlocks blocks that
// has run out of roots) -- takes the next kClqTake children with one atomic
// add.  A wave keeps the common neighbourhood of its current pick (AND of
// the picked rows and the live mask) for every depth on a stack, lanes over
// row words, and extends a pick only when every class after it still holds
// a candidate.  The key of a child is (root, j) in lexicographic order; the
// first clique a child's search meets is that child's smallest, so the
// smallest key with a clique holds the smallest clique overall: an atomic
// minimum over keys keeps it, and waves holding larger keys stop as soon as
// it is known.  Helpers only poll, a bounded number of times in a row, for
// work opened by waves that are already running; nothing else waits, so the
// launch cannot deadlock.
#include "kz_internal.h"

namespace kzi {

namespace {

constexpr int kClqWaves = 4;        // waves per workgroup
constexpr int kClqMaxWaves = 2048;  // waves of one launch (stack slots)
constexpr long long kClqNone = 0x7fffffffffffffffLL;
constexpr int kClqLdsWords = 1024;  // per-wave LDS stack (k * R words) when it fits
// share word of a slot: root << kClqSubBits | next child, or negative (no
// open children).  Vertices stay below kClqMaxN so that roots (< 2^40),
// children (< 2^21, plus at most one overshooting add of kClqTake per wave)
// and keys (root * s2 + j < 2^63) all fit.
constexpr int kClqSubBits = 22;
constexpr long long kClqSubMask = (1ll << kClqSubBits) - 1;
constexpr long long kClqClosed = -(1ll << 62);
constexpr int kClqMaxN = 1 << 21;
// a helper with no open child looks again at most this many times in a row
// (about 3.4 us apart) before it leaves: long enough for the long roots
// taken just before it to open, short enough not to hold the compute units
// from other work (other searches) while the last subtrees finish
constexpr int kClqIdlePolls = 32;
// a root opens its remaining children once its own wave has extended this
// many picks below it: short subtrees stay with their wave, long ones are
// shared
constexpr int kClqShareAfter = 64;
// only the waves of the first blocks help once the roots are gone; the rest
// leave, as their slots may serve other work
constexpr int kClqHelperBlocks = 64;
constexpr int kClqMaskWords = kClqMaxWaves / 64;  // bit t: slot t has an open root
constexpr int kClqTake = 8;  // children handed out per take (one atomic)

struct ClqHdr {
  long long best;    // smallest key with a clique
  long long next;    // next root to hand out
  long long nodes;   // picks extended
  int active;        // waves started and still taking roots
  int bad_colour, bad_layout;
  int coff[kBatchK + 1], soff[kBatchK + 1];
};

// Layout from the sorted colours (one workgroup): class starts by binary
// search, segment offsets, and the checks (colours in range, sorted, row
// words = sum of the class segments).
__global__ void __launch_bounds__(256) k_clique_setup(const int32_t *__restrict__ colour, int n, int k, int R,
                                                      ClqHdr *h, long long *__restrict__ share,
                                                      unsigned long long *__restrict__ omask) {
  const int tid = threadIdx.x;
  for (int t = tid; t < kClqMaxWaves; t += blockDim.x) share[t] = kClqClosed;
  if (tid < kClqMaskWords) omask[tid] = 0ull;
  if (tid == 0) {
    h->best = kClqNone;
    h->next = 0;
    h->nodes = 0;
    h->active = 0;
    h->bad_colour = 0;
    h->bad_layout = 0;
  }
  __syncthreads();
  for (int v = tid; v < n; v += blockDim.x) {
    const int c = colour[v];
    if (c < 0 || c >= k) h->bad_colour = 1;
    else if (v > 0 && colour[v - 1] > c) h->bad_layout = 1;
  }
  __syncthreads();
  if (h->bad_colour || h->bad_layout) return;
  for (int c = tid; c <= k; c += blockDim.x) {
    int lo = 0, hi = n;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (colour[mid] < c) lo = mid + 1;
      else hi = mid;
    }
    h->coff[c] = lo;
  }
  __syncthreads();
  if (tid == 0) {
    int w = 0;
    for (int c = 0; c < k; ++c) {
      h->soff[c] = w;
      w += (h->coff[c + 1] - h->coff[c] + 63) / 64;
    }
    h->soff[k] = w;
    if (w != R) h->bad_layout = 1;
  }
}

// The live mask in the rows' layout (bit j of word w of class c is vertex
// coff[c] + 64 (w - soff[c]) + j).  One thread per word.
__global__ void __launch_bounds__(256) k_clique_alive(const uint8_t *__restrict__ vmask, int k, int R,
                                                      const ClqHdr *__restrict__ h, uint64_t *__restrict__ am) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= R || h->bad_colour || h->bad_layout) return;
  int c = 0;
  while (c + 1 < k && h->soff[c + 1] <= w) ++c;
  const int v0 = h->coff[c] + 64 * (w - h->soff[c]), s_end = h->coff[c + 1];
  unsigned long long x = 0;
  for (int j = 0; j < 64 && v0 + j < s_end; ++j)
    if (!vmask || vmask[v0 + j]) x |= 1ull << j;
  am[w] = x;
}

// The smallest key with a clique so far, the same in every lane (lane 0's
// read, broadcast): the wave's control flow must not split on it.
__device__ __forceinline__ long long best_now(const ClqHdr *h) {
  const long long b = __hip_atomic_load(&h->best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return __shfl(b, 0, kWave);
}

// Takes the next kClqTake children of the root on a share word: (root, j),
// the first of them, or false when the word is closed or its children are
// all taken.  The add's old value decides, never an earlier read: an add
// that lands after the owner moved on to a new root takes that root's
// children; one past the last child only raises j further (at most one add
// per wave, far below the root bits).
__device__ __forceinline__ bool take_child(long long *share, long long S2, long long &r, int &j) {
  long long old = 0;
  if ((threadIdx.x & 63) == 0)
    old = __hip_atomic_fetch_add(share, (long long)kClqTake, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  old = __shfl(old, 0, kWave);
  if (old < 0 || (old & kClqSubMask) >= S2) return false;
  r = old >> kClqSubBits;
  j = (int)(old & kClqSubMask);
  return true;
}

// Writes the next depth's common neighbourhood over the words [lo, hi) of
// the classes after the pick (x(w) gives a word) and tells whether every one
// of those classes keeps a candidate.  The words load together, lanes over
// words; lane l then watches class c0 + l: whether the ballot of non-zero
// words has a bit in its word range.
template <typename F>
__device__ __forceinline__ bool extend_all(const int *soff, int c0, int k, int lane, uint64_t *out, F x) {
  const int lo = soff[c0], hi = soff[k];
  const int c = c0 + lane;
  const bool mine = c < k;
  const int cl = mine ? soff[c] : 0, ch = mine ? soff[c + 1] : 0;
  bool seen = false;
  for (int w0 = lo; w0 < hi; w0 += kWave) {
    const int w = w0 + lane;
    uint64_t v = 0;
    if (w < hi) {
      v = x(w);
      out[w] = v;
    }
    const unsigned long long nz = __ballot(v != 0ull);
    if (mine && !seen && cl < w0 + kWave && ch > w0) {
      const int a = max(cl, w0) - w0, b = min(ch, w0 + kWave) - w0;
      const unsigned long long m = (b - a == 64 ? ~0ull : ((1ull << (b - a)) - 1)) << a;
      seen = (nz & m) != 0ull;
    }
  }
  return __ballot(mine && !seen) == 0ull;
}

// The search.  stack: kClqMaxWaves slots of k * R words; share: a word per
// slot; omask: the open-slot bit mask; found: per slot the key (int64) and
// the k picks.
// LDS: the stack lives in LDS when it fits (k * R <= kClqLdsWords per wave).
template <bool LDS>
__global__ void __launch_bounds__(kClqWaves * 64) k_clique_search(const uint64_t *__restrict__ rows, int k, int R,
                                                                  const uint64_t *__restrict__ am, ClqHdr *h,
                                                                  uint64_t *__restrict__ stack,
                                                                  long long *__restrict__ share,
                                                                  unsigned long long *__restrict__ omask,
                                                                  long long *__restrict__ found_root,
                                                                  int *__restrict__ found_pick) {
  __shared__ uint64_t lstack[LDS ? kClqWaves * kClqLdsWords : 1];
  __shared__ int pos[kClqWaves][kBatchK];
  __shared__ int coff_s[kBatchK + 1], soff_s[kBatchK + 1];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int slot = blockIdx.x * kClqWaves + wid;
  if (h->bad_colour || h->bad_layout) return;
  for (int c = threadIdx.x; c <= k; c += blockDim.x) {
    coff_s[c] = h->coff[c];
    soff_s[c] = h->soff[c];
  }
  __syncthreads();
  const int *coff = coff_s, *soff = soff_s;
  int *P = pos[wid];
  uint64_t *cn = LDS ? lstack + wid * kClqLdsWords : stack + (long long)slot * k * R;
  const int s0 = coff[1] - coff[0];
  const int s1 = k > 1 ? coff[2] - coff[1] : 1;
  const long long nroots = (long long)s0 * s1;
  // children per root: the class-2 vertices (one pseudo-child below k = 3)
  const long long S2 = k > 2 ? max(coff[3] - coff[2], 1) : 1;
  long long nodes = 0;
  found_root[slot] = kClqNone;
  if (lane == 0) atomicAdd(&h->active, 1);

  // the stack's words are written by one lane and read by others: in
  // global memory the wave waits for its writes before it reads them back
  auto stack_written = [&]() {
    if constexpr (!LDS) __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  };

  auto record = [&](long long key) {
    if (lane == 0) {
      found_root[slot] = key;
      for (int c = 0; c < k; ++c) found_pick[(long long)slot * k + c] = P[c];
      atomicMin((long long *)&h->best, key);
    }
  };

  // The first candidate of class d at or after local index `from` in the
  // common neighbourhood of depth d (a local index), or -1.
  auto next_cand = [&](int d, int from) -> int {
    const uint64_t *cd = cn + (long long)d * R;
    const int ws0 = soff[d], ws1 = soff[d + 1];
    for (int w0 = ws0 + (from >> 6); w0 < ws1; w0 += kWave) {
      const int w = w0 + lane;
      uint64_t x = w < ws1 ? cd[w] : 0ull;
      if (w == ws0 + (from >> 6) && (from & 63)) x &= ~0ull << (from & 63);
      const unsigned long long b = __ballot(x != 0ull);
      if (b) {
        const int f = __builtin_ctzll(b);
        const uint64_t xf = __shfl(x, f, kWave);
        return 64 * (w0 + f - ws0) + __builtin_ctzll(xf);
      }
    }
    return -1;
  };

  // Depth-first search below the picks P[0..2] of child `key`, from the
  // common neighbourhood of depth 3 on the stack: true at the first clique
  // (the child's smallest), false when the subtree is exhausted or a smaller
  // key already has a clique (looked up every 32 steps: the load goes to
  // memory).
  auto dfs = [&](long long key) -> bool {
    int d = 3;
    if (lane == 0) P[3] = -1;
    int steps = 0;
    while (d >= 3) {
      if ((++steps & 31) == 0 && best_now(h) < key) return false;
      // next candidate of class d after P[d] in the common neighbourhood
      const uint64_t *cd = cn + (long long)d * R;
      const int after = __shfl(P[d], 0, kWave);  // vertex or -1
      const int from = after < 0 ? 0 : after - coff[d] + 1;
      const int lv = next_cand(d, from);
      const int v = lv < 0 ? -1 : coff[d] + lv;
      if (v < 0) {
        --d;
        continue;
      }
      if (lane == 0) P[d] = v;
      ++nodes;
      if (d == k - 1) return true;
      // extend: the common neighbourhood of the pick over classes d+1..k-1
      const uint64_t *rv = rows + (long long)v * R;
      uint64_t *cnext = cn + (long long)(d + 1) * R;
      const bool ok = extend_all(soff, d + 1, k, lane, cnext, [&](int w) { return cd[w] & rv[w]; });
      stack_written();
      if (ok) {
        ++d;
        if (lane == 0) P[d] = -1;
      }
    }
    return false;
  };

  // The common neighbourhood of root r's pair over classes 2..k-1 at depth
  // 2 of the stack, with P[0], P[1]: false when a class is left without a
  // candidate (k >= 3).
  auto open_root = [&](long long r) -> bool {
    const int v0 = coff[0] + (int)(r / s1), v1 = coff[1] + (int)(r % s1);
    const uint64_t *r0 = rows + (long long)v0 * R, *r1 = rows + (long long)v1 * R;
    if (lane == 0) {
      P[0] = v0;
      P[1] = v1;
    }
    const bool ok = extend_all(soff, 2, k, lane, cn + 2 * (long long)R, [&](int w) { return r0[w] & r1[w] & am[w]; });
    stack_written();
    return ok;
  };

  // Child j of the open root r: the class-2 vertex coff[2] + j, if it is in
  // the pair's common neighbourhood, and the search below it.
  auto child = [&](long long r, int j) -> bool {
    const uint64_t *c2 = cn + 2 * (long long)R;
    if (!((c2[soff[2] + (j >> 6)] >> (j & 63)) & 1ull)) return false;
    const long long key = r * S2 + j;
    const int v2 = coff[2] + j;
    if (lane == 0) P[2] = v2;
    ++nodes;
    if (k == 3) {
      record(key);
      return true;
    }
    const uint64_t *rv = rows + (long long)v2 * R;
    const bool ok = extend_all(soff, 3, k, lane, cn + 3 * (long long)R, [&](int w) { return c2[w] & rv[w]; });
    stack_written();
    if (!ok) return false;
    if (!dfs(key)) return false;
    record(key);
    return true;
  };

  // The children j0 .. j0 + kClqTake - 1 of root r in order, up to the
  // first clique: true then.
  auto children = [&](long long r, int j0) -> bool {
    const int j1 = (int)min((long long)j0 + kClqTake, S2);
    for (int j = j0; j < j1; ++j)
      if (child(r, j)) return true;
    return false;
  };

  bool done = false;
  // own roots, in the order of the counter
  for (;;) {
    long long r = 0;
    if (lane == 0) r = atomicAdd((unsigned long long *)&h->next, 1ull);
    r = __shfl(r, 0, kWave);
    if (r >= nroots || r * S2 > best_now(h)) break;
    const int v0 = coff[0] + (int)(r / s1);
    const int v1 = k > 1 ? coff[1] + (int)(r % s1) : -1;
    const uint64_t *r0 = rows + (long long)v0 * R;
    {
      const int l0 = v0 - coff[0];
      if (!((am[soff[0] + (l0 >> 6)] >> (l0 & 63)) & 1ull)) continue;
    }
    if (lane == 0) P[0] = v0;
    ++nodes;
    if (k == 1) {
      record(r);
      done = true;
      break;
    }
    {
      const int l1 = v1 - coff[1], w1 = soff[1] + (l1 >> 6);
      if (!((am[w1] >> (l1 & 63)) & 1ull) || !((r0[w1] >> (l1 & 63)) & 1ull)) continue;
    }
    if (lane == 0) P[1] = v1;
    ++nodes;
    if (k == 2) {
      record(r);
      done = true;
      break;
    }
    if (!open_root(r)) continue;
    // the children in order: the candidates one after another by this wave
    // while the root is young, then -- once it has cost kClqShareAfter picks
    // -- the rest opened to every wave and taken like any helper takes them
    const long long young = nodes + kClqShareAfter;
    bool shared = false;
    int j = 0;
    while (!done) {
      if (!shared) {
        j = next_cand(2, j);
        if (j < 0 || r * S2 + j > best_now(h)) break;
        done = child(r, j);
        ++j;
        if (!done && nodes > young && j < S2) {
          shared = true;
          if (lane == 0) {
            __hip_atomic_store(&share[slot], (r << kClqSubBits) | j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            atomicOr(&omask[slot >> 6], 1ull << (slot & 63));
          }
        }
      } else {
        long long rr;
        int j0;
        if (!take_child(&share[slot], S2, rr, j0) || rr * S2 + j0 > best_now(h)) break;
        done = children(rr, j0);
      }
    }
    if (shared && lane == 0) {
      atomicAnd(&omask[slot >> 6], ~(1ull << (slot & 63)));
      __hip_atomic_store(&share[slot], kClqClosed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (done) break;
  }

  if (lane == 0) atomicSub(&h->active, 1);

  // out of roots: the waves of the first kClqHelperBlocks blocks help with
  // the open children, the smallest key first.  With none open, sleep and
  // look again, until no started wave is taking roots any more or
  // kClqIdlePolls looks in a row found nothing (waves not yet started are
  // not waited for: they find the roots gone and help, or leave, in turn).
  long long have = -1;  // the root whose pair neighbourhood is on the stack
  int polls = 0;
  while (!done && k > 2 && blockIdx.x < kClqHelperBlocks) {
    long long bestkey = kClqNone;
    int bslot = -1;
    {
      // lane l reads word l of the open-slot mask, then the share words of
      // its set bits
      unsigned long long bits =
          lane < kClqMaskWords ? __hip_atomic_load(&omask[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0ull;
      while (bits) {
        const int t = 64 * lane + __builtin_ctzll(bits);
        bits &= bits - 1;
        const long long v = __hip_atomic_load(&share[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const long long key =
            v >= 0 && (v & kClqSubMask) < S2 ? (v >> kClqSubBits) * S2 + (v & kClqSubMask) : kClqNone;
        if (key < bestkey) {
          bestkey = key;
          bslot = t;
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const long long ok = __shfl_xor(bestkey, off, kWave);
        const int os = __shfl_xor(bslot, off, kWave);
        if (ok < bestkey || (ok == bestkey && os < bslot)) {
          bestkey = ok;
          bslot = os;
        }
      }
    }
    if (bestkey != kClqNone && bestkey <= best_now(h)) {
      polls = 0;  // look again at once after this child
      long long r;
      int j0;
      if (!take_child(&share[bslot], S2, r, j0)) continue;  // taken meanwhile
      if (r * S2 + j0 > best_now(h)) continue;
      if (r != have) {
        open_root(r);  // true: the owner opened it
        have = r;
      }
      done = children(r, j0);
      continue;
    }
    if (polls >= kClqIdlePolls ||
        __shfl(__hip_atomic_load(&h->active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), 0, kWave) == 0)
      break;
    __builtin_amdgcn_s_sleep(127);
    ++polls;
  }
  if (lane == 0 && nodes) atomicAdd((unsigned long long *)&h->nodes, (unsigned long long)nodes);
}

// Copies the picks of the smallest key's slot to the output (all -1 when
// there is no clique).
__global__ void k_clique_final(int k, const ClqHdr *__restrict__ h, const long long *__restrict__ found_root,
                               const int *__restrict__ found_pick, int slots, int32_t *__restrict__ clique) {
  const long long best = h->best;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (best == kClqNone) {
    if (t < k) clique[t] = -1;
    return;
  }
  if (t < slots && found_root[t] == best)
    for (int c = 0; c < k; ++c) clique[c] = found_pick[(long long)t * k + c];
}

struct ClqWs {
  size_t hdr, am, stack, share, omask, root, pick, total;
};

ClqWs clique_ws(int k, int R) {
  ClqWs z{};
  size_t o = 0;
  auto take = [&o](size_t b) {
    const size_t at = o;
    o += (b + 255) / 256 * 256;
    return at;
  };
  z.hdr = take(sizeof(ClqHdr));
  z.am = take(sizeof(uint64_t) * (size_t)(R > 0 ? R : 1));
  z.stack = take(sizeof(uint64_t) * (size_t)kClqMaxWaves * (size_t)k * (size_t)R);
  z.share = take(sizeof(long long) * kClqMaxWaves);
  z.omask = take(sizeof(uint64_t) * kClqMaskWords);
  z.root = take(sizeof(long long) * kClqMaxWaves);
  z.pick = take(sizeof(int) * (size_t)kClqMaxWaves * (size_t)k);
  z.total = o;
  return z;
}

}  // namespace
}  // namespace kzi

extern "C" {

int kz_clique_workspace_bytes(const kz_graph *g, int32_t k, size_t *bytes) {
  if (!g || !bytes || g->format != KZ_BITSET_U64 || k < 1 || k > kzi::kBatchK || g->n < 0 || g->row_words < 0)
    return KZ_EINVAL;
  *bytes = kzi::clique_ws(k, g->row_words).total;
  return KZ_OK;
}

int kz_find_clique(kz_ctx *ctx, const kz_graph *g, const int32_t *colour, int32_t k, const uint8_t *vmask, void *ws,
                   size_t ws_bytes, int32_t *clique, void *stream, kz_clique_result *res) {
  using namespace kzi;
  kz_clique_result r{};
  auto done = [&](int st) {
    r.status = st;
    if (res) *res = r;
    return st;
  };
  if (!ctx || !g || g->format != KZ_BITSET_U64 || k < 1 || g->n < 0 || g->row_words < 0) return done(KZ_EINVAL);
  if (k > kBatchK || g->n >= kClqMaxN) return done(KZ_ETOOLARGE);
  const int n = g->n, R = g->row_words;
  if (n > 0 && (!g->rows || !colour || !clique || !ws || (uintptr_t)ws % 256)) return done(KZ_EINVAL);
  if (n == 0) {  // no vertex: no clique
    if (clique && hipMemsetAsync(clique, 0xff, sizeof(int32_t) * (size_t)k, (hipStream_t)stream) != hipSuccess)
      return done(KZ_EHIP);
    return done(KZ_OK);
  }
  const ClqWs z = clique_ws(k, R);
  if (ws_bytes < z.total) return done(KZ_EWORKSPACE);
  if (hipSetDevice(ctx->device) != hipSuccess) return done(KZ_EHIP);
  hipStream_t s = (hipStream_t)stream;
  char *base = (char *)ws;
  ClqHdr *h = (ClqHdr *)(base + z.hdr);
  uint64_t *am = (uint64_t *)(base + z.am);
  uint64_t *stack = (uint64_t *)(base + z.stack);
  long long *share = (long long *)(base + z.share);
  unsigned long long *omask = (unsigned long long *)(base + z.omask);
  long long *froot = (long long *)(base + z.root);
  int *fpick = (int *)(base + z.pick);
  hipLaunchKernelGGL(k_clique_setup, dim3(1), dim3(256), 0, s, colour, n, k, R, h, share, omask);
  hipLaunchKernelGGL(k_clique_alive, dim3((R + 255) / 256 > 0 ? (R + 255) / 256 : 1), dim3(256), 0, s, vmask, k, R,
                     h, am);
  if ((long long)k * R <= kClqLdsWords)
    hipLaunchKernelGGL(k_clique_search<true>, dim3(kClqMaxWaves / kClqWaves), dim3(kClqWaves * 64), 0, s, g->rows,
                       k, R, am, h, stack, share, omask, froot, fpick);
  else
    hipLaunchKernelGGL(k_clique_search<false>, dim3(kClqMaxWaves / kClqWaves), dim3(kClqWaves * 64), 0, s,
                       g->rows, k, R, am, h, stack, share, omask, froot, fpick);
  hipLaunchKernelGGL(k_clique_final, dim3((kClqMaxWaves + 255) / 256), dim3(256), 0, s, k, h, froot, fpick,
                     kClqMaxWaves, clique);
  ClqHdr *hh = (ClqHdr *)ctx->pinned;
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(hh, h, sizeof(ClqHdr), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return done(KZ_EHIP);
  if (hh->bad_colour) return done(KZ_ECOLOUR);
  if (hh->bad_layout) return done(KZ_EINVAL);
  r.found = hh->best != kClqNone;
  r.nodes = hh->nodes;
  const long long nroots = (long long)(hh->coff[1] - hh->coff[0]) * (k > 1 ? hh->coff[2] - hh->coff[1] : 1);
  r.roots = hh->next < nroots ? hh->next : nroots;
  return done(KZ_OK);
}

}  // extern "C"
