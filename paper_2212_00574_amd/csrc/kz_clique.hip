// k-clique search on a (kernelized) legally k-coloured graph (gfx950): the
// search the kernel is handed to.  A k-clique holds one vertex of every
// class; the search returns the lexicographically smallest one (class 0's
// vertex first, then class 1's, ...) among the live vertices, or none.
//
// Roots are the pairs (v0, v1) of class 0 x class 1 in lexicographic order,
// handed out one at a time from an atomic counter; each wave runs a
// depth-first search from its root over classes 2, 3, ... in index order.
// The wave keeps the common neighbourhood of its current pick (AND of the
// picked rows and the live mask) for every depth on a stack in the
// workspace, lanes over row words, and extends a pick only when every class
// after it still holds a candidate.  The first clique a root's search meets
// is that root's smallest, and the smallest root with a clique holds the
// smallest clique overall: an atomic minimum over roots keeps it, and
// waves holding later roots stop as soon as it is known.  Nothing waits for
// anything, so the launch cannot deadlock.
#include "kz_internal.h"

namespace kzi {

namespace {

constexpr int kClqWaves = 4;        // waves per workgroup
constexpr int kClqMaxWaves = 2048;  // waves of one launch (stack slots)
constexpr long long kClqNone = 0x7fffffffffffffffLL;
constexpr int kClqLdsWords = 1024;  // per-wave LDS stack (k * R words) when it fits

struct ClqHdr {
  long long best;    // smallest root with a clique
  long long next;    // next root to hand out
  long long nodes;   // picks extended
  int bad_colour, bad_layout;
  int coff[kBatchK + 1], soff[kBatchK + 1];
};

// Layout from the sorted colours (one workgroup): class starts by binary
// search, segment offsets, and the checks (colours in range, sorted, row
// words = sum of the class segments).
__global__ void __launch_bounds__(256) k_clique_setup(const int32_t *__restrict__ colour, int n, int k, int R,
                                                      ClqHdr *h) {
  const int tid = threadIdx.x;
  if (tid == 0) {
    h->best = kClqNone;
    h->next = 0;
    h->nodes = 0;
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

// The smallest root with a clique so far, the same in every lane (lane 0's
// read, broadcast): the wave's control flow must not split on it.
__device__ __forceinline__ long long best_now(const ClqHdr *h) {
  const long long b = __hip_atomic_load(&h->best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return __shfl(b, 0, kWave);
}

// The search.  stack: kClqMaxWaves slots of k * R words; found: per slot the
// root (int64) and the k picks.
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

// LDS: the stack lives in LDS when it fits (k * R <= kClqLdsWords per wave).
template <bool LDS>
__global__ void __launch_bounds__(kClqWaves * 64) k_clique_search(const uint64_t *__restrict__ rows, int k, int R,
                                                                  const uint64_t *__restrict__ am, ClqHdr *h,
                                                                  uint64_t *__restrict__ stack,
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
  long long nodes = 0;
  found_root[slot] = kClqNone;
  for (;;) {
    long long r = 0;
    if (lane == 0) r = atomicAdd((unsigned long long *)&h->next, 1ull);
    r = __shfl(r, 0, kWave);
    if (r >= nroots || r > best_now(h)) break;
    const int v0 = coff[0] + (int)(r / s1);
    const int v1 = k > 1 ? coff[1] + (int)(r % s1) : -1;
    const uint64_t *r0 = rows + (long long)v0 * R;
    {
      const int l0 = v0 - coff[0];
      if (!((am[soff[0] + (l0 >> 6)] >> (l0 & 63)) & 1ull)) continue;
    }
    P[0] = v0;
    ++nodes;
    if (k == 1) {
      if (lane == 0) {
        found_root[slot] = r;
        found_pick[(long long)slot * k] = v0;
        atomicMin((long long *)&h->best, r);
      }
      break;
    }
    {
      const int l1 = v1 - coff[1], w1 = soff[1] + (l1 >> 6);
      if (!((am[w1] >> (l1 & 63)) & 1ull) || !((r0[w1] >> (l1 & 63)) & 1ull)) continue;
    }
    P[1] = v1;
    ++nodes;
    const uint64_t *r1 = rows + (long long)v1 * R;
    // depth 2: the common neighbourhood of v0, v1 over classes 2..k-1, each
    // of them non-empty
    uint64_t *c2 = cn + 2 * (long long)R;
    if (k > 2 && !extend_all(soff, 2, k, lane, c2, [&](int w) { return r0[w] & r1[w] & am[w]; })) continue;
    if (k == 2) {
      if (lane == 0) {
        found_root[slot] = r;
        found_pick[(long long)slot * k] = v0;
        found_pick[(long long)slot * k + 1] = v1;
        atomicMin((long long *)&h->best, r);
      }
      break;
    }
    int d = 2;
    if (lane == 0) P[2] = -1;
    bool done = false;
    int steps = 0;
    while (d >= 2 && !done) {
      // a smaller root already has a clique (looked up every 32 steps: the
      // load goes to memory)
      if ((++steps & 31) == 0 && best_now(h) < r) break;
      // next candidate of class d after P[d] in the common neighbourhood
      const uint64_t *cd = cn + (long long)d * R;
      const int cs = coff[d], ws0 = soff[d], ws1 = soff[d + 1];
      const int after = __shfl(P[d], 0, kWave);  // vertex or -1
      const int from = after < 0 ? 0 : after - cs + 1;
      int v = -1;
      for (int w0 = ws0 + (from >> 6); w0 < ws1 && v < 0; w0 += kWave) {
        const int w = w0 + lane;
        uint64_t x = w < ws1 ? cd[w] : 0ull;
        if (w == ws0 + (from >> 6) && (from & 63)) x &= ~0ull << (from & 63);
        const unsigned long long b = __ballot(x != 0ull);
        if (b) {
          const int f = __builtin_ctzll(b);
          const uint64_t xf = __shfl(x, f, kWave);
          v = cs + 64 * (w0 + f - ws0) + __builtin_ctzll(xf);
        }
      }
      if (v < 0) {
        --d;
        continue;
      }
      if (lane == 0) P[d] = v;
      ++nodes;
      if (d == k - 1) {
        if (lane == 0) {
          found_root[slot] = r;
          for (int c = 0; c < k; ++c) found_pick[(long long)slot * k + c] = P[c];
          atomicMin((long long *)&h->best, r);
        }
        done = true;
        break;
      }
      // extend: the common neighbourhood of the pick over classes d+1..k-1
      const uint64_t *rv = rows + (long long)v * R;
      uint64_t *cnext = cn + (long long)(d + 1) * R;
      if (extend_all(soff, d + 1, k, lane, cnext, [&](int w) { return cd[w] & rv[w]; })) {
        ++d;
        if (lane == 0) P[d] = -1;
      }
    }
    if (done) break;
  }
  if (lane == 0 && nodes) atomicAdd((unsigned long long *)&h->nodes, (unsigned long long)nodes);
}

// Copies the picks of the smallest root's slot to the output (all -1 when
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
  size_t hdr, am, stack, root, pick, total;
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
  if (k > kBatchK) return done(KZ_ETOOLARGE);
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
  long long *froot = (long long *)(base + z.root);
  int *fpick = (int *)(base + z.pick);
  hipLaunchKernelGGL(k_clique_setup, dim3(1), dim3(256), 0, s, colour, n, k, R, h);
  hipLaunchKernelGGL(k_clique_alive, dim3((R + 255) / 256 > 0 ? (R + 255) / 256 : 1), dim3(256), 0, s, vmask, k, R,
                     h, am);
  if ((long long)k * R <= kClqLdsWords)
    hipLaunchKernelGGL(k_clique_search<true>, dim3(kClqMaxWaves / kClqWaves), dim3(kClqWaves * 64), 0, s, g->rows,
                       k, R, am, h, stack, froot, fpick);
  else
    hipLaunchKernelGGL(k_clique_search<false>, dim3(kClqMaxWaves / kClqWaves), dim3(kClqWaves * 64), 0, s,
                       g->rows, k, R, am, h, stack, froot, fpick);
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
