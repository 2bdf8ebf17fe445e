// Dominance reductions (thesis section 4.3, Definitions 4.3.1 and 4.3.2,
// Algorithms 1 and 2) on plain bit rows (gfx950).
//
// The algorithms are sequential sweeps whose deletions are visible to every
// later test, repeated until a sweep deletes nothing.  One workgroup runs a
// graph's whole fixpoint on the device (one launch, no host round trip):
// the sweep stays sequential over its steps, and each step's tests run in
// parallel over the workgroup's threads.
//
// Vertex dominance, step b: b deletes every node it dominates.  The set is
// the one b dominates at the start of the step: deleting a dominated a
// cannot make another node dominated by the same b (a node adjacent to a is
// in N(a), so in N(b), so adjacent to b), and the nodes b dominates are
// pairwise non-adjacent, so the edges removed are the sum of their degrees.
//
// Edge dominance, step a: the pairs (a, u), u in N(a), in index order; the
// edge {a,u} goes when some b in N(u), b != a, b not in N(a), sees all of
// N(a) & N(u).  Within the step only N(a) changes (it loses the u's already
// deleted: D), and the test is monotone in D -- W = N(a) & N(u) shrinks, the
// candidates N(u) \ N(a) grow, N(b) stays (it can only lose a, which is not
// in W).  So u is deleted iff its test holds with D restricted to the u's
// before it, a recursion with one solution, reached by parallel passes that
// start from D = {} and add every u whose test holds, until none is added.
#include "kz_internal.h"

namespace kzi {

namespace {

constexpr int kDomMaxWords = 1024;  // rows of at most 1024 words (n <= 65536)

struct DomHdr {
  long long dirs;    // set bits of the input (twice the edges)
  long long dv, de;  // deleted vertices, edges
  long long sweeps;  // sweeps that deleted something
  long long events;  // steps (vertex) or edges (edge) that deleted something
  long long passes;  // edge: parallel passes over a step's neighbours
  int prio;          // worst input problem (P_*)
  int pad[3];
};

__global__ void k_dom_init(DomHdr *h) {
  if (threadIdx.x == 0) {
    h->dirs = 0;
    h->dv = 0;
    h->de = 0;
    h->sweeps = 0;
    h->events = 0;
    h->passes = 0;
    h->prio = P_NONE;
  }
}

// Copies the rows into the state, sets every node alive, counts the set
// bits and checks the input: no bit at or beyond n, no self-loop, every bit
// mirrored.  One thread per row word.
__global__ void __launch_bounds__(256) k_dom_setup(const uint64_t *__restrict__ rows, uint64_t *__restrict__ st,
                                                   uint8_t *__restrict__ alive, int n, int R, DomHdr *h) {
  const long long total = (long long)n * R;
  const long long stride = (long long)gridDim.x * blockDim.x;
  unsigned long long cnt = 0;
  int pr = P_NONE;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int v = (int)(i / R), w = (int)(i % R);
    unsigned long long x = rows[i];
    st[i] = x;
    if (w == 0) alive[v] = 1;
    cnt += __popcll(x);
    const long long base = 64LL * w;
    if (base >= n) {
      if (x) pr = max(pr, (int)P_EINVAL);
      continue;
    }
    if (base + 64 > n) {
      const int keep = (int)(n - base);
      if (x >> keep) pr = max(pr, (int)P_EINVAL);
      x &= (1ull << keep) - 1;
    }
    while (x) {
      const int t = (int)base + __builtin_ctzll(x);
      x &= x - 1;
      if (t == v) pr = max(pr, (int)P_ESELFLOOP);
      else if (!((rows[(long long)t * R + (v >> 6)] >> (v & 63)) & 1ull)) pr = max(pr, (int)P_EASYM);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    cnt += __shfl_xor(cnt, off, kWave);
    pr = max(pr, __shfl_xor(pr, off, kWave));
  }
  if ((threadIdx.x & 63) == 0) {
    if (cnt) atomicAdd((unsigned long long *)&h->dirs, cnt);
    if (pr != P_NONE) atomicMax(&h->prio, pr);
  }
}

// ---- vertex dominance (Definition 4.3.1): the whole fixpoint, one workgroup
//
// Most steps delete nothing, so the waves first test consecutive steps at
// once (wave w: does node b0 + w dominate anyone?), on the same graph; the
// first step in sweep order that does is then run in full by the whole
// workgroup, and the scan goes on right after it.  Steps before it saw the
// graph the sequential sweep would have shown them (nothing was deleted in
// between); the results of the steps after it are dropped.
__global__ void __launch_bounds__(1024) k_dom_vertex_run(uint64_t *__restrict__ st, uint8_t *__restrict__ alive,
                                                         int n, int R, DomHdr *h) {
  __shared__ uint64_t AL[kDomMaxWords];  // live nodes (bit v of word v / 64)
  __shared__ uint64_t rb[kDomMaxWords], D[kDomMaxWords];
  __shared__ int dw[kDomMaxWords];       // the words of D that hold a deleted node
  __shared__ unsigned long long nv, ne;
  __shared__ int any_sweep, ndw;
  __shared__ unsigned hits;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int nwaves = blockDim.x >> 6;
  if (h->prio != P_NONE) return;
  for (int w = tid; w < R; w += blockDim.x) {
    const int lo = 64 * w;
    AL[w] = lo + 64 <= n ? ~0ull : lo < n ? (1ull << (n - lo)) - 1 : 0ull;
  }
  long long sweeps = 0, steps = 0;
  for (;;) {
    // every thread has read the previous sweep's flag before it is reset
    __syncthreads();
    if (tid == 0) any_sweep = 0;
    int b0 = 0;
    while (b0 < n) {
      if (tid == 0) hits = 0;
      __syncthreads();
      // scan: wave w tests step b0 + w; its lanes take the row words of the
      // live non-neighbours of b and test those nodes one by one
      {
        const int b = b0 + wid;
        if (b < n && ((AL[b >> 6] >> (b & 63)) & 1ull)) {
          const uint64_t *rbg = st + (long long)b * R;
          bool hit = false;
          for (int w = lane; w < R && !hit; w += kWave) {
            uint64_t cand = AL[w] & ~rbg[w];
            if (w == (b >> 6)) cand &= ~(1ull << (b & 63));
            while (cand && !hit) {
              const int a = 64 * w + __builtin_ctzll(cand);
              cand &= cand - 1;
              const uint64_t *ra = st + (long long)a * R;
              bool sub = true;
              for (int w2 = 0; w2 < R; ++w2) {
                if (ra[w2] & ~rbg[w2]) {
                  sub = false;
                  break;
                }
              }
              hit = sub;
            }
          }
          if (__ballot(hit) != 0ull && lane == 0) atomicOr(&hits, 1u << wid);
        }
      }
      __syncthreads();
      const unsigned hm = hits;
      if (!hm) {
        b0 += nwaves;
        continue;
      }
      const int b = b0 + __builtin_ctz(hm);
      // the step in full: every node b dominates, deleted with its edges
      for (int w = tid; w < R; w += blockDim.x) {
        rb[w] = st[(long long)b * R + w];
        D[w] = 0;
      }
      if (tid == 0) {
        nv = 0;
        ne = 0;
        ndw = 0;
      }
      __syncthreads();
      for (int w = tid; w < R; w += blockDim.x) {
        uint64_t cand = AL[w] & ~rb[w];
        if (w == (b >> 6)) cand &= ~(1ull << (b & 63));
        while (cand) {
          const int a = 64 * w + __builtin_ctzll(cand);
          cand &= cand - 1;
          const uint64_t *ra = st + (long long)a * R;
          bool sub = true;
          unsigned long long deg = 0;
          for (int w2 = 0; w2 < R; ++w2) {
            const uint64_t x = ra[w2];
            deg += __popcll(x);
            if (x & ~rb[w2]) {
              sub = false;
              break;
            }
          }
          if (sub) {
            D[w] |= 1ull << (a & 63);   // word w belongs to this thread alone
            atomicAdd(&nv, 1ull);
            atomicAdd(&ne, deg);
          }
        }
        if (D[w]) dw[atomicAdd(&ndw, 1)] = w;
      }
      __syncthreads();
      // the deleted nodes lose their rows and their place in AL; their
      // neighbours (all in N(b)) lose them, in the words listed in dw
      const int nd = ndw;
      for (int w = tid; w < R; w += blockDim.x) AL[w] &= ~D[w];
      for (int x = tid; x < n; x += blockDim.x) {
        uint64_t *rx = st + (long long)x * R;
        if ((D[x >> 6] >> (x & 63)) & 1ull) {
          alive[x] = 0;
          for (int w = 0; w < R; ++w) rx[w] = 0;
        } else if ((rb[x >> 6] >> (x & 63)) & 1ull) {
          for (int i = 0; i < nd; ++i) {
            const int w = dw[i];
            if (rx[w] & D[w]) rx[w] &= ~D[w];
          }
        }
      }
      if (tid == 0) {
        h->dv += (long long)nv;
        h->de += (long long)ne;
        any_sweep = 1;
        ++steps;
      }
      b0 = b + 1;
      // every thread has read `hits` and the step is applied before the next scan
      __syncthreads();
    }
    __syncthreads();
    if (!any_sweep) break;
    ++sweeps;
  }
  if (tid == 0) {
    h->sweeps = sweeps;
    h->events = steps;
  }
}

// ---- edge dominance (Definition 4.3.2): the whole fixpoint, one workgroup
__global__ void __launch_bounds__(1024) k_dom_edge_run(uint64_t *__restrict__ st, int n, int R, DomHdr *h) {
  __shared__ uint64_t na[kDomMaxWords], D[kDomMaxWords];
  __shared__ int grew, any_sweep;
  __shared__ unsigned long long nd;
  const int tid = threadIdx.x;
  if (h->prio != P_NONE) return;
  long long sweeps = 0, passes = 0;
  for (;;) {
    // every thread has read the previous sweep's flag before it is reset
    __syncthreads();
    if (tid == 0) any_sweep = 0;
    for (int a = 0; a < n; ++a) {
      __syncthreads();
      for (int w = tid; w < R; w += blockDim.x) {
        na[w] = st[(long long)a * R + w];
        D[w] = 0;
      }
      if (tid == 0) nd = 0;
      for (;;) {
        // every thread has read the previous pass's flag (and the step's rows
        // and D are in place) before the flag is reset
        __syncthreads();
        if (tid == 0) grew = 0;
        __syncthreads();
        // one pass: every neighbour u of a not yet in D, tested with D below u
        for (int u = tid; u < n; u += blockDim.x) {
          const int uw = u >> 6;
          const uint64_t ub = 1ull << (u & 63);
          if (!(na[uw] & ub) || (D[uw] & ub)) continue;
          const uint64_t *ru = st + (long long)u * R;
          bool dom = false;
          for (int cw = 0; cw < R && !dom; ++cw) {
            const uint64_t below = cw < uw ? D[cw] : cw == uw ? (D[cw] & (ub - 1)) : 0ull;
            uint64_t cand = ru[cw] & (~na[cw] | below);
            if (cw == (a >> 6)) cand &= ~(1ull << (a & 63));
            while (cand && !dom) {
              const int bv = 64 * cw + __builtin_ctzll(cand);
              cand &= cand - 1;
              const uint64_t *rbv = st + (long long)bv * R;
              bool sub = true;
              for (int w2 = 0; w2 < R; ++w2) {
                const uint64_t b2 = w2 < uw ? D[w2] : w2 == uw ? (D[w2] & (ub - 1)) : 0ull;
                if (((na[w2] & ~b2) & ru[w2]) & ~rbv[w2]) {
                  sub = false;
                  break;
                }
              }
              dom = sub;
            }
          }
          if (dom) {
            atomicOr((unsigned long long *)&D[uw], ub);
            grew = 1;
          }
        }
        __syncthreads();
        if (tid == 0) ++passes;
        if (!grew) break;
      }
      // apply: {a, u} for every u in D
      for (int w = tid; w < R; w += blockDim.x) {
        if (D[w]) {
          st[(long long)a * R + w] = na[w] & ~D[w];
          atomicAdd(&nd, (unsigned long long)__popcll(D[w]));
        }
      }
      for (int u = tid; u < n; u += blockDim.x)
        if ((D[u >> 6] >> (u & 63)) & 1ull) st[(long long)u * R + (a >> 6)] &= ~(1ull << (a & 63));
      __syncthreads();
      if (tid == 0 && nd) {
        h->de += (long long)nd;
        any_sweep = 1;
      }
    }
    __syncthreads();
    if (!any_sweep) break;
    ++sweeps;
  }
  if (tid == 0) {
    h->sweeps = sweeps;
    h->events = h->de;
    h->passes = passes;
  }
}

int dom_status(int prio) {
  switch (prio) {
    case P_NONE: return KZ_OK;
    case P_ESELFLOOP: return KZ_ESELFLOOP;
    case P_EASYM: return KZ_EASYM;
    default: return KZ_EINVAL;
  }
}

}  // namespace
}  // namespace kzi

extern "C" {

int kz_dom_workspace_bytes(int32_t n, size_t *bytes) {
  if (!bytes || n < 0) return KZ_EINVAL;
  *bytes = 256;
  return KZ_OK;
}

int kz_dominance(kz_ctx *ctx, int32_t mode, int32_t n, const uint64_t *rows, int32_t row_words, void *ws,
                 size_t ws_bytes, uint8_t *vmask, uint64_t *emask, void *stream, kz_dom_result *res) {
  using namespace kzi;
  kz_dom_result r{};
  auto done = [&](int st) {
    r.status = st;
    if (res) *res = r;
    return st;
  };
  if (!ctx || (mode != KZ_DOM_VERTEX && mode != KZ_DOM_EDGE) || n < 0 || row_words < (n + 63) / 64)
    return done(KZ_EINVAL);
  if (n == 0) return done(KZ_OK);
  if (!rows || !ws || !vmask || !emask || (uintptr_t)ws % 256) return done(KZ_EINVAL);
  if (ws_bytes < sizeof(DomHdr)) return done(KZ_EWORKSPACE);
  if (row_words > kDomMaxWords) return done(KZ_ETOOLARGE);
  if (hipSetDevice(ctx->device) != hipSuccess) return done(KZ_EHIP);
  hipStream_t s = (hipStream_t)stream;
  DomHdr *h = (DomHdr *)ws;
  const int R = row_words;
  hipLaunchKernelGGL(k_dom_init, dim3(1), dim3(64), 0, s, h);
  const long long words = (long long)n * R;
  const int grid = (int)std::min<long long>((words + 255) / 256, 4096);
  hipLaunchKernelGGL(k_dom_setup, dim3(grid), dim3(256), 0, s, rows, emask, vmask, n, R, h);
  if (mode == KZ_DOM_VERTEX) hipLaunchKernelGGL(k_dom_vertex_run, dim3(1), dim3(1024), 0, s, emask, vmask, n, R, h);
  else hipLaunchKernelGGL(k_dom_edge_run, dim3(1), dim3(1024), 0, s, emask, n, R, h);
  DomHdr *hh = (DomHdr *)ctx->pinned;
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(hh, h, sizeof(DomHdr), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return done(KZ_EHIP);
  r.input_edges = hh->dirs / 2;
  const int st0 = dom_status(hh->prio);
  if (st0 != KZ_OK) return done(st0);
  r.sweeps = (int32_t)hh->sweeps;
  r.deleted_vertices = hh->dv;
  r.deleted_edges = hh->de;
  r.events = hh->events;
  r.scans = hh->passes;
  return done(KZ_OK);
}

}  // extern "C"
