// Batched kernelization (gfx950): many small graphs in one persistent launch.
//
// Every workgroup repeatedly takes the next graph from an atomic queue and
// runs that graph's synchronous rounds to the fixpoint on its own, using
// workgroup barriers as the per-graph round barriers (no workgroup ever waits
// for another, so the launch cannot deadlock).  Within a workgroup the waves
// take 64x64 block tiles one at a time (one wave per tile).
//
// Graph g's rows follow the bit-row layout of the single-graph path
// (class-major slots; class c's segment has ceil(s_c/64) words) and sit at
// word offset row_offset[g] of the rows arena; its colours and vertex mask at
// vertex_offset[g].  The state is kept in the emask arena (same layout);
// changed words of a round are staged in the workgroup's slice of scratch.
// Graphs too large for this path (k > kBatchK, row words > kBatchR, or
// n > kBatchN) get status KZ_ETOOLARGE in their result and are left to the
// single-graph path.
#include "kz_internal.h"

namespace kzi {

namespace {

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

__device__ __forceinline__ void tri(long long t, int NB, int &X, int &Y) {
  auto start = [NB](long long x) { return x * (2LL * NB - x - 1) / 2; };
  double d = 2.0 * NB - 1.0;
  long long x = (long long)((d - sqrt(d * d - 8.0 * (double)t)) * 0.5);
  if (x < 0) x = 0;
  if (x > NB - 2) x = NB - 2;
  while (x > 0 && start(x) > t) --x;
  while (x < NB - 2 && start(x + 1) <= t) ++x;
  X = (int)x;
  Y = (int)(t - start(x) + x + 1);
}

__device__ __forceinline__ bool tbit(const unsigned *b, int i) { return (b[i >> 5] >> (i & 31)) & 1u; }

struct BatchShared {
  int coff[kBatchK + 1], soff[kBatchK + 1];
  short bcls[kBatchR];
  int bstart[kBatchR];
  unsigned char blen[kBatchR];
  unsigned touched[2][kBatchN / 32];
  unsigned btouched[2][kBatchR / 32];
  int gi, bad_colour, bad_layout, prio, next_item, nchanged;
  unsigned long long removed_v, removed_e, tests;
};

// One graph, one workgroup.  NW waves, CH third classes per staging chunk.
template <int NW, int CH>
__device__ void batch_graph(const BatchArgs &a, BatchShared &S, unsigned long long (*sU)[CH][kBlk],
                            unsigned long long (*sU2)[CH][kBlk], unsigned long long (*sPw)[kBlk], int g) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const kz_batch_graph G = a.graphs[g];
  const int n = G.n, k = G.k, R = G.row_words;
  const uint64_t *rows = a.rows + G.row_offset;
  uint64_t *cur = a.emask + G.row_offset;
  const int *colour = a.colour + G.vertex_offset;
  uint8_t *valive = a.vmask + G.vertex_offset;
  kz_result res{};
  res.status = 0;
  if (n < 0 || k < 1 || R < 0) {
    res.status = KZ_EINVAL;
  } else if (k > kBatchK || R > kBatchR || n > kBatchN) {
    res.status = kBatchTooLarge;
  }
  if (res.status != 0 || n == 0) {
    if (tid == 0) {
      res.equals_input = res.status == 0;
      a.results[g] = res;
    }
    return;
  }
  uint64_t *scratch = a.scratch + (long long)blockIdx.x * a.scratch_words;
  int *changed = (int *)(scratch + a.list_offset);

  // ---- layout: colours are sorted class by class; class c starts at the
  // first vertex whose colour is >= c (binary search)
  if (tid == 0) {
    S.bad_colour = 0;
    S.bad_layout = 0;
    S.prio = 0;
  }
  __syncthreads();
  for (int v = tid; v < n; v += NW * kWave) {
    const int c = colour[v];
    if (c < 0 || c >= k) S.bad_colour = 1;
    else if (v > 0 && colour[v - 1] > c) S.bad_layout = 1;
  }
  __syncthreads();
  if (S.bad_colour | S.bad_layout) {
    if (tid == 0) {
      res.status = S.bad_colour ? KZ_ECOLOUR : KZ_EINVAL;
      a.results[g] = res;
    }
    return;
  }
  for (int c = tid; c <= k; c += NW * kWave) {
    int lo = 0, hi = n;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (colour[mid] < c) lo = mid + 1;
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
        S.bstart[w + b] = S.coff[c] + 64 * b;
        S.blen[w + b] = (unsigned char)min(64, s - 64 * b);
      }
      w += (s + 63) / 64;
    }
    S.soff[k] = w;
    if (w != R) S.bad_layout = 1;
  }
  __syncthreads();
  if (S.bad_layout) {
    if (tid == 0) {
      res.status = KZ_EINVAL;
      a.results[g] = res;
    }
    return;
  }
  // ---- state: copy the rows, everything alive and touched
  for (long long i = tid; i < (long long)n * R; i += NW * kWave) cur[i] = rows[i];
  for (int i = tid; i < kBatchN / 32; i += NW * kWave) {
    S.touched[0][i] = 0;
    S.touched[1][i] = ~0u;
  }
  for (int i = tid; i < kBatchR / 32; i += NW * kWave) {
    S.btouched[0][i] = 0;
    S.btouched[1][i] = ~0u;
  }
  __syncthreads();

  long long removed_v = 0, removed_e = 0, tests = 0, m = 0;
  int rounds = 0, pass = 0;
  for (;;) {
    ++pass;
    const bool first = pass == 1;
    const int tc = pass & 1, tn = tc ^ 1;
    if (tid == 0) {
      S.removed_v = 0;
      S.removed_e = 0;
      S.tests = 0;
      S.next_item = 0;
      S.nchanged = 0;
    }
    for (int i = tid; i < kBatchN / 32; i += NW * kWave) S.touched[tn][i] = 0;
    for (int i = tid; i < kBatchR / 32; i += NW * kWave) S.btouched[tn][i] = 0;
    __syncthreads();
    const uint64_t *src = first ? rows : cur;

    // ---- vertex test: lane v of a wave = vertex 64*i + v
    for (int v0 = wid * kWave; v0 < n; v0 += NW * kWave) {
      const int v = v0 + lane;
      const bool act = v < n && (first || (valive[v] && tbit(S.touched[tc], v)));
      if (!__ballot(act)) continue;
      const uint64_t *row = src + (long long)(act ? v : v0) * R;
      const int cv = act ? colour[v] : -1;
      bool fail = false;
      int pr = 0;
      for (int c = 0; c < k; ++c) {
        const int w0 = S.soff[c], w1 = S.soff[c + 1];
        const int s = S.coff[c + 1] - S.coff[c];
        if (!act) continue;
        if (w1 == w0) {
          fail |= c != cv;
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
        fail |= !nz;
      }
      if (pr) atomicMax(&S.prio, pr);
      fail = fail && act;
      if (act) {
        if (first) valive[v] = fail ? 0 : 1;
        else if (fail) valive[v] = 0;
      }
      const int nf = bsum(fail ? 1 : 0);
      if (lane == 0 && nf) atomicAdd(&S.removed_v, (unsigned long long)nf);
    }

    // ---- edge test: waves take tiles (X < Y)
    const long long T = (long long)R * (R - 1) / 2;
    const int nthird = k - 2;
    for (;;) {
      int t = 0;
      if (lane == 0) t = atomicAdd(&S.next_item, 1);
      t = __builtin_amdgcn_readfirstlane(t);
      if (t >= T) break;
      int X, Y;
      tri(t, R, X, Y);
      const int cx = S.bcls[X], cy = S.bcls[Y];
      if (cx == cy) continue;
      if (!first && !(tbit(S.btouched[tc], X) || tbit(S.btouched[tc], Y))) continue;
      const int xs = S.bstart[X], xl = S.blen[X], ys = S.bstart[Y], yl = S.blen[Y];
      const unsigned long long ymask = yl == 64 ? ~0ull : ((1ull << yl) - 1);
      const unsigned long long xmask = xl == 64 ? ~0ull : ((1ull << xl) - 1);
      const uint64_t *rowu_l = src + (long long)(xs + (lane < xl ? lane : 0)) * R;  // lane as row u
      const uint64_t *rowv = src + (long long)(ys + (lane < yl ? lane : 0)) * R;    // lane as row v
      const unsigned long long Eu = lane < xl ? (rowu_l[Y] & ymask) : 0ull;          // E(u) of row u = lane
      const unsigned long long ET = lane < yl ? rowv[X] : 0ull;
      sPw[wid][lane] = Eu;
      for (int q = 0; q < nthird; q += CH) {
        // stage the first two words of each third-class segment: row u's in
        // LDS (read as broadcasts), row v's in registers
        unsigned long long vv[CH], vv2[CH];
        int w2[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j) {
          const int i = q + j;
          if (i < nthird) {
            int c = i;
            if (c >= cx) ++c;
            if (c >= cy) ++c;
            const int w0 = S.soff[c], w1 = S.soff[c + 1];
            const bool has = w1 > w0, two = w1 > w0 + 1;
            sU[wid][j][lane] = (has && lane < xl) ? rowu_l[w0] : 0ull;
            sU2[wid][j][lane] = (two && lane < xl) ? rowu_l[w0 + 1] : 0ull;
            vv[j] = (has && lane < yl) ? rowv[w0] : 0ull;
            vv2[j] = (two && lane < yl) ? rowv[w0 + 1] : 0ull;
            w2[j] = w0 + 2 < w1 ? w0 + 2 : -1;
          } else {
            sU[wid][j][lane] = ~0ull;
            sU2[wid][j][lane] = 0ull;
            vv[j] = ~0ull;
            vv2[j] = 0ull;
            w2[j] = -1;
          }
        }
        __builtin_amdgcn_wave_barrier();
        for (int u = 0; u < xl; ++u) {
          unsigned long long P = bcast64(sPw[wid][lane], u);
          if (!P) continue;
          unsigned long long all = ~0ull;
#pragma unroll
          for (int j = 0; j < CH; ++j) all &= __ballot((sU[wid][j][u] & vv[j]) != 0ull);
          if (!(P & ~all)) continue;
          // level 2: the first two words
          all = ~0ull;
#pragma unroll
          for (int j = 0; j < CH; ++j)
            all &= __ballot(((sU[wid][j][u] & vv[j]) | (sU2[wid][j][u] & vv2[j])) != 0ull);
          if (!(P & ~all)) continue;
          // level 3: scan the rest of the segment in memory
          const uint64_t *rowu = src + (long long)(xs + u) * R;
#pragma unroll
          for (int j = 0; j < CH; ++j) {
            unsigned long long miss =
                P & ~__ballot(((sU[wid][j][u] & vv[j]) | (sU2[wid][j][u] & vv2[j])) != 0ull);
            if (!miss) continue;
            if (w2[j] >= 0) {
              const int i = q + j;
              int c = i;
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
          if (lane == u) sPw[wid][lane] = P;
        }
        __builtin_amdgcn_wave_barrier();
      }
      const unsigned long long Pu = sPw[wid][lane];
      unsigned long long newET = 0, trE = 0;
      for (int u = 0; u < xl; ++u) {
        const unsigned long long P = bcast64(Pu, u);
        newET |= ((P >> lane) & 1ull) << u;
        if (first) trE |= ((bcast64(Eu, u) >> lane) & 1ull) << u;
      }
      if (first && lane < yl && ((trE ^ ET) & xmask)) atomicMax(&S.prio, P_EASYM);
      const bool chU = lane < xl && Eu != Pu;
      const bool chV = lane < yl && (ET & xmask) != newET;
      const unsigned long long bu = __ballot(chU), bv = __ballot(chV);
      if (bu | bv) {
        if (lane < xl) scratch[(long long)(xs + lane) * R + Y] = Pu;
        if (lane < yl) scratch[(long long)(ys + lane) * R + X] = newET;
        if (chU) atomicOr(&S.touched[tn][(xs + lane) >> 5], 1u << ((xs + lane) & 31));
        if (chV) atomicOr(&S.touched[tn][(ys + lane) >> 5], 1u << ((ys + lane) & 31));
        const int rem = bsum(lane < xl ? __popcll(Eu & ~Pu) : 0);
        if (lane == 0) {
          if (bu) atomicOr(&S.btouched[tn][X >> 5], 1u << (X & 31));
          if (bv) atomicOr(&S.btouched[tn][Y >> 5], 1u << (Y & 31));
          changed[atomicAdd(&S.nchanged, 1)] = t;
          atomicAdd(&S.removed_e, (unsigned long long)rem);
        }
      }
      int cnt;
      if (first) {
        cnt = bsum(lane < xl ? __popcll(Eu) : 0);
      } else {
        const bool tU = lane < xl && tbit(S.touched[tc], xs + lane);
        const unsigned long long TV = __ballot(lane < yl && tbit(S.touched[tc], ys + lane));
        cnt = bsum(lane < xl ? __popcll(Eu & (tU ? ~0ull : TV)) : 0);
      }
      if (lane == 0 && cnt) atomicAdd(&S.tests, (unsigned long long)cnt);
    }
    __syncthreads();
    // ---- apply: copy changed tiles into the state
    const int nch = S.nchanged;
    for (int i = wid; i < nch; i += NW) {
      int X, Y;
      tri(changed[i], R, X, Y);
      const int xs = S.bstart[X], xl = S.blen[X], ys = S.bstart[Y], yl = S.blen[Y];
      if (lane < xl) cur[(long long)(xs + lane) * R + Y] = scratch[(long long)(xs + lane) * R + Y];
      if (lane < yl) cur[(long long)(ys + lane) * R + X] = scratch[(long long)(ys + lane) * R + X];
    }
    __syncthreads();
    if (first && S.prio) {
      if (tid == 0) {
        res.status = S.prio == P_EINVAL ? KZ_EINVAL
                     : S.prio == P_ESELFLOOP ? KZ_ESELFLOOP
                     : S.prio == P_EASYM ? KZ_EASYM
                                         : KZ_EILLEGAL;
        a.results[g] = res;
      }
      return;
    }
    const long long rv = (long long)S.removed_v, re = (long long)S.removed_e;
    if (first) m = (long long)S.tests;
    tests += (long long)S.tests;
    removed_v += rv;
    removed_e += re;
    __syncthreads();  // everyone has read the counters before they are reset
    if (rv + re == 0) break;
    ++rounds;
  }
  if (tid == 0) {
    res.rounds = rounds;
    res.equals_input = rounds == 0;
    res.passes = pass;
    res.surviving_vertices = n - removed_v;
    res.surviving_edges = m - removed_e;
    res.input_edges = m;
    res.edge_tests = tests;
    a.results[g] = res;
  }
}

template <int NW, int CH>
__global__ void __launch_bounds__(NW * 64) k_batch(BatchArgs a) {
  __shared__ BatchShared S;
  __shared__ unsigned long long sU[NW][CH][kBlk];
  __shared__ unsigned long long sU2[NW][CH][kBlk];
  __shared__ unsigned long long sPw[NW][kBlk];
  for (;;) {
    if (threadIdx.x == 0) S.gi = atomicAdd(a.queue, 1);
    __syncthreads();
    const int gi = S.gi;
    __syncthreads();
    if (gi >= a.G) break;
    batch_graph<NW, CH>(a, S, sU, sU2, sPw, a.order[gi]);
    __syncthreads();
  }
}

// Orders the graphs by an estimate of their work, largest first (so the
// persistent workgroups finish together), or keeps the given order.  One
// workgroup, bitonic sort in LDS for up to kBatchSortMax graphs.
__global__ void __launch_bounds__(1024) k_batch_order(BatchArgs a, int lpt) {
  __shared__ unsigned long long key[kBatchSortMax];
  const int t = threadIdx.x, G = a.G;
  if (t == 0) *a.queue = 0;
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

void launch_batch(const BatchArgs &a, const BatchConfig &cfg, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_order, dim3(1), dim3(1024), 0, s, a, cfg.lpt);
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
