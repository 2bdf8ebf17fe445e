// HIP kernels (gfx950) of the colour-index kernelizer.
//
// Layout.  Vertices are renumbered class by class ("slots"); class c owns
// slots [coff[c], coff[c+1]).  A row holds, for every class c, W_c =
// ceil(s_c/64) uint64 words starting at word soff[c]; bit j of class c's
// segment is adjacency to slot coff[c]+j.  Word index X of a row is also the
// index of a "block": the (up to) 64 slots of class bcls[X] starting at
// bstart[X].  So the 64x64 bit tile between blocks X and Y is stored twice:
// as word Y of the rows of block X and as word X of the rows of block Y.
// The edge pass gives each unordered inter-class block pair (X < Y) to one
// workgroup, which alone computes both copies of that tile for the next
// state -- no atomics on the adjacency, and every word of the next state
// has exactly one producer.
//
// Tests (thesis section 4.2, vertex and edge colour indices):
//   vertex v fails  <=> some class c != class(v) has an all-zero segment in
//                       row v (colour index below k-1);
//   edge {u,v} fails <=> some class c outside {class(u), class(v)} has
//                       row_u[c] & row_v[c] == 0 (colour index below k-2).
// Rounds are synchronous: the vertex and edge passes read the state A of
// the previous round; changed tiles are written to Anext and copied back by
// the apply pass.  Rows track alive EDGES, so a dead vertex has an empty row
// (every edge at a failing vertex fails the edge test in the same round).
#include "kz_internal.h"

namespace kzi {

namespace {

__device__ __forceinline__ bool stage1_bad(const Hdr *h) { return (h->bad_colour | h->bad_layout) != 0; }

__device__ __forceinline__ int wave_sum(int x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
  return x;
}

// Spreads workgroup ids so that each XCD (ids are dealt round-robin to the
// 8 XCDs) gets one contiguous range of tiles: neighbouring tiles share a
// block of rows, which then stays in that XCD's L2.
__device__ __forceinline__ long long xcd_remap(long long g, long long G) {
  long long q = G / 8, r = G % 8;
  long long x = g % 8, i = g / 8;
  return x * q + (x < r ? x : r) + i;
}

// Tile t of the upper triangle (X < Y) of an NB x NB block grid, row-major.
__device__ __forceinline__ void tri_decode(long long t, int NB, int &X, int &Y) {
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

// ---------------------------------------------------------------- setup

__global__ void k_init_header(Plan p, int dense) {
  long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long stride = (long long)gridDim.x * blockDim.x;
  if (tid == 0) {
    Hdr *h = p.hdr;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 4; ++b) h->ctr[a][b] = 0;
    h->tile_count = 0;
    h->prio = 0;
    h->bad_colour = 0;
    h->bad_layout = 0;
    h->R = 0;
    h->n = p.n;
    h->k = p.k;
  }
  for (long long i = tid; i < p.k; i += stride) p.counts[i] = 0;
  if (dense)
    for (long long i = tid; i < (long long)p.nchunks * p.k; i += stride) p.hist[i] = 0;
}

// Class sizes (and per-chunk histograms for the stable partition); stage-1
// colour checks.
__global__ void k_count(Plan p, const int *colour, int dense) {
  int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= p.n) return;
  int c = colour[u];
  if (c < 0 || c >= p.k) {
    p.hdr->bad_colour = 1;
    return;
  }
  atomicAdd(&p.counts[c], 1);
  if (dense)
    atomicAdd(&p.hist[(long long)blockIdx.x * p.k + c], 1);
  else if (u > 0 && colour[u - 1] > c)
    p.hdr->bad_layout = 1;
}

// One workgroup: class offsets, segment offsets and the block table.
__global__ void k_layout(Plan p, int row_words, int bitset) {
  Hdr *h = p.hdr;
  if (h->bad_colour) return;
  __shared__ int sa[256], sb[256];
  __shared__ int carry_a, carry_b;
  const int t = threadIdx.x;
  if (t == 0) {
    carry_a = 0;
    carry_b = 0;
  }
  __syncthreads();
  for (int base = 0; base < p.k; base += 256) {
    int c = base + t;
    int s = c < p.k ? p.counts[c] : 0;
    int a = s, b = (s + 63) / 64;
    sa[t] = a;
    sb[t] = b;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {  // inclusive Hillis-Steele scan
      int xa = t >= off ? sa[t - off] : 0;
      int xb = t >= off ? sb[t - off] : 0;
      __syncthreads();
      sa[t] += xa;
      sb[t] += xb;
      __syncthreads();
    }
    if (c < p.k) {
      p.coff[c] = carry_a + sa[t] - a;
      p.soff[c] = carry_b + sb[t] - b;
    }
    __syncthreads();
    if (t == 255) {
      carry_a += sa[255];
      carry_b += sb[255];
    }
    __syncthreads();
  }
  if (t == 0) {
    p.coff[p.k] = carry_a;
    p.soff[p.k] = carry_b;
    int R = carry_b;
    if (bitset && R != row_words) {
      h->bad_layout = 1;
      R = row_words;
    }
    h->R = R;
  }
  __syncthreads();
  if (h->bad_layout) return;
  for (int c = t; c < p.k; c += 256) {
    int s = p.counts[c];
    int w0 = p.soff[c];
    for (int b = 0; 64 * b < s; ++b) {
      p.bcls[w0 + b] = c;
      p.bstart[w0 + b] = p.coff[c] + 64 * b;
      p.blen[w0 + b] = min(64, s - 64 * b);
    }
  }
}

// Stable partition of caller vertices into class-major slots.
__global__ void k_rank(Plan p, const int *colour) {
  if (stage1_bad(p.hdr)) return;
  __shared__ int sc[kRankChunk];
  const int b = blockIdx.x, t = threadIdx.x;
  const int u = b * kRankChunk + t;
  const int c = u < p.n ? colour[u] : -1;
  sc[t] = c;
  __syncthreads();
  if (u >= p.n) return;
  int r = 0;
  for (int j = 0; j < t; ++j) r += sc[j] == c;
  int base = 0;
  for (int bb = 0; bb < b; ++bb) base += p.hist[(long long)bb * p.k + c];
  const int slot = p.coff[c] + base + r;
  p.perm[slot] = u;
  p.inv[u] = slot;
  p.scls[slot] = c;
}

__global__ void k_init_state(Plan p) {
  const Hdr *h = p.hdr;
  if (stage1_bad(h)) return;
  long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = tid; i < p.n; i += stride) {
    p.valive[i] = 1;
    p.touched[1][i] = 1;  // pass 1 reads parity 1: everything is "touched"
    p.touched[0][i] = 0;
  }
  for (long long i = tid; i < h->R; i += stride) {
    p.btouched[1][i] = 1;
    p.btouched[0][i] = 0;
  }
}

// Dense u8 adjacency (caller order) -> class-partitioned bit rows.  One
// workgroup per caller row; the row is assembled in LDS when it fits.
__global__ void __launch_bounds__(256) k_pack_dense(Plan p, const uint8_t *adj, const int *colour,
                                                    int use_lds) {
  const Hdr *h = p.hdr;
  if (stage1_bad(h)) return;
  extern __shared__ unsigned long long srow[];
  const int u = blockIdx.x, t = threadIdx.x;
  const int R = h->R, n = p.n;
  uint64_t *Arow = p.A + (long long)p.inv[u] * R;
  for (int w = t; w < R; w += 256) {
    if (use_lds)
      srow[w] = 0;
    else
      Arow[w] = 0;
  }
  __syncthreads();
  int bad = 0;
  const uint8_t *arow = adj + (long long)u * n;
  for (int v = t; v < n; v += 256) {
    const uint8_t a = arow[v];
    bad |= a > 1;
    if (a) {
      const int c = colour[v];
      const int j = p.inv[v] - p.coff[c];
      const int w = p.soff[c] + (j >> 6);
      const unsigned long long bit = 1ull << (j & 63);
      if (use_lds)
        atomicOr(&srow[w], bit);
      else
        atomicOr((unsigned long long *)&Arow[w], bit);
    }
  }
  if (bad) atomicMax(&p.hdr->prio, P_EINVAL);
  __syncthreads();
  if (use_lds)
    for (int w = t; w < R; w += 256) Arow[w] = srow[w];
}

// ---------------------------------------------------------------- passes

// Vertex test for alive vertices touched by the previous round (all of them
// in pass 1, which also validates every row).  One wave per slot; lane c
// looks at class c's segment.  Also resets the "next" bookkeeping of the pass.
__global__ void __launch_bounds__(256) k_vertex(Plan p, const int *scls, int pass, int validate) {
  Hdr *h = p.hdr;
  if (stage1_bad(h)) return;
  const int R = h->R, n = p.n, k = p.k;
  const int cur = pass & 1, nxt = cur ^ 1;
  {
    long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = tid; i < n; i += stride) p.touched[nxt][i] = 0;
    for (long long i = tid; i < R; i += stride) p.btouched[nxt][i] = 0;
    if (tid == 0) {
      h->tile_count = 0;
      for (int j = 0; j < 4; ++j) h->ctr[nxt][j] = 0;
    }
  }
  const int v = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (v >= n) return;
  if (!validate && (!p.valive[v] || !p.touched[cur][v])) return;
  const uint64_t *row = p.A + (long long)v * R;
  const int cv = scls[v];
  bool fail = false;
  int pr = P_NONE;
  for (int c = lane; c < k; c += kWave) {
    const int w0 = p.soff[c], w1 = p.soff[c + 1];
    const int s = p.coff[c + 1] - p.coff[c];
    if (validate && (s & 63) && w1 > w0 && (row[w1 - 1] >> (s & 63))) pr = max(pr, P_EINVAL);
    if (c == cv) {
      if (!validate) continue;
      // own segment must be empty: classify what is there
      const int jv = v - p.coff[c];
      for (int w = w0; w < w1; ++w) {
        unsigned long long x = row[w];
        if (w == w1 - 1 && (s & 63)) x &= (1ull << (s & 63)) - 1;
        while (x) {
          const int b = __builtin_ctzll(x);
          x &= x - 1;
          const int tslot = p.coff[c] + (w - w0) * 64 + b;
          if (tslot == v) {
            pr = max(pr, P_ESELFLOOP);
          } else {
            const uint64_t y = p.A[(long long)tslot * R + w0 + (jv >> 6)];
            pr = max(pr, ((y >> (jv & 63)) & 1ull) ? (int)P_EILLEGAL : (int)P_EASYM);
          }
        }
      }
      continue;
    }
    bool nz = false;
    if (validate) {
      for (int w = w0; w < w1; ++w) nz |= row[w] != 0;
    } else {
      for (int w = w0; w < w1; ++w)
        if (row[w]) {
          nz = true;
          break;
        }
    }
    fail |= !nz;
  }
  if (pr) atomicMax(&h->prio, pr);
  const unsigned long long fb = __ballot(fail);
  if (fb && lane == 0 && p.valive[v]) {
    p.valive[v] = 0;
    atomicAdd(&h->ctr[cur][0], 1ull);
  }
}

// Edge test for every edge of one inter-class block pair (X, Y), X < Y.
//
// Lane v of each wave stands for slot bstart[Y]+v; wave w handles 16 rows u
// of block X.  P(u) is the 64-bit set of v with {u,v} still passing.  For
// each third class c, the first word of both rows' class-c segments (staged
// in LDS) usually already holds a common neighbour; the lanes still missing
// one (a wave ballot) scan the remaining words of the segment straight from
// memory.  Lanes with no common neighbour in c drop out of P(u).  The tile's
// two copies of its new bits (word Y of X's rows, word X of Y's rows) go to
// Anext, and the tile is listed for the apply pass, only if a bit changed.
__global__ void __launch_bounds__(kEdgeThreads) k_edge(Plan p, int pass, int validate) {
  Hdr *h = p.hdr;
  if (stage1_bad(h)) return;
  const int R = h->R, k = p.k;
  int X, Y;
  tri_decode(xcd_remap(blockIdx.x, gridDim.x), p.Rmax, X, Y);
  if (Y >= R) return;
  const int cx = p.bcls[X], cy = p.bcls[Y];
  if (cx == cy) return;
  const int cur = pass & 1, nxt = cur ^ 1;
  if (!(p.btouched[cur][X] | p.btouched[cur][Y])) return;

  __shared__ unsigned long long sU[kClassChunk][kBlk];
  __shared__ unsigned long long sV[kClassChunk][kBlk];
  __shared__ unsigned long long sE[kBlk], sP[kBlk];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int xs = p.bstart[X], xl = p.blen[X];
  const int ys = p.bstart[Y], yl = p.blen[Y];
  const unsigned long long ymask = yl == 64 ? ~0ull : ((1ull << yl) - 1);
  const unsigned long long xmask = xl == 64 ? ~0ull : ((1ull << xl) - 1);
  const uint64_t *__restrict__ A = p.A;

  if (tid < kBlk) {
    const unsigned long long e = tid < xl ? A[(long long)(xs + tid) * R + Y] : 0ull;
    sE[tid] = e;
    sP[tid] = e & ymask;
  }
  __syncthreads();

  const uint64_t *rowv = A + (long long)(ys + lane) * R;  // dereferenced only for lanes < yl
  for (int c0 = 0; c0 < k; c0 += kClassChunk) {
    const int nc = min(kClassChunk, k - c0);
    for (int i = tid; i < nc * kBlk; i += kEdgeThreads) {
      const int cc = i >> 6, r = i & 63, c = c0 + cc;
      const int w0 = p.soff[c];
      const bool has = p.soff[c + 1] > w0;
      sU[cc][r] = (has && r < xl) ? A[(long long)(xs + r) * R + w0] : 0ull;
      sV[cc][r] = (has && r < yl) ? A[(long long)(ys + r) * R + w0] : 0ull;
    }
    __syncthreads();
    for (int ui = 0; ui < kBlk / 4; ++ui) {
      const int u = wid * (kBlk / 4) + ui;
      if (u >= xl) break;
      unsigned long long P = sP[u];
      if (!P) continue;
      const uint64_t *rowu = A + (long long)(xs + u) * R;
      for (int cc = 0; cc < nc; ++cc) {
        const int c = c0 + cc;
        if (c == cx || c == cy) continue;
        const unsigned long long hit = __ballot((sU[cc][u] & sV[cc][lane]) != 0ull);
        unsigned long long miss = P & ~hit;
        if (miss) {
          const int w1 = p.soff[c + 1];
          for (int w = p.soff[c] + 1; w < w1 && miss; ++w) {
            const unsigned long long a = rowu[w];
            const unsigned long long b = ((miss >> lane) & 1ull) ? rowv[w] : 0ull;
            miss &= ~__ballot((a & b) != 0ull);
          }
          P &= ~miss;
          if (!P) break;
        }
      }
      if (lane == 0) sP[u] = P;
    }
    __syncthreads();
  }

  if (wid != 0) return;
  const int v = lane;
  const unsigned long long ET = v < yl ? A[(long long)(ys + v) * R + X] : 0ull;
  unsigned long long newET = 0, trE = 0;
  for (int u = 0; u < xl; ++u) {
    newET |= ((sP[u] >> v) & 1ull) << u;
    if (validate) trE |= ((sE[u] >> v) & 1ull) << u;
  }
  if (validate && v < yl && ((trE ^ ET) & xmask)) atomicMax(&h->prio, P_EASYM);
  const unsigned long long Eu = sE[lane] & ymask, Pu = sP[lane];
  const bool chU = lane < xl && Eu != Pu;
  const bool chV = v < yl && (ET & xmask) != newET;
  const unsigned long long bu = __ballot(chU), bv = __ballot(chV);
  if (bu | bv) {
    if (lane < xl) p.Anext[(long long)(xs + lane) * R + Y] = Pu;
    if (v < yl) p.Anext[(long long)(ys + v) * R + X] = newET;
    if (chU) p.touched[nxt][xs + lane] = 1;
    if (chV) p.touched[nxt][ys + v] = 1;
    const int rem = wave_sum(lane < xl ? __popcll(Eu & ~Pu) : 0);
    if (lane == 0) {
      if (bu) p.btouched[nxt][X] = 1;
      if (bv) p.btouched[nxt][Y] = 1;
      const int pos = atomicAdd(&h->tile_count, 1);
      p.tiles[pos] = make_int2(X, Y);
      atomicAdd(&h->ctr[cur][1], (unsigned long long)rem);
    }
  }
  // exact worklist size: edges of this tile with a touched endpoint
  const int tU = lane < xl ? p.touched[cur][xs + lane] : 0;
  const int tV = v < yl ? p.touched[cur][ys + v] : 0;
  const unsigned long long TV = __ballot(tV != 0);
  const int cnt = wave_sum(lane < xl ? __popcll(Eu & (tU ? ~0ull : TV)) : 0);
  if (lane == 0 && cnt) atomicAdd(&h->ctr[cur][2], (unsigned long long)cnt);
}

// Copies the changed tiles of this pass from Anext into A.
__global__ void __launch_bounds__(128) k_apply(Plan p) {
  const Hdr *h = p.hdr;
  if (stage1_bad(h)) return;
  const int R = h->R;
  const int cnt = h->tile_count;
  for (int i = blockIdx.x; i < cnt; i += gridDim.x) {
    const int2 t = p.tiles[i];
    int j = threadIdx.x;
    long long idx = -1;
    if (j < 64) {
      if (j < p.blen[t.x]) idx = (long long)(p.bstart[t.x] + j) * R + t.y;
    } else {
      j -= 64;
      if (j < p.blen[t.y]) idx = (long long)(p.bstart[t.y] + j) * R + t.x;
    }
    if (idx >= 0) p.A[idx] = p.Anext[idx];
  }
}

// Bit rows -> dense u8 masks in caller order.  One workgroup per caller row.
__global__ void __launch_bounds__(256) k_unpack_dense(Plan p, const int *colour, uint8_t *vmask,
                                                      uint8_t *emask, int use_lds) {
  const Hdr *h = p.hdr;
  if (stage1_bad(h)) return;
  extern __shared__ unsigned long long srow[];
  const int u = blockIdx.x, t = threadIdx.x;
  const int R = h->R, n = p.n;
  const int s = p.inv[u];
  const uint64_t *row = p.A + (long long)s * R;
  if (use_lds) {
    for (int w = t; w < R; w += 256) srow[w] = row[w];
    __syncthreads();
  }
  uint8_t *out = emask + (long long)u * n;
  for (int v = t; v < n; v += 256) {
    const int c = colour[v];
    const int j = p.inv[v] - p.coff[c];
    const int w = p.soff[c] + (j >> 6);
    const unsigned long long x = use_lds ? srow[w] : row[w];
    out[v] = (uint8_t)((x >> (j & 63)) & 1ull);
  }
  if (t == 0) vmask[u] = p.valive[s];
}

inline unsigned grid_for(long long work, int threads, long long cap) {
  long long g = (work + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

}  // namespace

void launch_init_header(const Plan &p, bool dense, hipStream_t s) {
  long long work = p.k;
  if (dense) work = (long long)p.nchunks * p.k;
  hipLaunchKernelGGL(k_init_header, dim3(grid_for(work, 256, 1024)), dim3(256), 0, s, p, dense ? 1 : 0);
}

void launch_count(const Plan &p, const int *colour, bool dense, hipStream_t s) {
  hipLaunchKernelGGL(k_count, dim3(grid_for(p.n, kRankChunk, 1LL << 30)), dim3(kRankChunk), 0, s, p,
                     colour, dense ? 1 : 0);
}

void launch_layout(const Plan &p, int row_words, bool bitset, hipStream_t s) {
  hipLaunchKernelGGL(k_layout, dim3(1), dim3(256), 0, s, p, row_words, bitset ? 1 : 0);
}

void launch_rank(const Plan &p, const int *colour, hipStream_t s) {
  hipLaunchKernelGGL(k_rank, dim3(p.nchunks), dim3(kRankChunk), 0, s, p, colour);
}

void launch_init_state(const Plan &p, hipStream_t s) {
  hipLaunchKernelGGL(k_init_state, dim3(grid_for(p.n, 256, 2048)), dim3(256), 0, s, p);
}

void launch_pack_dense(const Plan &p, const uint8_t *adj, const int *colour, hipStream_t s) {
  const int use_lds = p.Rmax <= kPackLdsWords;
  const size_t lds = use_lds ? sizeof(unsigned long long) * (size_t)p.Rmax : 0;
  hipLaunchKernelGGL(k_pack_dense, dim3(p.n), dim3(256), lds, s, p, adj, colour, use_lds);
}

void launch_copy_rows(const Plan &p, const uint64_t *rows, hipStream_t s) {
  (void)hipMemcpyAsync(p.A, rows, sizeof(uint64_t) * (size_t)p.n * (size_t)p.Rmax, hipMemcpyDeviceToDevice, s);
}

void launch_vertex_pass(const Plan &p, const int *scls, int pass, bool validate, hipStream_t s) {
  hipLaunchKernelGGL(k_vertex, dim3(grid_for(p.n, 4, 1LL << 30)), dim3(256), 0, s, p, scls, pass,
                     validate ? 1 : 0);
}

void launch_edge_pass(const Plan &p, int pass, bool validate, hipStream_t s) {
  if (p.Tmax <= 0) return;
  hipLaunchKernelGGL(k_edge, dim3((unsigned)p.Tmax), dim3(kEdgeThreads), 0, s, p, pass, validate ? 1 : 0);
}

void launch_apply(const Plan &p, hipStream_t s) {
  if (p.Tmax <= 0) return;
  hipLaunchKernelGGL(k_apply, dim3(grid_for(p.Tmax, 1, 4096)), dim3(128), 0, s, p);
}

void launch_unpack_dense(const Plan &p, const int *colour, uint8_t *vmask, uint8_t *emask, hipStream_t s) {
  const int use_lds = p.Rmax <= kPackLdsWords;
  const size_t lds = use_lds ? sizeof(unsigned long long) * (size_t)p.Rmax : 0;
  hipLaunchKernelGGL(k_unpack_dense, dim3(p.n), dim3(256), lds, s, p, colour, vmask, emask, use_lds);
}

}  // namespace kzi
