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
// Rounds are synchronous: every test of a pass reads the state left by the
// previous round and writes only the next state.  Rows track alive EDGES, so
// a dead vertex has an empty row (every edge at a failing vertex fails the
// edge test in the same round).
#include "kz_internal.h"

namespace kzi {

namespace {

__device__ __forceinline__ bool stage1_bad(const Hdr *h) { return (h->bad_colour | h->bad_layout) != 0; }

__device__ __forceinline__ int wave_sum(int x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
  return x;
}

// A value every lane holds identically, moved to scalar registers.
__device__ __forceinline__ unsigned long long uniform64(unsigned long long x) {
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)x);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(x >> 32));
  return ((unsigned long long)hi << 32) | lo;
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

// Tile t of the edge pass.  Row-major over the triangle (p.Sq <= 1), or in
// squares of Sq x Sq block pairs: the squares (I, J), I <= J, row-major over
// the triangle of squares with its diagonal, the cells of a square
// row-major.  The tiles a chip's XCD has in flight then come from a few
// squares, whose rows and first words fit its L2, instead of from one or
// two block rows paired with every other block.  Cells with X >= Y or
// Y >= NB are not tiles: false.
__device__ __forceinline__ bool tile_decode(long long t, int NB, int Sq, int &X, int &Y) {
  if (Sq <= 1) {
    tri_decode(t, NB, X, Y);
    return true;
  }
  const int NS = (NB + Sq - 1) / Sq;
  const long long sq = t / ((long long)Sq * Sq);
  const int cell = (int)(t - sq * Sq * Sq);
  int I, J;
  tri_decode(sq, NS + 1, I, J);  // (I, J+1) over NS+1 blocks: I <= J over NS
  J -= 1;
  X = I * Sq + cell / Sq;
  Y = J * Sq + cell % Sq;
  return X < Y && Y < NB;
}

// ---------------------------------------------------------------- setup

// One workgroup: zeroes the header, counts the classes (stage-1 colour
// checks), scans class and segment offsets and fills the block table.  For
// dense input it also builds per-chunk class histograms for the stable
// partition; for CSR input it only zeroes the header.
__global__ void __launch_bounds__(kSetupThreads) k_setup(Plan p, const int *colour, int row_words,
                                                         int mode) {
  const bool dense = mode == SETUP_DENSE, bitset = mode == SETUP_BITSET;
  Hdr *h = p.hdr;
  const int t = threadIdx.x, n = p.n, k = p.k;
  __shared__ int sh[kSetupLdsClasses];
  __shared__ int sst[kSetupLdsClasses + 1];  // bit-row input: first vertex of each class
  __shared__ int sa[kSetupThreads / kWave], sb[kSetupThreads / kWave];
  __shared__ int s_bad_colour, s_bad_layout, carry_a, carry_b;
  const bool lds_hist = k <= kSetupLdsClasses;
  if (t == 0) {
    h->tile_count = 0;
    h->prio = 0;
    h->bad_colour = 0;
    h->bad_layout = 0;
    h->R = 0;
    h->n = n;
    h->k = k;
    h->done = 0;
    h->out = kz_out{};
    s_bad_colour = 0;
    s_bad_layout = 0;
    carry_a = 0;
    carry_b = 0;
  }
  for (int i = t; i < 2 * kCtrSlots * 4; i += kSetupThreads) h->ctr(i / (4 * kCtrSlots), (i / 4) % kCtrSlots, i % 4) = 0;
  // CSR kernels use no class table; their validation checks the colours
  if (mode == SETUP_CSR) return;
  for (int c = t; c < k; c += kSetupThreads) {
    if (lds_hist)
      sh[c] = 0;
    else
      p.counts[c] = 0;
  }
  if (dense)
    for (long long i = t; i < (long long)p.nchunks * k; i += kSetupThreads) p.hist[i] = 0;
  if (bitset && lds_hist)
    for (int c = t; c <= k; c += kSetupThreads) sst[c] = 0;
  __syncthreads();
  // four vertices per thread at a time, their colour loads issued together
  constexpr int kBatch = 4;
  for (int u0 = t; u0 < n; u0 += kBatch * kSetupThreads) {
    int cs[kBatch], ps[kBatch];
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      const int u = u0 + q * kSetupThreads;
      cs[q] = u < n ? colour[u] : 0;
      ps[q] = bitset && u < n && u > 0 ? colour[u - 1] : -1;
    }
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      const int u = u0 + q * kSetupThreads;
      if (u >= n) break;
      const int c = cs[q];
      if (c < 0 || c >= k) {
        s_bad_colour = 1;
        continue;
      }
      if (bitset) {
        // sorted colours: u is the first vertex of every class in
        // (colour[u-1], c], and the last vertex ends the classes above its own
        const int prev = ps[q];
        if (prev > c) {
          s_bad_layout = 1;
        } else if (lds_hist) {
          for (int x = max(prev + 1, 0); x <= c; ++x) sst[x] = u;
          if (u == n - 1)
            for (int x = c + 1; x <= k; ++x) sst[x] = n;
        }
        continue;
      }
      if (lds_hist)
        atomicAdd(&sh[c], 1);
      else
        atomicAdd(&p.counts[c], 1);
      if (dense) atomicAdd(&p.hist[(long long)(u / kRankChunk) * k + c], 1);
    }
  }
  if (bitset && lds_hist) {
    // class sizes from the class starts (meaningful only when the colours
    // are sorted; the layout check above flags them otherwise)
    __syncthreads();
    for (int c = t; c < k; c += kSetupThreads) sh[c] = sst[c + 1] - sst[c];
  } else if (bitset) {
    // class c holds the vertices from the first colour >= c to the first
    // colour >= c+1
    auto first_ge = [&](int c) {
      int lo = 0, hi = n;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (colour[mid] < c) lo = mid + 1;
        else hi = mid;
      }
      return lo;
    };
    for (int c = t; c < k; c += kSetupThreads) {
      const int cnt = first_ge(c + 1) - first_ge(c);
      if (lds_hist) sh[c] = cnt;
      else p.counts[c] = cnt;
    }
  }
  __syncthreads();
  if (s_bad_colour) {
    if (t == 0) h->bad_colour = 1;
    return;
  }
  // exclusive scans of class sizes and segment widths: shuffle scans inside
  // each wave, then a scan of the wave totals
  constexpr int kSetupWaves = kSetupThreads / kWave;
  const int lane = t & 63, wv = t >> 6;
  int my_s = 0, my_c0 = 0, my_w0 = 0;  // class t's size and offsets, kept for the block table
  for (int base = 0; base < k; base += kSetupThreads) {
    const int c = base + t;
    int s = 0;
    if (c < k) s = lds_hist ? sh[c] : atomicAdd(&p.counts[c], 0);
    const int a = s, b = (s + 63) / 64;
    int ia = a, ib = b;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const int xa = __shfl_up(ia, off, kWave), xb = __shfl_up(ib, off, kWave);
      if (lane >= off) {
        ia += xa;
        ib += xb;
      }
    }
    if (lane == kWave - 1) {
      sa[wv] = ia;
      sb[wv] = ib;
    }
    __syncthreads();
    if (t == 0) {
      int ra = carry_a, rb = carry_b;
      for (int w = 0; w < kSetupWaves; ++w) {
        const int xa = sa[w], xb = sb[w];
        sa[w] = ra;
        sb[w] = rb;
        ra += xa;
        rb += xb;
      }
      carry_a = ra;
      carry_b = rb;
    }
    __syncthreads();
    if (c < k) {
      const int c0 = sa[wv] + ia - a, w0 = sb[wv] + ib - b;
      p.counts[c] = a;
      p.coff[c] = c0;
      p.soff[c] = w0;
      if (base == 0) {
        my_s = a;
        my_c0 = c0;
        my_w0 = w0;
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    p.coff[k] = carry_a;
    p.soff[k] = carry_b;
    int R = bitset || dense ? carry_b : 0;
    if (bitset && R != row_words) s_bad_layout = 1;
    if (s_bad_layout) {
      h->bad_layout = 1;
      R = row_words;
    }
    h->R = R;
  }
  __syncthreads();
  if (s_bad_layout) return;
  // each thread reads back only the entries it wrote itself above
  for (int c = t; c < k; c += kSetupThreads) {
    const bool mine = c == t;
    const int s = mine ? my_s : p.counts[c];
    const int w0 = mine ? my_w0 : p.soff[c], c0 = mine ? my_c0 : p.coff[c];
    for (int b = 0; 64 * b < s; ++b) {
      p.bcls[w0 + b] = c;
      p.bstart[w0 + b] = c0 + 64 * b;
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

// Dense u8 adjacency (caller order) -> class-partitioned bit rows.  One
// workgroup per caller row; the row is assembled in LDS when it fits.
__global__ void __launch_bounds__(256) k_pack_dense(Plan p, const uint8_t *adj, const int *colour,
                                                    uint64_t *dst, int use_lds) {
  const Hdr *h = p.hdr;
  if (stage1_bad(h)) return;
  extern __shared__ unsigned long long srow[];
  const int u = blockIdx.x, t = threadIdx.x;
  const int R = h->R, n = p.n;
  uint64_t *Arow = dst + (long long)p.inv[u] * R;
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

// Vertex test of the passes after the first.  A workgroup takes 64 slots
// (lane v = slot 64*block + v) and its 4 waves split the classes (wave w
// walks c = w, w+4, ...); only alive vertices touched by the previous round
// are tested.  For each tested row it also refreshes the first-word matrix
// F[v*k + c] (the first word of row v's class-c segment), which the edge
// pass tests first.  Also resets the bookkeeping the edge pass of this pass
// fills.
__global__ void __launch_bounds__(256) k_vertex(Plan p, const int *scls, const uint64_t *__restrict__ src,
                                                int pass) {
  Hdr *h = p.hdr;
  if (stage1_bad(h) || h->done) return;
  const int R = h->R, n = p.n, k = p.k;
  const int cur = pass & 1, nxt = cur ^ 1;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  {
    const long long gt = (long long)blockIdx.x * blockDim.x + tid;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = gt; i < n; i += stride) p.touched[nxt][i] = 0;
    for (long long i = gt; i < R; i += stride) p.btouched[nxt][i] = 0;
    if (gt == 0) h->tile_count = 0;
    if (gt < kCtrSlots * 4) h->ctr(nxt, gt / 4, gt % 4) = 0;
  }
  __shared__ int sFail[kWave];
  __shared__ int sOff[kVertexLdsClasses + 1];  // soff
  const bool lds_off = k <= kVertexLdsClasses;
  const int v0 = blockIdx.x * kWave;
  if (tid < kWave) sFail[tid] = 0;
  if (lds_off)
    for (int c = tid; c <= k; c += 256) sOff[c] = p.soff[c];
  __syncthreads();
  const int v = v0 + lane;
  const bool active = v < n && p.valive[v] && p.touched[cur][v];
  if (__ballot(active)) {
    const int vc = active ? v : v0;  // clamped row for inactive lanes
    const uint64_t *row = src + (long long)vc * R;
    const int cv = scls[vc];
    bool fail = false;
    // the wave's classes c = wid, wid+4, ... in groups of kVG: all loads of
    // a group go out before any of them is used
    constexpr int kVG = 4;
    for (int cg = wid; cg < k; cg += 4 * kVG) {
      unsigned long long x0[kVG], x1[kVG];
#pragma unroll
      for (int g = 0; g < kVG; ++g) {
        const int c = cg + 4 * g;
        const int w0 = c < k ? (lds_off ? sOff[c] : p.soff[c]) : 0;
        const int w1 = c < k ? (lds_off ? sOff[c + 1] : p.soff[c + 1]) : 0;
        x0[g] = w1 > w0 ? row[w0] : 0ull;
        x1[g] = w1 - w0 >= 2 ? row[w0 + 1] : 0ull;
      }
#pragma unroll
      for (int g = 0; g < kVG; ++g) {
        const int c = cg + 4 * g;
        if (c >= k) break;
        const int w0 = lds_off ? sOff[c] : p.soff[c];
        const int w1 = lds_off ? sOff[c + 1] : p.soff[c + 1];
        if (active) {
          p.F[(long long)v * p.kF + c] = c == cv ? ~0ull : x0[g];
          p.S[(long long)v * p.kF + c] = x1[g];
        }
        if (c == cv) continue;
        // an empty class has no words: no neighbour possible
        bool nz = (x0[g] | x1[g]) != 0;
        if (active && !nz)
          for (int w = w0 + 2; w < w1; ++w)
            if (row[w]) {
              nz = true;
              break;
            }
        fail |= !nz;
      }
    }
    if (fail && active) atomicOr(&sFail[lane], 1);
  }
  __syncthreads();
  if (wid != 0 || !__ballot(active)) return;
  const bool fail = active && sFail[lane];
  if (fail) p.valive[v] = 0;
  const int nf = wave_sum(fail ? 1 : 0);
  if (lane == 0 && nf) atomicAdd(&h->ctr(cur, blockIdx.x % kCtrSlots, 0), (unsigned long long)nf);
}

// Pass-1 vertex test fused with the copy of the input into the output state.
// A workgroup takes kVfRows slots; wave w takes rows v0+w, v0+w+4, ... and lane l
// holds word 64*j+l of a row, so every load is one contiguous 512-byte
// piece, stored to `dst` as it is tested.  Per piece the lane knows its
// word's class, the word's place in that class's segment and its valid bits;
// the lanes that start a class in the piece ("heads") see, through a wave
// ballot of the nonzero words, whether their class has a bit in this row.  A
// class that runs on into the next piece carries its verdict there.  A row
// fails when a class other than its own has no bit, or when some class is
// empty.  Words of the row's own class must be zero (a nonzero one is
// classified: self-loop, edge inside a class, or asymmetry), and so must
// padding bits past a class's size.  The first word of every segment fills
// the first-word matrix F.  All loads of a piece are independent of
// each other, so one memory round serves the copy, the test and F.  Rh > 0:
// the caller's row width (bit-row input; a layout whose classes do not add up
// to it is flagged by the setup pass and nothing is written); 0: the setup
// pass's.
__global__ void __launch_bounds__(256) k_vertex_first(Plan p, const int *scls, const uint64_t *__restrict__ src,
                                                      uint64_t *__restrict__ dst, int Rh) {
  Hdr *h = p.hdr;
  const int n = p.n, k = p.k;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  constexpr int kRows = kVfRows / 4;  // rows per wave
  __shared__ int sOff[2][kVertexLdsClasses + 1];  // coff, soff
  const bool lds_off = k <= kVertexLdsClasses;
  const int v0 = blockIdx.x * kVfRows;
  const int nrows = min(kVfRows, n - v0);
  const int R = Rh > 0 ? Rh : h->R;
  const int nch = (R + kWave - 1) / kWave;
  // Every load of the first piece goes out before any is used: indices are
  // clamped into range (the values of clamped lanes and rows are unused), so
  // no load sits behind a branch.
  const int Rl = max(R - 1, 0);  // last word (a failed setup pass leaves R = 0)
  auto load_rows = [&](int ch, unsigned long long (&x)[kRows]) {
    const int w = min(ch * kWave + lane, Rl);
#pragma unroll
    for (int i = 0; i < kRows; ++i) {
      const int r = min(wid + 4 * i, nrows - 1);
      x[i] = src[(long long)(v0 + r) * R + w];
    }
  };
  // per-piece word facts: class of the word and of its neighbours two back
  // and one ahead, and the word's valid bits
  struct Meta {
    int c, cm1, cm2, cp1, bl;
  };
  auto load_meta = [&](int ch) {
    const int w = ch * kWave + lane;
    Meta m;
    m.c = p.bcls[min(w, Rl)];
    m.cm1 = p.bcls[min(max(w - 1, 0), Rl)];
    m.cm2 = p.bcls[min(max(w - 2, 0), Rl)];
    m.cp1 = p.bcls[min(w + 1, Rl)];
    m.bl = p.blen[min(w, Rl)];
    return m;
  };
  const int c0 = min(tid, k);
  const int off0 = p.coff[c0], soff0 = p.soff[c0];
  const int sc = scls[min(v0 + (lane & (kVfRows - 1)), n - 1)];  // class of slot v0 + lane % kVfRows
  unsigned long long x[kRows];
  load_rows(0, x);
  Meta m = load_meta(0);
  if (lds_off) {
    // every thread stores (threads past k repeat entry k), so the wait for
    // these loads is not behind a branch
    sOff[0][c0] = off0;
    sOff[1][c0] = soff0;
    for (int c = tid + 256; c <= k; c += 256) {
      sOff[0][c] = p.coff[c];
      sOff[1][c] = p.soff[c];
    }
  }
  if (stage1_bad(h)) return;
  // one wait for every load above (vmcnt(0)), so that no use further down
  // waits again -- such a wait would also wait for the stores issued since
  __builtin_amdgcn_s_waitcnt(0x0F70);
  const int cur = 1, nxt = 0;
  {
    const long long gt = (long long)blockIdx.x * blockDim.x + tid;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = gt; i < n; i += stride) p.touched[nxt][i] = 0;
    for (long long i = gt; i < R; i += stride) p.btouched[nxt][i] = 0;
    if (gt == 0) h->tile_count = 0;
    if (gt < kCtrSlots * 4) h->ctr(nxt, gt / 4, gt % 4) = 0;
  }
  __shared__ int sEmpty;
  if (tid == 0) sEmpty = 0;
  __syncthreads();
  // an empty class leaves every vertex without a neighbour there (a vertex's
  // own class is never empty); F of an empty class is zero
  auto empty_class = [&](int c) {
    sEmpty = 1;
    for (int r = 0; r < nrows; ++r) {
      p.F[(long long)(v0 + r) * p.kF + c] = 0ull;
      p.S[(long long)(v0 + r) * p.kF + c] = 0ull;
    }
  };
  if (lds_off) {
    for (int c = tid; c < k; c += 256)
      if (sOff[1][c] == sOff[1][c + 1]) empty_class(c);
  } else {
    for (int c = tid; c < k; c += 256)
      if (p.soff[c] == p.soff[c + 1]) empty_class(c);
  }
  // F's padding classes (k up to its row stride) pass every first-word test
  {
    const int pad = p.kF - k;
    for (int i = tid; i < nrows * pad; i += 256) p.F[(long long)(v0 + i / pad) * p.kF + k + i % pad] = ~0ull;
  }
  __syncthreads();
  const bool any_empty = sEmpty != 0;
  unsigned long long failRows = 0, carryRows = 0;
  int pr = P_NONE;
  // one piece: copy, test, F (the first piece is peeled off the loop so that
  // its values, already waited for, are not waited for again)
  auto piece = [&](int ch) {
    const int w = ch * kWave + lane;
    const bool valid = w < R;
    // the word's class, its place in the class's segment (0, 1, or 2 for
    // later), its valid bits, and whether the segment ends with it
    const int cw = valid ? m.c : -1;
    const int off = !valid ? 2 : (w < 1 || m.cm1 != m.c) ? 0 : (w < 2 || m.cm2 != m.c) ? 1 : 2;
    const int bl = valid ? m.bl : 64;
    const bool ends = !valid || w + 1 >= R || m.cp1 != m.c;
    const bool head = valid && (lane == 0 || off == 0);
    const unsigned long long heads = __ballot(head);
    // lanes of my class in this piece: from me up to the next head
    const unsigned long long above = lane == 63 ? 0ull : heads >> (lane + 1);
    const int nh = above ? lane + 1 + __builtin_ctzll(above) : 64;
    const unsigned long long mine = (nh == 64 ? ~0ull : (1ull << nh) - 1) & ~((1ull << lane) - 1);
    const bool cont0 = ch > 0 && __shfl(off, 0, kWave) != 0;  // lane 0's class began before
    const int lastLane = min(kWave, R - ch * kWave) - 1;
    const unsigned long long lastHead = 1ull << (63 - __builtin_clzll(heads));
    const bool contL = __shfl(ends ? 0 : 1, lastLane, kWave) != 0;  // the last class runs on
    unsigned bad_rows = 0;  // rows with a bit in this lane's word of their own class
#pragma unroll
    for (int i = 0; i < kRows; ++i) {
      const int r = wid + 4 * i;
      if (r >= nrows) continue;
      const int v = v0 + r;
      const unsigned long long xi = x[i];
      const int cvr = __builtin_amdgcn_readlane(sc, r);
      if (valid) {
        dst[(long long)v * R + w] = xi;
        if (off == 0) p.F[(long long)v * p.kF + cw] = cw == cvr ? ~0ull : xi;
        if (off == 1) p.S[(long long)v * p.kF + cw] = xi;
        if (off == 0 && ends) p.S[(long long)v * p.kF + cw] = 0ull;
        if (bl < 64 && (xi >> bl)) pr = max(pr, (int)P_EINVAL);
      }
      const unsigned long long nz = __ballot(valid && xi != 0);
      unsigned long long H = __ballot(head && (nz & mine) != 0);
      if (cont0 && ((carryRows >> i) & 1)) H |= 1ull;
      const unsigned long long own = __ballot(head && cw == cvr);
      const unsigned long long defer = contL ? lastHead : 0ull;
      if (heads & ~H & ~own & ~defer) failRows |= 1ull << i;
      carryRows = (carryRows & ~(1ull << i)) | ((contL && (H & lastHead)) ? 1ull << i : 0ull);
      if (valid && cw == cvr && xi) bad_rows |= 1u << i;
    }
    // bits inside a row's own class (invalid input): classify them
    while (bad_rows) {
      const int i = __builtin_ctz(bad_rows);
      bad_rows &= bad_rows - 1;
      const int v = v0 + wid + 4 * i;
      const unsigned long long xi = src[(long long)v * R + w];
      unsigned long long y = bl < 64 ? xi & ((1ull << bl) - 1) : xi;
      const int jv = v - (lds_off ? sOff[0][cw] : p.coff[cw]);
      const int wv = (lds_off ? sOff[1][cw] : p.soff[cw]) + (jv >> 6);
      const int b0 = p.bstart[w];
      while (y) {
        const int b = __builtin_ctzll(y);
        y &= y - 1;
        const int tslot = b0 + b;
        if (tslot == v) {
          pr = max(pr, (int)P_ESELFLOOP);
        } else {
          const uint64_t z = src[(long long)tslot * R + wv];
          pr = max(pr, ((z >> (jv & 63)) & 1ull) ? (int)P_EILLEGAL : (int)P_EASYM);
        }
      }
    }
  };
  piece(0);
  for (int ch = 1; ch < nch; ++ch) {
    load_rows(ch, x);
    m = load_meta(ch);
    piece(ch);
  }
  if (pr) atomicMax(&h->prio, pr);
  // lane i < kRows publishes row wid + 4i
  const int r = wid + 4 * lane;
  const bool fail = any_empty || ((failRows >> (lane & (kRows - 1))) & 1);
  const bool mine_row = lane < kRows && r < nrows;
  if (mine_row) p.valive[v0 + r] = fail ? 0 : 1;
  const int nf = wave_sum(mine_row && fail ? 1 : 0);
  if (lane == 0 && nf) atomicAdd(&h->ctr(cur, blockIdx.x % kCtrSlots, 0), (unsigned long long)nf);
}

// Reads lane l's 64-bit value into scalar registers.
__device__ __forceinline__ unsigned long long lane64(unsigned long long x, int l) {
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)x, l);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(x >> 32), l);
  return ((unsigned long long)hi << 32) | lo;
}

// x with lane l's value replaced by the uniform value y.
__device__ __forceinline__ unsigned long long set_lane64(unsigned long long x, unsigned long long y, int l,
                                                         int lane) {
  return lane == l ? y : x;
}

constexpr int kTileWaves = kEdgeThreads / kWave;  // waves per workgroup of the edge pass

// What a wave knows about its tile (X, Y): blocks of two different classes,
// lane l standing for row u = xs + l and for row v = ys + l.  A workgroup
// takes kTileWaves / TW tiles, TW waves each.
struct Tile {
  int X, Y, xs, xl, ys, yl, cx, cy;
  unsigned long long E;   // lane u: row u's word Y (its edges into block Y)
  unsigned long long ET;  // lane v: row v's word X
  unsigned long long TU, TV;  // rows of X / Y touched by the previous round (all in pass 1)
};

// Decodes this wave's tile and loads its words; false when the wave has no
// inter-class tile to test in this pass (the same answer for the TW waves of
// a tile).
template <bool FIRST, int TW>
__device__ __forceinline__ bool tile_begin(const Plan &p, const uint64_t *__restrict__ src, int cur, int lane,
                                           Tile &T) {
  const Hdr *h = p.hdr;
  const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const long long t = xcd_remap(blockIdx.x, gridDim.x) * (kTileWaves / TW) + wid / TW;
  if (t >= (p.Sq > 1 ? p.Tcells : p.Tmax)) return false;
  if (!tile_decode(t, p.Rmax, p.Sq, T.X, T.Y)) return false;
  // one round of independent loads (X, Y < Rmax: the block table is in
  // bounds even where this call's layout is shorter or invalid)
  const int bad = h->bad_colour | h->bad_layout | h->done, R = h->R;
  T.cx = p.bcls[T.X];
  T.cy = p.bcls[T.Y];
  T.xs = p.bstart[T.X];
  T.xl = p.blen[T.X];
  T.ys = p.bstart[T.Y];
  T.yl = p.blen[T.Y];
  const bool btouch = FIRST || (p.btouched[cur][T.X] | p.btouched[cur][T.Y]);
  if (bad || T.Y >= R || T.cx == T.cy || !btouch) return false;
  const unsigned long long ymask = T.yl == 64 ? ~0ull : ((1ull << T.yl) - 1);
  const int urc = lane < T.xl ? lane : T.xl - 1, vrc = lane < T.yl ? lane : T.yl - 1;  // clamped rows
  const unsigned long long e = src[(long long)(T.xs + urc) * R + T.Y];
  const unsigned long long et = src[(long long)(T.ys + vrc) * R + T.X];
  T.E = lane < T.xl ? e & ymask : 0ull;
  T.ET = lane < T.yl ? et : 0ull;
  // pairs to re-test: those with a touched endpoint (all of them in pass 1);
  // the others keep their outcome, so masks and rounds equal full sweeps
  T.TU = FIRST ? ~0ull : __ballot(lane < T.xl && p.touched[cur][T.xs + lane]);
  T.TV = FIRST ? ~0ull : __ballot(lane < T.yl && p.touched[cur][T.ys + lane]);
  return true;
}

// The tile's next state from P (lane u: the pairs of row u that still pass,
// a subset of E): wave-transposes P into the new word X of every row v (and,
// in pass 1, E against the rows' word X to check symmetry), writes both
// copies of the tile when a bit changed (pass 1: into the output state,
// which already holds the input; later passes: into scratch, the tile
// listed for the apply pass), marks touched rows and blocks, and counts the
// removed edges and the exact-worklist tests.
template <bool FIRST>
__device__ __forceinline__ void tile_finish(const Plan &p, uint64_t *__restrict__ dst, const Tile &T,
                                            unsigned long long P, int cur, int lane) {
  Hdr *h = p.hdr;
  const int R = h->R, nxt = cur ^ 1, slot = blockIdx.x % kCtrSlots;
  const unsigned long long xmask = T.xl == 64 ? ~0ull : ((1ull << T.xl) - 1);
  const unsigned long long newET = wave_transpose64(P, lane) & xmask;
  if (FIRST) {
    const unsigned long long trE = wave_transpose64(T.E, lane);
    if (lane < T.yl && ((trE ^ T.ET) & xmask)) atomicMax(&h->prio, P_EASYM);
  }
  const bool chU = lane < T.xl && T.E != P;
  const bool chV = lane < T.yl && (T.ET & xmask) != newET;
  const unsigned long long bu = __ballot(chU), bv = __ballot(chV);
  if (bu | bv) {
    if (lane < T.xl) dst[(long long)(T.xs + lane) * R + T.Y] = P;
    if (lane < T.yl) dst[(long long)(T.ys + lane) * R + T.X] = newET;
    if (chU) p.touched[nxt][T.xs + lane] = 1;
    if (chV) p.touched[nxt][T.ys + lane] = 1;
    const int rem = wave_sum(lane < T.xl ? __popcll(T.E & ~P) : 0);
    if (lane == 0) {
      if (bu) p.btouched[nxt][T.X] = 1;
      if (bv) p.btouched[nxt][T.Y] = 1;
      if (!FIRST) {
        const int pos = atomicAdd(&h->tile_count, 1);
        p.tiles[pos] = make_int2(T.X, T.Y);
      }
      atomicAdd(&h->ctr(cur, slot, 1), (unsigned long long)rem);
    }
  }
  // exact worklist size: edges of this tile with a touched endpoint
  const int cnt = wave_sum(lane < T.xl ? __popcll(T.E & (((T.TU >> lane) & 1ull) ? ~0ull : T.TV)) : 0);
  if (lane == 0 && cnt) atomicAdd(&h->ctr(cur, slot, 2), (unsigned long long)cnt);
}

// Edge test (witness search) for every edge of one inter-class block pair
// (X, Y), X < Y.  Edge {u,v} fails when some class other than class(X) and
// class(Y) holds no common neighbour.  The first-word matrix F (F[v*kF + c]
// = the first word of row v's class-c segment) feeds the common case: per
// chunk of KC classes, lane v holds its row's first words in registers; for
// each row u, u's first words of the chunk come in as one block of scalar
// loads (the address is uniform), and one AND, a compare and a wave ballot
// per class give the lanes with a common neighbour there.  No class needs a
// special case in this loop: F holds all-ones for a row's own class and for
// the padding classes past k, and the registers of class(X) are set to
// all-ones once per chunk, so the tile's own two classes and the padding
// pass (class(Y) is v's own class), and an empty class holds zero words.
// The one exception is a row u with no neighbour in the first word of
// class(Y): its ballots for that class are empty, and the row takes the rare
// path below like a row with a miss.  A lane that is still an edge and has
// no witness in some third class's first word tries the second words (the
// second-word matrix S, laid out like F and as small, so both sides come
// from the L2), then scans the rest of the segment in the rows.  TW = 1: the
// four waves of a workgroup test four neighbouring tiles (same X, so their
// scalar loads share the cache), with no LDS and no barrier; TW = 4 (graphs
// with few tiles): the workgroup's waves split one tile's rows u, 16 each,
// so four times as many waves hide the scalar loads' latency, and wave 0
// finishes the tile from the rows' results gathered in LDS.
template <bool FIRST, int KC, int TW>
__global__ void __launch_bounds__(kEdgeThreads) k_edge(Plan p, const uint64_t *__restrict__ src,
                                                       uint64_t *__restrict__ dst, int pass,
                                                       const uint64_t *__restrict__ F,
                                                       const uint64_t *__restrict__ S) {
  static_assert(TW == 1 || TW == kTileWaves, "a tile takes one wave or the whole workgroup");
  const int lane = threadIdx.x & 63, cur = pass & 1;
  Tile T;
  if (!tile_begin<FIRST, TW>(p, src, cur, lane, T)) return;
  const int k = p.k, kF = p.kF, R = p.hdr->R;
  const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int u0 = TW == 1 ? 0 : wid * (kBlk / TW), u1 = TW == 1 ? T.xl : min(u0 + kBlk / TW, T.xl);
  const int vrc = lane < T.yl ? lane : T.yl - 1;
  const uint64_t *rowv = src + (long long)(T.ys + vrc) * R;
  const uint64_t *Sv = S + (long long)(T.ys + vrc) * kF;
  unsigned long long P = T.E;
  for (int q = 0; q < k; q += KC) {
    // third classes of the tile in this chunk
    const int hi = min(q + KC, k);
    const int nthird = hi - q - (T.cx >= q && T.cx < hi) - (T.cy >= q && T.cy < hi);
    if (nthird <= 0) continue;
    const uint64_t *Fv = F + (long long)(T.ys + vrc) * kF + q;
    unsigned long long vf[KC];
#pragma unroll
    for (int j = 0; j < KC; ++j) vf[j] = q + j == T.cx ? ~0ull : Fv[j];
    unsigned third = 0;  // chunk positions of the tile's third classes
#pragma unroll
    for (int j = 0; j < KC; ++j)
      if (q + j < k && q + j != T.cx && q + j != T.cy) third |= 1u << j;
    const uint64_t *Fu = F + (long long)(T.xs + u0) * kF + q;  // row u's first words: uniform, scalar loads
    for (int u = u0; u < u1; ++u, Fu += kF) {
      unsigned long long Pu = lane64(P, u);
      const unsigned long long Pt = Pu & (((T.TU >> u) & 1ull) ? ~0ull : T.TV);
      if (!Pt) continue;
      unsigned long long uf[KC];
#pragma unroll
      for (int j = 0; j < KC; ++j) uf[j] = Fu[j];
      // lanes with a witness in every class of each quarter of the chunk
      constexpr int KQ = KC / 4;
      unsigned long long all[4] = {~0ull, ~0ull, ~0ull, ~0ull};
#pragma unroll
      for (int j = 0; j < KC; ++j) all[j / KQ] &= __ballot((uf[j] & vf[j]) != 0ull);
      if (!(Pt & ~(all[0] & all[1] & all[2] & all[3]))) continue;
      // some edge of u lacks a witness in a first word: in each quarter with
      // a miss, third class by third class (u's word reloaded, so the hot
      // loop's scalar registers need not live on into this path), the
      // second words (S sits in the L2), then the rest of the segment in the
      // rows; every load is made only by the lanes still missing a witness
      const uint64_t *Su = S + (long long)(T.xs + u) * kF;
      const uint64_t *rowu = src + (long long)(T.xs + u) * R;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        if (!(Pt & ~all[g])) continue;
#pragma unroll
        for (int jj = 0; jj < KQ; ++jj) {
          const int j = g * KQ + jj;
          const unsigned long long ufj = __builtin_nontemporal_load(Fu + j);
          unsigned long long m = Pt & ~__ballot((ufj & vf[j]) != 0ull);
          if (!m || !((third >> j) & 1u)) continue;
          const int c = q + j;
          const bool mine = (m >> lane) & 1ull;
          const unsigned long long x2 = mine ? Su[c] : 0ull, y2 = mine ? Sv[c] : 0ull;
          m &= ~__ballot((x2 & y2) != 0ull);
          if (!m) continue;
          const int w1 = p.soff[c + 1];
          for (int w = p.soff[c] + 2; w < w1 && m; ++w) {
            const bool still = (m >> lane) & 1ull;
            const unsigned long long x = still ? rowu[w] : 0ull, y = still ? rowv[w] : 0ull;
            m &= ~__ballot((x & y) != 0ull);
          }
          Pu &= ~m;
        }
      }
      P = set_lane64(P, Pu, u, lane);
    }
  }
  if (TW > 1) {
    // gather the rows' results (lane u of the wave that owns row u)
    __shared__ unsigned long long sP[kBlk];
    if (lane >= u0 && lane < u0 + kBlk / TW) sP[lane] = P;
    __syncthreads();
    if (wid != 0) return;
    P = sP[lane];
  }
  tile_finish<FIRST>(p, dst, T, P, cur, lane);
}

// The MFMA count path's tile epilogue: the pairs with a touched endpoint
// take the fail bits `fb` that k_mfma_count computed (same layout as the
// rows); the others keep their outcome.
template <bool FIRST>
__global__ void __launch_bounds__(kEdgeThreads) k_edge_mf(Plan p, const uint64_t *__restrict__ src,
                                                          uint64_t *__restrict__ dst, int pass,
                                                          const uint64_t *__restrict__ fb) {
  const int lane = threadIdx.x & 63, cur = pass & 1;
  Tile T;
  if (!tile_begin<FIRST, 1>(p, src, cur, lane, T)) return;
  const int R = p.hdr->R;
  unsigned long long P = T.E;
  if (lane < T.xl) {
    const unsigned long long Pt = ((T.TU >> lane) & 1ull) ? ~0ull : T.TV;
    P &= ~(fb[(long long)(T.xs + lane) * R + T.Y] & Pt);
  }
  tile_finish<FIRST>(p, dst, T, P, cur, lane);
}

// ---------------------------------------------------------------- MFMA count path
//
// count_c(u, v) = sum over w in class c of A[u][w] * A[v][w]: the number of
// common neighbours of u and v in class c, an int8 x int8 -> int32 block
// contraction (exact: counts stay below 2^31).  An edge {u, v} fails when
// some third class c has count_c(u, v) == 0 -- the same test as the witness
// search, computed for every pair of a tile.  One workgroup takes a group
// tile of two blocks by two blocks (up to 128 x 128 pairs of two classes);
// for every word of every third class it expands the 64 bits of each of its
// 256 rows to bytes in LDS (double-buffered) and each wave accumulates a
// 64 x 64 quarter with 32x32x32 int8 MFMAs.  A class with a zero count marks
// the pair in the fail bits `fb` (same layout as the rows; words of block Y
// and Y+1 in the rows of blocks X and X+1); k_edge<.., true> turns them
// into the next state with the usual worklist and counter epilogue.
typedef int mf_v4i __attribute__((ext_vector_type(4)));
typedef int mf_v16i __attribute__((ext_vector_type(16)));
constexpr int kMfRows = 128;   // rows per side of a group tile
constexpr int kMfPitch = 80;   // bytes per staged row: 64 + 16 of padding
constexpr int kMfAhead = 8;    // words fetched ahead of their staging

// bits 0..3 of x -> bytes 0..3 (0 or 1): the four shifted copies land on
// distinct bit positions, so the product has no carries
__device__ __forceinline__ int nib_bytes(unsigned x) { return (int)(((x & 0xFu) * 0x00204081u) & 0x01010101u); }

template <bool FIRST>
__global__ void __launch_bounds__(kMfThreads) k_mfma_count(Plan p, const uint64_t *__restrict__ src,
                                                          uint64_t *__restrict__ fb, int pass) {
  Hdr *h = p.hdr;
  if (stage1_bad(h) || h->done) return;
  const int R = h->R;
  int X, Y;
  tri_decode(xcd_remap(blockIdx.x, gridDim.x), p.Rmax, X, Y);
  if (Y >= R) return;
  const int cx = p.bcls[X], cy = p.bcls[Y];
  if (cx == cy) return;
  // group heads: the even-numbered blocks of each class
  if (((X - p.soff[cx]) & 1) || ((Y - p.soff[cy]) & 1)) return;
  const bool x2 = X + 1 < R && p.bcls[X + 1] == cx;
  const bool y2 = Y + 1 < R && p.bcls[Y + 1] == cy;
  const int cur = pass & 1;
  if (!FIRST && !(p.btouched[cur][X] | (x2 && p.btouched[cur][X + 1]) | p.btouched[cur][Y] |
                  (y2 && p.btouched[cur][Y + 1])))
    return;
  const int xs = p.bstart[X], ul = p.blen[X] + (x2 ? p.blen[X + 1] : 0);
  const int ys = p.bstart[Y], vl = p.blen[Y] + (y2 ? p.blen[Y + 1] : 0);

  __shared__ __attribute__((aligned(16))) signed char sA[2][kMfRows * kMfPitch];
  __shared__ __attribute__((aligned(16))) signed char sB[2][kMfRows * kMfPitch];
  __shared__ short sWord[kMfMaxWords];  // third-class words in order; bit 15: last word of its class
  __shared__ int sN, sEmpty;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  if (tid == 0) {
    int nw = 0, empty = 0;
    for (int c = 0; c < p.k; ++c) {
      if (c == cx || c == cy) continue;
      const int w0 = p.soff[c], w1 = p.soff[c + 1];
      if (w0 == w1) empty = 1;  // an empty third class: no pair has a common neighbour there
      for (int w = w0; w < w1 && nw < kMfMaxWords; ++w) sWord[nw++] = (short)(w | (w == w1 - 1 ? 0x8000 : 0));
    }
    sN = nw;
    sEmpty = empty;
  }
  __syncthreads();
  const int nwords = sN;

  // staging: thread t < 128 expands row t of the u side, t >= 128 row t-128 of the v side
  const int sr = tid & (kMfRows - 1);
  const bool sideB = tid >= kMfRows;
  const int slen = sideB ? vl : ul;
  const uint64_t *srow = src + (long long)((sideB ? ys : xs) + (sr < slen ? sr : 0)) * R;
  auto stage = [&](int buf, unsigned long long word) {
    mf_v4i *d = (mf_v4i *)((sideB ? sB[buf] : sA[buf]) + sr * kMfPitch);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const unsigned x = (unsigned)(word >> (16 * q));
      mf_v4i v;
      v.x = nib_bytes(x);
      v.y = nib_bytes(x >> 4);
      v.z = nib_bytes(x >> 8);
      v.w = nib_bytes(x >> 12);
      d[q] = v;
    }
  };
  mf_v16i acc[2][2];
  unsigned fail[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      acc[i][j] = mf_v16i{};
      fail[i][j] = sEmpty ? 0xffffu : 0u;
    }
  // words are fetched kMfAhead iterations before they are staged, so the
  // loads' latency hides behind that many words of MFMAs
  auto fetch = [&](int t) -> unsigned long long {
    return (t < nwords && sr < slen) ? srow[sWord[t] & 0x7fff] : 0ull;
  };
  unsigned long long ring[kMfAhead];  // ring[q]: the word staged at iteration t0 + q
  if (nwords > 0) stage(0, fetch(0));
#pragma unroll
  for (int q = 0; q < kMfAhead; ++q) ring[q] = fetch(q + 1);
  __syncthreads();
  const int koff = (lane >> 5) * 16;
  for (int t0 = 0; t0 < nwords; t0 += kMfAhead) {
#pragma unroll
    for (int q = 0; q < kMfAhead; ++q) {
      const int t = t0 + q;
      if (t < nwords) {
        const int buf = t & 1;
#pragma unroll
        for (int st = 0; st < 2; ++st) {
          mf_v4i a[2], b[2];
#pragma unroll
          for (int i = 0; i < 2; ++i)
            a[i] = *(const mf_v4i *)(sA[buf] + (64 * wr + 32 * i + (lane & 31)) * kMfPitch + st * 32 + koff);
#pragma unroll
          for (int j = 0; j < 2; ++j)
            b[j] = *(const mf_v4i *)(sB[buf] + (64 * wc + 32 * j + (lane & 31)) * kMfPitch + st * 32 + koff);
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        if (sWord[t] & 0x8000) {
          // end of a third class: a zero count fails the pair
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
#pragma unroll
              for (int e = 0; e < 16; ++e) fail[i][j] |= (acc[i][j][e] == 0 ? 1u : 0u) << e;
              acc[i][j] = mf_v16i{};
            }
        }
        if (t + 1 < nwords) stage(buf ^ 1, ring[q]);
        ring[q] = fetch(t + 1 + kMfAhead);
        __syncthreads();
      }
    }
  }
  // fail bits -> words: element e of lane l is pair (row 8*(e/4) + 4*(l/32) +
  // e%4, column l%32) of a 32x32 quarter, so one ballot per (e, quarter)
  // gives 32 columns of two rows
  unsigned long long myword = 0;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const unsigned long long b0 = __ballot((fail[i][0] >> e) & 1u), b1 = __ballot((fail[i][1] >> e) & 1u);
      const int r0 = 32 * i + 8 * (e >> 2) + (e & 3);
      if (lane == r0) myword = (b0 & 0xffffffffull) | (b1 << 32);
      if (lane == r0 + 4) myword = (b0 >> 32) | ((b1 >> 32) << 32);
    }
  const int row = 64 * wr + lane;
  if (row < ul && (wc == 0 || y2)) fb[(long long)(xs + row) * R + Y + wc] = myword;
}

// Copies the changed tiles of this pass from scratch into the state.
__global__ void __launch_bounds__(128) k_apply(Plan p, const uint64_t *__restrict__ scratch,
                                               uint64_t *__restrict__ cur) {
  const Hdr *h = p.hdr;
  if (stage1_bad(h) || h->done) return;
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
    if (idx >= 0) cur[idx] = scratch[idx];
  }
}

// Bit rows -> dense u8 masks in caller order.  One workgroup per caller row.
__global__ void __launch_bounds__(256) k_unpack_dense(Plan p, const int *colour, const uint64_t *cur,
                                                      uint8_t *vmask, uint8_t *emask, int use_lds) {
  const Hdr *h = p.hdr;
  // the caller's masks are written once, at the fixpoint
  if (stage1_bad(h) || !h->done || h->out.result.status != KZ_OK) return;
  extern __shared__ unsigned long long srow[];
  const int u = blockIdx.x, t = threadIdx.x;
  const int R = h->R, n = p.n;
  const int s = p.inv[u];
  const uint64_t *row = cur + (long long)s * R;
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

void launch_setup(const Plan &p, const int *colour, int row_words, SetupMode mode, hipStream_t s) {
  hipLaunchKernelGGL(k_setup, dim3(1), dim3(kSetupThreads), 0, s, p, colour, row_words, (int)mode);
}

void launch_rank(const Plan &p, const int *colour, hipStream_t s) {
  hipLaunchKernelGGL(k_rank, dim3(p.nchunks), dim3(kRankChunk), 0, s, p, colour);
}

void launch_pack_dense(const Plan &p, const uint8_t *adj, const int *colour, uint64_t *dst, hipStream_t s) {
  const int use_lds = p.Rmax <= kPackLdsWords;
  const size_t lds = use_lds ? sizeof(unsigned long long) * (size_t)p.Rmax : 0;
  hipLaunchKernelGGL(k_pack_dense, dim3(p.n), dim3(256), lds, s, p, adj, colour, dst, use_lds);
}

void launch_vertex_pass(const Plan &p, const int *scls, const uint64_t *src, uint64_t *dst, int pass,
                        bool first, int row_words, hipStream_t s) {
  const dim3 grid(grid_for(p.n, kWave, 1LL << 30));  // 64 slots per workgroup
  if (first)
    hipLaunchKernelGGL(k_vertex_first, dim3(grid_for(p.n, kVfRows, 1LL << 30)), dim3(256), 0, s, p, scls, src, dst,
                       row_words);
  else
    hipLaunchKernelGGL(k_vertex, grid, dim3(256), 0, s, p, scls, src, pass);
}

void launch_edge_pass(const Plan &plan, const uint64_t *src, uint64_t *dst, int pass, bool first,
                      hipStream_t s) {
  if (plan.Tmax <= 0) return;
  Plan p = plan;
  const uint64_t *F = p.F, *S = p.S;
  // a wave per tile when there are tiles enough to fill the chip many times
  // over, else a workgroup per tile
  const bool wide = p.Tmax < kEdgeWaveTiles;
  // many tiles: in squares of kEdgeSquare x kEdgeSquare block pairs
  p.Sq = wide ? 1 : kEdgeSquare;
  if (p.Sq > 1) {
    const long long NS = (p.Rmax + p.Sq - 1) / p.Sq;
    p.Tcells = NS * (NS + 1) / 2 * p.Sq * p.Sq;
  }
  const long long cells = p.Sq > 1 ? p.Tcells : p.Tmax;
  const dim3 grid((unsigned)(wide ? cells : (cells + kTileWaves - 1) / kTileWaves));
  // classes per chunk: edge_chunk(k), which F's row stride is a multiple of
#define KZ_EDGE(FI, KC)                                                                                       \
  do {                                                                                                        \
    if (wide)                                                                                                 \
      hipLaunchKernelGGL((k_edge<FI, KC, kTileWaves>), grid, dim3(kEdgeThreads), 0, s, p, src, dst, pass, F, S); \
    else                                                                                                      \
      hipLaunchKernelGGL((k_edge<FI, KC, 1>), grid, dim3(kEdgeThreads), 0, s, p, src, dst, pass, F, S);       \
  } while (0)
#define KZ_EDGE_K(FI)                \
  switch (edge_chunk(p.k)) {         \
    case 4: KZ_EDGE(FI, 4); break;   \
    case 8: KZ_EDGE(FI, 8); break;   \
    case 12: KZ_EDGE(FI, 12); break; \
    case 16: KZ_EDGE(FI, 16); break; \
    case 20: KZ_EDGE(FI, 20); break; \
    case 24: KZ_EDGE(FI, 24); break; \
    case 28: KZ_EDGE(FI, 28); break; \
    default: KZ_EDGE(FI, 32); break; \
  }
  if (first) {
    KZ_EDGE_K(true)
  } else {
    KZ_EDGE_K(false)
  }
#undef KZ_EDGE_K
#undef KZ_EDGE
}

void launch_edge_pass_mfma(const Plan &p, const uint64_t *src, uint64_t *dst, uint64_t *fb, int pass, bool first,
                           hipStream_t s) {
  if (p.Tmax <= 0) return;
  const dim3 grid((unsigned)p.Tmax), tgrid((unsigned)((p.Tmax + kTileWaves - 1) / kTileWaves));
  if (first) {
    hipLaunchKernelGGL((k_mfma_count<true>), grid, dim3(kMfThreads), 0, s, p, src, fb, pass);
    hipLaunchKernelGGL((k_edge_mf<true>), tgrid, dim3(kEdgeThreads), 0, s, p, src, dst, pass, (const uint64_t *)fb);
  } else {
    hipLaunchKernelGGL((k_mfma_count<false>), grid, dim3(kMfThreads), 0, s, p, src, fb, pass);
    hipLaunchKernelGGL((k_edge_mf<false>), tgrid, dim3(kEdgeThreads), 0, s, p, src, dst, pass, (const uint64_t *)fb);
  }
}

// End of pass `pass` (one wave): the pass's counters, summed over their
// slots, fold into the result; the run is done at the first pass that
// removes nothing (the fixpoint of section 4.2's iterated pruning), or at
// pass 1 when validation found an input error.
__global__ void __launch_bounds__(64) k_pass_end(Plan p, int pass, int csr, kz_out *out) {
  Hdr *h = p.hdr;
  if (h->done) return;
  const int lane = threadIdx.x, par = pass & 1;
  unsigned long long c0 = 0, c1 = 0, c2 = 0, c3 = 0;
  if (lane < kCtrSlots) {
    c0 = h->ctr(par, lane, 0);
    c1 = h->ctr(par, lane, 1);
    c2 = h->ctr(par, lane, 2);
    c3 = h->ctr(1, lane, 3);  // CSR: entries above minus below the diagonal, with pass 1's counters
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    c0 += (unsigned long long)__shfl_xor((long long)c0, off, kWave);
    c1 += (unsigned long long)__shfl_xor((long long)c1, off, kWave);
    c2 += (unsigned long long)__shfl_xor((long long)c2, off, kWave);
    c3 += (unsigned long long)__shfl_xor((long long)c3, off, kWave);
  }
  if (lane != 0) return;
  kz_out o = h->out;
  int st = KZ_OK;
  if (pass == 1) {
    int prio = h->prio;
    if (csr && c3 != 0 && prio < P_EASYM) prio = P_EASYM;  // an entry without its reverse
    st = h->bad_colour           ? KZ_ECOLOUR
         : h->bad_layout         ? KZ_EINVAL
         : prio == P_EINVAL      ? KZ_EINVAL
         : prio == P_ESELFLOOP   ? KZ_ESELFLOOP
         : prio == P_EASYM       ? KZ_EASYM
         : prio == P_EILLEGAL    ? KZ_EILLEGAL
                                 : KZ_OK;
  }
  if (st != KZ_OK) {
    o = kz_out{};
    o.result.status = st;
    o.converged = 1;
  } else {
    if (pass == 1) {
      // pass 1 tests every edge once: the input's edge count
      o.result.input_edges = (long long)c2;
      o.result.surviving_edges = (long long)c2;
      o.result.surviving_vertices = p.n;
    }
    o.result.edge_tests += (long long)c2;
    o.result.surviving_vertices -= (long long)c0;
    o.result.surviving_edges -= (long long)c1;
    o.result.passes = pass;
    o.last_removed = (long long)(c0 + c1);
    if (c0 + c1 == 0) o.converged = 1;
    else o.result.rounds += 1;
    o.result.equals_input = o.result.rounds == 0;
  }
  h->out = o;
  if (o.converged) h->done = 1;
  if (out) *out = o;
}

__global__ void k_write_out(kz_out *out, kz_out v) { *out = v; }

void launch_pass_end(const Plan &p, int pass, bool csr, kz_out *out, hipStream_t s) {
  hipLaunchKernelGGL(k_pass_end, dim3(1), dim3(64), 0, s, p, pass, csr ? 1 : 0, out);
}

void launch_write_out(kz_out *out, const kz_out &v, hipStream_t s) {
  hipLaunchKernelGGL(k_write_out, dim3(1), dim3(1), 0, s, out, v);
}

void launch_apply(const Plan &p, const uint64_t *scratch, uint64_t *cur, hipStream_t s) {
  if (p.Tmax <= 0) return;
  hipLaunchKernelGGL(k_apply, dim3(grid_for(p.Tmax, 1, 4096)), dim3(128), 0, s, p, scratch, cur);
}

void launch_unpack_dense(const Plan &p, const int *colour, const uint64_t *cur, uint8_t *vmask,
                         uint8_t *emask, hipStream_t s) {
  const int use_lds = p.Rmax <= kPackLdsWords;
  const size_t lds = use_lds ? sizeof(unsigned long long) * (size_t)p.Rmax : 0;
  hipLaunchKernelGGL(k_unpack_dense, dim3(p.n), dim3(256), lds, s, p, colour, cur, vmask, emask, use_lds);
}

}  // namespace kzi
