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
// F[c][v] (the first two words of row v's class-c segment), which the edge
// pass stages from.  Also resets the bookkeeping the edge pass of this pass
// fills.
__global__ void __launch_bounds__(256) k_vertex(Plan p, const int *scls, const uint64_t *__restrict__ src,
                                                int pass) {
  Hdr *h = p.hdr;
  if (stage1_bad(h)) return;
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
        ulonglong2 *Fcv = (ulonglong2 *)p.F + ((long long)c * n + v);
        if (active) *Fcv = make_ulonglong2(x0[g], x1[g]);
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
// padding bits past a class's size.  The first two words of every segment
// fill the first-word matrix F.  All loads of a piece are independent of
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
      p.F[2 * ((long long)c * n + v0 + r)] = 0ull;
      p.F[2 * ((long long)c * n + v0 + r) + 1] = 0ull;
    }
  };
  if (lds_off) {
    for (int c = tid; c < k; c += 256)
      if (sOff[1][c] == sOff[1][c + 1]) empty_class(c);
  } else {
    for (int c = tid; c < k; c += 256)
      if (p.soff[c] == p.soff[c + 1]) empty_class(c);
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
        if (off < 2) p.F[2 * ((long long)cw * n + v) + off] = xi;
        if (off == 0 && ends) p.F[2 * ((long long)cw * n + v) + 1] = 0ull;
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

// The i-th class other than cx and cy (cx < cy): the third classes of a tile.
__device__ __forceinline__ int third_class(int i, int cx, int cy) {
  int c = i;
  if (c >= cx) ++c;
  if (c >= cy) ++c;
  return c;
}

// Edge test for every edge of one inter-class block pair (X, Y), X < Y.
//
// Lane v of each wave stands for slot bstart[Y]+v; wave w handles 16 rows u
// of block X.  P(u) is the 64-bit set of v with {u,v} still passing.  The
// tile walks its third classes (every class but class(X) and class(Y)) in
// chunks of CH, staged from the first-word matrix: the first two words of
// every row's class-c segment, row u's in LDS (read as broadcasts), row v's
// in the lane's registers.  Level 1: the first words of u and v are ANDed
// and a wave ballot gives the lanes with a common neighbour there; the
// ballots of the chunk are ANDed.  Level 2, when some edge of u is not
// covered: the same with the first two words.  Level 3 (rare): class by
// class, the lanes still missing a witness scan the rest of the segment in
// memory.  Padding slots of the last chunk hold all-ones words, so they never
// drop a lane.  Wave 0 then turns the rows P(u) into the new word X of every
// row v with a lane butterfly transpose (and, in pass 1, checks the input's
// symmetry the same way).  When a bit of the tile changed, both copies of
// its new bits go to `dst` (pass 1: the output state, which already holds a
// copy of the input; later passes: scratch, and the tile is listed for the
// apply pass).  MF: the witness search is replaced by the fail bits `fb` of
// the MFMA count path (k_mfma_count), so both paths share this tile
// epilogue.  Six-class chunks keep the kernel within 80 registers, so six
// waves fit on a SIMD; eight-class chunks are held to five (96 registers),
// which lets every tile of a 50-block row width be resident at once.
template <bool FIRST, int CH, bool MF>
__global__ void __launch_bounds__(kEdgeThreads, CH == 6 ? 6 : 5) k_edge(Plan p, const uint64_t *__restrict__ src,
                                                       uint64_t *__restrict__ dst, int pass,
                                                       const uint64_t *__restrict__ fb) {
  Hdr *h = p.hdr;
  const int k = p.k;
  const int cur = pass & 1, nxt = cur ^ 1;
  int X, Y;
  tri_decode(xcd_remap(blockIdx.x, gridDim.x), p.Rmax, X, Y);
  // one round of independent loads (X, Y < Rmax: the block table is in
  // bounds even where this call's layout is shorter or invalid)
  const int bad = h->bad_colour | h->bad_layout, R = h->R;
  const int cx = p.bcls[X], cy = p.bcls[Y];
  const int xs = p.bstart[X], xl = p.blen[X];
  const int ys = p.bstart[Y], yl = p.blen[Y];
  const bool btouch = FIRST || (p.btouched[cur][X] | p.btouched[cur][Y]);
  if (bad || Y >= R || cx == cy || !btouch) return;

  constexpr int kWaves = kEdgeThreads / kWave;
  constexpr int kRowsPerWave = kBlk / kWaves;
  constexpr int kStage = (CH * kBlk + kEdgeThreads - 1) / kEdgeThreads;
  __shared__ ulonglong2 sU[CH][kBlk];
  __shared__ unsigned long long sV2[CH][kBlk];
  __shared__ unsigned long long sE[kBlk], sP[kBlk];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  const unsigned long long ymask = yl == 64 ? ~0ull : ((1ull << yl) - 1);
  const unsigned long long xmask = xl == 64 ? ~0ull : ((1ull << xl) - 1);
  const int nthird = MF ? 0 : k - 2;
  const int n = p.n;
  const ulonglong2 *F = (const ulonglong2 *)p.F;
  const int ur = tid & 63;                      // staging row of this thread
  const int urc = ur < xl ? ur : xl - 1;        // clamped into the block
  const int vrc = lane < yl ? lane : yl - 1;
  const uint64_t *rowv = src + (long long)(ys + vrc) * R;

  // Staging of one chunk of CH third classes from the first-word matrix:
  // `issue` loads (the third classes follow from cx and cy alone, so these
  // loads go out together with the tile's own), `stage` writes row u's two
  // first words to LDS (read as broadcasts) and keeps row v's first word in
  // the lane's registers.  Padding slots of the last chunk hold all-ones.
  // Row v's second words go to LDS too, class j by wave j % kWaves.
  constexpr int kV2 = (CH + kWaves - 1) / kWaves;
  ulonglong2 uu[kStage];
  unsigned long long vv[CH], vy[kV2];
  auto issue = [&](int q) {
#pragma unroll
    for (int e2 = 0; e2 < kStage; ++e2) {
      const int e = tid + e2 * kEdgeThreads;
      const int i = q + (e < CH * kBlk ? e >> 6 : 0);
      const int c = i < nthird ? third_class(i, cx, cy) : 0;
      uu[e2] = F[(long long)c * n + xs + urc];
    }
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const int c = q + j < nthird ? third_class(q + j, cx, cy) : 0;
      vv[j] = F[(long long)c * n + ys + vrc].x;
    }
#pragma unroll
    for (int jj = 0; jj < kV2; ++jj) {
      const int j = wid + jj * kWaves;
      const int c = j < CH && q + j < nthird ? third_class(q + j, cx, cy) : 0;
      vy[jj] = F[(long long)c * n + ys + vrc].y;
    }
  };
  auto stage = [&](int q) {
#pragma unroll
    for (int e2 = 0; e2 < kStage; ++e2) {
      const int e = tid + e2 * kEdgeThreads;
      if (e < CH * kBlk) {
        const int j = e >> 6;
        sU[j][ur] = q + j < nthird ? uu[e2] : make_ulonglong2(~0ull, ~0ull);
      }
    }
#pragma unroll
    for (int jj = 0; jj < kV2; ++jj) {
      const int j = wid + jj * kWaves;
      if (j < CH) sV2[j][lane] = q + j < nthird ? (lane < yl ? vy[jj] : 0ull) : ~0ull;
    }
#pragma unroll
    for (int j = 0; j < CH; ++j) vv[j] = q + j < nthird ? (lane < yl ? vv[j] : 0ull) : ~0ull;
  };

  // row index clamped into the block so the load is always in bounds
  const unsigned long long e0 = tid < kBlk ? src[(long long)(xs + urc) * R + Y] : 0ull;
  if (nthird > 0) issue(0);
  const unsigned long long ET = lane < yl ? rowv[X] : 0ull;  // used by the transpose
  // pairs to re-test: those with a touched endpoint (all of them in pass 1);
  // the others keep their outcome, so masks and rounds equal full sweeps
  const unsigned long long TU = FIRST ? ~0ull : __ballot(lane < xl && p.touched[cur][xs + lane]);
  const unsigned long long TV = FIRST ? ~0ull : __ballot(lane < yl && p.touched[cur][ys + lane]);
  if (tid < kBlk) {
    sE[tid] = tid < xl ? e0 : 0ull;
    sP[tid] = tid < xl ? (e0 & ymask) : 0ull;
  }
  if (MF) {
    // pairs with a touched endpoint take the MFMA path's outcome; the others
    // keep theirs (each thread updates the word it wrote itself)
    if (tid < xl) {
      const unsigned long long Pt = ((TU >> tid) & 1ull) ? ~0ull : TV;
      sP[tid] &= ~(fb[(long long)(xs + tid) * R + Y] & Pt);
    }
  }
  for (int q = 0; q < nthird; q += CH) {
    if (q > 0) {
      issue(q);
      __syncthreads();  // every wave is done with the previous chunk
    }
    stage(q);
    __syncthreads();    // also publishes sE / sP before the first chunk
    // P of the wave's rows, lane i holding row wid*kRowsPerWave + i: one LDS
    // read per chunk instead of one per row (a row's P changes only in its
    // own iteration below)
    const unsigned long long Pw = sP[wid * kRowsPerWave + (lane & (kRowsPerWave - 1))];
    for (int ui = 0; ui < kRowsPerWave; ++ui) {
      const int u = wid * kRowsPerWave + ui;
      if (u >= xl) break;
      unsigned long long P = ((unsigned long long)(unsigned)__builtin_amdgcn_readlane((int)(Pw >> 32), ui) << 32) |
                             (unsigned)__builtin_amdgcn_readlane((int)Pw, ui);
      const unsigned long long Pt = P & (((TU >> u) & 1ull) ? ~0ull : TV);
      if (!Pt) continue;
      unsigned long long all = ~0ull;
      {
        unsigned long long a[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j) a[j] = sU[j][u].x;
#pragma unroll
        for (int j = 0; j < CH; ++j) all &= __ballot((a[j] & vv[j]) != 0ull);
      }
      if (!(Pt & ~all)) continue;
      // level 2: the first two words (re-read from LDS; rare)
      all = ~0ull;
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        const ulonglong2 a = sU[j][u];
        all &= __ballot(((a.x & vv[j]) | (a.y & sV2[j][lane])) != 0ull);
      }
      if (!(Pt & ~all)) continue;
      // level 3: class by class, scanning the rest of the segment
      const uint64_t *rowu = src + (long long)(xs + u) * R;
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        if (q + j >= nthird) break;
        const ulonglong2 a = sU[j][u];
        unsigned long long miss = Pt & ~__ballot(((a.x & vv[j]) | (a.y & sV2[j][lane])) != 0ull);
        const int c = third_class(q + j, cx, cy);
        const int w1 = p.soff[c + 1];
        for (int w = p.soff[c] + 2; w < w1 && miss; ++w) {
          const unsigned long long x = rowu[w];
          const unsigned long long y = ((miss >> lane) & 1ull) ? rowv[w] : 0ull;
          miss &= ~__ballot((x & y) != 0ull);
        }
        P &= ~miss;
      }
      if (lane == 0) sP[u] = P;
    }
  }
  __syncthreads();

  if (wid != 0) return;

  // wave 0: lane v gets bit v of every P(u) -- the new word X of row v --
  // and, in pass 1, of every E(u), to check that the rows are symmetric
  const int v = lane;
  const unsigned long long newET = wave_transpose64(sP[lane], lane) & xmask;
  if (FIRST) {
    const unsigned long long trE = wave_transpose64(sE[lane], lane);
    if (v < yl && ((trE ^ ET) & xmask)) atomicMax(&h->prio, P_EASYM);
  }
  const unsigned long long Eu = sE[lane] & ymask, Pu = sP[lane];
  const bool chU = lane < xl && Eu != Pu;
  const bool chV = v < yl && (ET & xmask) != newET;
  const unsigned long long bu = __ballot(chU), bv = __ballot(chV);
  if (bu | bv) {
    if (lane < xl) dst[(long long)(xs + lane) * R + Y] = Pu;
    if (v < yl) dst[(long long)(ys + v) * R + X] = newET;
    if (chU) p.touched[nxt][xs + lane] = 1;
    if (chV) p.touched[nxt][ys + v] = 1;
    const int rem = wave_sum(lane < xl ? __popcll(Eu & ~Pu) : 0);
    if (lane == 0) {
      if (bu) p.btouched[nxt][X] = 1;
      if (bv) p.btouched[nxt][Y] = 1;
      if (!FIRST) {
        const int pos = atomicAdd(&h->tile_count, 1);
        p.tiles[pos] = make_int2(X, Y);
      }
      atomicAdd(&h->ctr(cur, blockIdx.x % kCtrSlots, 1), (unsigned long long)rem);
    }
  }
  // exact worklist size: edges of this tile with a touched endpoint
  int cnt;
  if (FIRST) {
    cnt = wave_sum(lane < xl ? __popcll(Eu) : 0);
  } else {
    const int tU = lane < xl ? p.touched[cur][xs + lane] : 0;
    const int tV = v < yl ? p.touched[cur][ys + v] : 0;
    const unsigned long long TV = __ballot(tV != 0);
    cnt = wave_sum(lane < xl ? __popcll(Eu & (tU ? ~0ull : TV)) : 0);
  }
  if (lane == 0 && cnt) atomicAdd(&h->ctr(cur, blockIdx.x % kCtrSlots, 2), (unsigned long long)cnt);
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
  if (stage1_bad(h)) return;
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
    if (idx >= 0) cur[idx] = scratch[idx];
  }
}

// Bit rows -> dense u8 masks in caller order.  One workgroup per caller row.
__global__ void __launch_bounds__(256) k_unpack_dense(Plan p, const int *colour, const uint64_t *cur,
                                                      uint8_t *vmask, uint8_t *emask, int use_lds) {
  const Hdr *h = p.hdr;
  if (stage1_bad(h)) return;
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

void launch_edge_pass(const Plan &p, const uint64_t *src, uint64_t *dst, int pass, bool first, hipStream_t s) {
  if (p.Tmax <= 0) return;
  const dim3 grid((unsigned)p.Tmax);
  // chunk of third classes: whichever of 6 and 8 pads the k-2 classes least
  const int nthird = p.k > 2 ? p.k - 2 : 0;
  const bool six = (nthird + 5) / 6 * 6 < (nthird + 7) / 8 * 8;
  const uint64_t *nofb = nullptr;
#define KZ_EDGE(F, C) hipLaunchKernelGGL((k_edge<F, C, false>), grid, dim3(kEdgeThreads), 0, s, p, src, dst, pass, nofb)
  if (first) {
    if (six) KZ_EDGE(true, 6);
    else KZ_EDGE(true, 8);
  } else {
    if (six) KZ_EDGE(false, 6);
    else KZ_EDGE(false, 8);
  }
#undef KZ_EDGE
}

void launch_edge_pass_mfma(const Plan &p, const uint64_t *src, uint64_t *dst, uint64_t *fb, int pass, bool first,
                           hipStream_t s) {
  if (p.Tmax <= 0) return;
  const dim3 grid((unsigned)p.Tmax);
  if (first) {
    hipLaunchKernelGGL((k_mfma_count<true>), grid, dim3(kMfThreads), 0, s, p, src, fb, pass);
    hipLaunchKernelGGL((k_edge<true, 8, true>), grid, dim3(kEdgeThreads), 0, s, p, src, dst, pass,
                       (const uint64_t *)fb);
  } else {
    hipLaunchKernelGGL((k_mfma_count<false>), grid, dim3(kMfThreads), 0, s, p, src, fb, pass);
    hipLaunchKernelGGL((k_edge<false, 8, true>), grid, dim3(kEdgeThreads), 0, s, p, src, dst, pass,
                       (const uint64_t *)fb);
  }
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
