// HIP kernels (gfx950) of the colour-index kernelizer for sparse graphs
// given as CSR (both directions, column ids strictly increasing per row).
//
// The state is kept in the caller's order, in the output buffers themselves:
// vmask[v] (vertex alive) and emask[e] (entry e of col_idx alive; both
// directions of an edge always agree).  Per vertex the pass keeps PM(v), the
// set of colour classes holding an alive neighbour of v (KW 64-bit words).
//
// Tests (thesis section 4.2, vertex and edge colour indices):
//   vertex v fails   <=> PM(v) misses a class other than class(v);
//   edge {u,v} fails <=> some class outside {class(u), class(v)} holds no
//                        common alive neighbour.  Quick reject: such a class
//                        is certainly empty when PM(u) & PM(v) misses it;
//                        otherwise the two sorted rows are merged and the
//                        classes of common alive neighbours collected, until
//                        every third class has one.
// Both directions of an edge are tested independently (same answer), so a
// failing entry clears only itself and no reverse-entry index is needed.
#include "kz_internal.h"

namespace kzi {

namespace {

__device__ __forceinline__ bool csr_bad(const Hdr *h) { return (h->bad_colour | h->bad_layout) != 0; }

__device__ __forceinline__ int wave_sum_i(int x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
  return x;
}

// Adds two per-wave counts into counter slots (par, slot, j0) and (par,
// slot, j1) with one atomic each per workgroup of 4 waves: the counter lines
// take one update per workgroup instead of one per wave.  Every thread of the
// workgroup calls it.
__device__ __forceinline__ void wg_add2(Hdr *h, int par, int j0, long long a, int j1, long long b) {
  __shared__ long long sRed[4][2];
  const int wv = threadIdx.x >> 6;
  a = (long long)wave_sum_i((int)a);
  b = (long long)wave_sum_i((int)b);
  if ((threadIdx.x & 63) == 0) {
    sRed[wv][0] = a;
    sRed[wv][1] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const long long ta = sRed[0][0] + sRed[1][0] + sRed[2][0] + sRed[3][0];
    const long long tb = sRed[0][1] + sRed[1][1] + sRed[2][1] + sRed[3][1];
    const int slot = blockIdx.x % kCtrSlots;
    if (ta) atomicAdd(&h->ctr(par, slot, j0), (unsigned long long)ta);
    if (tb) atomicAdd(&h->ctr(par, slot, j1), (unsigned long long)tb);
  }
}

// Row bounds of u, or false when they do not lie inside [0, nnz].
__device__ __forceinline__ bool row_ok(const int64_t *rp, int u, long long nnz, long long &b, long long &e) {
  b = rp[u];
  e = rp[u + 1];
  return b >= 0 && b <= e && e <= nnz;
}

// Whether u is among entries [vb, ve) of col_idx (strictly increasing).
// With `vec` (col_idx 16-byte aligned) the search walks aligned pieces of
// four entries, one 16-byte load each: a piece whose valid entries bracket u
// decides, otherwise half of the remaining pieces are dropped.  Entries of
// neighbouring rows that share a boundary piece are ignored; a piece that
// would reach past nnz is read entry by entry.
__device__ __forceinline__ bool row_has(const int32_t *ci, long long nnz, long long vb, long long ve, int u,
                                        bool vec) {
  if (vb >= ve) return false;
  if (!vec) {
    long long lo = vb, hi = ve;
    while (lo < hi) {
      const long long mid = lo + (hi - lo) / 2;
      if (ci[mid] < u) lo = mid + 1;
      else hi = mid;
    }
    return lo < ve && ci[lo] == u;
  }
  long long lo = vb >> 2, hi = (ve - 1) >> 2;  // pieces, inclusive
  while (lo <= hi) {
    const long long mid = lo + (hi - lo) / 2;
    const long long e0 = mid << 2;
    int x0, x1, x2, x3;
    if (e0 + 3 < nnz) {
      const int4 q = *(const int4 *)(ci + e0);
      x0 = q.x;
      x1 = q.y;
      x2 = q.z;
      x3 = q.w;
    } else {
      x0 = ci[e0];
      x1 = e0 + 1 < nnz ? ci[e0 + 1] : 0;
      x2 = e0 + 2 < nnz ? ci[e0 + 2] : 0;
      x3 = 0;
    }
    // the piece's entries inside [vb, ve): positions jf..jl
    const int jf = (int)(vb > e0 ? vb - e0 : 0);
    const int jl = (int)(ve - 1 - e0 < 3 ? ve - 1 - e0 : 3);
    const int f = jf == 0 ? x0 : jf == 1 ? x1 : jf == 2 ? x2 : x3;
    const int l = jl == 0 ? x0 : jl == 1 ? x1 : jl == 2 ? x2 : x3;
    if (u < f) {
      hi = mid - 1;
    } else if (u > l) {
      lo = mid + 1;
    } else {
      return (jf <= 0 && x0 == u) || (jf <= 1 && jl >= 1 && x1 == u) || (jf <= 2 && jl >= 2 && x2 == u) ||
             (jl >= 3 && x3 == u);
    }
  }
  return false;
}

// Pass 1's sweep over the rows, one wave per row u: the colour range (stage
// 1), the structure and stage-2 checks, the start of the state (every entry
// alive, every vertex touched, the row of every entry recorded) and pass 1's
// vertex test with u's presence mask, all from one read of the row.
template <int KW>
__global__ void __launch_bounds__(256) k_csr_first(Plan p, const int64_t *rp, const int32_t *ci,
                                                   long long nnz, const int *colour, uint8_t *vmask,
                                                   uint8_t *emask) {
  Hdr *h = p.hdr;
  __shared__ unsigned long long sPM[4][KW];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int u = blockIdx.x * 4 + wv;
  const int n = p.n, k = p.k;
  int balance = 0;  // entries above the diagonal minus entries below it
  bool uf = false;  // u fails pass 1's vertex test
  const bool vec = ((uintptr_t)ci & 15) == 0;
  long long b, e;
  // stage 1: every colour in [0,k) (also on rows whose bounds are broken)
  const int cu = u < n ? colour[u] : 0;
  if (u < n && lane == 0 && (cu < 0 || cu >= k)) h->bad_colour = 1;
  if (u < n && !row_ok(rp, u, nnz, b, e)) {
    if (lane == 0) atomicMax(&h->prio, P_EINVAL);
  } else if (u < n) {
    int pr = P_NONE;
    if (u == 0 && lane == 0 && rp[0] != 0) pr = P_EINVAL;
    if (u == n - 1 && lane == 0 && rp[n] != nnz) pr = P_EINVAL;
    if (lane < KW) sPM[wv][lane] = 0;
    __builtin_amdgcn_wave_barrier();
    for (long long i = b + lane; i < e; i += kWave) {
      const int v = ci[i];
      p.src[i] = u;
      emask[i] = 1;
      p.efail[i] = 0;
      if (v < 0 || v >= n || (i > b && ci[i - 1] >= v)) {
        pr = max(pr, P_EINVAL);
        continue;
      }
      if (v == u) {
        pr = max(pr, P_ESELFLOOP);
        continue;
      }
      const int cv = colour[v];
      if (cv == cu) pr = max(pr, P_EILLEGAL);
      if (cv >= 0 && cv < k) atomicOr(&sPM[wv][cv >> 6], 1ull << (cv & 63));
      // Symmetry: every entry (u,v) with v > u must have its reverse (v,u),
      // found by binary search in row v; with as many entries below the
      // diagonal as above it (summed on the host), reversal then maps the
      // upper entries onto the lower ones, so the lower ones need no search.
      if (v < u) {
        --balance;
        continue;
      }
      ++balance;
      long long vb, ve;
      const bool found = row_ok(rp, v, nnz, vb, ve) && row_has(ci, nnz, vb, ve, u, vec);
      if (!found) pr = max(pr, P_EASYM);
    }
    if (pr) atomicMax(&h->prio, pr);
    __builtin_amdgcn_wave_barrier();
    // pass 1's vertex test: u fails iff some class other than its own is
    // missing from PM(u)
    bool fail = false;
    if (lane == KW) p.pm[(long long)u * (KW + 1) + KW] = (unsigned long long)(unsigned)cu;  // record: colour
    if (lane < KW) {
      const unsigned long long pm = sPM[wv][lane];
      p.pm[(long long)u * (KW + 1) + lane] = pm;
      const int lo = lane * 64;
      unsigned long long want = 0;
      if (k > lo) want = (k - lo >= 64) ? ~0ull : ((1ull << (k - lo)) - 1);
      if ((cu >> 6) == lane) want &= ~(1ull << (cu & 63));
      fail = (want & ~pm) != 0;
    }
    uf = __ballot(fail) != 0;
    if (lane == 0) {
      vmask[u] = uf ? 0 : 1;
      p.touched[1][u] = 1;
      p.touched[0][u] = 0;
    }
  }
  // removed vertices and the balance, counted with pass 1's counters
  wg_add2(h, 1, 0, lane == 0 && uf ? 1 : 0, 3, balance);
}

// Vertex test and presence masks of passes after the first.  One wave per
// vertex, lanes over its entries; only the alive vertices touched by the
// previous round.  Also resets this pass's bookkeeping.
template <int KW>
__global__ void __launch_bounds__(256) k_csr_vertex(Plan p, const int64_t *rp, const int32_t *ci,
                                                    const int *colour, uint8_t *vmask,
                                                    const uint8_t *emask, int pass) {
  Hdr *h = p.hdr;
  if (csr_bad(h) || h->prio || h->done) return;
  const int n = p.n, k = p.k;
  const int cur = pass & 1, nxt = cur ^ 1;
  {
    const long long gt = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = gt; i < n; i += stride) p.touched[nxt][i] = 0;
    if (gt < kCtrSlots * 4) h->ctr(nxt, gt / 4, gt % 4) = 0;
  }
  __shared__ unsigned long long sPM[4][KW];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int v = blockIdx.x * 4 + wv;
  if (v >= n) return;
  if (!vmask[v] || !p.touched[cur][v]) return;
  if (lane < KW) sPM[wv][lane] = 0;
  __builtin_amdgcn_wave_barrier();
  const long long b = rp[v], e = rp[v + 1];
  for (long long i = b + lane; i < e; i += kWave) {
    if (!emask[i]) continue;
    const int c = colour[ci[i]];
    atomicOr(&sPM[wv][c >> 6], 1ull << (c & 63));
  }
  __builtin_amdgcn_wave_barrier();
  // v fails iff some class other than its own is missing from PM(v)
  const int cv = colour[v];
  bool fail = false;
  if (lane < KW) {
    const unsigned long long pm = sPM[wv][lane];
    p.pm[(long long)v * (KW + 1) + lane] = pm;
    const int lo = lane * 64;
    unsigned long long want = 0;
    if (k > lo) want = (k - lo >= 64) ? ~0ull : ((1ull << (k - lo)) - 1);
    if ((cv >> 6) == lane) want &= ~(1ull << (cv & 63));
    fail = (want & ~pm) != 0;
  }
  const bool vf = __ballot(fail) != 0;
  if (lane == 0) {
    if (vf) {
      vmask[v] = 0;
      atomicAdd(&h->ctr(cur, blockIdx.x % kCtrSlots, 0), 1ull);
    }
  }
}

// Edge test, one thread per directed entry.  A failing entry is flagged for
// the apply pass, counted once per undirected edge (u < v) and marks its row
// u touched for the next pass (the reverse entry fails too and marks v).
template <bool FIRST, int KW>
__global__ void __launch_bounds__(256) k_csr_edge(Plan p, const int64_t *rp, const int32_t *ci,
                                                  long long nnz, const int *colour, const uint8_t *emask,
                                                  int pass) {
  Hdr *h = p.hdr;
  if (csr_bad(h) || h->prio || h->done) return;
  const int k = p.k;
  const int cur = pass & 1, nxt = cur ^ 1;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  bool tested = false, removed = false;
  int marks = -1;  // row to mark touched (the entry failed)
  if (i < nnz && emask[i]) {
    const int u = p.src[i], v = ci[i];
    if (FIRST || p.touched[cur][u] || p.touched[cur][v]) {
      tested = u < v;
      // each endpoint's record: its presence mask, then its colour
      const uint64_t *ru = p.pm + (long long)u * (KW + 1), *rv = p.pm + (long long)v * (KW + 1);
      unsigned long long mu[KW + 1], mv[KW + 1];
      if constexpr (KW == 1) {
        const ulonglong2 a = *(const ulonglong2 *)ru, c = *(const ulonglong2 *)rv;
        mu[0] = a.x;
        mu[1] = a.y;
        mv[0] = c.x;
        mv[1] = c.y;
      } else {
#pragma unroll
        for (int j = 0; j <= KW; ++j) {
          mu[j] = ru[j];
          mv[j] = rv[j];
        }
      }
      const int cu = (int)mu[KW], cv = (int)mv[KW];
      unsigned long long need[KW];
      bool fail = false;
#pragma unroll
      for (int j = 0; j < KW; ++j) {
        const int lo = j * 64;
        need[j] = k > lo ? ((k - lo >= 64) ? ~0ull : ((1ull << (k - lo)) - 1)) : 0ull;
        if ((cu >> 6) == j) need[j] &= ~(1ull << (cu & 63));
        if ((cv >> 6) == j) need[j] &= ~(1ull << (cv & 63));
        fail |= (need[j] & ~(mu[j] & mv[j])) != 0;
      }
      if (!fail) {
        // merge the sorted rows; collect classes of common alive neighbours
        long long a = rp[u], ae = rp[u + 1], c = rp[v], ce = rp[v + 1];
        bool done = true;  // nothing left to find (k <= 2)?
#pragma unroll
        for (int j = 0; j < KW; ++j) done &= need[j] == 0;
        while (a < ae && c < ce && !done) {
          const int x = ci[a], y = ci[c];
          if (x < y) {
            ++a;
          } else if (y < x) {
            ++c;
          } else {
            if (emask[a] && emask[c]) {
              const int cw = colour[x];
              done = true;
#pragma unroll
              for (int j = 0; j < KW; ++j)
                if ((cw >> 6) == j) need[j] &= ~(1ull << (cw & 63));
#pragma unroll
              for (int j = 0; j < KW; ++j) done &= need[j] == 0;
            }
            ++a;
            ++c;
          }
        }
        fail = !done;
      }
      if (fail) {
        p.efail[i] = 1;
        marks = u;
        removed = u < v;
      }
    }
  }
  // entries are in row order: of the lanes marking one row, only the first
  // of each run stores the flag
  const int prev = __shfl_up(marks, 1, kWave);
  if (marks >= 0 && ((threadIdx.x & 63) == 0 || prev != marks)) p.touched[nxt][marks] = 1;
  wg_add2(h, cur, 2, tested ? 1 : 0, 1, removed ? 1 : 0);
}

// Removes the entries that failed this pass (after every test of the pass
// has read the old masks).  Four entries per thread.
__global__ void __launch_bounds__(256) k_csr_apply(Plan p, long long nnz, uint8_t *emask) {
  const Hdr *h = p.hdr;
  if (csr_bad(h) || h->prio || h->done) return;
  const long long i0 = ((long long)blockIdx.x * blockDim.x + threadIdx.x) * 4;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const long long i = i0 + j;
    if (i < nnz && p.efail[i]) {
      p.efail[i] = 0;
      emask[i] = 0;
    }
  }
}

inline unsigned grid_of(long long work, int per_block) {
  long long g = (work + per_block - 1) / per_block;
  return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace

int csr_words(int k) { return k <= 64 ? 1 : (k <= 256 ? 4 : 16); }

void launch_csr_first(const Plan &p, const int64_t *rp, const int32_t *ci, long long nnz, const int *colour,
                      uint8_t *vmask, uint8_t *emask, hipStream_t s) {
  const dim3 grid(grid_of(p.n, 4)), block(256);
  const int kw = csr_words(p.k);
  if (kw == 1) hipLaunchKernelGGL((k_csr_first<1>), grid, block, 0, s, p, rp, ci, nnz, colour, vmask, emask);
  else if (kw == 4) hipLaunchKernelGGL((k_csr_first<4>), grid, block, 0, s, p, rp, ci, nnz, colour, vmask, emask);
  else hipLaunchKernelGGL((k_csr_first<16>), grid, block, 0, s, p, rp, ci, nnz, colour, vmask, emask);
}

void launch_csr_vertex(const Plan &p, const int64_t *rp, const int32_t *ci, const int *colour, uint8_t *vmask,
                       const uint8_t *emask, int pass, hipStream_t s) {
  const dim3 grid(grid_of(p.n, 4)), block(256);
  const int kw = csr_words(p.k);
#define KZ_CSR_V(W) hipLaunchKernelGGL((k_csr_vertex<W>), grid, block, 0, s, p, rp, ci, colour, vmask, emask, pass)
  if (kw == 1) KZ_CSR_V(1);
  else if (kw == 4) KZ_CSR_V(4);
  else KZ_CSR_V(16);
#undef KZ_CSR_V
}

void launch_csr_edge(const Plan &p, const int64_t *rp, const int32_t *ci, long long nnz, const int *colour,
                     const uint8_t *emask, int pass, bool first, hipStream_t s) {
  if (nnz <= 0) return;
  const dim3 grid(grid_of(nnz, 256)), block(256);
  const int kw = csr_words(p.k);
#define KZ_CSR_E(F, W) hipLaunchKernelGGL((k_csr_edge<F, W>), grid, block, 0, s, p, rp, ci, nnz, colour, emask, pass)
  if (first) {
    if (kw == 1) KZ_CSR_E(true, 1);
    else if (kw == 4) KZ_CSR_E(true, 4);
    else KZ_CSR_E(true, 16);
  } else {
    if (kw == 1) KZ_CSR_E(false, 1);
    else if (kw == 4) KZ_CSR_E(false, 4);
    else KZ_CSR_E(false, 16);
  }
#undef KZ_CSR_E
}

void launch_csr_apply(const Plan &p, long long nnz, uint8_t *emask, hipStream_t s) {
  if (nnz <= 0) return;
  hipLaunchKernelGGL(k_csr_apply, dim3(grid_of(nnz, 1024)), dim3(256), 0, s, p, nnz, emask);
}

}  // namespace kzi
