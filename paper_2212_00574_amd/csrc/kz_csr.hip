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

// Row bounds of u, or false when they do not lie inside [0, nnz].
__device__ __forceinline__ bool row_ok(const int64_t *rp, int u, long long nnz, long long &b, long long &e) {
  b = rp[u];
  e = rp[u + 1];
  return b >= 0 && b <= e && e <= nnz;
}

// Colour range (stage 1), structure and stage-2 checks, one wave per row;
// also records the row of every entry and starts the state (everything
// alive, everything touched).
__global__ void __launch_bounds__(256) k_csr_validate(Plan p, const int64_t *rp, const int32_t *ci,
                                                      long long nnz, const int *colour, uint8_t *vmask,
                                                      uint8_t *emask) {
  Hdr *h = p.hdr;
  if (csr_bad(h)) return;
  const int u = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int n = p.n;
  if (u >= n) return;
  // stage 1: every colour in [0,k)
  const int cu = colour[u];
  if (lane == 0 && (cu < 0 || cu >= p.k)) h->bad_colour = 1;
  int pr = P_NONE;
  if (u == 0 && lane == 0 && rp[0] != 0) pr = P_EINVAL;
  if (u == n - 1 && lane == 0 && rp[n] != nnz) pr = P_EINVAL;
  long long b, e;
  if (!row_ok(rp, u, nnz, b, e)) {
    if (lane == 0) atomicMax(&h->prio, P_EINVAL);
    return;
  }
  if (lane == 0) {
    vmask[u] = 1;
    p.touched[1][u] = 1;
    p.touched[0][u] = 0;
  }
  int balance = 0;  // entries above the diagonal minus entries below it
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
    // Symmetry: every entry (u,v) with v > u must have its reverse (v,u),
    // found by binary search in row v; with as many entries below the
    // diagonal as above it (summed on the host), reversal then maps the
    // upper entries onto the lower ones, so the lower ones need no search.
    // The same-class check likewise covers both directions from above.
    if (v < u) {
      --balance;
      continue;
    }
    ++balance;
    long long vb, ve;
    bool found = false;
    if (row_ok(rp, v, nnz, vb, ve)) {
      long long lo = vb, hi = ve;
      while (lo < hi) {
        const long long mid = lo + (hi - lo) / 2;
        const int x = ci[mid];
        if (x < u) lo = mid + 1;
        else hi = mid;
      }
      found = lo < ve && ci[lo] == u;
    }
    if (!found) pr = max(pr, P_EASYM);
    if (colour[v] == cu) pr = max(pr, P_EILLEGAL);
  }
  if (pr) atomicMax(&h->prio, pr);
  balance = wave_sum_i(balance);
  if (lane == 0 && balance)
    atomicAdd(&h->ctr[1][blockIdx.x % kCtrSlots][3], (unsigned long long)(long long)balance);
}

// Vertex test and presence masks.  One wave per vertex, lanes over its
// entries.  Pass 1 processes every vertex; later passes the alive vertices
// touched by the previous round.  Also resets this pass's bookkeeping.
template <bool FIRST, int KW>
__global__ void __launch_bounds__(256) k_csr_vertex(Plan p, const int64_t *rp, const int32_t *ci,
                                                    const int *colour, uint8_t *vmask,
                                                    const uint8_t *emask, int pass) {
  Hdr *h = p.hdr;
  if (csr_bad(h) || h->prio) return;
  const int n = p.n, k = p.k;
  const int cur = pass & 1, nxt = cur ^ 1;
  {
    const long long gt = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    if (!FIRST)
      for (long long i = gt; i < n; i += stride) p.touched[nxt][i] = 0;
    if (gt < kCtrSlots * 4) (&h->ctr[nxt][0][0])[gt] = 0;
  }
  __shared__ unsigned long long sPM[4][KW];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int v = blockIdx.x * 4 + wv;
  if (v >= n) return;
  if (!FIRST && (!vmask[v] || !p.touched[cur][v])) return;
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
    p.pm[(long long)v * KW + lane] = pm;
    const int lo = lane * 64;
    unsigned long long want = 0;
    if (k > lo) want = (k - lo >= 64) ? ~0ull : ((1ull << (k - lo)) - 1);
    if ((cv >> 6) == lane) want &= ~(1ull << (cv & 63));
    fail = (want & ~pm) != 0;
  }
  const bool vf = __ballot(fail) != 0;
  if (lane == 0) {
    if (FIRST) vmask[v] = vf ? 0 : 1;
    else if (vf) vmask[v] = 0;
    if (vf) atomicAdd(&h->ctr[cur][blockIdx.x % kCtrSlots][0], 1ull);
  }
}

// Edge test, one thread per directed entry.
template <bool FIRST, int KW>
__global__ void __launch_bounds__(256) k_csr_edge(Plan p, const int64_t *rp, const int32_t *ci,
                                                  long long nnz, const int *colour, const uint8_t *emask,
                                                  int pass) {
  Hdr *h = p.hdr;
  if (csr_bad(h) || h->prio) return;
  const int k = p.k;
  const int cur = pass & 1;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  bool tested = false;
  if (i < nnz && emask[i]) {
    const int u = p.src[i], v = ci[i];
    if (FIRST || p.touched[cur][u] || p.touched[cur][v]) {
      tested = u < v;
      const int cu = colour[u], cv = colour[v];
      unsigned long long need[KW];
      bool fail = false;
#pragma unroll
      for (int j = 0; j < KW; ++j) {
        const int lo = j * 64;
        need[j] = k > lo ? ((k - lo >= 64) ? ~0ull : ((1ull << (k - lo)) - 1)) : 0ull;
        if ((cu >> 6) == j) need[j] &= ~(1ull << (cu & 63));
        if ((cv >> 6) == j) need[j] &= ~(1ull << (cv & 63));
        fail |= (need[j] & ~(p.pm[(long long)u * KW + j] & p.pm[(long long)v * KW + j])) != 0;
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
      if (fail) p.efail[i] = 1;
    }
  }
  const int cnt = wave_sum_i(tested ? 1 : 0);
  if ((threadIdx.x & 63) == 0 && cnt)
    atomicAdd(&h->ctr[cur][blockIdx.x % kCtrSlots][2], (unsigned long long)cnt);
}

// Removes the entries that failed this pass and marks their endpoints.
__global__ void __launch_bounds__(256) k_csr_apply(Plan p, const int32_t *ci, long long nnz, uint8_t *emask,
                                                   int pass) {
  Hdr *h = p.hdr;
  if (csr_bad(h) || h->prio) return;
  const int cur = pass & 1, nxt = cur ^ 1;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  bool removed = false;
  if (i < nnz && p.efail[i]) {
    const int u = p.src[i], v = ci[i];
    p.efail[i] = 0;
    emask[i] = 0;
    p.touched[nxt][u] = 1;
    p.touched[nxt][v] = 1;
    removed = u < v;
  }
  const int cnt = wave_sum_i(removed ? 1 : 0);
  if ((threadIdx.x & 63) == 0 && cnt)
    atomicAdd(&h->ctr[cur][blockIdx.x % kCtrSlots][1], (unsigned long long)cnt);
}

inline unsigned grid_of(long long work, int per_block) {
  long long g = (work + per_block - 1) / per_block;
  return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace

int csr_words(int k) { return k <= 64 ? 1 : (k <= 256 ? 4 : 16); }

void launch_csr_validate(const Plan &p, const int64_t *rp, const int32_t *ci, long long nnz, const int *colour,
                         uint8_t *vmask, uint8_t *emask, hipStream_t s) {
  hipLaunchKernelGGL(k_csr_validate, dim3(grid_of(p.n, 4)), dim3(256), 0, s, p, rp, ci, nnz, colour, vmask,
                     emask);
}

void launch_csr_vertex(const Plan &p, const int64_t *rp, const int32_t *ci, const int *colour, uint8_t *vmask,
                       const uint8_t *emask, int pass, bool first, hipStream_t s) {
  const dim3 grid(grid_of(p.n, 4)), block(256);
  const int kw = csr_words(p.k);
#define KZ_CSR_V(F, W) hipLaunchKernelGGL((k_csr_vertex<F, W>), grid, block, 0, s, p, rp, ci, colour, vmask, emask, pass)
  if (first) {
    if (kw == 1) KZ_CSR_V(true, 1);
    else if (kw == 4) KZ_CSR_V(true, 4);
    else KZ_CSR_V(true, 16);
  } else {
    if (kw == 1) KZ_CSR_V(false, 1);
    else if (kw == 4) KZ_CSR_V(false, 4);
    else KZ_CSR_V(false, 16);
  }
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

void launch_csr_apply(const Plan &p, const int32_t *ci, long long nnz, uint8_t *emask, int pass, hipStream_t s) {
  if (nnz <= 0) return;
  hipLaunchKernelGGL(k_csr_apply, dim3(grid_of(nnz, 256)), dim3(256), 0, s, p, ci, nnz, emask, pass);
}

}  // namespace kzi
