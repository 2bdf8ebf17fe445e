// Struction (thesis section 4.1, Definition 4.1.1) on plain bit rows
// (gfx950).  Around a pivot p: A = the neighbours of p and B = the other
// vertices except p; C holds a node c(x, y) for every edge {x, y} inside B
// with x < y.  G' has the nodes A (in vertex order) followed by C (ordered
// by x, then y):
//   A-A: as in G;  C-C: c(x,y) ~ c(x',y') iff x = x' and y ~ y';
//   A-C: a ~ c(x,y) iff a ~ x and a ~ y (the rule that makes Lemmas 1 and 2
//   hold; the thesis states none), so omega(G') = omega(G) - 1.
//
// Plan: B's mask, every vertex's place in A, and for every x in B the count
// of its C nodes (neighbours y > x in B), scanned into offsets.  Build: the
// node map; M[v] = row v compressed onto A's index space (bit t = v ~ A[t]);
// then one thread per output word: the A part of a word is M[a] (A row) or
// M[x] & M[y] (C row); the C part of a C row is non-zero only inside its own
// first vertex's block (y ~ y'), that of an A row holds a ~ x' and a ~ y'.
#include "kz_internal.h"

namespace kzi {

namespace {

struct StHdr {
  long long na, nc;    // |A|, |C|
  long long edges2;    // set bits of the input
  int prio;            // input problems (P_*)
  int pad;
};

__device__ __forceinline__ bool bit(const uint64_t *row, int v) { return (row[v >> 6] >> (v & 63)) & 1ull; }

// Validation (padding bits, self-loops, symmetry) and bit count; B's mask
// (one thread per word of the pivot's row).
__global__ void __launch_bounds__(256) k_st_check(const uint64_t *__restrict__ rows, int n, int R, int pivot,
                                                  uint64_t *__restrict__ bmask, StHdr *h) {
  const long long total = (long long)n * R;
  const long long stride = (long long)gridDim.x * blockDim.x;
  unsigned long long cnt = 0;
  int pr = P_NONE;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int v = (int)(i / R), w = (int)(i % R);
    unsigned long long x = rows[i];
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
      else if (!bit(rows + (long long)t * R, v)) pr = max(pr, (int)P_EASYM);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    cnt += __shfl_xor(cnt, off, kWave);
    pr = max(pr, __shfl_xor(pr, off, kWave));
  }
  if ((threadIdx.x & 63) == 0) {
    if (cnt) atomicAdd((unsigned long long *)&h->edges2, cnt);
    if (pr != P_NONE) atomicMax(&h->prio, pr);
  }
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w < R) {
    const long long lo = 64LL * w;
    uint64_t valid = lo + 64 <= n ? ~0ull : lo < n ? (1ull << (n - lo)) - 1 : 0ull;
    if (w == (pivot >> 6)) valid &= ~(1ull << (pivot & 63));
    bmask[w] = ~rows[(long long)pivot * R + w] & valid;
  }
}

// Every vertex's place in A (or -1), and every B vertex's count of C nodes.
__global__ void __launch_bounds__(256) k_st_count(const uint64_t *__restrict__ rows, int n, int R, int pivot,
                                                  const uint64_t *__restrict__ bmask, int *__restrict__ apos,
                                                  long long *__restrict__ ccount) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const uint64_t *rp = rows + (long long)pivot * R;
  const int vw = v >> 6;
  if (bit(rp, v)) {
    int before = __popcll(rp[vw] & ((1ull << (v & 63)) - 1));
    for (int w = 0; w < vw; ++w) before += __popcll(rp[w]);
    apos[v] = before;
    ccount[v] = 0;
  } else {
    apos[v] = -1;
    long long c = 0;
    if (bit(bmask, v)) {
      const uint64_t *rv = rows + (long long)v * R;
      // neighbours y > v inside B
      c = __popcll(rv[vw] & bmask[vw] & ((v & 63) == 63 ? 0ull : ~0ull << ((v & 63) + 1)));
      for (int w = vw + 1; w < R; ++w) c += __popcll(rv[w] & bmask[w]);
    }
    ccount[v] = c;
  }
}

// Exclusive scan of the counts into C offsets (one workgroup); |A| and |C|.
__global__ void __launch_bounds__(1024) k_st_scan(const long long *__restrict__ ccount, int n, int na,
                                                 long long *__restrict__ coff, StHdr *h) {
  __shared__ long long part[1024];
  const int tid = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int lo = tid * per, hi = min(n, lo + per);
  long long s = 0;
  for (int v = lo; v < hi; ++v) s += ccount[v];
  part[tid] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const long long x = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += x;
    __syncthreads();
  }
  long long run = part[tid] - s;
  for (int v = lo; v < hi; ++v) {
    coff[v] = run;
    run += ccount[v];
  }
  if (tid == 1023) {
    coff[n] = part[1023];
    h->na = na;
    h->nc = part[1023];
  }
}

// The node map: (v, -1) for A nodes, (x, y) for C nodes (one thread per vertex).
__global__ void __launch_bounds__(256) k_st_map(const uint64_t *__restrict__ rows, int n, int R,
                                                const uint64_t *__restrict__ bmask, const int *__restrict__ apos,
                                                const long long *__restrict__ coff, long long na,
                                                int *__restrict__ map) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  if (apos[v] >= 0) {
    map[2LL * apos[v]] = v;
    map[2LL * apos[v] + 1] = -1;
    return;
  }
  if (!bit(bmask, v)) return;
  const uint64_t *rv = rows + (long long)v * R;
  long long at = na + coff[v];
  const int vw = v >> 6;
  for (int w = vw; w < R; ++w) {
    uint64_t x = rv[w] & bmask[w];
    if (w == vw) x &= (v & 63) == 63 ? 0ull : ~0ull << ((v & 63) + 1);
    while (x) {
      const int y = 64 * w + __builtin_ctzll(x);
      x &= x - 1;
      map[2 * at] = v;
      map[2 * at + 1] = y;
      ++at;
    }
  }
}

// M[v][j] bit t = v ~ A[64 j + t] (one thread per word of M).
__global__ void __launch_bounds__(256) k_st_compress(const uint64_t *__restrict__ rows, int n, int R,
                                                     const int *__restrict__ map, int na, int RA,
                                                     uint64_t *__restrict__ M) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)n * RA) return;
  const int v = (int)(i / RA), j = (int)(i % RA);
  const uint64_t *rv = rows + (long long)v * R;
  uint64_t x = 0;
  for (int t = 0; t < 64 && 64 * j + t < na; ++t)
    if (bit(rv, map[2 * (64 * j + t)])) x |= 1ull << t;
  M[i] = x;
}

// One output word: node i's adjacency to the nodes 64 j .. 64 j + 63.
__global__ void __launch_bounds__(256) k_st_rows(const uint64_t *__restrict__ rows, int R,
                                                 const uint64_t *__restrict__ M, int RA,
                                                 const int *__restrict__ map, const long long *__restrict__ coff,
                                                 long long na, long long np, int RP, uint64_t *__restrict__ out) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= np * RP) return;
  const long long i = idx / RP;
  const int j = (int)(idx % RP);
  const long long lo = 64LL * j;
  uint64_t x = 0;
  if (lo < np) {
    const int xi = map[2 * i], yi = map[2 * i + 1];
    // A part: nodes lo .. min(lo + 64, na)
    if (lo < na) {
      uint64_t a = M[(long long)xi * RA + j];
      if (yi >= 0) a &= M[(long long)yi * RA + j];
      if (na - lo < 64) a &= (1ull << (na - lo)) - 1;
      x |= a;
    }
    // C part: nodes max(lo, na) .. min(lo + 64, np)
    const long long c0 = lo > na ? lo : na, c1 = lo + 64 < np ? lo + 64 : np;
    if (c0 < c1) {
      if (yi < 0) {
        const uint64_t *ra = rows + (long long)xi * R;
        for (long long q = c0; q < c1; ++q) {
          const int xq = map[2 * q], yq = map[2 * q + 1];
          if (bit(ra, xq) && bit(ra, yq)) x |= 1ull << (q - lo);
        }
      } else {
        // only the block of C nodes whose first vertex is xi
        const long long b0 = na + coff[xi], b1 = na + coff[xi + 1];
        const long long s0 = c0 > b0 ? c0 : b0, s1 = c1 < b1 ? c1 : b1;
        const uint64_t *ry = rows + (long long)yi * R;
        for (long long q = s0; q < s1; ++q)
          if (bit(ry, map[2 * q + 1])) x |= 1ull << (q - lo);
      }
    }
    if (i >= lo && i < lo + 64) x &= ~(1ull << (i - lo));
  }
  out[idx] = x;
}

struct StWs {
  size_t hdr, bmask, apos, ccount, coff, M, total;
};

StWs st_ws(int n, int R) {
  StWs z{};
  size_t o = 0;
  auto take = [&o](size_t b) {
    const size_t at = o;
    o += (b + 255) / 256 * 256;
    return at;
  };
  z.hdr = take(sizeof(StHdr));
  z.bmask = take(sizeof(uint64_t) * (size_t)(R > 0 ? R : 1));
  z.apos = take(sizeof(int) * (size_t)(n > 0 ? n : 1));
  z.ccount = take(sizeof(long long) * (size_t)(n > 0 ? n : 1));
  z.coff = take(sizeof(long long) * (size_t)(n + 1));
  z.M = take(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1) * (size_t)(R > 0 ? R : 1));
  z.total = o;
  return z;
}

int st_status(int prio) {
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

int kz_struction_workspace_bytes(int32_t n, int32_t row_words, size_t *bytes) {
  if (!bytes || n < 0 || row_words < (n + 63) / 64) return KZ_EINVAL;
  *bytes = kzi::st_ws(n, row_words).total;
  return KZ_OK;
}

int kz_struction(kz_ctx *ctx, int32_t n, const uint64_t *rows, int32_t row_words, int32_t pivot, void *ws,
                 size_t ws_bytes, uint64_t *out, int32_t out_row_words, int64_t out_nodes, int32_t *map,
                 void *stream, kz_struction_result *res) {
  using namespace kzi;
  kz_struction_result r{};
  auto done = [&](int st) {
    r.status = st;
    if (res) *res = r;
    return st;
  };
  if (!ctx || n < 1 || pivot < 0 || pivot >= n || row_words < (n + 63) / 64 || !rows || !ws || (uintptr_t)ws % 256)
    return done(KZ_EINVAL);
  const StWs z = st_ws(n, row_words);
  if (ws_bytes < z.total) return done(KZ_EWORKSPACE);
  if (hipSetDevice(ctx->device) != hipSuccess) return done(KZ_EHIP);
  hipStream_t s = (hipStream_t)stream;
  char *base = (char *)ws;
  StHdr *h = (StHdr *)(base + z.hdr);
  uint64_t *bmask = (uint64_t *)(base + z.bmask);
  int *apos = (int *)(base + z.apos);
  long long *ccount = (long long *)(base + z.ccount);
  long long *coff = (long long *)(base + z.coff);
  uint64_t *M = (uint64_t *)(base + z.M);
  const int R = row_words;
  if (hipMemsetAsync(h, 0, sizeof(StHdr), s) != hipSuccess) return done(KZ_EHIP);
  {
    const long long words = (long long)n * R;
    const int grid = (int)std::max<long long>(std::min<long long>((words + 255) / 256, 4096), (R + 255) / 256);
    hipLaunchKernelGGL(k_st_check, dim3(grid), dim3(256), 0, s, rows, n, R, pivot, bmask, h);
  }
  StHdr *hh = (StHdr *)ctx->pinned;
  if (hipGetLastError() != hipSuccess || hipMemcpyAsync(hh, h, sizeof(StHdr), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return done(KZ_EHIP);
  r.input_edges = hh->edges2 / 2;
  const int st0 = st_status(hh->prio);
  if (st0 != KZ_OK) return done(st0);
  hipLaunchKernelGGL(k_st_count, dim3((n + 255) / 256), dim3(256), 0, s, rows, n, R, pivot, bmask, apos, ccount);
  // |A| = the pivot's degree, from its row
  int na = 0;
  {
    std::vector<uint64_t> rp(R);
    if (hipMemcpyAsync(rp.data(), rows + (long long)pivot * R, sizeof(uint64_t) * R, hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return done(KZ_EHIP);
    for (int w = 0; w < R; ++w) na += __builtin_popcountll(rp[w]);
  }
  hipLaunchKernelGGL(k_st_scan, dim3(1), dim3(1024), 0, s, ccount, n, na, coff, h);
  if (hipGetLastError() != hipSuccess || hipMemcpyAsync(hh, h, sizeof(StHdr), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return done(KZ_EHIP);
  const long long np = hh->na + hh->nc;
  r.a_nodes = hh->na;
  r.c_nodes = hh->nc;
  r.nodes = np;
  r.row_words = (int32_t)((np + 63) / 64);
  if (!out) return done(KZ_OK);  // plan only
  if (!map || out_nodes < np || out_row_words < (np + 63) / 64) return done(KZ_EWORKSPACE);
  if (np == 0) return done(KZ_OK);
  const int RA = (int)((hh->na + 63) / 64);
  hipLaunchKernelGGL(k_st_map, dim3((n + 255) / 256), dim3(256), 0, s, rows, n, R, bmask, apos, coff, hh->na, map);
  if (RA > 0) {
    const long long mw = (long long)n * RA;
    hipLaunchKernelGGL(k_st_compress, dim3((unsigned)((mw + 255) / 256)), dim3(256), 0, s, rows, n, R, map,
                       (int)hh->na, RA, M);
  }
  const long long ow = np * out_row_words;
  hipLaunchKernelGGL(k_st_rows, dim3((unsigned)((ow + 255) / 256)), dim3(256), 0, s, rows, R, M, RA, map, coff,
                     hh->na, np, out_row_words, out);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return done(KZ_EHIP);
  return done(KZ_OK);
}

}  // extern "C"
