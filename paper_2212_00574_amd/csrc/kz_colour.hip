// Upstream legal colouring (gfx950): Jones and Plassmann's parallel greedy
// colouring (SIAM J. Sci. Comput. 14(3), 1993) of a graph given as plain bit
// rows, for inputs that arrive without the legal colouring the colour-index
// method of section 4.2 needs.
//
// Every vertex v has the key (priority[v], v), compared lexicographically.
// A round takes every uncoloured vertex whose key beats the key of each of
// its uncoloured neighbours; each vertex taken gets the smallest colour that
// no neighbour coloured in an earlier round holds.  Vertices taken in one
// round are pairwise non-adjacent, so the colouring is legal and independent
// of the order in which a round's vertices are coloured.
//
// Layout: U, a bit set of the uncoloured vertices (ceil(n/64) words); per
// round one wave per vertex tests row & U (only uncoloured neighbours can
// beat it), then one wave per taken vertex marks the colours of row & ~U in
// an LDS bitmap and takes its lowest zero bit.  A taken vertex clears its own
// bit of U in the same kernel: the other vertices taken in the round are not
// its neighbours, so no one reads that bit for it.
#include <string.h>

#include <algorithm>

#include "kz.h"
#include "kz_internal.h"

namespace {

constexpr int kColWaves = 4;                // waves (vertices) per workgroup
constexpr int kColMaxWords = 1024;          // row words (65536 vertices)
constexpr size_t kColAlign = 256;
constexpr int kColFirstChunk = 8;           // rounds enqueued before the first look at the count
constexpr int kColMaxChunk = 128;           // ... and at most between two looks

struct ColCtr {
  int left;    // vertices not yet coloured; every round kernel returns at once at 0
  int bad;     // validation: a KZ_* status, most severe first (see k_col_check)
  int maxc;    // largest colour given
  int rounds;  // rounds that ran
};

size_t col_up(size_t x) { return (x + kColAlign - 1) / kColAlign * kColAlign; }

struct ColWs {
  size_t ctr, U, sel, total;
};

ColWs col_ws(int n) {
  ColWs w{};
  size_t o = 0;
  w.ctr = o;
  o += col_up(sizeof(ColCtr));
  w.U = o;
  o += col_up(sizeof(uint64_t) * (size_t)((n + 63) / 64 + 1));
  w.sel = o;
  o += col_up((size_t)n + 1);
  w.total = o;
  return w;
}

__device__ __forceinline__ bool key_beats(unsigned long long pu, int u, unsigned long long pv, int v) {
  return pu > pv || (pu == pv && u > v);
}

// Validation and set-up, one wave per row: no bit at or beyond n
// (KZ_EINVAL), no self-loop (KZ_ESELFLOOP), symmetric (KZ_EASYM); the
// most severe found wins (EINVAL, then ESELFLOOP, then EASYM).  colour = -1,
// U = every vertex.
__global__ void __launch_bounds__(kColWaves * 64) k_col_check(int n, const uint64_t *__restrict__ rows, int R,
                                                              int *colour, uint64_t *U, ColCtr *ctr) {
  const int lane = threadIdx.x & 63;
  const int v = blockIdx.x * kColWaves + (threadIdx.x >> 6);
  if (v >= n) return;
  const uint64_t *row = rows + (long long)v * R;
  int bad = 0;  // 3 EINVAL, 2 ESELFLOOP, 1 EASYM
  for (int w = lane; w < R; w += 64) {
    unsigned long long x = row[w];
    const int lo = 64 * w;
    if (lo + 64 > n) {
      const unsigned long long past = lo >= n ? ~0ull : ~0ull << (n - lo);
      if (x & past) bad = max(bad, 3);
      x &= ~past;
    }
    while (x) {
      const int b = __builtin_ctzll(x);
      x &= x - 1;
      const int u = lo + b;
      if (u == v) bad = max(bad, 2);
      else if (!((rows[(long long)u * R + (v >> 6)] >> (v & 63)) & 1ull)) bad = max(bad, 1);
    }
  }
  for (int off = 32; off > 0; off >>= 1) bad = max(bad, __shfl_xor(bad, off, 64));
  if (lane == 0) {
    colour[v] = -1;
    if (bad) atomicMax(&ctr->bad, bad);
    if (v == 0) ctr->left = n;
  }
  if (lane == 0 && (v & 63) == 0) {
    const int nb = min(64, n - v);
    U[v >> 6] = nb == 64 ? ~0ull : (1ull << nb) - 1;
  }
}

// One round's choice, one wave per vertex: sel[v] = v is uncoloured and its
// key beats every uncoloured neighbour's.
__global__ void __launch_bounds__(kColWaves * 64) k_col_select(int n, const uint64_t *__restrict__ rows, int R,
                                                               const uint64_t *__restrict__ pri,
                                                               const uint64_t *__restrict__ U, uint8_t *sel,
                                                               ColCtr *ctr) {
  const int lane = threadIdx.x & 63;
  const int v = blockIdx.x * kColWaves + (threadIdx.x >> 6);
  if (ctr->left == 0) return;  // coloured in an earlier round of this chunk
  if (v == 0 && lane == 0) atomicAdd(&ctr->rounds, 1);
  if (v >= n) return;
  const bool unc = (U[v >> 6] >> (v & 63)) & 1ull;
  if (!unc) {
    if (lane == 0) sel[v] = 0;
    return;
  }
  const uint64_t *row = rows + (long long)v * R;
  const unsigned long long pv = pri[v];
  const int W = (n + 63) >> 6;
  bool beaten = false;
  for (int w0 = 0; w0 < W; w0 += 64) {
    const int w = w0 + lane;
    if (w < W) {
      unsigned long long x = row[w] & U[w];
      while (x && !beaten) {
        const int b = __builtin_ctzll(x);
        x &= x - 1;
        const int u = 64 * w + b;
        beaten = key_beats(pri[u], u, pv, v);
      }
    }
    if (__ballot(beaten)) break;
  }
  const bool taken = __ballot(beaten) == 0ull;
  if (lane == 0) sel[v] = taken ? 1 : 0;
}

// One round's colours, one wave per vertex taken: the smallest colour that
// no neighbour coloured earlier holds; then v leaves U.
__global__ void __launch_bounds__(kColWaves * 64) k_col_colour(int n, const uint64_t *__restrict__ rows, int R,
                                                               const uint8_t *__restrict__ sel, uint64_t *U,
                                                               int *colour, ColCtr *ctr) {
  __shared__ unsigned long long used[kColWaves][kColMaxWords];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int v = blockIdx.x * kColWaves + wid;
  // left is 0 here only if it was 0 when this round's select kernel read it
  // (that kernel then returned at once and sel is a previous round's): a
  // vertex taken in this round keeps it positive until its own wave below
  // has coloured it
  if (v >= n || ctr->left == 0 || !sel[v]) return;
  const int W = (n + 63) >> 6;
  unsigned long long *mine = used[wid];
  for (int w = lane; w < W; w += 64) mine[w] = 0ull;
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  const uint64_t *row = rows + (long long)v * R;
  for (int w = lane; w < W; w += 64) {
    unsigned long long x = row[w] & ~U[w];  // neighbours coloured in earlier rounds
    while (x) {
      const int b = __builtin_ctzll(x);
      x &= x - 1;
      const int c = colour[64 * w + b];
      if (c >= 0 && c < 64 * W) atomicOr(&mine[c >> 6], 1ull << (c & 63));
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  // the lowest zero bit: the first word with a zero, in lane order
  int c = -1;
  for (int w0 = 0; w0 < W && c < 0; w0 += 64) {
    const int w = w0 + lane;
    const unsigned long long free = w < W ? ~mine[w] : 0ull;
    const unsigned long long has = __ballot(free != 0ull);
    if (has) {
      const int first = __builtin_ctzll(has);
      const unsigned long long f = __shfl(free, first, 64);
      c = 64 * (w0 + first) + __builtin_ctzll(f);
    }
  }
  if (c < 0) c = 64 * W;  // every colour below 64*W held (cannot happen: v has fewer than n neighbours)
  if (lane == 0) {
    colour[v] = c;
    atomicMax(&ctr->maxc, c);
    atomicAnd(&U[v >> 6], ~(1ull << (v & 63)));
    atomicSub(&ctr->left, 1);
  }
}

}  // namespace

extern "C" {

int kz_colour_workspace_bytes(int32_t n, size_t *bytes) {
  if (!bytes || n < 0) return KZ_EINVAL;
  *bytes = col_ws(n).total;
  return KZ_OK;
}

int kz_colour_jp(kz_ctx *ctx, int32_t n, const uint64_t *rows, int32_t row_words, const uint64_t *priority,
                 void *ws, size_t ws_bytes, int32_t *colour, void *stream, kz_colour_result *res) {
  kz_colour_result r{};
  r.status = KZ_EINVAL;
  auto done = [&]() {
    if (res) *res = r;
    return r.status;
  };
  if (!ctx || n < 0 || row_words < 0) return done();
  if (n == 0) {
    r.status = KZ_OK;
    return done();
  }
  if (!rows || !priority || !colour || !ws || (uintptr_t)ws % kColAlign) return done();
  if (row_words < (n + 63) / 64) return done();
  if (row_words > kColMaxWords) {
    r.status = KZ_ETOOLARGE;
    return done();
  }
  const ColWs z = col_ws(n);
  if (ws_bytes < z.total) {
    r.status = KZ_EWORKSPACE;
    return done();
  }
  r.status = KZ_EHIP;
  if (hipSetDevice(ctx->device) != hipSuccess) return done();
  hipStream_t s = (hipStream_t)stream;
  char *base = (char *)ws;
  ColCtr *ctr = (ColCtr *)(base + z.ctr);
  uint64_t *U = (uint64_t *)(base + z.U);
  uint8_t *sel = (uint8_t *)(base + z.sel);
  ColCtr *h = (ColCtr *)ctx->pinned;  // the context's pinned readback buffer (4 KiB)
  const dim3 grid((unsigned)((n + kColWaves - 1) / kColWaves)), block(kColWaves * 64);
  if (hipMemsetAsync(ctr, 0, sizeof(ColCtr), s) != hipSuccess) return done();
  hipLaunchKernelGGL(k_col_check, grid, block, 0, s, n, rows, (int)row_words, colour, U, ctr);
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(h, ctr, sizeof(ColCtr), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return done();
  if (h->bad) {
    r.status = h->bad == 3 ? KZ_EINVAL : h->bad == 2 ? KZ_ESELFLOOP : KZ_EASYM;
    return done();
  }
  // rounds in chunks, ended on the device: one readback per chunk (rounds
  // past the last one return at once)
  int chunk = kColFirstChunk, last_left = n;
  for (;;) {
    for (int i = 0; i < chunk; ++i) {
      hipLaunchKernelGGL(k_col_select, grid, block, 0, s, n, rows, (int)row_words, priority, U, sel, ctr);
      hipLaunchKernelGGL(k_col_colour, grid, block, 0, s, n, rows, (int)row_words, sel, U, colour, ctr);
    }
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(h, ctr, sizeof(ColCtr), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return done();
    if (h->left == 0) break;
    if (h->left >= last_left) return done();  // cannot happen: every round takes the largest uncoloured key
    last_left = h->left;
    chunk = std::min(2 * chunk, kColMaxChunk);
  }
  r.status = KZ_OK;
  r.rounds = h->rounds;
  r.colours = h->maxc + 1;
  return done();
}

}  // extern "C"
