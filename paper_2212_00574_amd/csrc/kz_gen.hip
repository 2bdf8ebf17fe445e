// Synthetic workload materialiser (gfx950): writes the class-major bit rows
// of a seeded random legally coloured graph straight into device memory, so
// large served requests need no host generation or upload.
//
// Edge rule (the same draw the host generator uses): an inter-class slot
// pair {a < b} of graph `gid` under `seed` is an edge iff
//   splitmix64(splitmix64((seed << 32) | gid) ^ ((a << 32) | b)) < thr,
// with thr = floor(p * 2^64) and splitmix64 the output function of Steele,
// Lea and Flood's SplitMix64 generator (OOPSLA 2014).  Pairs inside a class
// are never edges.  A planted clique (one slot per class) forces every pair
// among its slots.  Nothing here is part of the kernelization method.
#include "kz_internal.h"

namespace kzi {

namespace {

__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ int class_of(const int *off, int k, int x) {
  int lo = 0, hi = k - 1;  // last c with off[c] <= x
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// One thread per output word (row v, word w).
__global__ void __launch_bounds__(256) k_gen_rows(GenArgs g, uint64_t *rows, int *colour) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = (long long)g.n * g.R;
  if (i >= total) return;
  const int v = (int)(i / g.R), w = (int)(i % g.R);
  const int cv = class_of(g.coff, g.k, v);
  if (colour && w == 0) colour[v] = cv;
  const int c = class_of(g.soff, g.k, w);  // first class whose segment holds word w
  unsigned long long word = 0;
  if (c != cv) {
    const int b0 = g.coff[c] + 64 * (w - g.soff[c]), b1 = min(b0 + 64, g.coff[c + 1]);
    const bool vp = g.planted && g.pl[cv] == v;
    for (int b = b0; b < b1; ++b) {
      const unsigned long long lo = (unsigned long long)min(v, b), hi = (unsigned long long)max(v, b);
      bool e = mix64(g.base ^ ((lo << 32) | hi)) < g.thr;
      if (vp && g.pl[c] == b) e = true;
      word |= (unsigned long long)e << (b - b0);
    }
  }
  rows[i] = word;
}

}  // namespace

void launch_gen_rows(const GenArgs &g, uint64_t *rows, int *colour, hipStream_t s) {
  const long long total = (long long)g.n * g.R;
  if (total <= 0) return;
  const unsigned blocks = (unsigned)((total + 255) / 256);
  hipLaunchKernelGGL(k_gen_rows, dim3(blocks), dim3(256), 0, s, g, rows, colour);
}

}  // namespace kzi
