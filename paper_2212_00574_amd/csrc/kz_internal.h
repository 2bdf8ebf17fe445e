// Internal declarations shared by the kernels and the host driver of the
// colour-index kernelizer (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>
#include <stdint.h>

#include "kz.h"

namespace kzi {

constexpr int kWave = 64;          // CDNA wavefront
constexpr int kBlk = 64;           // slots per block == bits per word
constexpr int kEdgeThreads = 256;  // edge pass: 4 waves per workgroup
constexpr long long kEdgeWaveTiles = 16384;  // tiles from which the edge pass gives a tile one wave, not four
constexpr int kEdgeSquare = 16;              // then the side of its squares of tiles (in blocks)
constexpr int kMfThreads = 256;    // MFMA count path: 4 waves per 128x128 group tile
constexpr int kMfMaxWords = 2048;  // MFMA count path: row words it supports
constexpr int kRankChunk = 256;    // vertices per stable-partition chunk
constexpr int kPackLdsWords = 8192;  // dense pack: row assembled in LDS up to this many words
constexpr int kSetupThreads = 1024;  // the single setup workgroup
constexpr int kVertexLdsClasses = 2048;  // vertex pass keeps class offsets in LDS up to this k
constexpr int kVfRows = 16;  // rows per workgroup of the pass-1 vertex test (4 per wave)
constexpr int kSetupLdsClasses = 4096;  // class histogram kept in LDS up to this k

constexpr int kCtrSlots = 32;      // spread of the per-pass counters
constexpr int kCtrStride = 16;     // words per counter slot: 4 per pass parity, one cache line

// stage-2 status priorities (largest wins)
enum : int { P_NONE = 0, P_EILLEGAL = 1, P_EASYM = 2, P_ESELFLOOP = 3, P_EINVAL = 4 };

// Transposes a 64x64 bit matrix held one row per lane (lane l holds row l,
// bit b = column b): returns row l of the transpose, i.e. bit b of the
// result is bit l of lane b's input.  Six butterfly stages: at stage j,
// lanes l and l^j swap the j-wide column groups on the wrong side of the
// diagonal.  Every lane of the wave must take part.
__device__ __forceinline__ unsigned long long wave_transpose64(unsigned long long x, int lane) {
  constexpr unsigned long long kM[6] = {0xFFFFFFFF00000000ull, 0xFFFF0000FFFF0000ull, 0xFF00FF00FF00FF00ull,
                                        0xF0F0F0F0F0F0F0F0ull, 0xCCCCCCCCCCCCCCCCull, 0xAAAAAAAAAAAAAAAAull};
#pragma unroll
  for (int st = 0; st < 6; ++st) {
    const int j = 32 >> st;
    const unsigned long long m = kM[st];
    const unsigned long long y = (unsigned long long)__shfl_xor((long long)x, j, kWave);
    x = (lane & j) ? ((x & m) | ((y & m) >> j)) : ((x & ~m) | ((y & ~m) << j));
  }
  return x;
}

// Device-resident header at the start of the workspace.
struct Hdr {
  // Per slot and pass parity: removed vertices, removed edges, edge tests,
  // and a fourth counter that only the CSR validation uses (ctr(1, *, 3):
  // entries above minus entries below the diagonal, read with pass 1's
  // counters).  Workgroups add into slot (id % kCtrSlots) so that thousands
  // of same-address atomics do not serialise; each slot is one 128-byte
  // cache line holding both parities (atomics on one line serialise too,
  // and the host copies the header back every pass, so it stays 4 KiB); the
  // host sums the slots.
  unsigned long long ctrw[kCtrSlots][kCtrStride];
  __host__ __device__ unsigned long long &ctr(int par, int slot, int j) { return ctrw[slot][par * 4 + j]; }
  __host__ __device__ const unsigned long long &ctr(int par, int slot, int j) const {
    return ctrw[slot][par * 4 + j];
  }
  int tile_count;        // changed tiles appended by the edge pass
  int prio;              // stage-2 status priority
  int bad_colour;        // stage 1: some colour outside [0,k)
  int bad_layout;        // stage 1: bitset colours unsorted / row stride mismatch
  int R;                 // words per row == number of 64-slot blocks
  int n, k, pad;
  // the pass loop's state on the device (k_pass_end): set once a pass
  // removed nothing or pass 1 found an input error; every later pass kernel
  // of the run then returns at once
  int done, pad2;
  kz_out out;  // the result so far
};

// Device pointers of one kernelization (workspace carve-up + caller buffers).
struct Plan {
  Hdr *hdr;
  int *counts;       // [k] class sizes
  int *coff;         // [k+1] first slot of each class
  int *soff;         // [k+1] first word of each class segment
  int *bcls;         // [Rmax] class of block / word index
  int *bstart;       // [Rmax] first slot of block
  int *blen;         // [Rmax] slots in block (1..64)
  int *hist;         // [nchunks*k] per-chunk class histograms (dense only)
  int *perm;         // [n] slot -> caller vertex (dense only)
  int *inv;          // [n] caller vertex -> slot (dense only)
  int *scls;         // [n] class of each slot (dense; bitset uses colour)
  uint8_t *valive;   // [n] slot order (bitset: the caller's vmask)
  uint8_t *touched[2];   // [n]
  uint8_t *btouched[2];  // [Rmax]
  int2 *tiles;       // [Tmax] changed tiles of the current pass
  uint64_t *packed;  // [n*Rmax] dense input packed into bit rows (dense only)
  uint64_t *spare;   // [n*Rmax] second state buffer
  uint64_t *F;       // [n*kF] F[slot*kF + c]: the first word of the slot's class-c segment
                     // (0 for an empty class); all-ones for the slot's own class and
                     // for c >= k (so those classes never fail a first-word test)
  uint64_t *S;       // [n*kF] S[slot*kF + c]: the second word of the slot's class-c segment
                     // (0 where the segment is shorter)
  uint64_t *fb;      // [n*Rmax] MFMA count path: fail bits of the pairs of a pass
  int32_t *src;      // [nnz] csr: row of every entry
  uint8_t *efail;    // [nnz] csr: entry failed the edge test this pass
  uint64_t *pm;      // [n*(KW+1)] csr: per vertex the KW words of classes holding an alive
                     // neighbour, then its colour (one record, one gather per endpoint)
  int n, k, Rmax, nchunks;
  int kF;            // row stride of F: k rounded up to the edge pass's class chunk
  long long Tmax;    // Rmax*(Rmax-1)/2
  // the edge pass's tile order (set by its launcher): 0 or 1, row-major over
  // the triangle of block pairs; else squares of Sq x Sq block pairs, the
  // squares row-major over the triangle of squares, Tcells cells in all
  int Sq;
  long long Tcells;
};

// Classes per chunk of the bit-row edge test (the rows' first words of a
// chunk are held in 2*KC registers), and the row stride of F that makes
// every chunk's load of a row in bounds.
__host__ __device__ inline int edge_chunk(int k) { return k <= 4 ? 4 : k <= 32 ? (k + 3) / 4 * 4 : 32; }
__host__ __device__ inline int f_stride(int k) {
  const int c = edge_chunk(k);
  return (k + c - 1) / c * c;
}

struct WsSizes {
  size_t total;
  size_t off_counts, off_coff, off_soff, off_bcls, off_bstart, off_blen, off_hist, off_perm,
      off_inv, off_scls, off_valive, off_touched0, off_touched1, off_bt0, off_bt1, off_tiles,
      off_packed, off_spare, off_F, off_S, off_fb, off_src, off_efail, off_pm;
  int Rmax, nchunks;
  long long Tmax;
};

// Kernel launchers (kz_kernels.hip).  All asynchronous on `s`.
//
// Pass 1 ("first") reads the input rows `src`; its vertex pass copies them
// into `dst` and its edge pass rewrites the tiles that change, so `dst` ends
// up holding the state after round 1.  Later passes read the state `cur`,
// write changed tiles into `scratch`, and the apply pass copies them back
// into `cur`.  `row_words` of the vertex pass: the caller's row width for
// bit-row input, 0 for dense input (the width the setup pass computed).
enum SetupMode : int { SETUP_BITSET = 0, SETUP_DENSE = 1, SETUP_CSR = 2 };
void launch_setup(const Plan &p, const int *colour, int row_words, SetupMode mode, hipStream_t s);
void launch_rank(const Plan &p, const int *colour, hipStream_t s);
void launch_pack_dense(const Plan &p, const uint8_t *adj, const int *colour, uint64_t *dst,
                       hipStream_t s);
void launch_vertex_pass(const Plan &p, const int *scls, const uint64_t *src, uint64_t *dst, int pass,
                        bool first, int row_words, hipStream_t s);
void launch_edge_pass(const Plan &p, const uint64_t *src, uint64_t *dst, int pass, bool first,
                      hipStream_t s);
// The int8 MFMA count path of the edge test: fail bits of every pair (into
// `fb`, n*Rmax words), then the shared tile epilogue.
void launch_edge_pass_mfma(const Plan &p, const uint64_t *src, uint64_t *dst, uint64_t *fb, int pass, bool first,
                           hipStream_t s);
void launch_apply(const Plan &p, const uint64_t *scratch, uint64_t *cur, hipStream_t s);
// Ends pass `pass` on the device (one wave): folds its counters into the
// header's result, sets `done` at the fixpoint or on an input error, and
// copies the result to `out` when it is not null.
void launch_pass_end(const Plan &p, int pass, bool csr, kz_out *out, hipStream_t s);
void launch_write_out(kz_out *out, const kz_out &v, hipStream_t s);
void launch_unpack_dense(const Plan &p, const int *colour, const uint64_t *cur, uint8_t *vmask,
                         uint8_t *emask, hipStream_t s);

// Sparse path (kz_csr.hip).  State in place: vmask / emask (per entry).
int csr_words(int k);  // 64-bit words of a class set: 1, 4 or 16 (k <= 1024)
// Pass 1's validation, state start and vertex test in one sweep; later
// passes' vertex tests.
void launch_csr_first(const Plan &p, const int64_t *rp, const int32_t *ci, long long nnz, const int *colour,
                      uint8_t *vmask, uint8_t *emask, hipStream_t s);
void launch_csr_vertex(const Plan &p, const int64_t *rp, const int32_t *ci, const int *colour, uint8_t *vmask,
                       const uint8_t *emask, int pass, hipStream_t s);
void launch_csr_edge(const Plan &p, const int64_t *rp, const int32_t *ci, long long nnz, const int *colour,
                     const uint8_t *emask, int pass, bool first, hipStream_t s);
void launch_csr_apply(const Plan &p, long long nnz, uint8_t *emask, hipStream_t s);

// Batched path (kz_batch.hip).
constexpr int kBatchK = 64;          // classes
constexpr int kBatchR = 512;         // words per row (blocks)
constexpr int kBatchN = 32768;       // vertices
constexpr int kBatchSortMax = 8192;  // graphs ordered by work on the device up to this count
constexpr int kBatchBoard = 256;     // board of shared passes (job g posts at g mod its size): default
                                     // size, and the part one scan step of a wave reads
constexpr int kBatchTooLarge = KZ_ETOOLARGE;

// Per-graph buffers when graphs do not sit in shared arenas (served requests).
struct BatchPtrs {
  const uint64_t *rows;
  const int *colour;
  uint8_t *vmask;
  uint64_t *emask;
  uint64_t *next;  // n*row_words words
  int *lists;      // changed tiles: 2*n*row_words ints
  int *items;      // pass items: 2*n*row_words ints
};                 // every buffer starts on a 128-byte line

// One graph's job state in device memory.  Every word other workgroups
// update with atomics is only ever accessed with (agent-scope) atomics, and
// those words sit on cache lines of their own: a plain store to such a word
// could linger dirty in one XCD's L2 and overwrite atomic updates made
// meanwhile when it is written back.
struct alignas(128) BatchJob {
  // shared-pass control and merged counts (atomics only)
  unsigned long long claim;  // (pass << 40) | (items << 20) | next unclaimed item of a shared pass
  unsigned done;             // items finished in the shared pass
  int prio, nchanged, pad0;
  unsigned long long removed_v, removed_e, tests;
  unsigned touched[2][kBatchN / 32];                  // per pass parity: touched vertices
  unsigned btouched[2][kBatchR / 32];                 // and blocks
  // totals, kept by the carriers (atomic loads and stores)
  alignas(128) long long tot_removed_v, tot_removed_e, tot_tests, m;
  int rounds;
  // the number of the job's first pass, and the last pass opened in this
  // slot: a slot that takes a new job while the launch runs numbers its
  // passes on from the previous job's, so a workgroup holding a copy of an
  // earlier job's pass never mistakes it for one of the new job's
  int pass0, lastpass;
  // session mode: the request's descriptor, buffers and ticket, copied from
  // the host slot when the job starts (plain; read after the job's fences)
  alignas(128) kz_batch_graph sdesc;
  BatchPtrs sptrs;
  unsigned long long ticket;
  // layout, written when the job starts, read by helpers (plain)
  alignas(128) int coff[kBatchK + 1], soff[kBatchK + 1];
  short bcls[kBatchR];
  unsigned short bstart[kBatchR];
  unsigned char blen[kBatchR];
};


struct BatchArgs {
  const kz_batch_graph *graphs;
  const BatchPtrs *ptrs;  // [G] or null: then the arenas below and the descriptors' offsets
  int G;          // graphs (session mode: slots)
  int share;      // 0: share passes once the queue is empty; 1: share every pass; 2: never
  int *order;     // [G]
  int *queue;     // next graph to take
  int *finished;  // graphs finished
  int *board;     // [board_mask + 1] jobs with a shared pass (job g posts at g & board_mask)
  int board_mask; // a power of two of at least kBatchBoard, less one (0: kBatchBoard - 1)
  BatchJob *jobs; // [G]
  const uint64_t *rows;
  const int *colour;
  uint64_t *emask;
  uint8_t *vmask;
  kz_result *results;
  uint64_t *next;  // next-state words, same layout as rows
  int *lists;      // changed tiles: graph g's at int offset 2*row_offset
  int *items;      // pass items: graph g's at int offset 2*row_offset
  // session mode (a server's continuous feed): jobs are slots of pinned host
  // memory that the host publishes through a ring, and workgroups take them
  // while the launch runs
  int session;                        // 1: the fields below feed the queue
  unsigned long long *squeue;         // next sequence number to take (device, atomics only)
  unsigned long long *dhead;          // the host's count as last seen (device, atomics only)
  unsigned long long *hpoll;          // when a workgroup last read the host's words (device)
  int cap;                            // ring length (>= slots)
  unsigned *ring;                     // [cap] slot of the request at each sequence number;
                                      // the device marks an entry it has read kRingFree
  const unsigned long long *head;     // requests published (host-written)
  const kz_batch_graph *hgraphs;      // [slots] descriptors (row/vertex offsets unused)
  const BatchPtrs *hptrs;             // [slots] buffers
  const unsigned long long *htickets; // [slots] the request's ticket
  kz_result *hres;                    // [slots] results
  unsigned long long *hdone;          // [slots] ticket of the request whose result is in the slot
  unsigned long long idle_ticks;      // leave after this long without work (wall_clock64 ticks)
  unsigned long long lease_ticks;     // take no new request after this long (0: no limit)
};

constexpr unsigned kRingFree = 0xffffffffu;  // a ring entry the device has read

struct BatchConfig {
  int waves, chunk, lpt, workgroups, share;
};

void launch_batch(const BatchArgs &a, const BatchConfig &cfg, hipStream_t s);

// Synthetic input materialiser (kz_gen.hip).
constexpr int kGenK = 64;
struct GenArgs {
  int n, k, R, planted;
  unsigned long long base, thr;  // splitmix64((seed << 32) | gid), floor(p * 2^64)
  int coff[kGenK + 1], soff[kGenK + 1], pl[kGenK];
};
void launch_gen_rows(const GenArgs &g, uint64_t *rows, int *colour, hipStream_t s);

}  // namespace kzi

// ---- the library context (kz_api.hip, kz_server.hip)
struct kz_ctx {
  int device;
  kzi::Hdr *pinned;  // host staging for the per-pass counter readback
  // optional per-kernel timing (kz_profile_enable)
  bool prof;
  struct Pending {
    hipEvent_t a, b;
    int kind;
  };
  std::vector<hipEvent_t> pool;
  std::vector<Pending> pending;
  double total_ms[KZ_KERNEL_COUNT];
  int64_t launches[KZ_KERNEL_COUNT];
  // batched path
  kzi::BatchConfig batch_cfg;
  bool batch_cfg_set;
  int cus;        // compute units of the device
  int edge_path;  // KZ_EDGE_BITSET or KZ_EDGE_MFMA_I8
  void *scratch;  // device address of the no-allocation workspace on this device
};

