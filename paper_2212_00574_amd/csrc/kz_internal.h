// Internal declarations shared by the kernels and the host driver of the
// colour-index kernelizer (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kzi {

constexpr int kWave = 64;          // CDNA wavefront
constexpr int kBlk = 64;           // slots per block == bits per word
constexpr int kEdgeThreads = 256;  // 4 waves per edge tile
constexpr int kClassChunk = 32;    // classes staged in LDS at a time
constexpr int kRankChunk = 256;    // vertices per stable-partition chunk
constexpr int kPackLdsWords = 8192;  // dense pack: row assembled in LDS up to this many words

// stage-2 status priorities (largest wins)
enum : int { P_NONE = 0, P_EILLEGAL = 1, P_EASYM = 2, P_ESELFLOOP = 3, P_EINVAL = 4 };

// Device-resident header at the start of the workspace.
struct Hdr {
  unsigned long long ctr[2][4];  // per pass parity: removed vertices, removed edges, edge tests, spare
  int tile_count;        // changed tiles appended by the edge pass
  int prio;              // stage-2 status priority
  int bad_colour;        // stage 1: some colour outside [0,k)
  int bad_layout;        // stage 1: bitset colours unsorted / row stride mismatch
  int R;                 // words per row == number of 64-slot blocks
  int n, k, pad;
};

// Device pointers of one kernelization (workspace carve-up + caller buffers).
struct Plan {
  Hdr *hdr;
  int *counts;       // [k]
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
  uint64_t *A;       // [n*Rmax] working adjacency (bitset: the caller's emask)
  uint64_t *Anext;   // [n*Rmax]
  int n, k, Rmax, nchunks;
  long long Tmax;    // Rmax*(Rmax-1)/2
};

struct WsSizes {
  size_t total;
  size_t off_counts, off_coff, off_soff, off_bcls, off_bstart, off_blen, off_hist, off_perm,
      off_inv, off_scls, off_valive, off_touched0, off_touched1, off_bt0, off_bt1, off_tiles,
      off_A, off_Anext;
  int Rmax, nchunks;
  long long Tmax;
};

// Kernel launchers (kz_kernels.hip).  All asynchronous on `s`.
void launch_init_header(const Plan &p, bool dense, hipStream_t s);
void launch_count(const Plan &p, const int *colour, bool dense, hipStream_t s);
void launch_layout(const Plan &p, int row_words, bool bitset, hipStream_t s);
void launch_rank(const Plan &p, const int *colour, hipStream_t s);
void launch_init_state(const Plan &p, hipStream_t s);
void launch_pack_dense(const Plan &p, const uint8_t *adj, const int *colour, hipStream_t s);
void launch_copy_rows(const Plan &p, const uint64_t *rows, hipStream_t s);
void launch_vertex_pass(const Plan &p, const int *scls, int pass, bool validate, hipStream_t s);
void launch_edge_pass(const Plan &p, int pass, bool validate, hipStream_t s);
void launch_apply(const Plan &p, hipStream_t s);
void launch_unpack_dense(const Plan &p, const int *colour, uint8_t *vmask, uint8_t *emask,
                         hipStream_t s);

}  // namespace kzi
