/*
 * kz.h -- C ABI of the MI355X (gfx950) colour-index kernelizer.
 *
 * The operation (thesis section 4.2, Definition 4.2.1 and the vertex and edge
 * colour indices defined after it): the input is a finite simple graph whose
 * vertices carry a legal colouring with k colours (no edge joins two vertices
 * of one colour).  The colour index of a vertex is the number of colour
 * classes holding a neighbour of it; a vertex whose index is below k-1 cannot
 * be in a k-clique and is deleted (with its edges).  The colour index of an
 * edge {u,v} is the number of colour classes holding a common neighbour of u
 * and v; an edge whose index is below k-2 cannot be in a k-clique and is
 * deleted, u and v staying.  With exactly k classes these read: a vertex goes
 * when some other class holds no neighbour of it; an edge goes when some
 * class other than its endpoints' holds no common neighbour.
 *
 * The library applies both tests in synchronous rounds (every test of round r
 * reads the graph left by round r-1; the round's removals then apply
 * together) until a round removes nothing.  The kernel reached is unique and
 * does not depend on the order of removals; `rounds` counts the rounds that
 * removed something, so the kernel equals the input iff rounds == 0, which
 * is known after the first pass.  Every k-clique survives.
 *
 * Memory.  Every graph, colour, mask and workspace pointer is HIP device
 * memory owned by the caller (PyTorch allocates it in the Python binding).
 * The library allocates no device memory per call; a context owns a small
 * pinned host staging buffer.  All device work is ordered on the caller's
 * stream.  kz_kernelize blocks the calling host thread: it reads a few
 * counters back after each pass to decide whether to go on.
 *
 * Threading.  A context belongs to one host thread at a time.
 */
#ifndef KZ_H
#define KZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status */
#define KZ_OK          0
#define KZ_EINVAL     (-1)  /* bad argument or malformed input (see formats)    */
#define KZ_ECOLOUR    (-2)  /* a colour outside [0, k)                           */
#define KZ_EILLEGAL   (-3)  /* an edge joins two vertices of one colour class    */
#define KZ_EASYM      (-4)  /* adjacency not symmetric                           */
#define KZ_ESELFLOOP  (-5)  /* a vertex adjacent to itself                       */
#define KZ_EWORKSPACE (-6)  /* workspace smaller than kz_workspace_bytes()       */
#define KZ_ENOMEM     (-7)  /* host staging allocation failed                    */
#define KZ_EHIP       (-8)  /* a HIP runtime call failed                         */
#define KZ_EAGAIN     (-9)  /* serving: no slot or memory free yet               */
#define KZ_ETOOLARGE  (-10) /* a size beyond an entry point's stated limits     */

/* Input validation happens in two stages and reports one code:
 *   1. colours: any colour outside [0,k) -> KZ_ECOLOUR; otherwise, for the
 *      bitset format, colours not sorted ascending or a row stride that does
 *      not match the class sizes -> KZ_EINVAL;
 *   2. graph entries, highest priority first: malformed entry (KZ_EINVAL) >
 *      self-loop (KZ_ESELFLOOP) > asymmetry (KZ_EASYM) > edge inside a colour
 *      class (KZ_EILLEGAL).
 * On any error the masks are undefined; nothing outside the masks and the
 * workspace is written. */

/* ------------------------------------------------------------ formats */
typedef enum {
  KZ_DENSE_U8   = 0,  /* adj: n*n bytes, row-major, entries 0/1, symmetric,
                         zero diagonal; vertices in any order.               */
  KZ_BITSET_U64 = 1,  /* rows: n rows of row_words uint64 words.  Vertices
                         are numbered class by class (colour sorted
                         ascending).  Class c has s_c vertices and its
                         segment holds W_c = ceil(s_c/64) words starting at
                         word sum_{c'<c} W_c'; bit j of the segment (word
                         j/64, bit j%64) is adjacency to the j-th vertex of
                         class c.  row_words = sum_c W_c.  Padding bits (j >=
                         s_c) must be zero.                                   */
  KZ_CSR        = 2   /* row_ptr[n+1] (int64), col_idx[nnz] (int32): both
                         directions of every edge, column ids strictly
                         increasing within a row; row_ptr[0] = 0 and
                         row_ptr[n] = nnz; vertices in any order.  k must
                         not exceed 1024 (host check, KZ_EINVAL).  Suited to
                         sparse graphs: the edge test first compares the
                         endpoints' sets of neighbour classes, then merges
                         the two rows.                                        */
} kz_format;

typedef struct kz_graph {
  int32_t format;            /* kz_format                                   */
  int32_t n;                 /* vertices, >= 0                              */
  const uint8_t *adj;        /* KZ_DENSE_U8                                 */
  const uint64_t *rows;      /* KZ_BITSET_U64                               */
  int32_t row_words;         /* KZ_BITSET_U64                               */
  int32_t reserved0;
  const int64_t *row_ptr;    /* KZ_CSR                                      */
  const int32_t *col_idx;    /* KZ_CSR                                      */
  int64_t nnz;               /* KZ_CSR                                      */
} kz_graph;

/* Outputs (device memory, caller-owned):
 *   vmask: uint8[n], 1 = vertex survives, in the input's vertex order;
 *   emask: surviving edges in the input's format --
 *          KZ_DENSE_U8:   uint8[n*n] (both directions);
 *          KZ_BITSET_U64: uint64 rows, same layout as the input rows;
 *          KZ_CSR:        uint8[nnz] aligned with col_idx.
 * For KZ_BITSET_U64 the library also uses emask as its working copy of the
 * adjacency; it must not overlap the input rows. */
typedef struct kz_result {     /* host memory, filled on return            */
  int32_t status;              /* same as the return value                 */
  int32_t rounds;              /* productive synchronous rounds            */
  int32_t equals_input;        /* 1 iff rounds == 0                        */
  int32_t passes;              /* passes run (rounds + 1 when n > 0)       */
  int64_t surviving_vertices;
  int64_t surviving_edges;     /* undirected                               */
  int64_t input_edges;         /* undirected                               */
  int64_t edge_tests;          /* edge tests on exact worklists: pass 1
                                  tests every edge; pass r+1 the edges still
                                  alive that have an endpoint which lost an
                                  edge in round r                           */
} kz_result;

/* The result of the asynchronous call, written by the device in stream
 * order after every pass: device memory or pinned, device-mapped host
 * memory. */
typedef struct kz_out {
  kz_result result;      /* as kz_kernelize reports it, for the passes run so
                            far (status: input errors found in pass 1)      */
  int32_t converged;     /* 1 once a pass removed nothing (the fixpoint) or
                            pass 1 found an input error; later passes of
                            the same run then do nothing                    */
  int32_t pad;
  int64_t last_removed;  /* vertices plus edges the latest pass removed     */
} kz_out;

typedef struct kz_ctx kz_ctx;

/* Creates a context on HIP device `device`.  Returns KZ_OK or KZ_EHIP /
 * KZ_ENOMEM; *out is NULL on failure. */
int kz_create(kz_ctx **out, int device);

/* Releases a context (NULL is allowed). */
void kz_destroy(kz_ctx *ctx);

/* Static text for a status code. */
const char *kz_strerror(int status);

/* Workspace bytes kz_kernelize needs for this graph shape and k (an upper
 * bound that depends only on format, n, k and nnz).  Returns KZ_OK or
 * KZ_EINVAL for arguments kz_kernelize would reject on the host. */
int kz_workspace_bytes(const kz_ctx *ctx, const kz_graph *g, int32_t k, size_t *bytes);

/* Kernelizes one graph to the fixpoint.
 *   colour: int32[n] device array, the colour of each vertex (input order);
 *   ws, ws_bytes: device workspace of at least kz_workspace_bytes() bytes,
 *                 256-byte aligned, contents ignored on entry;
 *   vmask, emask: outputs as described above;
 *   stream: a hipStream_t (NULL = the null stream);
 *   res: host struct receiving the scalar results.
 * Returns KZ_OK or a status code (also stored in res->status when res is
 * not NULL).  Host-detectable argument errors return before any device
 * work. */
int kz_kernelize(kz_ctx *ctx, const kz_graph *g, const int32_t *colour, int32_t k,
                 void *ws, size_t ws_bytes, uint8_t *vmask, void *emask,
                 void *stream, kz_result *res);

/* The asynchronous form of kz_kernelize (section 4.2's pruning, repeated to
 * the fixpoint): enqueues passes first_pass .. first_pass + npasses - 1 on
 * `stream` and returns without waiting.  Every pass ends with a one-wave
 * kernel that folds the pass's removals into the result and, at the first
 * pass that removes nothing (or at pass 1 on an input error), marks the run
 * converged; the kernels of later passes of the run then return at once.
 * There is no host synchronisation inside, so the call can be captured in a
 * HIP graph (it issues kernel launches only).
 *   first_pass: 1 starts from the input (setup and validation included);
 *               a larger value continues a run whose passes up to
 *               first_pass - 1 were enqueued by earlier calls with the same
 *               arguments and workspace;
 *   npasses:    passes to enqueue (>= 1); a run needs rounds + 1 passes;
 *   out:        NULL, or a kz_out in device memory or in pinned,
 *               device-mapped host memory, written in stream order after
 *               every pass (after the last call's work completes: the final
 *               result when out->converged is 1, else the result so far).
 * The masks hold the kernel once out->converged is 1 and status is KZ_OK
 * (dense input: they are written only then).  Returns KZ_OK once enqueued,
 * or a host-detectable error (KZ_EINVAL also for first_pass < 1 or
 * npasses < 1) with nothing enqueued.  kz_kernelize is this call in chunks
 * of passes, with one look at the result between chunks. */
int kz_kernelize_async(kz_ctx *ctx, const kz_graph *g, const int32_t *colour, int32_t k,
                       void *ws, size_t ws_bytes, uint8_t *vmask, void *emask,
                       int32_t first_pass, int32_t npasses, void *stream, kz_out *out);

/* The same as kz_kernelize, with the library's own workspace instead of a
 * caller's: for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  It
 * allocates nothing and calls no allocating routine.  The workspace is a
 * fixed array of KZ_NOALLOC_SCRATCH_BYTES in device memory, one per GPU,
 * held until the process ends; a graph whose kz_workspace_bytes exceeds it
 * gets KZ_EWORKSPACE before any device work (use kz_kernelize with a larger
 * workspace).  Every call on one GPU uses that GPU's one array: calls that
 * overlap on a GPU (from two threads, or on two streams without ordering
 * between them) race and give undefined results.  Contents left by the
 * previous call are ignored (every kernel initialises what it reads).
 * Arguments, outputs, errors and blocking behaviour as kz_kernelize. */
#define KZ_NOALLOC_SCRATCH_BYTES (64u << 20)
int kz_kernelize_noalloc(kz_ctx *ctx, const kz_graph *g, const int32_t *colour, int32_t k,
                         uint8_t *vmask, void *emask, void *stream, kz_result *res);

/* Edge-test implementation used by kz_kernelize for KZ_DENSE_U8 and
 * KZ_BITSET_U64 input (CSR always uses its own):
 *   KZ_EDGE_BITSET  (default) witness search on the bit rows: per third
 *                   class, the first common neighbour ends the search;
 *   KZ_EDGE_MFMA_I8 per-class common-neighbour counts of every pair of a
 *                   tile as int8 x int8 -> int32 MFMA block contractions
 *                   (exact), an edge failing where some third class counts
 *                   zero; identical masks, rounds and counts.  Needs 8 bytes
 *                   per vertex per row word more workspace (query
 *                   kz_workspace_bytes after setting it) and row_words <=
 *                   2048 (else KZ_ETOOLARGE).
 * Applies to later calls on the context; KZ_EINVAL for another value. */
#define KZ_EDGE_BITSET 0
#define KZ_EDGE_MFMA_I8 1
int kz_set_edge_path(kz_ctx *ctx, int32_t path);

/* ------------------------------------------------------------ batches
 * Many small graphs kernelized together in one persistent launch (same
 * results as kz_kernelize on each graph alone).  Each graph is a job of
 * synchronous passes; a workgroup takes the next graph from a device queue
 * and runs its passes; once the queue is empty, workgroups without a graph
 * claim items (vertex chunks, block tiles) of the passes still running, and
 * whichever workgroup finishes a pass carries the graph on (nobody waits for
 * anybody).  All graphs use the KZ_BITSET_U64 layout and sit in shared
 * arenas:
 *   rows   (uint64): graph g's n*row_words words start at rows + row_offset;
 *   colour (int32) and vmask (uint8): graph g's n entries start at
 *          vertex_offset;
 *   emask  (uint64): same layout as rows (must not overlap it).
 * The graphs' row ranges must not overlap.  Every graph's ranges start on a
 * 128-byte line: row_offset a multiple of 16 words and vertex_offset a
 * multiple of 128 vertices, and the four arena pointers 128-byte aligned
 * (else the call returns KZ_EINVAL before any device work).  Workgroups on
 * different XCDs work on different graphs at once, and each XCD's L2 is a
 * write-back cache: a line holding two graphs' bytes could be read stale.
 * Limits of the batched path: k <= 64, row_words <= 512, n <= 32768; a graph
 * beyond them gets status KZ_ETOOLARGE in its result (run it through
 * kz_kernelize); negative offsets give KZ_EINVAL.  The call is
 * asynchronous: it enqueues the work on the stream and returns; results[g]
 * (device memory) is valid in stream order.  It performs no host
 * synchronisation, so a caller may capture it in a hipGraph and replay it. */
/* clique: the clique size when it is below the number of colour classes k
 * (1 <= clique < k; 0 or k: the clique size is k).  A k'-clique of a graph
 * legally coloured with k colours uses k' distinct classes, so section
 * 4.2's argument gives thresholds k'-1 and k'-2: a vertex fails when more
 * than k - k' other classes hold no neighbour, an edge when more than k - k'
 * third classes hold no common neighbour.  Outside [0, k]: KZ_EINVAL in the
 * graph's result. */
typedef struct kz_batch_graph {
  int32_t n, k, row_words, clique;
  int64_t row_offset;     /* in uint64 words */
  int64_t vertex_offset;  /* in vertices */
} kz_batch_graph;

typedef struct kz_batch_config {
  int32_t waves;       /* waves per workgroup: 4, 8 or 16                 */
  int32_t chunk;       /* third classes staged per step: 4 or 8 (4 when
                          waves is 16)                                     */
  int32_t lpt;         /* 1: largest graphs first; 0: given order         */
  int32_t workgroups;  /* persistent workgroups (0 = fill the device)     */
  int32_t share;       /* 0: a pass with more items than the workgroup has
                          waves is shared once the queue is empty;
                          1: every pass is shared (tests the cross-
                          workgroup path); 2: never (one workgroup per
                          graph)                                           */
} kz_batch_config;

/* Workspace bytes kz_kernelize_batch needs for these graphs (host array),
 * the same for every configuration: the queue, a job record per graph
 * (about 11 KB), and per row word one next-state word and four list ints
 * (changed tiles, items) up to the highest row_offset + n*row_words. */
int kz_batch_workspace_bytes(const kz_ctx *ctx, const kz_batch_graph *graphs, int32_t G, size_t *bytes);

/* Kernelizes G graphs.  graphs_host and graphs_dev hold the same
 * descriptors (the host copy sizes the work, the device copy is read by the
 * kernels).  results: kz_result[G] in device memory. */
int kz_kernelize_batch(kz_ctx *ctx, const kz_batch_graph *graphs_host, const kz_batch_graph *graphs_dev,
                       int32_t G, const uint64_t *rows, const int32_t *colour, void *ws, size_t ws_bytes,
                       uint8_t *vmask, uint64_t *emask, kz_result *results, void *stream);

/* Times the candidate configurations on this batch (synchronously, on the
 * stream) and keeps the fastest for later kz_kernelize_batch calls on this
 * context; *best receives it. */
int kz_batch_autotune(kz_ctx *ctx, const kz_batch_graph *graphs_host, const kz_batch_graph *graphs_dev,
                      int32_t G, const uint64_t *rows, const int32_t *colour, void *ws, size_t ws_bytes,
                      uint8_t *vmask, uint64_t *emask, kz_result *results, void *stream,
                      kz_batch_config *best);

/* Sets / reads the configuration kz_kernelize_batch uses (for example one
 * the autotuner picked in an earlier process). */
int kz_batch_set_config(kz_ctx *ctx, const kz_batch_config *cfg);
int kz_batch_get_config(const kz_ctx *ctx, kz_batch_config *cfg);

/* ------------------------------------------------------------ serving
 * A server admits requests one at a time and runs them with continuous
 * batching in two lanes that share the device.
 *
 * Session lane: requests go, once the inputs written on the server's stream
 * before their submission are complete, into a ring in pinned host memory
 * that a running launch of the batched path's job runtime (the persistent
 * workgroups above) reads while it runs: a workgroup that frees up takes the
 * next request, so a new request never waits for a whole batch to end.  A
 * launch has session_cus workgroups of 16 waves (each fills a compute unit's
 * registers, so the other units stay free for the other lane); a workgroup
 * takes no new request once lease_us has passed since it started, and
 * leaves once idle, so under load a launch ends about every lease_us -- or
 * when its longest job does, which for requests just under split_n can be
 * tens of ms -- and the server starts the next when requests wait (queued
 * behind the running launch, so they wait for that job: a lower split_n
 * shortens the wait).
 *
 * Single-graph lane: requests of split_n vertices or more (default 2048),
 * or beyond the batched path's k and row-word limits, go to worker threads
 * (six by default), each with a stream of its own, that run them through
 * the single-graph path beside the session lane: a worker runs the request
 * at the front of the lane's queue for two passes (the asynchronous call,
 * continued from the request's workspace) and puts it back at the end of
 * the queue until its fixpoint, so a long cascade does not hold a worker
 * while short requests wait.  The process then has workers + 2 streams of its own besides the
 * caller's; with fewer hardware queues than streams (HIP's
 * GPU_MAX_HW_QUEUES, 4 by default) streams share queues, and a short
 * kernel can wait behind a long one of another lane; work on a stream that
 * shares the session launch's queue (the caller's input stream, say) waits
 * for that launch to end, up to lease_us.
 *
 * A request is a KZ_BITSET_U64 graph in caller-owned device buffers (vmask
 * and emask 128-byte aligned, else KZ_EINVAL); results are the same as
 * kz_kernelize on the graph alone.  The server takes a fixed part of a
 * caller-provided device arena for the runtime's state and carves each
 * admitted request's scratch from the rest (first fit).  It admits a request
 * only when a slot, its scratch and (when a limit is set) its resident bytes
 * fit, else KZ_EAGAIN.  It allocates no device memory of its own; when it is
 * created it allocates pinned host memory for the ring and the per-slot
 * descriptors and results, a stream for session launches, and per worker a
 * context, a stream and a thread.  A server belongs to one host thread (the
 * workers are internal). */
typedef struct kz_server kz_server;

typedef struct kz_request {
  int32_t n, k, row_words, clique;  /* clique: as in kz_batch_graph (0 = k);
                                       a request with clique in [1, k) is
                                       served by the batched lane, so it must
                                       fit that lane's limits (KZ_EINVAL
                                       otherwise) */
  const uint64_t *rows;   /* device, n*row_words words (layout of KZ_BITSET_U64) */
  const int32_t *colour;  /* device, n colours sorted class by class            */
  uint8_t *vmask;         /* device output, n bytes                             */
  uint64_t *emask;        /* device output, n*row_words words (not overlapping
                             rows); all four buffers must stay valid and
                             unchanged until the request is done               */
} kz_request;

/* Fixed arena bytes of a server with max_slots slots (1..4096): the
 * session runtime's counters, board and per-slot job states; the arena must
 * be larger by the scratch of the requests it is to hold at once. */
size_t kz_server_fixed_bytes(int32_t max_slots);

/* Arena bytes an admitted request holds until it is done: in the batch
 * lane its next-state words and tile lists (16 bytes per row word), in the
 * single-graph lane kz_kernelize's workspace; 256-byte aligned.  0 for an
 * invalid request. */
size_t kz_server_request_bytes(const kz_server *srv, const kz_request *req);

/* Creates a server on ctx's device.  arena: device memory, 256-byte aligned,
 * arena_bytes > kz_server_fixed_bytes(max_slots), owned by the caller and
 * not touched by it until kz_server_destroy returns.  stream: the stream all
 * inputs are written on (NULL = the null stream): what a caller writes on
 * it before kz_server_submit is complete before the request runs. */
int kz_server_create(kz_ctx *ctx, void *arena, size_t arena_bytes, int32_t max_slots, void *stream,
                     kz_server **out);

typedef struct kz_server_config {
  int32_t split_n;        /* requests with at least this many vertices take the
                             single-graph lane (0 = 2048); a value above 32768
                             keeps every request the batched path takes in
                             the session lane                                */
  int32_t idle_us;        /* a session launch ends after this long without
                             work, in microseconds (0 = 20000; at most 1e6)  */
  int32_t lease_us;       /* a session workgroup takes no new request this
                             long after it started (0 = 10000; at most 1e6)  */
  int32_t session_cus;    /* compute units a session launch fills, up to the
                             device's (0 = 3/16 of them)                     */
  int32_t workers;        /* single-graph lane: requests in flight at once,
                             each with a worker thread, context and stream
                             of its own (0 = 6; at most 8)                   */
  int32_t partition;      /* 1: the session lane's stream is masked to
                             session_cus compute units and the other lane's
                             streams to the rest, so neither lane waits for
                             the other's workgroups to leave a unit (masked
                             streams are blocking streams: pass the server a
                             stream other than the legacy null stream);
                             0: both lanes may use every unit               */
  size_t resident_limit;  /* admit while the admitted, unfinished requests'
                             rows, colours and masks (2*8*n*row_words + 5*n
                             bytes each) total at most this; 0 = no limit    */
} kz_server_config;

/* Sets the configuration; only while no request is admitted (KZ_EAGAIN
 * otherwise).  KZ_EINVAL for negative fields, times above 1e6 or more
 * compute units than the device has. */
int kz_server_configure(kz_server *srv, const kz_server_config *cfg);

/* Admits a request: KZ_OK and *ticket, KZ_EAGAIN (no slot, scratch or
 * resident budget now: retry after kz_server_poll has retired finished
 * requests), or KZ_EINVAL (bad arguments, or a request whose resident bytes
 * alone exceed the limit). */
int kz_server_submit(kz_server *srv, const kz_request *req, uint64_t *ticket);

/* Collects finished requests (freeing their scratch, slot and resident
 * bytes), publishes requests whose inputs are complete and starts a session
 * launch when published requests wait.  Returns the number of admitted
 * requests not yet retired by kz_server_poll, or a negative status.  Call
 * it (or kz_server_poll) while requests are outstanding: the server has no
 * thread of its own for this. */
int kz_server_progress(kz_server *srv);

/* 1: the request is done; *res (if not NULL) receives its result and the
 * ticket is retired.  0: not done yet.  KZ_EINVAL: unknown ticket.  Calls
 * kz_server_progress first. */
int kz_server_poll(kz_server *srv, uint64_t ticket, kz_result *res);

/* Retires up to max finished requests, oldest completion first: their
 * tickets go to tickets[0..), their results (if res is not NULL) to
 * res[0..).  Calls kz_server_progress first.  Returns the number retired
 * (0 when none has finished), or a negative status.  One call replaces a
 * kz_server_poll per outstanding ticket. */
int kz_server_done(kz_server *srv, uint64_t *tickets, kz_result *res, int32_t max);

/* Waits for the requests in flight (a session launch ends once idle) and
 * releases the server; requests whose inputs were not yet complete are
 * dropped. */
void kz_server_destroy(kz_server *srv);

/* ------------------------------------------------------------ measurement
 * When enabled, kz_kernelize brackets every kernel launch with HIP events
 * recorded on the caller's stream and accumulates the elapsed time per
 * kernel family (read after the call returns).  Costs a few microseconds
 * per launch; off by default. */
typedef enum {
  KZ_KERNEL_SETUP = 0,   /* header, colour count, layout, partition, state init */
  KZ_KERNEL_PACK = 1,    /* dense input -> class-partitioned bit rows         */
  KZ_KERNEL_VERTEX = 2,  /* vertex colour-index test (CSR pass 1: also the
                            validation sweep over the rows)                   */
  KZ_KERNEL_EDGE = 3,    /* edge colour-index test (tiles / CSR entries)      */
  KZ_KERNEL_APPLY = 4,   /* changed tiles into the state / failed CSR entries
                            cleared                                           */
  KZ_KERNEL_UNPACK = 5,  /* bit rows -> output masks                          */
  KZ_KERNEL_COUNT = 6
} kz_kernel;

/* Turns timing on (on != 0) or off; clears the accumulated times. */
int kz_profile_enable(kz_ctx *ctx, int on);

/* Accumulated milliseconds and launch count of one kernel family. */
int kz_profile_read(const kz_ctx *ctx, int kernel, double *total_ms, int64_t *launches);

/* ------------------------------------------------------------ synthetic inputs
 * Not part of the method: materialises a seeded random legally coloured
 * graph in the KZ_BITSET_U64 layout directly in device memory (for
 * benchmarks and servers that must not generate large graphs on the host).
 * Class c holds sizes[c] vertices (class-major slots); an inter-class slot
 * pair {a < b} is an edge iff
 *   splitmix64(splitmix64((seed << 32) | gid) ^ ((a << 32) | b)) < floor(p * 2^64)
 * (splitmix64 = the output function of Steele, Lea and Flood's SplitMix64,
 * OOPSLA 2014); pairs inside a class never are.  planted (host, k slot ids,
 * one per class, or NULL) forces a k-clique on those slots.
 *   k: 1..64; sizes: host int32[k], >= 0; p in [0, 1];
 *   rows: device uint64[n * row_words], row_words = sum ceil(sizes[c]/64)
 *         (KZ_EINVAL otherwise);
 *   colour: device int32[n] receiving the sorted colours, or NULL.
 * Asynchronous on the stream. */
int kz_gen_bitset(kz_ctx *ctx, int32_t k, const int32_t *sizes, double p, uint32_t seed, uint32_t gid,
                  const int32_t *planted, uint64_t *rows, int32_t row_words, int32_t *colour, void *stream);

/* ------------------------------------------------------------ colouring
 * An upstream legal colouring, for graphs that arrive uncoloured: the
 * colour-index method (section 4.2, Definition 4.2.1) needs a legal
 * colouring of its input, and the thesis assumes one is given without
 * naming an algorithm.  This is Jones and Plassmann's parallel greedy
 * colouring (SIAM J. Sci. Comput. 14(3), 1993): vertex v has the key
 * (priority[v], v); each round takes every uncoloured vertex whose key
 * beats the key of each uncoloured neighbour, and each vertex taken gets
 * the smallest colour no neighbour coloured in an earlier round holds.  The
 * result is legal, uses at most max degree + 1 colours, and is the same for
 * any order inside a round.  With m colours the graph goes to the
 * colour-index method as m classes, with a clique size k <= m (the batched
 * path's kz_batch_graph.clique).
 *   rows: device uint64[n * row_words], plain rows as for kz_dominance
 *         (bit w % 64 of word w / 64 of row v set iff {v, w} is an edge);
 *         ceil(n / 64) <= row_words <= 1024 (else KZ_EINVAL / KZ_ETOOLARGE);
 *         symmetric (KZ_EASYM), no self-loop (KZ_ESELFLOOP), no bit at or
 *         beyond n (KZ_EINVAL);
 *   priority: device uint64[n], the vertices' priorities (random numbers
 *         the caller draws; equal ones are broken by the index);
 *   ws, ws_bytes: device workspace of kz_colour_workspace_bytes() bytes,
 *         256-byte aligned;
 *   colour: device int32[n] out, in [0, colours).
 * Blocking: rounds end on the device and go out in chunks, with one small
 * readback per chunk. */
typedef struct kz_colour_result {
  int32_t status;
  int32_t rounds;
  int32_t colours;  /* 1 + the largest colour given                      */
  int32_t pad;
} kz_colour_result;

int kz_colour_workspace_bytes(int32_t n, size_t *bytes);
int kz_colour_jp(kz_ctx *ctx, int32_t n, const uint64_t *rows, int32_t row_words, const uint64_t *priority,
                 void *ws, size_t ws_bytes, int32_t *colour, void *stream, kz_colour_result *res);

/* ------------------------------------------------------------ dominance
 * Dominance reductions (thesis section 4.3).  A different method from the
 * colour index and kept apart from it: it uses no colouring, and vertex
 * dominance may delete k-cliques (never all of the largest ones -- every
 * deletion trades a for b inside any clique through it, so the clique number
 * is unchanged).
 *   KZ_DOM_VERTEX  Definition 4.3.1, Algorithm 1: node b dominates node a
 *                  when they are not adjacent and N(a) is a subset of N(b).
 *                  A sweep visits b in index order; each step deletes, with
 *                  their edges, the nodes b dominates in the current graph.
 *   KZ_DOM_EDGE    Definition 4.3.2, Algorithm 2: for distinct a, u, b the
 *                  edge {u,b} dominates {a,u} when b is not a neighbour of a
 *                  and N(a) & N(u) is a subset of N(b).  A sweep visits the
 *                  pairs (a, u), u a neighbour of a, in index order and
 *                  deletes {a,u} when some b makes it dominated in the
 *                  current graph (a and u stay).
 * Sweeps repeat until one deletes nothing.
 *   rows: device uint64[n * row_words], bit w % 64 of word w / 64 of row v
 *         set iff {v, w} is an edge; row_words >= ceil(n / 64) and <= 1024
 *         (else KZ_ETOOLARGE); symmetric (KZ_EASYM), no self-loop
 *         (KZ_ESELFLOOP), no bit at or beyond n (KZ_EINVAL);
 *   ws, ws_bytes: device workspace of kz_dom_workspace_bytes() bytes,
 *         256-byte aligned;
 *   vmask: device uint8[n], 1 = node kept;
 *   emask: device uint64[n * row_words], the adjacency left, same layout
 *         (may be the rows buffer itself);
 *   res: host struct receiving the counts.
 * Blocking: the sweep is a chain of parallel scans, each followed by one
 * small readback; returns after the fixpoint.  Outputs are unspecified
 * when the status is not KZ_OK. */
#define KZ_DOM_VERTEX 0
#define KZ_DOM_EDGE 1

typedef struct kz_dom_result {
  int32_t status;
  int32_t sweeps;            /* sweeps that deleted something               */
  int64_t deleted_vertices;
  int64_t deleted_edges;     /* undirected; vertex mode: edges of deleted
                                nodes                                       */
  int64_t input_edges;       /* undirected                                  */
  int64_t events;            /* steps (vertex) or edges (edge) that deleted
                                something                                   */
  int64_t scans;             /* parallel scans run                          */
} kz_dom_result;

int kz_dom_workspace_bytes(int32_t n, size_t *bytes);
int kz_dominance(kz_ctx *ctx, int32_t mode, int32_t n, const uint64_t *rows, int32_t row_words, void *ws,
                 size_t ws_bytes, uint8_t *vmask, uint64_t *emask, void *stream, kz_dom_result *res);

/* ------------------------------------------------------------ clique search
 * The search the kernel is handed to (the thesis's problem: is there a
 * k-clique?).  On a legally k-coloured graph a k-clique holds one vertex of
 * every class.  kz_find_clique returns the lexicographically smallest
 * k-clique among the live vertices -- ordered by its class-0 vertex, then
 * its class-1 vertex, ... (vertex ids are the slot ids of the bit rows) --
 * or reports that there is none.  Run it on kz_kernelize's output (rows =
 * its emask, vmask = its vmask): every k-clique survives the kernel, so the
 * answer is the same as on the input, found in less work.
 *   g: KZ_BITSET_U64 (class-major slots; the rows are not re-validated, they
 *      must be a valid kz_kernelize input or output);
 *   colour: device int32[n], sorted, in [0, k) (KZ_ECOLOUR / KZ_EINVAL);
 *   k: 1..64, and n below 2^21 (KZ_ETOOLARGE beyond);
 *   vmask: device uint8[n] (0 = deleted), or NULL for all vertices;
 *   ws, ws_bytes: device workspace of kz_clique_workspace_bytes() bytes,
 *      256-byte aligned;
 *   clique: device int32[k], the clique's vertex of each class, or all -1.
 * Blocking: returns after the search with res->found. */
typedef struct kz_clique_result {
  int32_t status;
  int32_t found;             /* 1 iff a k-clique exists                     */
  int64_t nodes;             /* partial cliques the search extended (a
                                measure; it depends on the schedule)        */
  int64_t roots;             /* (class 0, class 1) pairs handed out         */
} kz_clique_result;

int kz_clique_workspace_bytes(const kz_graph *g, int32_t k, size_t *bytes);
int kz_find_clique(kz_ctx *ctx, const kz_graph *g, const int32_t *colour, int32_t k, const uint8_t *vmask,
                   void *ws, size_t ws_bytes, int32_t *clique, void *stream, kz_clique_result *res);

/* ------------------------------------------------------------ struction
 * Struction (thesis section 4.1, Definition 4.1.1, Theorem 1): a graph G'
 * whose clique number is one less than G's.  Around the pivot p: A = the
 * neighbours of p, B = the other vertices except p, and a node c(x, y) for
 * every edge {x, y} of G inside B with x < y.  G' has the nodes A (in vertex
 * order) followed by the nodes c(x, y) (ordered by x, then y):
 *   a ~ a'           iff {a, a'} is an edge of G;
 *   c(x,y) ~ c(x',y') iff x = x' and {y, y'} is an edge of G;
 *   a ~ c(x, y)      iff a ~ x and a ~ y (the thesis states no rule for
 *                    these pairs; this one makes its Lemmas 1 and 2 hold).
 *   rows: device uint64[n * row_words], plain bit rows (bit w % 64 of word
 *         w / 64 of row v: {v, w} is an edge), row_words >= ceil(n / 64),
 *         symmetric, no self-loop, no bit at or beyond n (else KZ_EASYM /
 *         KZ_ESELFLOOP / KZ_EINVAL); n >= 1, 0 <= pivot < n;
 *   ws, ws_bytes: device workspace of kz_struction_workspace_bytes() bytes,
 *         256-byte aligned;
 *   out == NULL: plan only -- res gets the node counts and the row words
 *         G' needs (ceil(n' / 64));
 *   out: device uint64[out_nodes * out_row_words], G' in the same bit-row
 *         layout; map: device int32[out_nodes * 2], per node (v, -1) for
 *         A nodes and (x, y) for C nodes; KZ_EWORKSPACE when out_nodes or
 *         out_row_words is too small for G'.
 * Blocking (two small readbacks). */
typedef struct kz_struction_result {
  int32_t status;
  int32_t row_words;         /* ceil(nodes / 64)                            */
  int64_t nodes;             /* n' = a_nodes + c_nodes                      */
  int64_t a_nodes;           /* the pivot's degree                          */
  int64_t c_nodes;           /* edges inside B                              */
  int64_t input_edges;       /* undirected                                  */
} kz_struction_result;

int kz_struction_workspace_bytes(int32_t n, int32_t row_words, size_t *bytes);
int kz_struction(kz_ctx *ctx, int32_t n, const uint64_t *rows, int32_t row_words, int32_t pivot, void *ws,
                 size_t ws_bytes, uint64_t *out, int32_t out_row_words, int64_t out_nodes, int32_t *map,
                 void *stream, kz_struction_result *res);

#ifdef __cplusplus
}
#endif

#endif /* KZ_H */
