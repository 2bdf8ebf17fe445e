/*
 * kz_oracle.c -- plain CPU oracle for iterated colour-index pruning
 * (kernelization of the k-clique problem on a legally k-coloured graph).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg do.  It shares no code, header, table or helper with the GPU
 * library: it reads the caller's arrays itself and keeps its own plain
 * adjacency lists.
 *
 * What it computes (thesis section 4.2, Definition 4.2.1 and the two colour
 * indices that follow it):
 *   - a legal colouring puts every vertex in one of k colour classes and no
 *     edge joins two vertices of the same class;
 *   - the colour index of a vertex v is the number of colour classes that
 *     hold at least one vertex adjacent to v; a vertex whose index is below
 *     k-1 lies in no k-clique and is deleted;
 *   - the colour index of an edge {u,v} is the number of colour classes that
 *     hold at least one vertex adjacent to both u and v; an edge whose index
 *     is below k-2 lies in no k-clique and is deleted, while u and v stay.
 *
 * The thesis states each rule once and is silent on repetition and order.
 * Reading used here (it is also the library's contract): the two tests are
 * applied in synchronous rounds -- every test of round r looks at the graph
 * left by round r-1 and all removals of the round take effect together --
 * until a round removes nothing.  "rounds" counts the rounds that removed
 * something; the kernel equals the input iff rounds == 0.  Deleting a vertex
 * deletes its incident edges.
 *
 * Two independent algorithms are given:
 *   O1 kzo_fixpoint              -- the synchronous rounds above, recomputing
 *                                   every index from the current graph;
 *   O2 kzo_fixpoint_random_order -- one element at a time in a seeded random
 *                                   order with incremental counters (masks
 *                                   only).  The greatest "stable" subgraph is
 *                                   unique, so both must give the same masks.
 * plus a brute-force enumerator of k-cliques (one vertex per class, pairwise
 * adjacent) for the soundness check: every vertex and edge of every k-clique
 * must survive.
 *
 * Input validation follows the library's documented order: colours first
 * (a colour outside [0,k) -> -2; for the bitset format, colours not sorted by
 * class or a row stride that does not match the class sizes -> -1), then the
 * graph entries with priority: malformed entry (-1) > self-loop (-5) >
 * asymmetric adjacency (-4) > edge inside a colour class (-3).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ST_OK 0
#define ST_EINVAL (-1)
#define ST_ECOLOUR (-2)
#define ST_EILLEGAL (-3)
#define ST_EASYM (-4)
#define ST_ESELFLOOP (-5)
#define ST_ENOMEM (-7)

enum { FMT_DENSE = 0, FMT_BITSET = 1, FMT_CSR = 2 };

typedef struct {
  int32_t n, k;
  int fmt;
  int32_t row_words;   /* bitset format only */
  int32_t *col;        /* colour of each vertex (input order) */
  int64_t *rp;         /* n+1 row pointers of the directed entry lists */
  int32_t *nb;         /* neighbour of each entry; strictly increasing per row */
  int32_t *src;        /* row of each entry */
  int64_t *mate;       /* entry (v,u) for entry (u,v) */
  uint8_t *ea;         /* entry alive (both directions kept equal) */
  uint8_t *va;         /* vertex alive */
  int64_t nent;
  /* bitset format: class sizes / offsets, to place bits on output */
  int64_t *coff;       /* k+1 first vertex of each class (class-major ids) */
  int64_t *soff;       /* k+1 first word of each class segment */
  int32_t *stamp;      /* k scratch for "seen colour" marks */
  int32_t stamp_now;
} og_t;

static void og_free(og_t *g) {
  if (!g) return;
  free(g->col); free(g->rp); free(g->nb); free(g->src); free(g->mate);
  free(g->ea); free(g->va); free(g->coff); free(g->soff); free(g->stamp);
  free(g);
}

/* ------------------------------------------------------------------ input */

/* Stage 1: colours.  Returns status. */
static int check_colours(int32_t n, const int32_t *col, int32_t k) {
  for (int32_t v = 0; v < n; ++v)
    if (col[v] < 0 || col[v] >= k) return ST_ECOLOUR;
  return ST_OK;
}

/* Builds the directed entry lists from per-row neighbour lists already in
 * increasing order.  cnt[v] = entries of row v, lists concatenated in nbuf. */
static int og_alloc_entries(og_t *g, int64_t nent) {
  g->nent = nent;
  g->nb = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nent ? nent : 1));
  g->src = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nent ? nent : 1));
  g->mate = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nent ? nent : 1));
  g->ea = (uint8_t *)malloc((size_t)(nent ? nent : 1));
  return (g->nb && g->src && g->mate && g->ea) ? ST_OK : ST_ENOMEM;
}

static int64_t find_entry(const og_t *g, int32_t v, int32_t w) {
  int64_t lo = g->rp[v], hi = g->rp[v + 1];
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (g->nb[mid] < w) lo = mid + 1; else hi = mid;
  }
  if (lo < g->rp[v + 1] && g->nb[lo] == w) return lo;
  return -1;
}

/* Stage 2 checks on the entry lists (structure already checked). */
static int check_graph(og_t *g) {
  int has_loop = 0, has_asym = 0, has_intra = 0;
  for (int32_t u = 0; u < g->n; ++u) {
    for (int64_t e = g->rp[u]; e < g->rp[u + 1]; ++e) {
      int32_t v = g->nb[e];
      g->src[e] = u;
      if (v == u) { has_loop = 1; g->mate[e] = e; continue; }
      int64_t m = find_entry(g, v, u);
      if (m < 0) has_asym = 1;
      g->mate[e] = m;
      if (g->col[u] == g->col[v]) has_intra = 1;
    }
  }
  if (has_loop) return ST_ESELFLOOP;
  if (has_asym) return ST_EASYM;
  if (has_intra) return ST_EILLEGAL;
  return ST_OK;
}

static og_t *og_new(int32_t n, int32_t k, const int32_t *col, int fmt) {
  og_t *g = (og_t *)calloc(1, sizeof(og_t));
  if (!g) return NULL;
  g->n = n; g->k = k; g->fmt = fmt;
  g->col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
  g->rp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  g->va = (uint8_t *)malloc((size_t)(n ? n : 1));
  g->stamp = (int32_t *)calloc((size_t)k, sizeof(int32_t));
  if (!g->col || !g->rp || !g->va || !g->stamp) { og_free(g); return NULL; }
  if (n) memcpy(g->col, col, sizeof(int32_t) * (size_t)n);
  return g;
}

/* DENSE: adj is n*n bytes, row-major. */
static int load_dense(og_t *g, const uint8_t *adj) {
  int32_t n = g->n;
  int64_t nent = 0;
  for (int64_t i = 0; i < (int64_t)n * n; ++i) {
    if (adj[i] > 1) return ST_EINVAL;
    nent += adj[i];
  }
  if (og_alloc_entries(g, nent)) return ST_ENOMEM;
  int64_t e = 0;
  for (int32_t u = 0; u < n; ++u) {
    g->rp[u] = e;
    for (int32_t v = 0; v < n; ++v)
      if (adj[(int64_t)u * n + v]) g->nb[e++] = v;
  }
  g->rp[n] = e;
  return ST_OK;
}

/* CSR: row_ptr[n+1], col_idx[nnz]; rows must be strictly increasing. */
static int load_csr(og_t *g, const int64_t *rp, const int32_t *ci, int64_t nnz) {
  int32_t n = g->n;
  if (rp[0] != 0 || rp[n] != nnz) return ST_EINVAL;
  for (int32_t u = 0; u < n; ++u) {
    if (rp[u + 1] < rp[u]) return ST_EINVAL;
    for (int64_t e = rp[u]; e < rp[u + 1]; ++e) {
      if (ci[e] < 0 || ci[e] >= n) return ST_EINVAL;
      if (e > rp[u] && ci[e] <= ci[e - 1]) return ST_EINVAL;
    }
  }
  if (og_alloc_entries(g, nnz)) return ST_ENOMEM;
  memcpy(g->rp, rp, sizeof(int64_t) * ((size_t)n + 1));
  if (nnz) memcpy(g->nb, ci, sizeof(int32_t) * (size_t)nnz);
  return ST_OK;
}

/* BITSET: vertices are numbered class by class; colour must be sorted.
 * Row v has, for each class c, ceil(s_c/64) words; bit j of class c's
 * segment (word j/64, bit j%64) is adjacency to the j-th vertex of class c. */
static int load_bitset(og_t *g, const uint64_t *rows, int32_t row_words) {
  int32_t n = g->n, k = g->k;
  g->coff = (int64_t *)calloc((size_t)k + 1, sizeof(int64_t));
  g->soff = (int64_t *)calloc((size_t)k + 1, sizeof(int64_t));
  if (!g->coff || !g->soff) return ST_ENOMEM;
  for (int32_t v = 1; v < n; ++v)
    if (g->col[v] < g->col[v - 1]) return ST_EINVAL;
  for (int32_t v = 0; v < n; ++v) g->coff[g->col[v] + 1] += 1;
  for (int32_t c = 0; c < k; ++c) {
    int64_t s = g->coff[c + 1];
    g->soff[c + 1] = g->soff[c] + (s + 63) / 64;
    g->coff[c + 1] += g->coff[c];
  }
  if (g->soff[k] != row_words) return ST_EINVAL;
  g->row_words = row_words;
  /* padding bits must be zero */
  for (int32_t v = 0; v < n; ++v) {
    const uint64_t *row = rows + (int64_t)v * row_words;
    for (int32_t c = 0; c < k; ++c) {
      int64_t s = g->coff[c + 1] - g->coff[c];
      for (int64_t j = s; j < 64 * (g->soff[c + 1] - g->soff[c]); ++j)
        if ((row[g->soff[c] + j / 64] >> (j % 64)) & 1u) return ST_EINVAL;
    }
  }
  int64_t nent = 0;
  for (int32_t v = 0; v < n; ++v) {
    const uint64_t *row = rows + (int64_t)v * row_words;
    for (int32_t c = 0; c < k; ++c)
      for (int64_t j = 0; j < g->coff[c + 1] - g->coff[c]; ++j)
        nent += (row[g->soff[c] + j / 64] >> (j % 64)) & 1u;
  }
  if (og_alloc_entries(g, nent)) return ST_ENOMEM;
  int64_t e = 0;
  for (int32_t v = 0; v < n; ++v) {
    const uint64_t *row = rows + (int64_t)v * row_words;
    g->rp[v] = e;
    for (int32_t c = 0; c < k; ++c)   /* classes in order => ids increasing */
      for (int64_t j = 0; j < g->coff[c + 1] - g->coff[c]; ++j)
        if ((row[g->soff[c] + j / 64] >> (j % 64)) & 1u) g->nb[e++] = (int32_t)(g->coff[c] + j);
  }
  g->rp[n] = e;
  return ST_OK;
}

void kzo_reset(void *h) {
  og_t *g = (og_t *)h;
  memset(g->va, 1, (size_t)(g->n ? g->n : 1));
  if (g->nent) memset(g->ea, 1, (size_t)g->nent);
}

/* Loads one graph.  *status receives the validation result; NULL unless OK. */
void *kzo_load(int fmt, int32_t n, const uint8_t *adj, const uint64_t *rows, int32_t row_words,
               const int64_t *row_ptr, const int32_t *col_idx, int64_t nnz,
               const int32_t *colour, int32_t k, int32_t *status) {
  *status = ST_EINVAL;
  if (n < 0 || k < 1 || fmt < 0 || fmt > 2) return NULL;
  if (n > 0 && !colour) return NULL;
  int st = check_colours(n, colour, k);
  if (st) { *status = st; return NULL; }
  og_t *g = og_new(n, k, colour, fmt);
  if (!g) { *status = ST_ENOMEM; return NULL; }
  if (fmt == FMT_DENSE) st = (n && !adj) ? ST_EINVAL : load_dense(g, adj);
  else if (fmt == FMT_BITSET) st = (row_words < 0 || (n && !rows)) ? ST_EINVAL : load_bitset(g, rows, row_words);
  else st = (!row_ptr || nnz < 0 || (nnz && !col_idx)) ? ST_EINVAL : load_csr(g, row_ptr, col_idx, nnz);
  if (st == ST_OK) st = check_graph(g);
  if (st) { og_free(g); *status = st; return NULL; }
  kzo_reset(g);
  *status = ST_OK;
  return g;
}

void kzo_free(void *h) { og_free((og_t *)h); }
int64_t kzo_num_entries(void *h) { return ((og_t *)h)->nent; }

/* ------------------------------------------------------------- the indices */

static int edge_alive(const og_t *g, int32_t v, int32_t w) {
  int64_t e = find_entry(g, v, w);
  return e >= 0 && g->ea[e];
}

static void new_stamp(og_t *g) {
  if (++g->stamp_now == INT32_MAX) {
    memset(g->stamp, 0, sizeof(int32_t) * (size_t)g->k);
    g->stamp_now = 1;
  }
}

/* Colour index of vertex v in the current graph, counted up to `cap`
 * (cap = k gives the exact index). */
static int32_t ci_vertex(og_t *g, int32_t v, int32_t cap) {
  int32_t count = 0;
  new_stamp(g);
  for (int64_t e = g->rp[v]; e < g->rp[v + 1] && count < cap; ++e) {
    if (!g->ea[e]) continue;
    int32_t c = g->col[g->nb[e]];
    if (g->stamp[c] != g->stamp_now) { g->stamp[c] = g->stamp_now; ++count; }
  }
  return count;
}

/* Colour index of edge {u,v}: classes holding a vertex w with {u,w} and
 * {v,w} both alive.  Counted up to `cap`. */
static int32_t ci_edge(og_t *g, int32_t u, int32_t v, int32_t cap) {
  int32_t count = 0;
  new_stamp(g);
  for (int64_t e = g->rp[u]; e < g->rp[u + 1] && count < cap; ++e) {
    if (!g->ea[e]) continue;
    int32_t w = g->nb[e];
    int32_t c = g->col[w];
    if (g->stamp[c] == g->stamp_now) continue;
    if (edge_alive(g, v, w)) { g->stamp[c] = g->stamp_now; ++count; }
  }
  return count;
}

int32_t kzo_ci_vertex(void *h, int32_t v) {
  og_t *g = (og_t *)h;
  if (v < 0 || v >= g->n) return -1;
  return ci_vertex(g, v, g->k);
}

/* -1 if {u,v} is not an alive edge. */
int32_t kzo_ci_edge(void *h, int32_t u, int32_t v) {
  og_t *g = (og_t *)h;
  if (u < 0 || v < 0 || u >= g->n || v >= g->n || !edge_alive(g, u, v)) return -1;
  return ci_edge(g, u, v, g->k);
}

static int vertex_fails(og_t *g, int32_t v) {
  return g->k >= 1 && ci_vertex(g, v, g->k - 1) < g->k - 1;
}

static int edge_fails(og_t *g, int32_t u, int32_t v) {
  return g->k >= 3 && ci_edge(g, u, v, g->k - 2) < g->k - 2;
}

static void kill_entry(og_t *g, int64_t e) {
  g->ea[e] = 0;
  g->ea[g->mate[e]] = 0;
}

/* ------------------------------------------------------------------- O1 */

/* Synchronous rounds to the fixpoint.
 * stats[0] rounds, [1] equals_input, [2] surviving vertices,
 * [3] surviving undirected edges, [4] edge tests on exact worklists:
 * the first pass tests every edge; pass r+1 tests the edges still alive
 * after round r that have an endpoint which lost an incident edge in round r. */
int kzo_fixpoint(void *h, int64_t *stats) {
  og_t *g = (og_t *)h;
  int32_t n = g->n;
  uint8_t *fv = (uint8_t *)calloc((size_t)(n ? n : 1), 1);
  uint8_t *fe = (uint8_t *)calloc((size_t)(g->nent ? g->nent : 1), 1);
  uint8_t *touched = (uint8_t *)calloc((size_t)(n ? n : 1), 1);
  if (!fv || !fe || !touched) { free(fv); free(fe); free(touched); return ST_ENOMEM; }
  int64_t rounds = 0, tests = 0;
  for (int64_t e = 0; e < g->nent; ++e)
    if (g->ea[e] && g->src[e] < g->nb[e]) ++tests;
  for (;;) {
    int any = 0;
    for (int32_t v = 0; v < n; ++v)
      if (g->va[v] && vertex_fails(g, v)) { fv[v] = 1; any = 1; }
    for (int64_t e = 0; e < g->nent; ++e) {
      int32_t u = g->src[e], v = g->nb[e];
      if (u < v && g->ea[e] && edge_fails(g, u, v)) { fe[e] = 1; any = 1; }
    }
    if (!any) break;
    /* apply every removal of the round at once */
    memset(touched, 0, (size_t)(n ? n : 1));
    for (int64_t e = 0; e < g->nent; ++e) {
      int32_t u = g->src[e], v = g->nb[e];
      if (!g->ea[e] || u > v) continue;
      if (fe[e] || fv[u] || fv[v]) { kill_entry(g, e); touched[u] = touched[v] = 1; }
    }
    for (int32_t v = 0; v < n; ++v)
      if (fv[v]) g->va[v] = 0;
    memset(fv, 0, (size_t)(n ? n : 1));
    memset(fe, 0, (size_t)(g->nent ? g->nent : 1));
    ++rounds;
    for (int64_t e = 0; e < g->nent; ++e) {
      int32_t u = g->src[e], v = g->nb[e];
      if (u < v && g->ea[e] && (touched[u] || touched[v])) ++tests;
    }
  }
  int64_t sv = 0, se = 0;
  for (int32_t v = 0; v < n; ++v) sv += g->va[v];
  for (int64_t e = 0; e < g->nent; ++e)
    if (g->ea[e] && g->src[e] < g->nb[e]) ++se;
  stats[0] = rounds;
  stats[1] = rounds == 0;
  stats[2] = sv;
  stats[3] = se;
  stats[4] = tests;
  free(fv); free(fe); free(touched);
  return ST_OK;
}

/* ------------------------------------------------------------------- O2 */

typedef struct { uint64_t s; } rng_t;
static uint64_t rng_next(rng_t *r) {   /* SplitMix64 (Steele, Lea, Flood 2014) */
  uint64_t z = (r->s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

typedef struct {
  int64_t *items; int64_t len, cap;
  uint8_t *in;
} bag_t;

static void bag_push(bag_t *b, int64_t x) {
  if (b->in[x]) return;
  b->in[x] = 1;
  b->items[b->len++] = x;
}

typedef struct {
  og_t *g;
  int32_t *nbr_cnt;   /* [n*k]  alive neighbours of v in class c */
  int32_t *com_cnt;   /* [nent*k] common alive neighbours of entry's edge in class c (canonical entry) */
  bag_t bag;
} o2_t;

static int64_t canon(const og_t *g, int64_t e) { return g->src[e] < g->nb[e] ? e : g->mate[e]; }

static int o2_vertex_fails(o2_t *s, int32_t v) {
  og_t *g = s->g;
  int32_t ci = 0;
  for (int32_t c = 0; c < g->k; ++c) ci += s->nbr_cnt[(int64_t)v * g->k + c] > 0;
  return ci < g->k - 1;
}

static int o2_edge_fails(o2_t *s, int64_t ce) {
  og_t *g = s->g;
  int32_t ci = 0;
  for (int32_t c = 0; c < g->k; ++c) ci += s->com_cnt[ce * g->k + c] > 0;
  return ci < g->k - 2;
}

static void o2_remove_edge(o2_t *s, int64_t ce) {
  og_t *g = s->g;
  int32_t u = g->src[ce], v = g->nb[ce];
  int32_t k = g->k;
  kill_entry(g, ce);
  s->nbr_cnt[(int64_t)u * k + g->col[v]]--;
  s->nbr_cnt[(int64_t)v * k + g->col[u]]--;
  bag_push(&s->bag, u);
  bag_push(&s->bag, v);
  /* every alive w adjacent to both loses v (resp. u) as a common neighbour */
  for (int64_t e = g->rp[u]; e < g->rp[u + 1]; ++e) {
    if (!g->ea[e]) continue;
    int32_t w = g->nb[e];
    int64_t f = find_entry(g, v, w);
    if (f < 0 || !g->ea[f]) continue;
    int64_t cuw = canon(g, e), cvw = canon(g, f);
    s->com_cnt[cuw * k + g->col[v]]--;
    s->com_cnt[cvw * k + g->col[u]]--;
    bag_push(&s->bag, g->n + cuw);
    bag_push(&s->bag, g->n + cvw);
  }
}

/* O2: seeded random order, one removal at a time, incremental counters.
 * Leaves the final masks in the handle. */
int kzo_fixpoint_random_order(void *h, uint64_t seed) {
  og_t *g = (og_t *)h;
  int32_t n = g->n, k = g->k;
  o2_t s;
  s.g = g;
  s.nbr_cnt = (int32_t *)calloc((size_t)n * k + 1, sizeof(int32_t));
  s.com_cnt = (int32_t *)calloc((size_t)g->nent * k + 1, sizeof(int32_t));
  int64_t tot = (int64_t)n + g->nent;
  s.bag.items = (int64_t *)malloc(sizeof(int64_t) * (size_t)(tot + 1));
  s.bag.in = (uint8_t *)calloc((size_t)tot + 1, 1);
  s.bag.len = 0; s.bag.cap = tot;
  if (!s.nbr_cnt || !s.com_cnt || !s.bag.items || !s.bag.in) {
    free(s.nbr_cnt); free(s.com_cnt); free(s.bag.items); free(s.bag.in);
    return ST_ENOMEM;
  }
  for (int64_t e = 0; e < g->nent; ++e) {
    if (!g->ea[e]) continue;
    int32_t u = g->src[e], v = g->nb[e];
    s.nbr_cnt[(int64_t)u * k + g->col[v]]++;
    if (u > v) continue;
    for (int64_t f = g->rp[u]; f < g->rp[u + 1]; ++f) {
      if (!g->ea[f]) continue;
      int32_t w = g->nb[f];
      if (edge_alive(g, v, w)) s.com_cnt[e * k + g->col[w]]++;
    }
  }
  for (int32_t v = 0; v < n; ++v) if (g->va[v]) bag_push(&s.bag, v);
  for (int64_t e = 0; e < g->nent; ++e)
    if (g->ea[e] && g->src[e] < g->nb[e]) bag_push(&s.bag, n + e);
  rng_t r = {seed};
  while (s.bag.len) {
    int64_t i = (int64_t)(rng_next(&r) % (uint64_t)s.bag.len);
    int64_t x = s.bag.items[i];
    s.bag.items[i] = s.bag.items[--s.bag.len];
    s.bag.in[x] = 0;
    if (x < n) {
      int32_t v = (int32_t)x;
      if (!g->va[v] || !o2_vertex_fails(&s, v)) continue;
      g->va[v] = 0;
      for (int64_t e = g->rp[v]; e < g->rp[v + 1]; ++e)
        if (g->ea[e]) o2_remove_edge(&s, canon(g, e));
    } else {
      int64_t ce = x - n;
      if (!g->ea[ce] || !o2_edge_fails(&s, ce)) continue;
      o2_remove_edge(&s, ce);
    }
  }
  free(s.nbr_cnt); free(s.com_cnt); free(s.bag.items); free(s.bag.in);
  return ST_OK;
}

/* ---------------------------------------------------------- brute force */

typedef struct {
  og_t *g;
  int32_t **cls; int32_t *clen;
  int32_t *pick;
  uint8_t *vin, *ein;
  int64_t count;
} bf_t;

static void bf_rec(bf_t *b, int32_t c) {
  og_t *g = b->g;
  for (int32_t i = 0; i < b->clen[c]; ++i) {
    int32_t v = b->cls[c][i];
    int ok = 1;
    for (int32_t j = 0; j < c && ok; ++j) ok = find_entry(g, b->pick[j], v) >= 0;
    if (!ok) continue;
    b->pick[c] = v;
    if (c + 1 < g->k) { bf_rec(b, c + 1); continue; }
    b->count++;
    for (int32_t a = 0; a < g->k; ++a) {
      b->vin[b->pick[a]] = 1;
      for (int32_t d = 0; d < g->k; ++d)
        if (a != d) b->ein[find_entry(g, b->pick[a], b->pick[d])] = 1;
    }
  }
}

/* Every k-clique of the INPUT graph (one vertex per class, pairwise
 * adjacent).  vin[n], ein[entries] receive the union.  Returns the count. */
int64_t kzo_kcliques(void *h, uint8_t *vin, uint8_t *ein) {
  og_t *g = (og_t *)h;
  int32_t n = g->n, k = g->k;
  memset(vin, 0, (size_t)(n ? n : 1));
  memset(ein, 0, (size_t)(g->nent ? g->nent : 1));
  bf_t b;
  b.g = g; b.vin = vin; b.ein = ein; b.count = 0;
  b.clen = (int32_t *)calloc((size_t)k, sizeof(int32_t));
  b.cls = (int32_t **)calloc((size_t)k, sizeof(int32_t *));
  b.pick = (int32_t *)calloc((size_t)k, sizeof(int32_t));
  for (int32_t v = 0; v < n; ++v) b.clen[g->col[v]]++;
  for (int32_t c = 0; c < k; ++c) { b.cls[c] = (int32_t *)malloc(sizeof(int32_t) * (size_t)(b.clen[c] + 1)); b.clen[c] = 0; }
  for (int32_t v = 0; v < n; ++v) b.cls[g->col[v]][b.clen[g->col[v]]++] = v;
  int empty = 0;
  for (int32_t c = 0; c < k; ++c) empty |= b.clen[c] == 0;
  if (!empty && n > 0) bf_rec(&b, 0);
  for (int32_t c = 0; c < k; ++c) free(b.cls[c]);
  free(b.cls); free(b.clen); free(b.pick);
  return b.count;
}

/* -------------------------------------------------------------- masks */

/* Current masks.  vmask[n]; emask in the loaded graph's format:
 * dense u8[n*n]; bitset uint64 rows (row_words per row); csr u8[nnz]. */
void kzo_get_masks(void *h, uint8_t *vmask, void *emask) {
  og_t *g = (og_t *)h;
  int32_t n = g->n;
  for (int32_t v = 0; v < n; ++v) vmask[v] = g->va[v];
  if (g->fmt == FMT_CSR) {
    for (int64_t e = 0; e < g->nent; ++e) ((uint8_t *)emask)[e] = g->ea[e];
  } else if (g->fmt == FMT_DENSE) {
    uint8_t *m = (uint8_t *)emask;
    memset(m, 0, (size_t)n * n);
    for (int64_t e = 0; e < g->nent; ++e)
      if (g->ea[e]) m[(int64_t)g->src[e] * n + g->nb[e]] = 1;
  } else {
    uint64_t *m = (uint64_t *)emask;
    memset(m, 0, sizeof(uint64_t) * (size_t)n * g->row_words);
    for (int64_t e = 0; e < g->nent; ++e) {
      if (!g->ea[e]) continue;
      int32_t w = g->nb[e], c = g->col[w];
      int64_t j = w - g->coff[c];
      m[(int64_t)g->src[e] * g->row_words + g->soff[c] + j / 64] |= 1ull << (j % 64);
    }
  }
}

/* Installs a state (e.g. a result to be checked) given as masks in the
 * graph's format.  Returns -1 if a mask names an edge that is not in the
 * input, or an edge alive in one direction only, or an alive edge at a dead
 * vertex. */
int kzo_set_masks(void *h, const uint8_t *vmask, const void *emask) {
  og_t *g = (og_t *)h;
  int32_t n = g->n;
  int64_t bits = 0;
  for (int32_t v = 0; v < n; ++v) {
    if (vmask[v] > 1) return -1;
    g->va[v] = vmask[v];
  }
  for (int64_t e = 0; e < g->nent; ++e) {
    int32_t u = g->src[e], w = g->nb[e];
    uint8_t a;
    if (g->fmt == FMT_CSR) {
      a = ((const uint8_t *)emask)[e];
      if (a > 1) return -1;
    } else if (g->fmt == FMT_DENSE) {
      a = ((const uint8_t *)emask)[(int64_t)u * n + w];
      if (a > 1) return -1;
    } else {
      int32_t c = g->col[w];
      int64_t j = w - g->coff[c];
      a = (((const uint64_t *)emask)[(int64_t)u * g->row_words + g->soff[c] + j / 64] >> (j % 64)) & 1u;
    }
    g->ea[e] = a;
    bits += a;
  }
  /* no mask bit outside the input's edges */
  int64_t total = 0;
  if (g->fmt == FMT_DENSE) {
    for (int64_t i = 0; i < (int64_t)n * n; ++i) total += ((const uint8_t *)emask)[i] != 0;
  } else if (g->fmt == FMT_BITSET) {
    for (int64_t i = 0; i < (int64_t)n * g->row_words; ++i)
      total += __builtin_popcountll(((const uint64_t *)emask)[i]);
  } else {
    total = bits;
  }
  if (total != bits) return -1;
  for (int64_t e = 0; e < g->nent; ++e) {
    if (g->ea[e] != g->ea[g->mate[e]]) return -1;
    if (g->ea[e] && (!g->va[g->src[e]] || !g->va[g->nb[e]])) return -1;
  }
  return 0;
}

/* For the listed vertices (vs) and edges (us[i], ws[i]) of the CURRENT
 * state: 1 where the element is alive and fails its test, else 0. */
void kzo_failing(void *h, const int32_t *vs, int64_t nv, uint8_t *vfail,
                 const int32_t *us, const int32_t *ws, int64_t ne, uint8_t *efail) {
  og_t *g = (og_t *)h;
  for (int64_t i = 0; i < nv; ++i)
    vfail[i] = g->va[vs[i]] && vertex_fails(g, vs[i]);
  for (int64_t i = 0; i < ne; ++i)
    efail[i] = edge_alive(g, us[i], ws[i]) && edge_fails(g, us[i], ws[i]);
}

/* ------------------------------------------------------------------- O3 */

/* O3: the synchronous rounds of O1 (same tests, same schedule, same counts),
 * computed on plain bit rows instead of adjacency lists, so that graphs with
 * 10^8 edges finish in seconds.  Input: the BITSET format (vertices class by
 * class, colour sorted; class c's segment holds ceil(s_c/64) words).  Its
 * own layout arithmetic and loops; nothing shared with O1/O2 except the
 * status codes.  Outputs: vmask[n], emask in the input's row layout (n *
 * row_words words), stats as kzo_fixpoint.  Returns a status code (input
 * validation in the documented order, checked on the rows themselves).
 *
 * One round, on the state A (alive edges as bits; a dead vertex has an
 * empty row):
 *   vertex v fails  <=> v alive and some class c != colour(v) has no bit in
 *                       A[v]'s segment c                   (index < k-1);
 *   edge {u,v} fails <=> some class c outside {colour(u), colour(v)} has
 *                       A[u][c] AND A[v][c] all zero         (index < k-2);
 * every failure is decided on A before any removal; then failed edges and
 * every edge of a failed vertex are cleared (both directions). */
#define O3_BIT(row, w) (((row)[(w) >> 6] >> ((w) & 63)) & 1ull)

/* More colours than the clique size (kk <= k classes): a k-clique still
 * uses kk distinct classes, so the same argument gives thresholds kk-1 and
 * kk-2: a vertex fails when more than k - kk other classes hold no
 * neighbour, an edge when more than k - kk third classes hold no common
 * neighbour.  kk = k is the rule above. */
static int o3_run(int32_t n, int32_t k, int32_t kk, const int32_t *col, const uint64_t *rows, int32_t row_words,
                  uint8_t *vmask, uint64_t *emask, int64_t *stats) {
  if (n < 0 || k < 1 || kk < 1 || kk > k || row_words < 0 || (n > 0 && (!col || !rows || !vmask || !emask)))
    return ST_EINVAL;
  const int32_t slack = k - kk;  /* classes a test may find without a witness */
  for (int32_t v = 0; v < n; ++v)
    if (col[v] < 0 || col[v] >= k) return ST_ECOLOUR;
  for (int32_t v = 1; v < n; ++v)
    if (col[v] < col[v - 1]) return ST_EINVAL;
  int64_t *first = (int64_t *)calloc((size_t)k + 1, sizeof(int64_t));  /* first vertex of class c */
  int64_t *seg = (int64_t *)calloc((size_t)k + 1, sizeof(int64_t));    /* first word of segment c */
  if (!first || !seg) { free(first); free(seg); return ST_ENOMEM; }
  for (int32_t v = 0; v < n; ++v) first[col[v] + 1] += 1;
  for (int32_t c = 0; c < k; ++c) {
    seg[c + 1] = seg[c] + (first[c + 1] + 63) / 64;
    first[c + 1] += first[c];
  }
  if (seg[k] != row_words) { free(first); free(seg); return ST_EINVAL; }
  const int64_t R = row_words;
  /* vertex id of bit j of word w: first[c] + 64*(w - seg[c]) + j for the
   * class c owning word w */
  int32_t *wcls = (int32_t *)malloc(sizeof(int32_t) * (size_t)(R ? R : 1));
  if (!wcls) { free(first); free(seg); return ST_ENOMEM; }
  for (int32_t c = 0; c < k; ++c)
    for (int64_t w = seg[c]; w < seg[c + 1]; ++w) wcls[w] = c;
  /* validation: malformed (padding bit) > self-loop > asymmetry > intra-class */
  int bad_pad = 0, bad_loop = 0, bad_asym = 0, bad_intra = 0;
  for (int32_t u = 0; u < n; ++u) {
    const uint64_t *ru = rows + (int64_t)u * R;
    for (int64_t w = 0; w < R; ++w) {
      uint64_t x = ru[w];
      while (x) {
        int j = __builtin_ctzll(x);
        x &= x - 1;
        int32_t c = wcls[w];
        int64_t v = first[c] + 64 * (w - seg[c]) + j;
        if (v >= first[c + 1]) { bad_pad = 1; continue; }
        if (v == u) { bad_loop = 1; continue; }
        int32_t cu = col[u];
        int64_t wu = seg[cu] + (u - first[cu]) / 64;
        if (!((rows[v * R + wu] >> ((u - first[cu]) % 64)) & 1ull)) bad_asym = 1;
        if (c == cu) bad_intra = 1;
      }
    }
  }
  int st = bad_pad ? ST_EINVAL : bad_loop ? ST_ESELFLOOP : bad_asym ? ST_EASYM : bad_intra ? ST_EILLEGAL : ST_OK;
  if (st) { free(first); free(seg); free(wcls); return st; }

  uint64_t *A = emask;                                    /* the state, in place */
  if (n) memcpy(A, rows, sizeof(uint64_t) * (size_t)n * (size_t)R);
  uint64_t *Fe = (uint64_t *)calloc((size_t)n * (size_t)R + 1, sizeof(uint64_t));  /* failed edges, u < v bits */
  uint8_t *fv = (uint8_t *)calloc((size_t)n + 1, 1);
  uint8_t *touched = (uint8_t *)calloc((size_t)n + 1, 1);
  if (!Fe || !fv || !touched) { free(first); free(seg); free(wcls); free(Fe); free(fv); free(touched); return ST_ENOMEM; }
  for (int32_t v = 0; v < n; ++v) vmask[v] = 1;
  int64_t m = 0;
  for (int32_t u = 0; u < n; ++u)
    for (int64_t w = 0; w < R; ++w) m += __builtin_popcountll(A[(int64_t)u * R + w]);
  m /= 2;
  int64_t rounds = 0, tests = m;
  for (;;) {
    int any = 0;
    /* vertex tests on the snapshot */
    for (int32_t v = 0; v < n; ++v) {
      fv[v] = 0;
      if (!vmask[v]) continue;
      const uint64_t *rv = A + (int64_t)v * R;
      int32_t miss = 0;
      for (int32_t c = 0; c < k && miss <= slack; ++c) {
        if (c == col[v]) continue;
        int has = 0;
        for (int64_t w = seg[c]; w < seg[c + 1] && !has; ++w) has = rv[w] != 0;
        if (!has) ++miss;
      }
      fv[v] = miss > slack;
      any |= fv[v];
    }
    /* edge tests on the snapshot: every alive edge u < v */
    for (int32_t u = 0; u < n; ++u) {
      const uint64_t *ru = A + (int64_t)u * R;
      uint64_t *fu = Fe + (int64_t)u * R;
      for (int64_t w = 0; w < R; ++w) {
        fu[w] = 0;
        uint64_t x = ru[w];
        while (x) {
          int j = __builtin_ctzll(x);
          x &= x - 1;
          int32_t cv = wcls[w];
          int64_t v = first[cv] + 64 * (w - seg[cv]) + j;
          if (v <= u || kk < 3) continue;
          const uint64_t *rv = A + v * R;
          int32_t miss = 0;
          for (int32_t c = 0; c < k && miss <= slack; ++c) {
            if (c == col[u] || c == cv) continue;
            int common = 0;
            for (int64_t t = seg[c]; t < seg[c + 1] && !common; ++t) common = (ru[t] & rv[t]) != 0;
            if (!common) ++miss;
          }
          if (miss > slack) { fu[w] |= 1ull << j; any = 1; }
        }
      }
    }
    if (!any) break;
    /* apply the round: failed edges, then every edge at a failed vertex */
    memset(touched, 0, (size_t)n + 1);
    for (int32_t u = 0; u < n; ++u) {
      uint64_t *ru = A + (int64_t)u * R;
      for (int64_t w = 0; w < R; ++w) {
        uint64_t x = Fe[(int64_t)u * R + w];
        while (x) {
          int j = __builtin_ctzll(x);
          x &= x - 1;
          int32_t cv = wcls[w];
          int64_t v = first[cv] + 64 * (w - seg[cv]) + j;
          int32_t cu = col[u];
          ru[w] &= ~(1ull << j);
          A[v * R + seg[cu] + (u - first[cu]) / 64] &= ~(1ull << ((u - first[cu]) % 64));
          touched[u] = touched[v] = 1;
        }
      }
    }
    for (int32_t u = 0; u < n; ++u) {
      if (!fv[u]) continue;
      uint64_t *ru = A + (int64_t)u * R;
      int32_t cu = col[u];
      for (int64_t w = 0; w < R; ++w) {
        uint64_t x = ru[w];
        while (x) {
          int j = __builtin_ctzll(x);
          x &= x - 1;
          int32_t cv = wcls[w];
          int64_t v = first[cv] + 64 * (w - seg[cv]) + j;
          A[v * R + seg[cu] + (u - first[cu]) / 64] &= ~(1ull << ((u - first[cu]) % 64));
          touched[u] = touched[v] = 1;
        }
        ru[w] = 0;
      }
      vmask[u] = 0;
    }
    ++rounds;
    /* next pass's exact worklist: alive edges with a touched endpoint */
    for (int32_t u = 0; u < n; ++u) {
      const uint64_t *ru = A + (int64_t)u * R;
      for (int64_t w = 0; w < R; ++w) {
        uint64_t x = ru[w];
        while (x) {
          int j = __builtin_ctzll(x);
          x &= x - 1;
          int32_t cv = wcls[w];
          int64_t v = first[cv] + 64 * (w - seg[cv]) + j;
          if (v > u && (touched[u] || touched[v])) ++tests;
        }
      }
    }
  }
  int64_t sv = 0, se = 0;
  for (int32_t v = 0; v < n; ++v) sv += vmask[v];
  for (int64_t i = 0; i < (int64_t)n * R; ++i) se += __builtin_popcountll(A[i]);
  const int64_t out[5] = {rounds, rounds == 0, sv, se / 2, tests};
  memcpy(stats, out, sizeof out);
  free(first); free(seg); free(wcls); free(Fe); free(fv); free(touched);
  return ST_OK;
}

int kzo_fixpoint_rows(int32_t n, int32_t k, const int32_t *col, const uint64_t *rows, int32_t row_words,
                      uint8_t *vmask, uint64_t *emask, int64_t *stats) {
  return o3_run(n, k, k, col, rows, row_words, vmask, emask, stats);
}

/* k classes, cliques of size kk <= k (section 4.2's indices with thresholds
 * kk-1 and kk-2 on a graph coloured with more colours than the clique size). */
int kzo_fixpoint_rows_mk(int32_t n, int32_t k, int32_t kk, const int32_t *col, const uint64_t *rows,
                         int32_t row_words, uint8_t *vmask, uint64_t *emask, int64_t *stats) {
  return o3_run(n, k, kk, col, rows, row_words, vmask, emask, stats);
}

/* ------------------------------------------------- witness-search work */

/* Measurement, not a result: over every edge {u,v} (u < v) of the input and
 * every class c other than the endpoints' classes, the number of words of
 * the two class-c segments that a search in word order reads up to and
 * including the first word holding a common neighbour (the whole segment
 * when there is none).  This is the least work of a test that stops at the
 * first witness of each class (section 4.2's edge index only needs to know
 * whether each class holds a common neighbour).  Input: the BITSET format,
 * assumed valid (validate it with kzo_fixpoint_rows or kzo_load first).
 * *pairs receives the number of (edge, class) pairs, *nowit those without a
 * common neighbour. */
int64_t kzo_witness_words(int32_t n, int32_t k, const int32_t *col, const uint64_t *rows, int32_t row_words,
                          int64_t *pairs, int64_t *nowit) {
  int64_t *first = (int64_t *)calloc((size_t)k + 1, sizeof(int64_t));
  int64_t *seg = (int64_t *)calloc((size_t)k + 1, sizeof(int64_t));
  if (!first || !seg) { free(first); free(seg); return -1; }
  for (int32_t v = 0; v < n; ++v) first[col[v] + 1] += 1;
  for (int32_t c = 0; c < k; ++c) {
    seg[c + 1] = seg[c] + (first[c + 1] + 63) / 64;
    first[c + 1] += first[c];
  }
  const int64_t R = row_words;
  int64_t words = 0, np = 0, nw = 0;
  for (int32_t u = 0; u < n; ++u) {
    const uint64_t *ru = rows + (int64_t)u * R;
    for (int32_t cv = 0; cv < k; ++cv) {
      for (int64_t j = 0; j < first[cv + 1] - first[cv]; ++j) {
        int64_t v = first[cv] + j;
        if (v <= u || !((ru[seg[cv] + j / 64] >> (j % 64)) & 1ull)) continue;
        const uint64_t *rv = rows + v * R;
        for (int32_t c = 0; c < k; ++c) {
          if (c == col[u] || c == cv) continue;
          int64_t w = seg[c];
          while (w < seg[c + 1] && !(ru[w] & rv[w])) ++w;
          if (w < seg[c + 1]) words += w - seg[c] + 1;
          else { words += seg[c + 1] - seg[c]; ++nw; }
          ++np;
        }
      }
    }
  }
  free(first); free(seg);
  *pairs = np;
  *nowit = nw;
  return words;
}
