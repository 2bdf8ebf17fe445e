/*
 * kz_oracle_ext.c -- plain CPU oracles for the reductions and searches that
 * sit beside colour-index pruning.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg do.  It shares no code with the GPU library.  Graphs are a
 * dense n*n matrix of 0/1 bytes (adj[v*n+w]), symmetric, zero diagonal.
 *
 * Dominance (thesis section 4.3).
 *
 *   Definition 4.3.1: node b dominates node a when a and b are distinct and
 *   not adjacent and N(a) is a subset of N(b).  A dominated node is deleted
 *   with its edges.  (Non-adjacency is implied by the subset: if a and b were
 *   adjacent, b would be in N(a) but not in N(b).)
 *
 *   Definition 4.3.2: for distinct a, u, b, the edge {u,b} dominates the
 *   edge {a,u} when b is not a neighbour of a and the common neighbourhood
 *   N(a) & N(u) is a subset of N(u) & N(b), i.e. of N(b).  The dominated edge
 *   is deleted; a and u stay.  (The thesis writes the first condition as
 *   "b is not in N(a) & N(b)", which holds in every simple graph; it is read
 *   as "b is not in N(a)", the condition that lets {u,b} replace {a,u} in a
 *   clique.)
 *
 *   Algorithm 1 (vertex dominance), as read here: for every node b in index
 *   order (skipping deleted ones), for every node a in index order: if b
 *   dominates a in the current graph, delete a at once (so later tests see
 *   the smaller graph).  The printed listing loops over a in N(node) and
 *   tests "N(a) & N(node)" with no comparison; both contradict Definition
 *   4.3.1 and are read as its non-adjacency and subset test.
 *
 *   Algorithm 2 (edge dominance), as read here: for every node a in index
 *   order, for every neighbour u of a in index order, for every neighbour b
 *   of u in index order with b != a: if b is not a neighbour of a and
 *   N(a) & N(u) is a subset of N(b) (current graph), delete the edge {a,u}
 *   and go on with the next u.  The printed listing's condition 1 ("b in
 *   N(a) & N(u)") contradicts Definition 4.3.2 and is read as "b not in
 *   N(a)"; its condition 2 compares a set with itself and is read as the
 *   definition's inclusion; it deletes "{a,b}", read as the dominated edge
 *   {a,u}.
 *
 *   One run of either algorithm is a sweep; sweeps repeat until one deletes
 *   nothing.  Each deletion keeps some maximum clique (a clique through the
 *   deleted vertex or edge trades a for b), so the clique number never
 *   changes; vertex dominance may delete some k-cliques, which is why it is
 *   kept apart from the clique-preserving colour-index path.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* b dominates a in the current graph (Definition 4.3.1). */
static int vertex_dominates(int32_t n, const uint8_t *adj, const uint8_t *alive, int32_t b, int32_t a) {
  if (a == b || !alive[a] || !alive[b] || adj[(int64_t)a * n + b]) return 0;
  for (int32_t x = 0; x < n; ++x)
    if (adj[(int64_t)a * n + x] && !adj[(int64_t)b * n + x]) return 0;
  return 1;
}

static int64_t delete_vertex(int32_t n, uint8_t *adj, uint8_t *alive, int32_t a) {
  int64_t removed = 0;
  alive[a] = 0;
  for (int32_t x = 0; x < n; ++x) {
    if (adj[(int64_t)a * n + x]) {
      adj[(int64_t)a * n + x] = 0;
      adj[(int64_t)x * n + a] = 0;
      ++removed;
    }
  }
  return removed;
}

/* Sweeps of Algorithm 1 until one deletes nothing.  adj is updated in place
 * (deleted vertices lose their edges); alive[v] = 1 for survivors.
 * stats: [0] sweeps that deleted something, [1] deleted vertices,
 * [2] deleted edges, [3] steps (node b) that deleted something. */
int kzo_dom_vertex(int32_t n, uint8_t *adj, uint8_t *alive, int64_t *stats) {
  int64_t sweeps = 0, dv = 0, de = 0, steps = 0;
  for (int32_t v = 0; v < n; ++v) alive[v] = 1;
  for (;;) {
    int any = 0;
    for (int32_t b = 0; b < n; ++b) {
      if (!alive[b]) continue;
      int here = 0;
      for (int32_t a = 0; a < n; ++a) {
        if (vertex_dominates(n, adj, alive, b, a)) {
          de += delete_vertex(n, adj, alive, a);
          ++dv;
          here = 1;
        }
      }
      steps += here;
      any |= here;
    }
    if (!any) break;
    ++sweeps;
  }
  stats[0] = sweeps;
  stats[1] = dv;
  stats[2] = de;
  stats[3] = steps;
  return 0;
}

/* The edge {u,b} dominates {a,u} in the current graph (Definition 4.3.2). */
static int edge_dominates(int32_t n, const uint8_t *adj, int32_t a, int32_t u, int32_t b) {
  if (b == a || b == u || a == u) return 0;
  if (!adj[(int64_t)a * n + u] || !adj[(int64_t)u * n + b] || adj[(int64_t)a * n + b]) return 0;
  for (int32_t x = 0; x < n; ++x)
    if (adj[(int64_t)a * n + x] && adj[(int64_t)u * n + x] && !adj[(int64_t)b * n + x]) return 0;
  return 1;
}

/* Sweeps of Algorithm 2 until one deletes nothing.  adj is updated in place.
 * stats: [0] sweeps that deleted something, [1] deleted edges. */
int kzo_dom_edge(int32_t n, uint8_t *adj, int64_t *stats) {
  int64_t sweeps = 0, de = 0;
  for (;;) {
    int any = 0;
    for (int32_t a = 0; a < n; ++a) {
      for (int32_t u = 0; u < n; ++u) {
        if (!adj[(int64_t)a * n + u]) continue;
        for (int32_t b = 0; b < n; ++b) {
          if (!adj[(int64_t)u * n + b]) continue;
          if (edge_dominates(n, adj, a, u, b)) {
            adj[(int64_t)a * n + u] = 0;
            adj[(int64_t)u * n + a] = 0;
            ++de;
            any = 1;
            break;
          }
        }
      }
    }
    if (!any) break;
    ++sweeps;
  }
  stats[0] = sweeps;
  stats[1] = de;
  return 0;
}

/*
 * k-clique search (the thesis's problem statement: the kernel is handed to
 * a standard solver that looks for a k-clique; section 4.2 names the
 * problem, no solver is given).  On a legally k-coloured graph a k-clique
 * holds one vertex of every class.  The search picks a vertex of class 0,
 * then of class 1, ... in increasing index order, each adjacent to every
 * vertex picked before, among the live vertices (alive[v] != 0; all when
 * alive is NULL).  The first complete pick is the lexicographically smallest
 * k-clique (ordered by class 0's vertex, then class 1's, ...).
 *   adj: n*n bytes, colour: int32[n] in [0, k), clique: int32[k] out.
 * Returns 1 and fills clique when one exists, 0 otherwise; *nodes counts the
 * partial picks extended (a measure of the search, not a result).
 */
static int clique_rec(int32_t n, const uint8_t *adj, const int32_t *colour, int32_t k, const uint8_t *alive,
                      int32_t c, int32_t *pick, int64_t *nodes) {
  if (c == k) return 1;
  for (int32_t v = 0; v < n; ++v) {
    if (colour[v] != c || (alive && !alive[v])) continue;
    int ok = 1;
    for (int32_t j = 0; j < c && ok; ++j) ok = adj[(int64_t)pick[j] * n + v] != 0;
    if (!ok) continue;
    pick[c] = v;
    ++*nodes;
    if (clique_rec(n, adj, colour, k, alive, c + 1, pick, nodes)) return 1;
  }
  return 0;
}

int kzo_find_clique(int32_t n, const uint8_t *adj, const int32_t *colour, int32_t k, const uint8_t *alive,
                    int32_t *clique, int64_t *nodes) {
  *nodes = 0;
  if (k < 1) return 0;
  int32_t *pick = (int32_t *)calloc((size_t)k, sizeof(int32_t));
  if (!pick) return -1;
  const int found = clique_rec(n, adj, colour, k, alive, 0, pick, nodes);
  for (int32_t c = 0; c < k; ++c) clique[c] = found ? pick[c] : -1;
  free(pick);
  return found;
}

/*
 * Struction (thesis section 4.1, Definition 4.1.1, Lemmas 1-2, Theorem 1).
 * Pivot p; A = the neighbours of p, B = the other vertices except p, both
 * in increasing order.  C holds a node c(x, y) for every edge {x, y} of G
 * inside B with x < y.  G' has the nodes A (in order) followed by C (ordered
 * by x, then y):
 *   a, a' in A are adjacent iff {a, a'} is an edge of G;
 *   c(x, y), c(x', y') in C are adjacent iff x = x' and {y, y'} is an edge
 *     of G (the thesis's "ordered pair {bY, bM}" is read as this edge);
 *   a in A and c(x, y) in C are adjacent iff a is adjacent to both x and y
 *     (the thesis gives no rule for these pairs; this one makes both lemmas
 *     hold: the C nodes of a clique of G' share their first vertex x, and
 *     x with their second vertices and the clique's A nodes is a clique of G
 *     one larger; a clique of G that avoids p maps back through its smallest
 *     B vertex).
 * So omega(G') = omega(G) - 1 (Theorem 1).
 *   adj: n*n bytes; out: n'*n' bytes (capacity cap nodes; call with out =
 *   NULL to get n' only); map: int32[n'][2] = (vertex, -1) for A nodes and
 *   (x, y) for C nodes.  Returns n', or -1 when cap is too small.
 */
int64_t kzo_struction(int32_t n, const uint8_t *adj, int32_t pivot, uint8_t *out, int64_t cap, int32_t *map) {
  if (pivot < 0 || pivot >= n) return -1;
  int64_t na = 0, nc = 0;
  for (int32_t v = 0; v < n; ++v) {
    if (v == pivot) continue;
    if (adj[(int64_t)pivot * n + v]) ++na;
  }
  for (int32_t x = 0; x < n; ++x) {
    if (x == pivot || adj[(int64_t)pivot * n + x]) continue;
    for (int32_t y = x + 1; y < n; ++y)
      if (y != pivot && !adj[(int64_t)pivot * n + y] && adj[(int64_t)x * n + y]) ++nc;
  }
  const int64_t np = na + nc;
  if (!out) return np;
  if (np > cap) return -1;
  int64_t i = 0;
  for (int32_t v = 0; v < n; ++v) {
    if (v != pivot && adj[(int64_t)pivot * n + v]) {
      map[2 * i] = v;
      map[2 * i + 1] = -1;
      ++i;
    }
  }
  for (int32_t x = 0; x < n; ++x) {
    if (x == pivot || adj[(int64_t)pivot * n + x]) continue;
    for (int32_t y = x + 1; y < n; ++y) {
      if (y != pivot && !adj[(int64_t)pivot * n + y] && adj[(int64_t)x * n + y]) {
        map[2 * i] = x;
        map[2 * i + 1] = y;
        ++i;
      }
    }
  }
  for (int64_t s = 0; s < np; ++s) {
    for (int64_t t = 0; t < np; ++t) {
      uint8_t e = 0;
      if (s != t) {
        const int32_t xs = map[2 * s], ys = map[2 * s + 1], xt = map[2 * t], yt = map[2 * t + 1];
        if (ys < 0 && yt < 0) e = adj[(int64_t)xs * n + xt];
        else if (ys >= 0 && yt >= 0) e = xs == xt && adj[(int64_t)ys * n + yt];
        else if (ys < 0) e = adj[(int64_t)xs * n + xt] && adj[(int64_t)xs * n + yt];
        else e = adj[(int64_t)xt * n + xs] && adj[(int64_t)xt * n + ys];
      }
      out[s * np + t] = e;
    }
  }
  return np;
}

/*
 * Upstream legal colouring.  The colour-index method (thesis section 4.2)
 * needs a legal colouring of its input; the thesis assumes one is given
 * and names no algorithm.  This is Jones and Plassmann's parallel greedy
 * colouring (SIAM J. Sci. Comput. 14(3), 1993).  Every vertex v has the key
 * (pri[v], v), compared lexicographically, so keys are distinct.  In each
 * round, every uncoloured vertex whose key exceeds the key of each of its
 * uncoloured neighbours is taken; each vertex taken receives the smallest
 * colour that none of its neighbours coloured in earlier rounds holds.  Two
 * vertices taken in one round are never adjacent (one of them has the larger
 * key), so the colouring is legal and does not depend on the order in which
 * a round's vertices are coloured.
 *   adj: n*n bytes (symmetric, zero diagonal); pri: uint64[n];
 *   colour: int32[n] out; *ncolours = 1 + the largest colour (0 for n = 0).
 * Returns the number of rounds, or -1 if a round takes no vertex (cannot
 * happen with distinct keys: the largest uncoloured key is always taken).
 */
static int jp_beats(const uint64_t *pri, int32_t u, int32_t v) {
  return pri[u] > pri[v] || (pri[u] == pri[v] && u > v);
}

int kzo_colour_jp(int32_t n, const uint8_t *adj, const uint64_t *pri, int32_t *colour, int32_t *ncolours) {
  int rounds = 0, left = n, top = -1;
  uint8_t *taken = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
  uint8_t *used = (uint8_t *)calloc((size_t)(n > 0 ? n : 1) + 1, 1);
  if (!taken || !used) {
    free(taken);
    free(used);
    return -1;
  }
  for (int32_t v = 0; v < n; ++v) colour[v] = -1;
  while (left > 0) {
    /* the vertices this round takes, from the colours at its start */
    int any = 0;
    for (int32_t v = 0; v < n; ++v) {
      taken[v] = 0;
      if (colour[v] >= 0) continue;
      int best = 1;
      for (int32_t u = 0; u < n && best; ++u)
        if (adj[(int64_t)v * n + u] && colour[u] < 0 && jp_beats(pri, u, v)) best = 0;
      taken[v] = (uint8_t)best;
      any |= best;
    }
    if (!any) {
      free(taken);
      free(used);
      return -1;
    }
    /* each takes the smallest colour its coloured neighbours leave free */
    for (int32_t v = 0; v < n; ++v) {
      if (!taken[v]) continue;
      memset(used, 0, (size_t)n + 1);
      for (int32_t u = 0; u < n; ++u)
        if (adj[(int64_t)v * n + u] && colour[u] >= 0 && !taken[u]) used[colour[u]] = 1;
      int c = 0;
      while (used[c]) ++c;
      colour[v] = c;
      if (c > top) top = c;
      --left;
    }
    ++rounds;
  }
  *ncolours = top + 1;
  free(taken);
  free(used);
  return rounds;
}
