/* ORACLE -- test infrastructure only.  Only tests/, __graft_entry__.smoke()
 * and bench.py's cpu_baseline leg may load this file's library.  It shares no
 * code with the GPU decoder.
 *
 * Plain, slow CPU computation of the minimum-weight embedded matching (MWEM)
 * of the decoding task (Results, "Decoding task"): given a detector graph
 * G = (V, E) with positive integer weights and a set D of active detectors,
 * find the minimum-weight M subset of E such that every detector in D has odd
 * degree in M, every other detector even degree, and boundary vertices any
 * degree.
 *
 * Method (textbook reduction, no blocking or reordering):
 *   1. Tie-broken integer weights.  With uniform weights the optimum is
 *      highly degenerate, so every solver here and on the GPU minimises the
 *      integer weight  wt(e) = 2*w(e)*2^64 + 2*h(e),  where h(e) is the
 *      (e+1)-th output of a SplitMix64 stream (Steele, Lea & Flood 2014)
 *      seeded with the tie-break seed, shifted right by 24 (40 bits).  Since
 *      sum_e 2*h(e) < 2^64 for |E| < 2^23, a wt-optimum is also a w-optimum;
 *      the wt-optimum is unique except with probability <= |E| / 2^40
 *      (isolation lemma).  Even weights make every event time of sparse
 *      blossom integral (Supplementary S1, where weights are scaled to even
 *      integers).
 *   2. Dijkstra from every defect on wt; a boundary vertex is a sink, so a
 *      defect's boundary distance is min over boundary edges (u, b) of
 *      dist(u) + wt(u, b).
 *   3. Minimum-weight perfect matching on the defect graph: nodes D and one
 *      boundary copy s' per defect s; costs dist(s, t), dist_bd(s) on (s, s'),
 *      and 0 on (s', t').  Solved exactly with Edmonds' weighted blossom
 *      algorithm (Edmonds 1965; the O(n^3) organisation of Gabow/Galil with
 *      per-vertex best-edge tracking) as a maximum-weight matching of
 *      K - cost with K large enough that every maximum-weight matching is
 *      perfect.  The matcher's organisation (vertex and blossom ids in one
 *      array, S/T labels, per-node best slack edge, the LCA walk with
 *      stamps, pairing within a blossom cycle by i ^ 1 after rotating to the
 *      base, halving the slack step) follows the widely circulated O(n^3)
 *      weighted general-matching routine of competitive programming, whose
 *      routines it mirrors one for one under other names; it is test
 *      infrastructure, and every call checks its output with the LP
 *      certificate of step 5.
 *   4. M = symmetric difference of the shortest paths of the matched pairs
 *      (and of the path to the nearest boundary edge for (s, s') pairs).
 *   5. Certificate: the final duals are checked for feasibility and
 *      complementary slackness and primal weight == dual objective
 *      (Supplementary S1, primal-dual pair), all in exact integers.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;
#define I128_INF (((i128)0x3FFFFFFFFFFFFFFFLL << 64) | (i128)0xFFFFFFFFFFFFFFFFULL)

enum { OF_TIE = 1, OF_INFEASIBLE = 2, OF_CERT_FAIL = 4, OF_CAPACITY = 8 };

/* ------------------------------------------------------------------ */
/* tie-break weights                                                    */
/* ------------------------------------------------------------------ */
static uint64_t splitmix_output(uint64_t seed, uint64_t k) {
  uint64_t z = seed + k * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static i128 tiebroken_weight(int32_t w, uint64_t seed, int64_t e) {
  uint64_t h = splitmix_output(seed, (uint64_t)e + 1ULL) >> 24;
  return ((i128)(2 * (int64_t)w) << 64) + (i128)(2 * h);
}

/* ------------------------------------------------------------------ */
/* graph                                                                */
/* ------------------------------------------------------------------ */
typedef struct {
  int32_t n;           /* detectors */
  int64_t m;           /* edges */
  int32_t* eu; int32_t* ev; int32_t* w; uint64_t* obs;
  i128* wt;            /* tie-broken weights */
  int64_t* adj_off;    /* CSR over detectors */
  int64_t* adj_edge;   /* edge ids */
} og_graph;

void* oracle_graph_create(int32_t n, int64_t m, const int32_t* eu, const int32_t* ev,
                          const int32_t* w, const uint64_t* obs, uint64_t seed) {
  if (n <= 0 || m < 0) return NULL;
  for (int64_t e = 0; e < m; ++e) {
    if (eu[e] < 0 || eu[e] >= n || ev[e] < -1 || ev[e] >= n || w[e] <= 0 || eu[e] == ev[e]) return NULL;
  }
  og_graph* g = (og_graph*)calloc(1, sizeof(og_graph));
  g->n = n; g->m = m;
  g->eu = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
  g->ev = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
  g->w = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
  g->obs = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(m ? m : 1));
  g->wt = (i128*)malloc(sizeof(i128) * (size_t)(m ? m : 1));
  memcpy(g->eu, eu, sizeof(int32_t) * (size_t)m);
  memcpy(g->ev, ev, sizeof(int32_t) * (size_t)m);
  memcpy(g->w, w, sizeof(int32_t) * (size_t)m);
  memcpy(g->obs, obs, sizeof(uint64_t) * (size_t)m);
  for (int64_t e = 0; e < m; ++e) g->wt[e] = tiebroken_weight(w[e], seed, e);
  g->adj_off = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  for (int64_t e = 0; e < m; ++e) {
    g->adj_off[eu[e] + 1]++;
    if (ev[e] >= 0) g->adj_off[ev[e] + 1]++;
  }
  for (int32_t i = 0; i < n; ++i) g->adj_off[i + 1] += g->adj_off[i];
  g->adj_edge = (int64_t*)malloc(sizeof(int64_t) * (size_t)(g->adj_off[n] ? g->adj_off[n] : 1));
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  for (int32_t i = 0; i < n; ++i) fill[i] = g->adj_off[i];
  for (int64_t e = 0; e < m; ++e) {
    g->adj_edge[fill[eu[e]]++] = e;
    if (ev[e] >= 0) g->adj_edge[fill[ev[e]]++] = e;
  }
  free(fill);
  return g;
}

void oracle_graph_destroy(void* p) {
  og_graph* g = (og_graph*)p;
  if (!g) return;
  free(g->eu); free(g->ev); free(g->w); free(g->obs); free(g->wt);
  free(g->adj_off); free(g->adj_edge); free(g);
}

/* ------------------------------------------------------------------ */
/* Dijkstra with a binary heap (lazy deletion)                          */
/* ------------------------------------------------------------------ */
typedef struct { i128 key; int32_t node; } heap_item;

typedef struct {
  i128* dist;        /* [n] */
  int64_t* pred;     /* [n] edge used to reach the node, -1 for the source */
  uint8_t* tie;      /* [n] a second shortest path reaches the node (or its pred chain) */
  i128 bd_dist;      /* distance to the nearest boundary vertex */
  int64_t bd_edge;   /* the boundary edge achieving it, -1 if none */
  int bd_tie;        /* two boundary edges at the same distance */
} sp_tree;

static void sp_alloc(sp_tree* t, int32_t n) {
  t->dist = (i128*)malloc(sizeof(i128) * (size_t)n);
  t->pred = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  t->tie = (uint8_t*)malloc((size_t)n);
}
static void sp_free(sp_tree* t) { free(t->dist); free(t->pred); free(t->tie); }

static void heap_push(heap_item* h, int64_t* sz, i128 key, int32_t node) {
  int64_t i = (*sz)++;
  h[i].key = key; h[i].node = node;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (h[p].key <= h[i].key) break;
    heap_item t = h[p]; h[p] = h[i]; h[i] = t; i = p;
  }
}
static heap_item heap_pop(heap_item* h, int64_t* sz) {
  heap_item top = h[0];
  h[0] = h[--(*sz)];
  int64_t i = 0;
  for (;;) {
    int64_t l = 2 * i + 1, r = l + 1, s = i;
    if (l < *sz && h[l].key < h[s].key) s = l;
    if (r < *sz && h[r].key < h[s].key) s = r;
    if (s == i) break;
    heap_item t = h[s]; h[s] = h[i]; h[i] = t; i = s;
  }
  return top;
}

/* Shortest paths from `src` (boundary vertices are sinks, never relaxed through). */
static void dijkstra(const og_graph* g, int32_t src, sp_tree* t) {
  const int32_t n = g->n;
  for (int32_t i = 0; i < n; ++i) { t->dist[i] = I128_INF; t->pred[i] = -1; t->tie[i] = 0; }
  uint8_t* done = (uint8_t*)calloc((size_t)n, 1);
  heap_item* h = (heap_item*)malloc(sizeof(heap_item) * (size_t)(g->adj_off[n] + 2));
  int64_t sz = 0;
  t->dist[src] = 0;
  heap_push(h, &sz, 0, src);
  t->bd_dist = I128_INF; t->bd_edge = -1; t->bd_tie = 0;
  while (sz > 0) {
    heap_item it = heap_pop(h, &sz);
    int32_t u = it.node;
    if (done[u] || it.key != t->dist[u]) continue;
    done[u] = 1;
    if (t->pred[u] >= 0) {
      int64_t pe = t->pred[u];
      int32_t pu = g->eu[pe] == u ? g->ev[pe] : g->eu[pe];
      t->tie[u] |= t->tie[pu];
    }
    for (int64_t k = g->adj_off[u]; k < g->adj_off[u + 1]; ++k) {
      int64_t e = g->adj_edge[k];
      int32_t v = g->eu[e] == u ? g->ev[e] : g->eu[e];
      i128 nd = t->dist[u] + g->wt[e];
      if (v < 0) {
        if (nd < t->bd_dist) { t->bd_dist = nd; t->bd_edge = e; t->bd_tie = t->tie[u]; }
        else if (nd == t->bd_dist) t->bd_tie = 1;
        continue;
      }
      if (done[v]) continue;
      if (nd < t->dist[v]) { t->dist[v] = nd; t->pred[v] = e; t->tie[v] = 0; heap_push(h, &sz, nd, v); }
      else if (nd == t->dist[v]) t->tie[v] = 1;
    }
  }
  free(done); free(h);
}

/* Exported: distances from one source (as hi/lo 64-bit halves), for tests. */
int oracle_dijkstra(void* pg, int32_t src, int64_t* dist_hi, uint64_t* dist_lo, int64_t* pred,
                    int64_t* bd_hi, uint64_t* bd_lo, int64_t* bd_edge) {
  og_graph* g = (og_graph*)pg;
  if (!g || src < 0 || src >= g->n) return -1;
  sp_tree t; sp_alloc(&t, g->n);
  dijkstra(g, src, &t);
  for (int32_t i = 0; i < g->n; ++i) {
    dist_hi[i] = (int64_t)(t.dist[i] >> 64);
    dist_lo[i] = (uint64_t)t.dist[i];
    pred[i] = t.pred[i];
  }
  *bd_hi = (int64_t)(t.bd_dist >> 64); *bd_lo = (uint64_t)t.bd_dist; *bd_edge = t.bd_edge;
  sp_free(&t);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Edmonds' weighted matching (maximum weight, general graph)           */
/* ------------------------------------------------------------------ */
/* Vertices 1..nv, blossoms nv+1 .. 2*nv.  Weights are doubled internally so
 * that all duals stay integral.  A node x (vertex or top-level blossom) has
 * label S (0, outer), T (1, inner) or free (-1). */
typedef struct { int32_t a, b; i128 wgt; } m_edge;   /* a, b vertices; wgt 0 = no edge */

typedef struct {
  int32_t nv, nx;                 /* vertices, highest blossom id in use */
  int32_t cap;                    /* 2*nv + 1 */
  m_edge* g;                      /* [cap*cap] best edge between two nodes */
  i128* dual;                     /* [cap] */
  int32_t* mate;                  /* [cap] vertex on the other side of the matched edge */
  int32_t* best;                  /* [cap] S-vertex giving the least-slack edge into node x */
  int32_t* top;                   /* [cap] top-level blossom containing x */
  int32_t* parent;                /* [cap] for T nodes: the S vertex they hang from */
  int32_t* label;                 /* [cap] */
  int32_t* stamp;                 /* [cap] for the LCA search */
  int32_t stamp_now;
  int32_t** child;                /* [cap] cycle of sub-blossoms, base first */
  int32_t* nchild;                /* [cap] */
  int32_t* inner_of;              /* [cap*(nv+1)] sub-blossom of b holding vertex v */
  int32_t* queue; int32_t qh, qt;
} matcher;

#define G(M, x, y) ((M)->g[(size_t)(x) * (size_t)(M)->cap + (size_t)(y)])
#define INNER(M, b, v) ((M)->inner_of[(size_t)(b) * (size_t)((M)->nv + 1) + (size_t)(v)])

static i128 slack_of(const matcher* M, m_edge e) {
  return M->dual[e.a] + M->dual[e.b] - 2 * e.wgt;
}

static void q_add(matcher* M, int32_t x) {
  if (x <= M->nv) { M->queue[M->qt++] = x; return; }
  for (int32_t i = 0; i < M->nchild[x]; ++i) q_add(M, M->child[x][i]);
}

static void set_top(matcher* M, int32_t x, int32_t b) {
  M->top[x] = b;
  if (x > M->nv) for (int32_t i = 0; i < M->nchild[x]; ++i) set_top(M, M->child[x][i], b);
}

static void consider_best(matcher* M, int32_t u, int32_t x) {
  if (!M->best[x] || slack_of(M, G(M, u, x)) < slack_of(M, G(M, M->best[x], x))) M->best[x] = u;
}

static void recompute_best(matcher* M, int32_t x) {
  M->best[x] = 0;
  for (int32_t u = 1; u <= M->nv; ++u)
    if (G(M, u, x).wgt > 0 && M->top[u] != x && M->label[M->top[u]] == 0) consider_best(M, u, x);
}

/* Rotate the cycle of blossom b so that the walk from the base to sub-blossom
 * xr has even length; returns the position of xr. */
static int32_t even_position(matcher* M, int32_t b, int32_t xr) {
  int32_t k = M->nchild[b], pos = 0;
  while (M->child[b][pos] != xr) ++pos;
  if (pos % 2 == 1) {
    /* reverse children 1..k-1 so the walk goes the other way round */
    for (int32_t i = 1, j = k - 1; i < j; ++i, --j) {
      int32_t t = M->child[b][i]; M->child[b][i] = M->child[b][j]; M->child[b][j] = t;
    }
    return k - pos;
  }
  return pos;
}

/* Match node x through its edge towards node y, fixing the blossom interior. */
static void match_through(matcher* M, int32_t x, int32_t y) {
  M->mate[x] = G(M, x, y).b;
  if (x <= M->nv) return;
  m_edge e = G(M, x, y);
  int32_t xr = INNER(M, x, e.a);
  int32_t pos = even_position(M, x, xr);
  for (int32_t i = 0; i < pos; ++i) match_through(M, M->child[x][i], M->child[x][i ^ 1]);
  match_through(M, xr, y);
  /* make xr the new base: rotate the cycle left by pos */
  int32_t k = M->nchild[x];
  int32_t* tmp = (int32_t*)malloc(sizeof(int32_t) * (size_t)k);
  for (int32_t i = 0; i < k; ++i) tmp[i] = M->child[x][(i + pos) % k];
  memcpy(M->child[x], tmp, sizeof(int32_t) * (size_t)k);
  free(tmp);
}

static void augment_from(matcher* M, int32_t u, int32_t v) {
  for (;;) {
    int32_t next = M->top[M->mate[u]];
    match_through(M, u, v);
    if (!next) return;
    match_through(M, next, M->top[M->parent[next]]);
    u = M->top[M->parent[next]];
    v = next;
  }
}

static int32_t common_ancestor(matcher* M, int32_t u, int32_t v) {
  ++M->stamp_now;
  while (u || v) {
    if (u == 0) { int32_t t = u; u = v; v = t; continue; }
    if (M->stamp[u] == M->stamp_now) return u;
    M->stamp[u] = M->stamp_now;
    u = M->top[M->mate[u]];
    if (u) u = M->top[M->parent[u]];
    int32_t t = u; u = v; v = t;
  }
  return 0;
}

static void make_blossom(matcher* M, int32_t u, int32_t anc, int32_t v) {
  int32_t b = M->nv + 1;
  while (b <= M->nx && M->top[b]) ++b;
  if (b > M->nx) ++M->nx;
  M->dual[b] = 0; M->label[b] = 0;
  M->mate[b] = M->mate[anc];
  int32_t* cyc = M->child[b];
  int32_t k = 0;
  cyc[k++] = anc;
  int32_t start = k;
  for (int32_t x = u, y; x != anc; x = M->top[M->parent[y]]) {
    cyc[k++] = x; y = M->top[M->mate[x]]; cyc[k++] = y; q_add(M, y);
  }
  for (int32_t i = start, j = k - 1; i < j; ++i, --j) { int32_t t = cyc[i]; cyc[i] = cyc[j]; cyc[j] = t; }
  for (int32_t x = v, y; x != anc; x = M->top[M->parent[y]]) {
    cyc[k++] = x; y = M->top[M->mate[x]]; cyc[k++] = y; q_add(M, y);
  }
  M->nchild[b] = k;
  set_top(M, b, b);
  for (int32_t x = 1; x <= M->nx; ++x) { G(M, b, x).wgt = 0; G(M, x, b).wgt = 0; }
  for (int32_t x = 1; x <= M->nv; ++x) INNER(M, b, x) = 0;
  for (int32_t i = 0; i < k; ++i) {
    int32_t xs = cyc[i];
    for (int32_t x = 1; x <= M->nx; ++x) {
      if (G(M, b, x).wgt == 0 || (G(M, xs, x).wgt > 0 && slack_of(M, G(M, xs, x)) < slack_of(M, G(M, b, x)))) {
        G(M, b, x) = G(M, xs, x); G(M, x, b) = G(M, x, xs);
      }
    }
    for (int32_t x = 1; x <= M->nv; ++x) if (INNER(M, xs, x)) INNER(M, b, x) = xs;
  }
  recompute_best(M, b);
}

static void dissolve_blossom(matcher* M, int32_t b) {
  for (int32_t i = 0; i < M->nchild[b]; ++i) set_top(M, M->child[b][i], M->child[b][i]);
  int32_t xr = INNER(M, b, G(M, b, M->parent[b]).a);
  int32_t pos = even_position(M, b, xr);
  for (int32_t i = 0; i < pos; i += 2) {
    int32_t xs = M->child[b][i], xns = M->child[b][i + 1];
    M->parent[xs] = G(M, xns, xs).a;
    M->label[xs] = 1; M->label[xns] = 0;
    M->best[xs] = 0; recompute_best(M, xns);
    q_add(M, xns);
  }
  M->label[xr] = 1; M->parent[xr] = M->parent[b];
  for (int32_t i = pos + 1; i < M->nchild[b]; ++i) {
    int32_t xs = M->child[b][i];
    M->label[xs] = -1; recompute_best(M, xs);
  }
  M->top[b] = 0;
}

/* An edge became tight; returns 1 if an augmentation happened. */
static int tight_edge(matcher* M, m_edge e) {
  int32_t u = M->top[e.a], v = M->top[e.b];
  if (M->label[v] == -1) {
    M->parent[v] = e.a; M->label[v] = 1;
    int32_t nu = M->top[M->mate[v]];
    M->best[v] = 0; M->best[nu] = 0;
    M->label[nu] = 0; q_add(M, nu);
  } else if (M->label[v] == 0) {
    int32_t anc = common_ancestor(M, u, v);
    if (!anc) { augment_from(M, u, v); augment_from(M, v, u); return 1; }
    make_blossom(M, u, anc, v);
  }
  return 0;
}

/* One stage: grow alternating trees from all exposed nodes until an
 * augmentation (returns 1) or until no augmentation can raise the weight. */
static int stage(matcher* M) {
  for (int32_t x = 1; x <= M->nx; ++x) { M->label[x] = -1; M->best[x] = 0; }
  M->qh = M->qt = 0;
  for (int32_t x = 1; x <= M->nx; ++x)
    if (M->top[x] == x && !M->mate[x]) { M->parent[x] = 0; M->label[x] = 0; q_add(M, x); }
  if (M->qh == M->qt) return 0;
  for (;;) {
    while (M->qh < M->qt) {
      int32_t u = M->queue[M->qh++];
      if (M->label[M->top[u]] == 1) continue;
      for (int32_t v = 1; v <= M->nv; ++v) {
        if (G(M, u, v).wgt > 0 && M->top[u] != M->top[v]) {
          if (slack_of(M, G(M, u, v)) == 0) { if (tight_edge(M, G(M, u, v))) return 1; }
          else consider_best(M, u, M->top[v]);
        }
      }
    }
    i128 delta = I128_INF;
    for (int32_t b = M->nv + 1; b <= M->nx; ++b)
      if (M->top[b] == b && M->label[b] == 1 && M->dual[b] / 2 < delta) delta = M->dual[b] / 2;
    for (int32_t x = 1; x <= M->nx; ++x) {
      if (M->top[x] == x && M->best[x]) {
        i128 s = slack_of(M, G(M, M->best[x], x));
        if (M->label[x] == -1 && s < delta) delta = s;
        else if (M->label[x] == 0 && s / 2 < delta) delta = s / 2;
      }
    }
    /* an S vertex whose dual would reach zero ends the search: the current
     * matching is then of maximum weight; apply the update first so the
     * final duals remain a valid certificate */
    int finished = 0;
    for (int32_t u = 1; u <= M->nv; ++u)
      if (M->label[M->top[u]] == 0 && M->dual[u] <= delta) { delta = M->dual[u]; finished = 1; }
    for (int32_t u = 1; u <= M->nv; ++u) {
      if (M->label[M->top[u]] == 0) M->dual[u] -= delta;
      else if (M->label[M->top[u]] == 1) M->dual[u] += delta;
    }
    for (int32_t b = M->nv + 1; b <= M->nx; ++b) {
      if (M->top[b] == b) {
        if (M->label[b] == 0) M->dual[b] += 2 * delta;
        else if (M->label[b] == 1) M->dual[b] -= 2 * delta;
      }
    }
    if (finished) return 0;
    M->qh = M->qt = 0;
    for (int32_t x = 1; x <= M->nx; ++x) {
      if (M->top[x] == x && M->best[x] && M->top[M->best[x]] != x &&
          slack_of(M, G(M, M->best[x], x)) == 0) {
        if (tight_edge(M, G(M, M->best[x], x))) return 1;
      }
    }
    for (int32_t b = M->nv + 1; b <= M->nx; ++b)
      if (M->top[b] == b && M->label[b] == 1 && M->dual[b] == 0) dissolve_blossom(M, b);
  }
}

static matcher* matcher_new(int32_t nv) {
  matcher* M = (matcher*)calloc(1, sizeof(matcher));
  M->nv = nv; M->nx = nv; M->cap = 2 * nv + 1;
  size_t c = (size_t)M->cap;
  M->g = (m_edge*)calloc(c * c, sizeof(m_edge));
  M->dual = (i128*)calloc(c, sizeof(i128));
  M->mate = (int32_t*)calloc(c, sizeof(int32_t));
  M->best = (int32_t*)calloc(c, sizeof(int32_t));
  M->top = (int32_t*)calloc(c, sizeof(int32_t));
  M->parent = (int32_t*)calloc(c, sizeof(int32_t));
  M->label = (int32_t*)calloc(c, sizeof(int32_t));
  M->stamp = (int32_t*)calloc(c, sizeof(int32_t));
  M->child = (int32_t**)calloc(c, sizeof(int32_t*));
  for (size_t i = 0; i < c; ++i) M->child[i] = (int32_t*)calloc(c, sizeof(int32_t));
  M->nchild = (int32_t*)calloc(c, sizeof(int32_t));
  M->inner_of = (int32_t*)calloc(c * ((size_t)nv + 1), sizeof(int32_t));
  M->queue = (int32_t*)calloc(c * 8 + 8, sizeof(int32_t));
  for (int32_t u = 1; u <= nv; ++u)
    for (int32_t v = 1; v <= nv; ++v) { G(M, u, v).a = u; G(M, u, v).b = v; G(M, u, v).wgt = 0; }
  return M;
}

static void matcher_free(matcher* M) {
  size_t c = (size_t)M->cap;
  free(M->g); free(M->dual); free(M->mate); free(M->best); free(M->top); free(M->parent);
  free(M->label); free(M->stamp);
  for (size_t i = 0; i < c; ++i) free(M->child[i]);
  free(M->child); free(M->nchild); free(M->inner_of); free(M->queue); free(M);
}

static void matcher_solve(matcher* M) {
  i128 wmax = 0;
  for (int32_t u = 1; u <= M->nv; ++u) {
    M->top[u] = u; M->mate[u] = 0;
    for (int32_t v = 1; v <= M->nv; ++v) {
      INNER(M, u, v) = (u == v) ? u : 0;
      if (G(M, u, v).wgt > wmax) wmax = G(M, u, v).wgt;
    }
  }
  for (int32_t u = 1; u <= M->nv; ++u) M->dual[u] = wmax;
  while (stage(M)) {}
}

/* Collect the vertex set of blossom b into out (returns count). */
static int32_t blossom_vertices(const matcher* M, int32_t b, int32_t* out) {
  if (b <= M->nv) { out[0] = b; return 1; }
  int32_t k = 0;
  for (int32_t i = 0; i < M->nchild[b]; ++i) k += blossom_vertices(M, M->child[b][i], out + k);
  return k;
}

/* LP certificate for the maximum-weight matching (doubled weights):
 * dual[v] >= 0, dual[b] >= 0 for live blossoms, reduced cost
 * dual[u] + dual[v] + sum_{live b containing u and v} dual[b] - 2 w(u,v) >= 0
 * on every edge, == 0 on matched edges, exposed vertices have dual 0, and
 * primal 2*sum w(matched) == sum dual[v] + sum dual[b] * (|b| - 1) / 2.
 * Returns 1 if the certificate holds. */
static int matcher_certificate(const matcher* M, const i128* W /* [nv+1][nv+1] */) {
  const int32_t nv = M->nv;
  const size_t stride = (size_t)nv + 1;
  i128* cover = (i128*)calloc(stride * stride, sizeof(i128));
  int32_t* verts = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nv + 1));
  i128 dual_obj = 0;
  for (int32_t v = 1; v <= nv; ++v) {
    if (M->dual[v] < 0) goto fail;
    dual_obj += M->dual[v];
  }
  for (int32_t b = nv + 1; b <= M->nx; ++b) {
    if (!M->top[b]) continue;            /* dissolved */
    if (M->dual[b] < 0) goto fail;
    int32_t k = blossom_vertices(M, b, verts);
    if (k % 2 == 0) goto fail;
    dual_obj += M->dual[b] * (i128)((k - 1) / 2);
    for (int32_t i = 0; i < k; ++i)
      for (int32_t j = 0; j < k; ++j) cover[(size_t)verts[i] * stride + (size_t)verts[j]] += M->dual[b];
  }
  i128 primal = 0;
  for (int32_t u = 1; u <= nv; ++u) {
    if (!M->mate[u] && M->dual[u] != 0) goto fail;
    for (int32_t v = u + 1; v <= nv; ++v) {
      i128 w = W[(size_t)u * stride + (size_t)v];
      if (w <= 0) continue;
      i128 rc = M->dual[u] + M->dual[v] + cover[(size_t)u * stride + (size_t)v] - 2 * w;
      if (rc < 0) goto fail;
      if (M->mate[u] == v) {
        if (rc != 0) goto fail;
        primal += 2 * w;
      }
    }
  }
  if (primal != dual_obj) goto fail;
  free(cover); free(verts);
  return 1;
fail:
  free(cover); free(verts);
  return 0;
}

/* Exported for tests: maximum-weight matching of a small explicit graph.
 * w is a dense (nv x nv) row-major matrix of non-negative weights (0 = no
 * edge), given as hi/lo halves.  mate_out[i] = matched vertex (0-based) or -1.
 * Returns 1 if the LP certificate holds, 0 if not. */
int oracle_max_weight_matching(int32_t nv, const int64_t* w_hi, const uint64_t* w_lo, int32_t* mate_out) {
  matcher* M = matcher_new(nv);
  const size_t stride = (size_t)nv + 1;
  i128* W = (i128*)calloc(stride * stride, sizeof(i128));
  for (int32_t i = 0; i < nv; ++i)
    for (int32_t j = 0; j < nv; ++j) {
      i128 x = ((i128)w_hi[(size_t)i * nv + j] << 64) | (i128)w_lo[(size_t)i * nv + j];
      W[(size_t)(i + 1) * stride + (size_t)(j + 1)] = x;
      G(M, i + 1, j + 1).wgt = x;
    }
  matcher_solve(M);
  int ok = matcher_certificate(M, W);
  for (int32_t i = 0; i < nv; ++i) mate_out[i] = M->mate[i + 1] ? M->mate[i + 1] - 1 : -1;
  free(W); matcher_free(M);
  return ok;
}

/* ------------------------------------------------------------------ */
/* MWEM                                                                 */
/* ------------------------------------------------------------------ */
static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* Append the shortest path from the tree's source to node t (edge ids). */
static int64_t path_to(const og_graph* g, const sp_tree* t, int32_t node, int32_t* buf, int64_t n) {
  while (t->pred[node] >= 0) {
    int64_t e = t->pred[node];
    buf[n++] = (int32_t)e;
    node = g->eu[e] == node ? g->ev[e] : g->eu[e];
  }
  return n;
}

/* Decodes one shot.  out_edges receives the MWEM edge ids in ascending
 * order (capacity out_cap).  Returns flags (OF_*); weight/obs are written
 * unless OF_INFEASIBLE. */
int oracle_mwem(void* pg, int32_t nd, const int32_t* defects, int32_t* out_edges, int64_t out_cap,
                int64_t* out_n, int64_t* out_weight, uint64_t* out_obs) {
  og_graph* g = (og_graph*)pg;
  int flags = 0;
  *out_n = 0; *out_weight = 0; *out_obs = 0;
  if (nd == 0) return 0;
  sp_tree* trees = (sp_tree*)malloc(sizeof(sp_tree) * (size_t)nd);
  for (int32_t i = 0; i < nd; ++i) { sp_alloc(&trees[i], g->n); dijkstra(g, defects[i], &trees[i]); }

  /* defect graph: vertex i+1 = defect i, vertex nd+i+1 = its boundary copy */
  const int32_t nv = 2 * nd;
  const size_t stride = (size_t)nv + 1;
  i128 cmax = 0;
  for (int32_t i = 0; i < nd; ++i) {
    if (trees[i].bd_dist < I128_INF && trees[i].bd_dist > cmax) cmax = trees[i].bd_dist;
    for (int32_t j = 0; j < nd; ++j)
      if (trees[i].dist[defects[j]] < I128_INF && trees[i].dist[defects[j]] > cmax) cmax = trees[i].dist[defects[j]];
  }
  const i128 K = (cmax + 1) * (i128)(nd + 1);   /* > cost of any perfect matching */
  matcher* M = matcher_new(nv);
  i128* W = (i128*)calloc(stride * stride, sizeof(i128));
#define SETW(a, b, x) do { W[(size_t)(a) * stride + (size_t)(b)] = (x); W[(size_t)(b) * stride + (size_t)(a)] = (x); \
                           G(M, a, b).wgt = (x); G(M, b, a).wgt = (x); } while (0)
  for (int32_t i = 0; i < nd; ++i) {
    for (int32_t j = i + 1; j < nd; ++j) {
      i128 c = trees[i].dist[defects[j]];
      if (c < I128_INF) SETW(i + 1, j + 1, K - c);
      SETW(nd + i + 1, nd + j + 1, K);
    }
    if (trees[i].bd_edge >= 0) SETW(i + 1, nd + i + 1, K - trees[i].bd_dist);
  }
#undef SETW
  matcher_solve(M);
  if (!matcher_certificate(M, W)) flags |= OF_CERT_FAIL;
  for (int32_t x = 1; x <= nv; ++x) if (!M->mate[x]) flags |= OF_INFEASIBLE;

  if (!(flags & OF_INFEASIBLE)) {
    /* collect paths of matched pairs, then cancel repeated edges */
    int64_t cap = 1024, n = 0;
    int32_t* buf = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
    for (int32_t i = 0; i < nd; ++i) {
      int32_t m = M->mate[i + 1];
      int32_t need = g->n + 1;
      if (n + need > cap) { while (n + need > cap) cap *= 2; buf = (int32_t*)realloc(buf, sizeof(int32_t) * (size_t)cap); }
      if (m == nd + i + 1) {                 /* matched to the boundary */
        int64_t e = trees[i].bd_edge;
        buf[n++] = (int32_t)e;
        int32_t u = g->eu[e] >= 0 && g->ev[e] == -1 ? g->eu[e] : g->ev[e];
        if (trees[i].tie[u] || trees[i].bd_tie) flags |= OF_TIE;
        n = path_to(g, &trees[i], u, buf, n);
      } else if (m >= 1 && m <= nd && m - 1 > i) {
        int32_t j = m - 1;
        if (trees[i].tie[defects[j]]) flags |= OF_TIE;
        n = path_to(g, &trees[i], defects[j], buf, n);
      }
    }
    qsort(buf, (size_t)n, sizeof(int32_t), cmp_i32);
    int64_t k = 0;
    for (int64_t a = 0; a < n;) {
      int64_t b = a;
      while (b < n && buf[b] == buf[a]) ++b;
      if ((b - a) % 2 == 1) {
        if (k < out_cap) out_edges[k] = buf[a];
        else flags |= OF_CAPACITY;
        ++k;
        *out_weight += g->w[buf[a]];
        *out_obs ^= g->obs[buf[a]];
      }
      a = b;
    }
    *out_n = k;
    free(buf);
  }
  free(W); matcher_free(M);
  for (int32_t i = 0; i < nd; ++i) sp_free(&trees[i]);
  free(trees);
  return flags;
}

/* Pairwise tie-broken distances between defects and defect->boundary
 * distances (hi/lo halves); infinity is reported as hi = INT64_MAX. */
int oracle_defect_distances(void* pg, int32_t nd, const int32_t* defects, int64_t* d_hi, uint64_t* d_lo,
                            int64_t* bd_hi, uint64_t* bd_lo) {
  og_graph* g = (og_graph*)pg;
  sp_tree t; sp_alloc(&t, g->n);
  for (int32_t i = 0; i < nd; ++i) {
    dijkstra(g, defects[i], &t);
    for (int32_t j = 0; j < nd; ++j) {
      i128 x = t.dist[defects[j]];
      if (x >= I128_INF) { d_hi[(size_t)i * nd + j] = INT64_MAX; d_lo[(size_t)i * nd + j] = 0; }
      else { d_hi[(size_t)i * nd + j] = (int64_t)(x >> 64); d_lo[(size_t)i * nd + j] = (uint64_t)x; }
    }
    if (t.bd_dist >= I128_INF) { bd_hi[i] = INT64_MAX; bd_lo[i] = 0; }
    else { bd_hi[i] = (int64_t)(t.bd_dist >> 64); bd_lo[i] = (uint64_t)t.bd_dist; }
  }
  sp_free(&t);
  return 0;
}

/* All-pairs-to-boundary-vertices distances for the clustering oracle:
 * out[i * nb + k] = distance from defect i to the boundary vertex of the k-th
 * boundary edge (edge ids in bedges). */
int oracle_defect_boundary_table(void* pg, int32_t nd, const int32_t* defects, int32_t nb, const int64_t* bedges,
                                 int64_t* d_hi, uint64_t* d_lo) {
  og_graph* g = (og_graph*)pg;
  sp_tree t; sp_alloc(&t, g->n);
  for (int32_t i = 0; i < nd; ++i) {
    dijkstra(g, defects[i], &t);
    for (int32_t k = 0; k < nb; ++k) {
      int64_t e = bedges[k];
      int32_t u = g->ev[e] == -1 ? g->eu[e] : g->ev[e];
      i128 x = t.dist[u] < I128_INF ? t.dist[u] + g->wt[e] : I128_INF;
      if (x >= I128_INF) { d_hi[(size_t)i * nb + k] = INT64_MAX; d_lo[(size_t)i * nb + k] = 0; }
      else { d_hi[(size_t)i * nb + k] = (int64_t)(x >> 64); d_lo[(size_t)i * nb + k] = (uint64_t)x; }
    }
  }
  sp_free(&t);
  return 0;
}

/* Exported so tests can compare the tie-break against an independent
 * reimplementation of the published SplitMix64 definition. */
void oracle_tiebroken_weights(void* pg, int64_t* hi, uint64_t* lo) {
  og_graph* g = (og_graph*)pg;
  for (int64_t e = 0; e < g->m; ++e) { hi[e] = (int64_t)(g->wt[e] >> 64); lo[e] = (uint64_t)g->wt[e]; }
}
