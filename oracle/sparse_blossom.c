/* ORACLE -- test infrastructure only.  Only tests/, __graft_entry__.smoke()
 * and bench.py's cpu_baseline leg may load this file's library.  It shares no
 * code with the GPU decoder, and none with mwem.c either (the MWEM reference
 * it is checked against): it has its own graph, its own searches and its own
 * matcher.
 *
 * Serial global sparse blossom and serial partition-and-fuse, written plainly
 * from the paper:
 *
 *   - Sparse blossom (Supplementary S1).  Every detection event owns a
 *     graph-fill region; a region has a radius y (its dual variable) that
 *     changes at rate +1 (growing, outer), 0 (frozen) or -1 (shrinking,
 *     inner).  The flooder produces the events ARRIVE (a growing region enters
 *     an empty detector), LEAVE (a shrinking region leaves a detector),
 *     COLLIDE (a growing region meets another region or the boundary) and
 *     IMPLODE (a shrinking region reaches radius zero); the matcher turns
 *     collisions and implosions into the events (a) tree hits match,
 *     (b) tree hits tree, (c) tree hits itself, (d) blossom shatters,
 *     (e) node shrinks to zero, (f) tree hits boundary and (g) tree hits
 *     boundary match.  Weights are the tie-broken even integers of the
 *     decoding task (below), so the dual step is 1 and every event happens at
 *     an integer time.
 *   - Algorithm "Clustering" (Methods): around every residual detection event
 *     an exploring region of radius b_k/2; two such regions touch when their
 *     events are at most b_k apart; a component of touching regions is a
 *     level-k processing cluster when the diameter of its event set is at most
 *     d_k and it has an even number of events or satisfies the boundary
 *     condition.
 *   - The hierarchical execution rule and Algorithm "Parallel sparse blossom"
 *     (Methods), run sequentially as in the paper's own simulator (Methods,
 *     numerical evaluation): level by level, the detection events of that
 *     level start growing at time 0 while every stopped lower-level matching
 *     configuration stays in place, frozen; a configuration that a running
 *     tree touches is continued by that tree's dynamics and belongs to it from
 *     then on.
 *   - The parallel event count E_ideal (Methods, numerical evaluation): every
 *     event is charged to the processing cluster whose alternating tree drives
 *     it; per level, t(C) = max(t_<k, s(C)) and
 *     E(C) = max(E_<k, E_C(t_<k)) + E_C(t(C)) - E_C(t_<k).
 *
 * Deliberately plain and slow: the next event is found by scanning every
 * region and every incident edge of every reached detector; a detector's local
 * radius is computed from its chain of enclosing regions; each compressed edge
 * stores the list of graph edges of its path, and the output edge set is the
 * symmetric difference of the paths of the final matching.
 *
 * Readings (where the paper is silent):
 *   - Tie-broken weights wt(e) = 2 w(e) 2^64 + 2 h(e), h(e) the (e+1)-th
 *     SplitMix64 output of the tie-break seed shifted right by 24.
 *   - A boundary vertex per boundary edge; no path passes through one.
 *   - Events at the same time are taken in the order: region events (IMPLODE,
 *     shatter) before LEAVE before edge events, each kind by the smaller
 *     region, detector or edge id.  When a blossom shatters, detectors still
 *     in its own shell (radius zero there) are released by the shatter itself.
 *   - Each level restarts the clock at 0; frozen regions keep their radii.
 *   - An event is charged to the tree of the growing (or shrinking) region
 *     that causes it: for a collision of a growing region with a frozen one,
 *     the growing region's tree.  A cluster's stopping time s(C) is its last
 *     event's time.
 *   - Clusters are identified by their smallest detection-event index.
 *   - Parity condition, "strict": one boundary vertex within d_k of every
 *     member; "loose": some member within b_k/2 of a boundary vertex.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;
#define SB_INF (((i128)1) << 124)

enum {
  SBF_INFEASIBLE = 1,    /* an alternating tree could not be resolved */
  SBF_INTERNAL = 2,      /* a state the dynamics must never reach */
  SBF_DUAL = 4,          /* sum of the final radii differs from the matching's weight */
  SBF_UNCLUSTERED = 8,   /* some event was not accepted within the given levels */
  SBF_REACHED_LATER = 16,/* a region reached the detector of a later level's event */
  SBF_CROSS_CLUSTER = 32 /* two trees of different processing clusters collided */
};

/* ------------------------------------------------------------------ */
/* graph                                                                */
/* ------------------------------------------------------------------ */
static uint64_t sm64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + k * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

typedef struct {
  int32_t n;
  int64_t m;
  int32_t *eu, *ev, *w;
  uint64_t* obs;
  i128* wt;
  int64_t *off, *adj;      /* incident edges of each detector */
  int32_t* comp;           /* connected component of each detector */
  i128* comp_bound;        /* per component: upper bound on any distance inside it */
  uint8_t* comp_bd;        /* per component: has a boundary edge */
} sb_graph;

typedef struct { i128 key; int32_t node; } hitem;
static void hpush(hitem* h, int64_t* sz, i128 k, int32_t x) {
  int64_t i = (*sz)++;
  h[i].key = k; h[i].node = x;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (h[p].key < h[i].key || (h[p].key == h[i].key && h[p].node <= h[i].node)) break;
    hitem t = h[p]; h[p] = h[i]; h[i] = t; i = p;
  }
}
static hitem hpop(hitem* h, int64_t* sz) {
  hitem top = h[0];
  h[0] = h[--(*sz)];
  int64_t i = 0;
  for (;;) {
    int64_t l = 2 * i + 1, r = l + 1, s = i;
    if (l < *sz && (h[l].key < h[s].key || (h[l].key == h[s].key && h[l].node < h[s].node))) s = l;
    if (r < *sz && (h[r].key < h[s].key || (h[r].key == h[s].key && h[r].node < h[s].node))) s = r;
    if (s == i) break;
    hitem t = h[s]; h[s] = h[i]; h[i] = t; i = s;
  }
  return top;
}

static int32_t other_end(const sb_graph* g, int64_t e, int32_t x) { return g->eu[e] == x ? g->ev[e] : g->eu[e]; }

/* Dijkstra from detector s, every detector settled (boundary vertices are
 * sinks); returns the largest distance to a detector of s's component. */
static i128 eccentricity(const sb_graph* g, int32_t s) {
  i128* dist = (i128*)malloc(sizeof(i128) * (size_t)g->n);
  for (int32_t i = 0; i < g->n; ++i) dist[i] = SB_INF;
  hitem* h = (hitem*)malloc(sizeof(hitem) * (size_t)(g->off[g->n] + 2));
  int64_t sz = 0;
  dist[s] = 0; hpush(h, &sz, 0, s);
  i128 ecc = 0;
  while (sz > 0) {
    hitem it = hpop(h, &sz);
    if (it.key != dist[it.node]) continue;
    if (it.key > ecc) ecc = it.key;
    for (int64_t k = g->off[it.node]; k < g->off[it.node + 1]; ++k) {
      const int64_t e = g->adj[k];
      const int32_t y = other_end(g, e, it.node);
      if (y < 0) continue;
      const i128 nd = it.key + g->wt[e];
      if (nd < dist[y]) { dist[y] = nd; hpush(h, &sz, nd, y); }
    }
  }
  free(dist); free(h);
  return ecc;
}

void* oracle_sb_graph_create(int32_t n, int64_t m, const int32_t* eu, const int32_t* ev, const int32_t* w,
                             const uint64_t* obs, uint64_t seed) {
  if (n <= 0 || m < 0) return NULL;
  for (int64_t e = 0; e < m; ++e)
    if (eu[e] < 0 || eu[e] >= n || ev[e] < -1 || ev[e] >= n || eu[e] == ev[e] || w[e] <= 0) return NULL;
  sb_graph* g = (sb_graph*)calloc(1, sizeof(sb_graph));
  const size_t mm = (size_t)(m ? m : 1);
  g->n = n; g->m = m;
  g->eu = (int32_t*)malloc(4 * mm); g->ev = (int32_t*)malloc(4 * mm); g->w = (int32_t*)malloc(4 * mm);
  g->obs = (uint64_t*)malloc(8 * mm); g->wt = (i128*)malloc(16 * mm);
  memcpy(g->eu, eu, 4 * (size_t)m); memcpy(g->ev, ev, 4 * (size_t)m); memcpy(g->w, w, 4 * (size_t)m);
  memcpy(g->obs, obs, 8 * (size_t)m);
  i128 wmax = 0;
  for (int64_t e = 0; e < m; ++e) {
    g->wt[e] = ((i128)(2 * (int64_t)w[e]) << 64) + (i128)(2 * (sm64(seed, (uint64_t)e + 1) >> 24));
    if (g->wt[e] > wmax) wmax = g->wt[e];
  }
  g->off = (int64_t*)calloc((size_t)n + 1, 8);
  for (int64_t e = 0; e < m; ++e) { g->off[eu[e] + 1]++; if (ev[e] >= 0) g->off[ev[e] + 1]++; }
  for (int32_t i = 0; i < n; ++i) g->off[i + 1] += g->off[i];
  g->adj = (int64_t*)malloc(8 * (size_t)(g->off[n] + 1));
  int64_t* fill = (int64_t*)malloc(8 * (size_t)n);
  for (int32_t i = 0; i < n; ++i) fill[i] = g->off[i];
  for (int64_t e = 0; e < m; ++e) { g->adj[fill[eu[e]]++] = e; if (ev[e] >= 0) g->adj[fill[ev[e]]++] = e; }
  free(fill);
  /* connected components (plain flood fill) and, per component, a bound on
   * every distance inside it: any two vertices (boundary vertices included)
   * are within ecc(x0) + (ecc(x0) + w_max) of each other through x0 */
  g->comp = (int32_t*)malloc(4 * (size_t)n);
  for (int32_t i = 0; i < n; ++i) g->comp[i] = -1;
  int32_t* stack = (int32_t*)malloc(4 * (size_t)n);
  int32_t nc = 0;
  g->comp_bound = (i128*)malloc(16 * (size_t)n);
  g->comp_bd = (uint8_t*)calloc((size_t)n, 1);
  for (int32_t s = 0; s < n; ++s) {
    if (g->comp[s] >= 0) continue;
    int32_t sp = 0;
    stack[sp++] = s; g->comp[s] = nc;
    while (sp > 0) {
      const int32_t x = stack[--sp];
      for (int64_t k = g->off[x]; k < g->off[x + 1]; ++k) {
        const int32_t y = other_end(g, g->adj[k], x);
        if (y >= 0 && g->comp[y] < 0) { g->comp[y] = nc; stack[sp++] = y; }
      }
    }
    g->comp_bound[nc] = 2 * (eccentricity(g, s) + wmax);
    ++nc;
  }
  free(stack);
  for (int64_t e = 0; e < m; ++e) if (ev[e] < 0) g->comp_bd[g->comp[eu[e]]] = 1;
  return g;
}

void oracle_sb_graph_destroy(void* p) {
  sb_graph* g = (sb_graph*)p;
  if (!g) return;
  free(g->eu); free(g->ev); free(g->w); free(g->obs); free(g->wt); free(g->off); free(g->adj);
  free(g->comp); free(g->comp_bound); free(g->comp_bd); free(g);
}

/* ------------------------------------------------------------------ */
/* per-shot state                                                       */
/* ------------------------------------------------------------------ */
typedef struct { int32_t sa, sb; int64_t off, len; } cedge;   /* ends (detection events; -1 boundary), path */

typedef struct {
  i128 base; int32_t rate;   /* y(t) = base + rate * t */
  int32_t alive;
  int32_t bpar;              /* blossom parent, -1 for an active region */
  int32_t cyc_off, cyc_len;  /* blossom cycle: (child, compressed edge to the next child) pairs */
  int32_t root;              /* detection event at the root of its alternating tree, -1 if none */
  int32_t tpar, tpe;         /* tree parent and the compressed edge to it */
  int32_t mate, me;          /* matched region (-2 boundary, -1 none) and the compressed edge */
} region;

#define MATE_BD (-2)

typedef struct {
  const sb_graph* g;
  int32_t nd;
  const int32_t* det;        /* detector of each detection event */
  int32_t* dix;              /* [n] detection-event index of a detector, -1 */
  int8_t* level;             /* [nd] processing-cluster level (1-based) */
  int32_t* cid;              /* [nd] processing cluster (its smallest event index) */
  /* detectors */
  int32_t* reg;              /* region in whose own shell the detector lies, -1 empty */
  i128* arr;                 /* that region's radius when the detector was entered */
  int32_t* src;              /* detection event the fill traces back to */
  int64_t* pe;               /* edge the fill entered through, -1 at a detection event */
  int32_t* pn;               /* detector it came from */
  uint8_t* seen;
  int32_t* reached; int64_t nreached;
  /* regions (0..nd-1: detector regions of the detection events) */
  region* R; int64_t nR, capR;
  cedge* CE; int64_t nCE, capCE;
  int32_t* path; int64_t npath, cappath;
  int32_t* cyc; int64_t ncyc, capcyc;
  i128* ysum; int32_t* top; int64_t capscan;
  i128 now;
  int flags;
  int64_t n_events, n_arrive, max_events;
  int64_t n_tied;            /* events applied while another, different event was due at the same time */
  /* parallel event count */
  int64_t *c_n, *c_early;
  i128* c_last;
  i128 t_lt;
  int64_t e_lt;
} shot;

#define GROW(p, cap, need)                                                    \
  do {                                                                        \
    if ((int64_t)(need) > (cap)) {                                            \
      int64_t nc_ = (cap) ? (cap) : 64;                                       \
      while (nc_ < (int64_t)(need)) nc_ *= 2;                                 \
      (p) = realloc((p), sizeof(*(p)) * (size_t)nc_);                         \
      (cap) = nc_;                                                            \
    }                                                                         \
  } while (0)

static i128 yr(const shot* S, int32_t r, i128 t) {
  const region* x = &S->R[r];
  return x->base + (x->rate > 0 ? t : (x->rate < 0 ? -t : (i128)0));
}

static void set_rate(shot* S, int32_t r, int32_t rate) {
  const i128 y = yr(S, r, S->now);
  S->R[r].rate = rate;
  S->R[r].base = y - (rate > 0 ? S->now : (rate < 0 ? -S->now : (i128)0));
}

static int32_t new_region(shot* S) {
  GROW(S->R, S->capR, S->nR + 1);
  region* x = &S->R[S->nR];
  memset(x, 0, sizeof(*x));
  x->alive = 1; x->bpar = -1; x->root = -1; x->tpar = -1; x->tpe = -1; x->mate = -1; x->me = -1;
  return (int32_t)S->nR++;
}

static void touch(shot* S, int32_t v) {
  if (!S->seen[v]) { S->seen[v] = 1; S->reached[S->nreached++] = v; }
}

/* Is detection event s inside region r (r or one of its blossom descendants)? */
static int inside(const shot* S, int32_t s, int32_t r) {
  int32_t x = s;
  int guard = 0;
  while (x >= 0 && guard++ < 1 << 24) { if (x == r) return 1; x = S->R[x].bpar; }
  return 0;
}

/* child of blossom b that contains detection event s */
static int32_t child_with(const shot* S, int32_t b, int32_t s) {
  int32_t x = s;
  int guard = 0;
  while (x >= 0 && S->R[x].bpar != b && guard++ < 1 << 24) x = S->R[x].bpar;
  return x;
}

/* the path of detector v back to its detection event, appended to the pool */
static void append_fill_path(shot* S, int32_t v) {
  int64_t guard = 0;
  while (v >= 0 && S->pe[v] >= 0) {
    GROW(S->path, S->cappath, S->npath + 1);
    S->path[S->npath++] = (int32_t)S->pe[v];
    v = S->pn[v];
    if (++guard > S->g->n) { S->flags |= SBF_INTERNAL; return; }
  }
}

/* compressed edge from a collision through graph edge e between detectors u and x (x < 0: boundary) */
static int32_t ce_collision(shot* S, int32_t u, int32_t x, int64_t e) {
  GROW(S->CE, S->capCE, S->nCE + 1);
  cedge* c = &S->CE[S->nCE];
  c->sa = S->src[u]; c->sb = x >= 0 ? S->src[x] : -1;
  c->off = S->npath;
  append_fill_path(S, u);
  GROW(S->path, S->cappath, S->npath + 1);
  S->path[S->npath++] = (int32_t)e;
  if (x >= 0) append_fill_path(S, x);
  c->len = S->npath - c->off;
  return (int32_t)S->nCE++;
}

/* compressed edge joining the far ends of two compressed edges that meet at detection event s */
static int32_t ce_join(shot* S, int32_t a, int32_t b, int32_t s) {
  GROW(S->CE, S->capCE, S->nCE + 1);
  GROW(S->path, S->cappath, S->npath + S->CE[a].len + S->CE[b].len);
  cedge* c = &S->CE[S->nCE];
  c->sa = S->CE[a].sa == s ? S->CE[a].sb : S->CE[a].sa;
  c->sb = S->CE[b].sa == s ? S->CE[b].sb : S->CE[b].sa;
  c->off = S->npath;
  memcpy(S->path + S->npath, S->path + S->CE[a].off, 4 * (size_t)S->CE[a].len); S->npath += S->CE[a].len;
  memcpy(S->path + S->npath, S->path + S->CE[b].off, 4 * (size_t)S->CE[b].len); S->npath += S->CE[b].len;
  c->len = S->npath - c->off;
  return (int32_t)S->nCE++;
}

/* end of compressed edge c that lies inside region r */
static int32_t end_inside(const shot* S, int32_t c, int32_t r) {
  return (S->CE[c].sa >= 0 && inside(S, S->CE[c].sa, r)) ? S->CE[c].sa : S->CE[c].sb;
}

/* ------------------------------------------------------------------ */
/* matcher (Supplementary S1: GROW, AUGMENT, SHRINK, EXPAND)            */
/* ------------------------------------------------------------------ */

/* AUGMENT: along the tree path from outer region a to its root, every inner
 * region is re-matched to its tree parent. */
static void augment_to_root(shot* S, int32_t a) {
  int32_t cur = a;
  int guard = 0;
  while (S->R[cur].tpar >= 0) {
    const int32_t in = S->R[cur].tpar, out = S->R[in].tpar;
    if (out < 0 || ++guard > S->nR) { S->flags |= SBF_INTERNAL; return; }
    S->R[in].mate = out; S->R[in].me = S->R[in].tpe;
    S->R[out].mate = in; S->R[out].me = S->R[in].tpe;
    cur = out;
  }
}

/* every region of the tree rooted at `root` leaves it and freezes */
static void dissolve_tree(shot* S, int32_t root) {
  for (int64_t r = 0; r < S->nR; ++r) {
    if (!S->R[r].alive || S->R[r].bpar >= 0 || S->R[r].root != root) continue;
    S->R[r].root = -1; S->R[r].tpar = -1; S->R[r].tpe = -1;
    set_rate(S, (int32_t)r, 0);
  }
}

/* SHRINK: outer regions a and b of one tree are joined by compressed edge c;
 * the odd cycle through their lowest common outer ancestor becomes a blossom. */
static void form_blossom(shot* S, int32_t a, int32_t b, int32_t c) {
  /* outer ancestors of a: a, grandparent(a), ... */
  int32_t* anc = (int32_t*)malloc(sizeof(int32_t) * (size_t)(S->nR + 1));
  int32_t na = 0;
  for (int32_t x = a;;) {
    anc[na++] = x;
    if (S->R[x].tpar < 0) break;
    x = S->R[S->R[x].tpar].tpar;
    if (x < 0 || na > S->nR) { S->flags |= SBF_INTERNAL; free(anc); return; }
  }
  int32_t lca = -1, nb = 0;
  int32_t* pb = (int32_t*)malloc(sizeof(int32_t) * (size_t)(S->nR + 1));   /* path b -> lca, lca excluded */
  for (int32_t y = b;;) {
    int found = 0;
    for (int32_t i = 0; i < na; ++i) if (anc[i] == y) found = 1;
    if (found) { lca = y; break; }
    pb[nb++] = y;
    const int32_t in = S->R[y].tpar;
    if (in < 0 || S->R[in].tpar < 0 || nb > S->nR) { S->flags |= SBF_INTERNAL; free(anc); free(pb); return; }
    pb[nb++] = in;
    y = S->R[in].tpar;
  }
  int32_t npa = 0;                       /* path a -> lca, lca excluded, with the inner regions */
  int32_t* pa = (int32_t*)malloc(sizeof(int32_t) * (size_t)(S->nR + 1));
  for (int32_t x = a; x != lca;) {
    pa[npa++] = x;
    const int32_t in = S->R[x].tpar;
    pa[npa++] = in;
    x = S->R[in].tpar;
  }
  /* cycle: lca, then down to a, then across c to b, then up to lca */
  const int32_t m = 1 + npa + nb;
  GROW(S->cyc, S->capcyc, S->ncyc + 2 * m);
  int32_t* cy = S->cyc + S->ncyc;
  int32_t k = 0;
  cy[2 * k++] = lca;
  for (int32_t i = npa - 1; i >= 0; --i) cy[2 * k++] = pa[i];
  for (int32_t i = 0; i < nb; ++i) cy[2 * k++] = pb[i];
  for (int32_t i = 0; i < m; ++i) {
    const int32_t x = cy[2 * i], y = cy[2 * ((i + 1) % m)];
    int32_t e;
    if (i < npa) e = S->R[y].tpe;          /* downwards: the child's tree edge */
    else if (i == npa) e = c;              /* a -> b */
    else e = S->R[x].tpe;                  /* upwards: the child's tree edge */
    cy[2 * i + 1] = e;
  }
  const int64_t off = S->ncyc;
  S->ncyc += 2 * m;
  const int32_t X = new_region(S);
  region* B = &S->R[X];
  B->base = -S->now; B->rate = 1;         /* y_X(now) = 0, growing */
  B->cyc_off = (int32_t)off; B->cyc_len = m;
  B->root = S->R[lca].root;
  B->tpar = S->R[lca].tpar; B->tpe = S->R[lca].tpe;
  B->mate = S->R[lca].mate; B->me = S->R[lca].me;
  if (B->tpar >= 0) S->R[B->tpar].mate = X;
  /* tree children of cycle members that are not on the cycle now hang from X */
  for (int64_t r = 0; r < S->nR; ++r) {
    if (r == X || !S->R[r].alive || S->R[r].bpar >= 0 || S->R[r].tpar < 0) continue;
    int on = 0, par_on = 0;
    for (int32_t i = 0; i < m; ++i) { on |= (cy[2 * i] == r); par_on |= (cy[2 * i] == S->R[r].tpar); }
    if (!on && par_on) S->R[r].tpar = X;
  }
  for (int32_t i = 0; i < m; ++i) {
    const int32_t ch = cy[2 * i];
    set_rate(S, ch, 0);
    S->R[ch].bpar = X; S->R[ch].root = -1; S->R[ch].tpar = -1; S->R[ch].tpe = -1;
    S->R[ch].mate = -1; S->R[ch].me = -1;
  }
  free(anc); free(pa); free(pb);
}

/* EXPAND ((d) blossom shatters): inner blossom B has reached radius zero. */
static void shatter(shot* S, int32_t B) {
  const region Bv = S->R[B];
  const int32_t m = Bv.cyc_len;
  const int32_t* cy = S->cyc + Bv.cyc_off;
  const int32_t P = Bv.tpar, C = Bv.mate;
  if (P < 0 || C < 0) { S->flags |= SBF_INTERNAL; return; }
  const int32_t c_in = child_with(S, B, end_inside(S, Bv.tpe, B));
  const int32_t c_out = child_with(S, B, end_inside(S, Bv.me, B));
  int32_t i_in = -1, i_out = -1;
  for (int32_t i = 0; i < m; ++i) { if (cy[2 * i] == c_in) i_in = i; if (cy[2 * i] == c_out) i_out = i; }
  if (i_in < 0 || i_out < 0) { S->flags |= SBF_INTERNAL; return; }
  const int32_t fwd = ((i_out - i_in) % m + m) % m;
  const int32_t dir = (fwd % 2 == 0) ? 1 : -1;
  const int32_t L = dir == 1 ? fwd : m - fwd;
  for (int32_t i = 0; i < m; ++i) S->R[cy[2 * i]].bpar = -1;
  /* detectors in B's own shell sit at radius zero: the shatter releases them */
  for (int64_t q = 0; q < S->nreached; ++q) {
    const int32_t v = S->reached[q];
    if (S->reg[v] == B) { S->reg[v] = -1; S->pe[v] = -1; S->pn[v] = -1; S->src[v] = -1; }
  }
  /* the even path from c_in to c_out joins the tree, alternately inner and outer */
  int32_t prev = P;
  for (int32_t j = 0; j <= L; ++j) {
    const int32_t idx = ((i_in + dir * j) % m + m) % m;
    const int32_t ch = cy[2 * idx];
    int32_t e;
    if (j == 0) e = Bv.tpe;
    else {
      const int32_t pidx = ((i_in + dir * (j - 1)) % m + m) % m;
      e = dir == 1 ? cy[2 * pidx + 1] : cy[2 * idx + 1];
    }
    S->R[ch].root = Bv.root; S->R[ch].tpar = prev; S->R[ch].tpe = e;
    if (j % 2 == 1) {
      S->R[ch].mate = prev; S->R[ch].me = e; S->R[prev].mate = ch; S->R[prev].me = e;
      set_rate(S, ch, 1);
    } else {
      set_rate(S, ch, -1);
    }
    prev = ch;
  }
  S->R[prev].mate = C; S->R[prev].me = Bv.me;
  S->R[C].tpar = prev; S->R[C].tpe = Bv.me; S->R[C].mate = prev; S->R[C].me = Bv.me;
  /* the rest of the cycle pairs up and freezes */
  for (int32_t j = 1; j + 1 <= m - L - 1; j += 2) {
    const int32_t ia = ((i_out + dir * j) % m + m) % m, ib = ((i_out + dir * (j + 1)) % m + m) % m;
    const int32_t a = cy[2 * ia], b = cy[2 * ib];
    const int32_t e = dir == 1 ? cy[2 * ia + 1] : cy[2 * ib + 1];
    S->R[a].mate = b; S->R[a].me = e; S->R[b].mate = a; S->R[b].me = e;
    S->R[a].root = -1; S->R[a].tpar = -1; S->R[a].tpe = -1;
    S->R[b].root = -1; S->R[b].tpar = -1; S->R[b].tpe = -1;
    set_rate(S, a, 0); set_rate(S, b, 0);
  }
  S->R[B].alive = 0; S->R[B].root = -1;
}

/* (e) node shrinks to zero: inner detector region T's parent and child meet at
 * its detection event and form a blossom with it. */
static void implode(shot* S, int32_t T) {
  const int32_t P = S->R[T].tpar, C = S->R[T].mate;
  if (P < 0 || C < 0) { S->flags |= SBF_INTERNAL; return; }
  const int32_t c = ce_join(S, S->R[T].me, S->R[T].tpe, T);
  form_blossom(S, C, P, c);
}

/* growing active region a (in a tree) meets region b (b < 0: the boundary) through compressed edge c */
static void collide(shot* S, int32_t a, int32_t b, int32_t c) {
  const int32_t ta = S->R[a].root;
  if (S->R[a].rate != 1 || ta < 0) { S->flags |= SBF_INTERNAL; return; }
  if (b < 0) {                                      /* (f) tree hits boundary */
    augment_to_root(S, a);
    S->R[a].mate = MATE_BD; S->R[a].me = c;
    dissolve_tree(S, ta);
    return;
  }
  const int32_t rb = S->R[b].rate;
  if (rb == 1) {
    const int32_t tb = S->R[b].root;
    if (tb == ta) { form_blossom(S, a, b, c); return; }   /* (c) tree hits itself */
    augment_to_root(S, a); augment_to_root(S, b);         /* (b) tree hits tree */
    S->R[a].mate = b; S->R[a].me = c; S->R[b].mate = a; S->R[b].me = c;
    dissolve_tree(S, ta); dissolve_tree(S, tb);
    return;
  }
  if (rb != 0) { S->flags |= SBF_INTERNAL; return; }
  const int32_t mb = S->R[b].mate;
  if (mb == MATE_BD) {                              /* (g) tree hits boundary match */
    augment_to_root(S, a);
    S->R[a].mate = b; S->R[a].me = c; S->R[b].mate = a; S->R[b].me = c;
    dissolve_tree(S, ta);
    return;
  }
  if (mb < 0) { S->flags |= SBF_INTERNAL; return; }
  /* (a) tree hits match: b joins as inner, its partner as outer (GROW) */
  S->R[b].root = ta; S->R[b].tpar = a; S->R[b].tpe = c;
  S->R[mb].root = ta; S->R[mb].tpar = b; S->R[mb].tpe = S->R[b].me;
  set_rate(S, b, -1);
  set_rate(S, mb, 1);
}

/* ------------------------------------------------------------------ */
/* flooder: the next event by a plain scan                               */
/* ------------------------------------------------------------------ */
enum { EV_REGION = 0, EV_LEAVE = 1, EV_EDGE = 2 };
typedef struct { i128 t; int32_t kind; int64_t key; int32_t u, x; int32_t tied; } event;

static int earlier(const event* a, const event* b) {
  if (a->t != b->t) return a->t < b->t;
  if (a->kind != b->kind) return a->kind < b->kind;
  return a->key < b->key;
}

/* active region and summed radius (the detector's local radius plus its
 * arrival radius) of every region, for the current time */
static void scan_regions(shot* S) {
  if (S->nR > S->capscan) {
    S->capscan = 2 * S->nR;
    S->ysum = (i128*)realloc(S->ysum, sizeof(i128) * (size_t)S->capscan);
    S->top = (int32_t*)realloc(S->top, sizeof(int32_t) * (size_t)S->capscan);
  }
  for (int64_t r = S->nR - 1; r >= 0; --r) {   /* a blossom has a larger id than its children */
    if (!S->R[r].alive) { S->top[r] = -1; continue; }
    const i128 y = yr(S, (int32_t)r, S->now);
    if (S->R[r].bpar < 0) { S->top[r] = (int32_t)r; S->ysum[r] = y; }
    else { S->top[r] = S->top[S->R[r].bpar]; S->ysum[r] = y + S->ysum[S->R[r].bpar]; }
  }
}

static i128 local_radius(const shot* S, int32_t v) { return S->ysum[S->reg[v]] - S->arr[v]; }

/* keeps the earliest event; `tied` records whether another, different event
 * (not the same edge seen from its other end) is due at that same time */
static void consider(event* best, i128 t, int32_t kind, int64_t key, int32_t u, int32_t x) {
  event c; c.t = t; c.kind = kind; c.key = key; c.u = u; c.x = x; c.tied = 0;
  const int same_time = (t == best->t);
  const int distinct = !(kind == best->kind && key == best->key);
  if (earlier(&c, best)) {
    c.tied = same_time && distinct && best->t < SB_INF;
    *best = c;
  } else if (same_time && distinct) {
    best->tied = 1;
  }
}

static event next_event(shot* S) {
  const sb_graph* g = S->g;
  event best; best.t = SB_INF; best.kind = 99; best.key = 0; best.u = -1; best.x = -1; best.tied = 0;
  scan_regions(S);
  /* IMPLODE / shatter: an active shrinking region reaches radius zero */
  for (int64_t r = 0; r < S->nR; ++r) {
    if (!S->R[r].alive || S->R[r].bpar >= 0 || S->R[r].rate >= 0) continue;
    consider(&best, S->now + yr(S, (int32_t)r, S->now), EV_REGION, r, (int32_t)r, -1);
  }
  for (int64_t q = 0; q < S->nreached; ++q) {
    const int32_t u = S->reached[q];
    if (S->reg[u] < 0) continue;
    const int32_t T = S->top[S->reg[u]];
    const int32_t ru = S->R[T].rate;
    const i128 lu = local_radius(S, u);
    if (ru < 0) {
      /* LEAVE: a detector of the shrinking region's own shell (not its detection event) */
      if (S->reg[u] == T && !(T < S->nd && S->det[T] == u)) consider(&best, S->now + lu, EV_LEAVE, u, u, -1);
      continue;
    }
    for (int64_t k = g->off[u]; k < g->off[u + 1]; ++k) {
      const int64_t e = g->adj[k];
      const int32_t x = other_end(g, e, u);
      const i128 W = g->wt[e];
      if (x < 0 || S->reg[x] < 0) {                 /* boundary or an empty detector */
        if (ru == 1) consider(&best, S->now + (W - lu), EV_EDGE, e, u, x);
        continue;
      }
      const int32_t T2 = S->top[S->reg[x]];
      if (T2 == T) continue;
      const int32_t rs = ru + S->R[T2].rate;
      if (rs <= 0) continue;
      const i128 num = W - lu - local_radius(S, x);
      if (num < 0 || (rs == 2 && (num & 1))) { S->flags |= SBF_INTERNAL; continue; }
      consider(&best, S->now + num / rs, EV_EDGE, e, u, x);
    }
  }
  return best;
}

/* tree charged with an event (the tree of the region that drives it) */
static int32_t driving_root(shot* S, const event* ev) {
  if (ev->kind == EV_REGION) return S->R[ev->u].root;
  if (ev->kind == EV_LEAVE) return S->R[S->top[S->reg[ev->u]]].root;
  const int32_t A = S->top[S->reg[ev->u]];
  if (S->R[A].rate == 1) {
    if (ev->x >= 0 && S->reg[ev->x] >= 0) {
      const int32_t B = S->top[S->reg[ev->x]];
      if (S->R[B].rate == 1 && S->R[B].root != S->R[A].root &&
          S->cid[S->R[B].root] != S->cid[S->R[A].root]) S->flags |= SBF_CROSS_CLUSTER;
    }
    return S->R[A].root;
  }
  return S->R[S->top[S->reg[ev->x]]].root;
}

static void charge(shot* S, int32_t root, i128 t) {
  if (root < 0) { S->flags |= SBF_INTERNAL; return; }
  const int32_t c = S->cid[root];
  S->c_n[c]++;
  if (t <= S->t_lt) S->c_early[c]++;
  S->c_last[c] = t;
}

static void apply(shot* S, const event* ev) {
  if (ev->kind == EV_REGION) {
    if (S->R[ev->u].cyc_len > 0) shatter(S, ev->u); else implode(S, ev->u);
    return;
  }
  if (ev->kind == EV_LEAVE) {
    const int32_t v = ev->u;
    S->reg[v] = -1; S->pe[v] = -1; S->pn[v] = -1; S->src[v] = -1;
    return;
  }
  const int32_t u = ev->u, x = ev->x;
  const int64_t e = ev->key;
  if (x >= 0 && S->reg[x] < 0) {                       /* ARRIVE */
    if (S->dix[x] >= 0) { S->flags |= SBF_REACHED_LATER; return; }
    const int32_t T = S->top[S->reg[u]];
    S->reg[x] = T; S->arr[x] = yr(S, T, S->now); S->src[x] = S->src[u]; S->pe[x] = e; S->pn[x] = u;
    touch(S, x);
    S->n_arrive++;
    return;
  }
  /* COLLIDE: the growing side drives the matcher */
  int32_t a = u, b = x;
  if (S->R[S->top[S->reg[a]]].rate != 1) { a = x; b = u; }
  const int32_t c = ce_collision(S, a, b, e);
  collide(S, S->top[S->reg[a]], b >= 0 ? S->top[S->reg[b]] : -1, c);
}

/* ------------------------------------------------------------------ */
/* Algorithm "Clustering"                                               */
/* ------------------------------------------------------------------ */
typedef struct { int32_t j; i128 d; } hit;

static int32_t uf_find(int32_t* p, int32_t x) { while (p[x] != x) { p[x] = p[p[x]]; x = p[x]; } return x; }

/* Dijkstra from detector s up to distance `limit`: detection events reached
 * (index, distance), boundary vertices reached (boundary edge, distance) and
 * the number of detectors settled within b/2 (the exploring region of radius b/2). */
static void search(const shot* S, int32_t s, i128 limit, i128 b, i128* dist, hitem* heap, hit** ev_out,
                   int64_t* nev, hit** bd_out, int64_t* nbd, int64_t* n_explore) {
  const sb_graph* g = S->g;
  int64_t sz = 0, cap_e = 0, cap_b = 0;
  int32_t* settled = (int32_t*)malloc(sizeof(int32_t) * (size_t)g->n);
  int64_t ns = 0;
  *nev = 0; *nbd = 0;
  dist[s] = 0; hpush(heap, &sz, 0, s);
  while (sz > 0) {
    hitem it = hpop(heap, &sz);
    const int32_t x = it.node;
    if (it.key != dist[x]) continue;
    settled[ns++] = x;
    if (2 * it.key <= b) ++*n_explore;
    if (S->dix[x] >= 0 && x != s) {
      GROW(*ev_out, cap_e, *nev + 1);
      (*ev_out)[*nev].j = S->dix[x]; (*ev_out)[*nev].d = it.key; ++*nev;
    }
    for (int64_t k = g->off[x]; k < g->off[x + 1]; ++k) {
      const int64_t e = g->adj[k];
      const int32_t y = other_end(g, e, x);
      const i128 nd = it.key + g->wt[e];
      if (nd > limit) continue;
      if (y < 0) {
        GROW(*bd_out, cap_b, *nbd + 1);
        (*bd_out)[*nbd].j = (int32_t)e; (*bd_out)[*nbd].d = nd; ++*nbd;
        continue;
      }
      if (nd < dist[y]) { dist[y] = nd; hpush(heap, &sz, nd, y); }
    }
  }
  for (int64_t i = 0; i < ns; ++i) dist[settled[i]] = SB_INF;
  /* nodes pushed but never settled */
  for (int64_t i = 0; i < sz; ++i) dist[heap[i].node] = SB_INF;
  free(settled);
}

static void clustering(shot* S, int32_t nl, const i128* dk, const i128* bk, int reading, int64_t* n_lvl1) {
  const sb_graph* g = S->g;
  const int32_t nd = S->nd;
  i128* dist = (i128*)malloc(sizeof(i128) * (size_t)g->n);
  for (int32_t i = 0; i < g->n; ++i) dist[i] = SB_INF;
  hitem* heap = (hitem*)malloc(sizeof(hitem) * (size_t)(g->off[g->n] + 2));
  hit** evl = (hit**)calloc((size_t)nd, sizeof(hit*));
  hit** bdl = (hit**)calloc((size_t)nd, sizeof(hit*));
  int64_t* nev = (int64_t*)calloc((size_t)nd, 8);
  int64_t* nbd = (int64_t*)calloc((size_t)nd, 8);
  int32_t* par = (int32_t*)malloc(4 * (size_t)nd);
  int32_t* mark = (int32_t*)malloc(4 * (size_t)nd);
  *n_lvl1 = 0;
  for (int32_t k = 0; k < nl; ++k) {
    int32_t nres = 0;
    for (int32_t i = 0; i < nd; ++i) nres += (S->level[i] == 0);
    if (nres == 0) break;
    for (int32_t i = 0; i < nd; ++i) { par[i] = i; free(evl[i]); free(bdl[i]); evl[i] = NULL; bdl[i] = NULL; }
    /* how far each exploring search has to look: pairs up to b_k (component
     * links), d_k (diameter, strict boundary condition), b_k/2 (loose
     * boundary condition).  When b_k exceeds every distance inside a graph
     * component, every residual event of it is linked to every other one and
     * only the diameter and boundary conditions need distances. */
    int32_t* whole = (int32_t*)calloc((size_t)nd, 4);   /* decided without distances (below) */
    for (int32_t i = 0; i < nd; ++i) {
      if (S->level[i] != 0) continue;
      const int32_t u = S->det[i];
      const i128 cb = g->comp_bound[g->comp[u]];
      const int all_linked = bk[k] >= cb;
      if (dk[k] >= cb && (reading == 0 || bk[k] / 2 >= cb)) {
        /* every distance inside the graph component is within d_k (and b_k/2
         * for the loose reading): all its residual events form one component
         * whose diameter and boundary conditions hold, the latter exactly when
         * the graph component has a boundary edge */
        whole[i] = 1;
        for (int32_t j = 0; j < nd; ++j)
          if (S->level[j] == 0 && g->comp[S->det[j]] == g->comp[u]) { int32_t a = uf_find(par, i), b = uf_find(par, j); if (a != b) par[a < b ? b : a] = a < b ? a : b; }
        continue;
      }
      i128 lim = all_linked ? dk[k] : bk[k];
      if (all_linked && reading == 1 && bk[k] / 2 > lim) lim = bk[k] / 2;
      int64_t nexp = 0;
      search(S, u, lim, bk[k], dist, heap, &evl[i], &nev[i], &bdl[i], &nbd[i], &nexp);
      if (k == 0) *n_lvl1 += nexp;
      if (all_linked) {
        for (int32_t j = 0; j < nd; ++j)
          if (S->level[j] == 0 && g->comp[S->det[j]] == g->comp[u]) { int32_t a = uf_find(par, i), b = uf_find(par, j); if (a != b) par[a < b ? b : a] = a < b ? a : b; }
      } else {
        for (int64_t q = 0; q < nev[i]; ++q) {
          const int32_t j = evl[i][q].j;
          if (S->level[j] != 0 || evl[i][q].d > bk[k]) continue;
          int32_t a = uf_find(par, i), b = uf_find(par, j);
          if (a != b) par[a < b ? b : a] = a < b ? a : b;
        }
      }
    }
    /* acceptance, component by component (root = smallest member) */
    for (int32_t r = 0; r < nd; ++r) {
      if (S->level[r] != 0 || uf_find(par, r) != r) continue;
      int32_t size = 0;
      for (int32_t i = 0; i < nd; ++i) if (S->level[i] == 0 && uf_find(par, i) == r) ++size;
      if (whole[r]) {
        const int ok = !(size & 1) || g->comp_bd[g->comp[S->det[r]]];
        if (ok) for (int32_t i = 0; i < nd; ++i) if (S->level[i] == 0 && uf_find(par, i) == r) S->cid[i] = r;
        continue;
      }
      int ok = 1;
      /* diameter: every member within d_k of every other member */
      for (int32_t i = 0; i < nd && ok; ++i) {
        if (S->level[i] != 0 || uf_find(par, i) != r) continue;
        int32_t within = 0;
        for (int32_t j = 0; j < nd; ++j) mark[j] = 0;
        for (int64_t q = 0; q < nev[i]; ++q) {
          const int32_t j = evl[i][q].j;
          if (S->level[j] == 0 && uf_find(par, j) == r && evl[i][q].d <= dk[k] && !mark[j]) { mark[j] = 1; ++within; }
        }
        if (within != size - 1) ok = 0;
      }
      if (ok && (size & 1)) {
        int found = 0;
        if (reading == 1) {
          for (int32_t i = 0; i < nd && !found; ++i) {
            if (S->level[i] != 0 || uf_find(par, i) != r) continue;
            for (int64_t q = 0; q < nbd[i] && !found; ++q) if (2 * bdl[i][q].d <= bk[k]) found = 1;
          }
        } else {
          /* a boundary vertex (boundary edge) within d_k of every member: try those of the root */
          for (int64_t q = 0; q < nbd[r] && !found; ++q) {
            if (bdl[r][q].d > dk[k]) continue;
            const int32_t be = bdl[r][q].j;
            int all = 1;
            for (int32_t i = 0; i < nd && all; ++i) {
              if (S->level[i] != 0 || uf_find(par, i) != r) continue;
              int has = 0;
              for (int64_t t = 0; t < nbd[i]; ++t) if (bdl[i][t].j == be && bdl[i][t].d <= dk[k]) has = 1;
              all = has;
            }
            found = all;
          }
        }
        ok = found;
      }
      if (ok) for (int32_t i = 0; i < nd; ++i) if (S->level[i] == 0 && uf_find(par, i) == r) S->cid[i] = r;
    }
    for (int32_t i = 0; i < nd; ++i) if (S->level[i] == 0 && S->cid[i] >= 0) S->level[i] = (int8_t)(k + 1);
    free(whole);
  }
  for (int32_t i = 0; i < nd; ++i) if (S->level[i] == 0) S->flags |= SBF_UNCLUSTERED;
  for (int32_t i = 0; i < nd; ++i) { free(evl[i]); free(bdl[i]); }
  free(evl); free(bdl); free(nev); free(nbd); free(par); free(mark); free(dist); free(heap);
}

/* ------------------------------------------------------------------ */
/* fuse: the final matching's compressed edges (blossoms expanded)       */
/* ------------------------------------------------------------------ */
static void add_final(shot* S, int32_t c, uint8_t* parity) {
  for (int64_t i = 0; i < S->CE[c].len; ++i) parity[S->path[S->CE[c].off + i]] ^= 1;
}

/* blossom X is matched through detection event s inside it */
static void expand(shot* S, int32_t X, int32_t s, uint8_t* parity, int depth) {
  if (S->R[X].cyc_len == 0) return;
  if (depth > 1 << 16) { S->flags |= SBF_INTERNAL; return; }
  const int32_t m = S->R[X].cyc_len;
  const int32_t* cy = S->cyc + S->R[X].cyc_off;
  const int32_t ch = child_with(S, X, s);
  int32_t p = -1;
  for (int32_t i = 0; i < m; ++i) if (cy[2 * i] == ch) p = i;
  if (p < 0) { S->flags |= SBF_INTERNAL; return; }
  expand(S, ch, s, parity, depth + 1);
  for (int32_t j = 1; j < m; j += 2) {
    const int32_t ia = (p + j) % m, ib = (p + j + 1) % m;
    const int32_t a = cy[2 * ia], b = cy[2 * ib], c = cy[2 * ia + 1];
    add_final(S, c, parity);
    expand(S, a, end_inside(S, c, a), parity, depth + 1);
    expand(S, b, end_inside(S, c, b), parity, depth + 1);
  }
}

/* ------------------------------------------------------------------ */
/* one shot                                                             */
/* ------------------------------------------------------------------ */
/* stats[0] applied events, [1] ARRIVE events, [2] E_ideal, [3] processing
 * clusters, [4] highest level, [5] detectors inside the level-1 exploring
 * regions (summed over events), [6] flags, [7] events applied while a
 * different event was due at the same time.  With such ties the result is
 * unique (the MWEM), but which of the simultaneous events remain valid after
 * the first is applied can depend on their order, and so can the counts. */
int oracle_sb_decode(void* pg, int32_t nd, const int32_t* det, int32_t n_levels, const int64_t* d_hi,
                     const uint64_t* d_lo, const int64_t* b_hi, const uint64_t* b_lo, int32_t reading, int32_t global,
                     int32_t* out_edges, int64_t out_cap, int64_t* n_out, int64_t* weight, uint64_t* obs,
                     int8_t* levels_out, int64_t* stats) {
  const sb_graph* g = (const sb_graph*)pg;
  for (int k = 0; k < 8; ++k) stats[k] = 0;
  *n_out = 0; *weight = 0; *obs = 0;
  if (!g || nd < 0) return SBF_INTERNAL;
  if (nd == 0) return 0;
  shot S;
  memset(&S, 0, sizeof(S));
  S.g = g; S.nd = nd; S.det = det;
  const int32_t n = g->n;
  S.dix = (int32_t*)malloc(4 * (size_t)n);
  for (int32_t i = 0; i < n; ++i) S.dix[i] = -1;
  for (int32_t i = 0; i < nd; ++i) {
    if (det[i] < 0 || det[i] >= n || S.dix[det[i]] >= 0) { free(S.dix); return SBF_INTERNAL; }
    S.dix[det[i]] = i;
  }
  S.level = (int8_t*)calloc((size_t)nd, 1);
  S.cid = (int32_t*)malloc(4 * (size_t)nd);
  for (int32_t i = 0; i < nd; ++i) S.cid[i] = -1;
  S.reg = (int32_t*)malloc(4 * (size_t)n); S.arr = (i128*)calloc((size_t)n, 16);
  S.src = (int32_t*)malloc(4 * (size_t)n); S.pe = (int64_t*)malloc(8 * (size_t)n);
  S.pn = (int32_t*)malloc(4 * (size_t)n); S.seen = (uint8_t*)calloc((size_t)n, 1);
  S.reached = (int32_t*)malloc(4 * (size_t)n);
  for (int32_t i = 0; i < n; ++i) { S.reg[i] = -1; S.src[i] = -1; S.pe[i] = -1; S.pn[i] = -1; }
  S.c_n = (int64_t*)calloc((size_t)nd, 8); S.c_early = (int64_t*)calloc((size_t)nd, 8);
  S.c_last = (i128*)calloc((size_t)nd, 16);
  S.max_events = 64 * ((int64_t)n + 64 * (int64_t)nd);
  /* detector regions 0..nd-1, created unseeded */
  for (int32_t i = 0; i < nd; ++i) { new_region(&S); S.R[i].alive = 0; }
  i128* dk = (i128*)malloc(16 * (size_t)(n_levels > 0 ? n_levels : 1));
  i128* bk = (i128*)malloc(16 * (size_t)(n_levels > 0 ? n_levels : 1));
  for (int32_t k = 0; k < n_levels; ++k) {
    dk[k] = ((i128)d_hi[k] << 64) | (i128)d_lo[k];
    bk[k] = ((i128)b_hi[k] << 64) | (i128)b_lo[k];
  }
  int64_t n_lvl1 = 0;
  if (global) {
    for (int32_t i = 0; i < nd; ++i) { S.level[i] = 1; S.cid[i] = 0; }
  } else {
    clustering(&S, n_levels, dk, bk, reading, &n_lvl1);
  }
  int32_t max_level = 0, n_clusters = 0;
  for (int32_t i = 0; i < nd; ++i) {
    if (S.level[i] > max_level) max_level = S.level[i];
    if (S.cid[i] == i || (global && i == 0)) ++n_clusters;
  }
  /* hierarchical execution: one level after the other, lower levels frozen */
  for (int32_t lvl = 1; lvl <= max_level && !(S.flags & ~SBF_DUAL); ++lvl) {
    int any = 0;
    for (int32_t i = 0; i < nd; ++i) any |= (S.level[i] == lvl);
    if (!any) continue;
    S.now = 0;
    for (int32_t i = 0; i < nd; ++i) {
      if (S.level[i] != lvl) continue;
      region* r = &S.R[i];
      r->alive = 1; r->base = 0; r->rate = 1; r->root = i;
      const int32_t v = det[i];
      S.reg[v] = i; S.arr[v] = 0; S.src[v] = i; S.pe[v] = -1; S.pn[v] = -1;
      touch(&S, v);
    }
    for (int32_t i = 0; i < nd; ++i) if (S.level[i] == lvl && S.cid[i] == i) { S.c_n[i] = 0; S.c_early[i] = 0; S.c_last[i] = 0; }
    if (global) { S.c_n[0] = 0; S.c_early[0] = 0; S.c_last[0] = 0; }
    for (;;) {
      event ev = next_event(&S);
      if (ev.t >= SB_INF || (S.flags & ~SBF_DUAL)) break;
      if (ev.t < S.now) { S.flags |= SBF_INTERNAL; break; }
      S.now = ev.t;
      S.n_tied += ev.tied;
      charge(&S, driving_root(&S, &ev), ev.t);
      apply(&S, &ev);
      if (++S.n_events > S.max_events) { S.flags |= SBF_INTERNAL; break; }
    }
    for (int64_t r = 0; r < S.nR; ++r)
      if (S.R[r].alive && S.R[r].bpar < 0 && S.R[r].root >= 0) S.flags |= SBF_INFEASIBLE;
    /* critical-path roll-up of this level's clusters */
    i128 t_next = S.t_lt;
    int64_t e_next = S.e_lt;
    for (int32_t i = 0; i < nd; ++i) {
      const int is_root = global ? (i == 0) : (S.level[i] == lvl && S.cid[i] == i);
      if (!is_root) continue;
      const i128 tC = S.c_last[i] > S.t_lt ? S.c_last[i] : S.t_lt;
      const int64_t EC = (S.c_early[i] > S.e_lt ? S.c_early[i] : S.e_lt) + S.c_n[i] - S.c_early[i];
      if (tC > t_next) t_next = tC;
      if (EC > e_next) e_next = EC;
    }
    S.t_lt = t_next; S.e_lt = e_next;
  }
  /* final matching: every active region is matched; expand blossoms */
  uint8_t* parity = (uint8_t*)calloc((size_t)(g->m ? g->m : 1), 1);
  i128 ysum = 0;
  if (!S.flags) {
    for (int64_t r = 0; r < S.nR; ++r) {
      if (!S.R[r].alive) continue;
      ysum += yr(&S, (int32_t)r, S.now);
      if (S.R[r].bpar >= 0) continue;
      const int32_t mt = S.R[r].mate, c = S.R[r].me;
      if (mt == -1 || c < 0) { S.flags |= SBF_INFEASIBLE; break; }
      if (mt != MATE_BD && mt < r) continue;
      add_final(&S, c, parity);
      expand(&S, (int32_t)r, end_inside(&S, c, (int32_t)r), parity, 0);
      if (mt != MATE_BD) expand(&S, mt, end_inside(&S, c, mt), parity, 0);
    }
  }
  if (!S.flags) {
    i128 wsum = 0;
    int64_t cnt = 0;
    for (int64_t e = 0; e < g->m; ++e) {
      if (!parity[e]) continue;
      if (cnt < out_cap) out_edges[cnt] = (int32_t)e;
      ++cnt;
      *weight += g->w[e]; *obs ^= g->obs[e]; wsum += g->wt[e];
    }
    *n_out = cnt;
    /* Supplementary S1, primal-dual pair: at the optimum the regions' radii
     * (the dual objective) add up to the weight of the matching */
    if (wsum != ysum) S.flags |= SBF_DUAL;
  }
  free(parity);
  if (levels_out) for (int32_t i = 0; i < nd; ++i) levels_out[i] = S.level[i];
  stats[0] = S.n_events; stats[1] = S.n_arrive; stats[2] = S.e_lt; stats[3] = n_clusters;
  stats[4] = max_level; stats[5] = n_lvl1; stats[6] = S.flags; stats[7] = S.n_tied;
  free(S.dix); free(S.level); free(S.cid); free(S.reg); free(S.arr); free(S.src); free(S.pe); free(S.pn);
  free(S.seen); free(S.reached); free(S.c_n); free(S.c_early); free(S.c_last);
  free(S.R); free(S.CE); free(S.path); free(S.cyc); free(S.ysum); free(S.top); free(dk); free(bk);
  return S.flags;
}
