// Per-shot decoding engine: one wavefront decodes one shot.
//
// Steps (paper: "Sparse-Blossom Decoding in o(1) Time", Mikami & Yamasaki):
//   1. syndrome intake: packed detector bits -> sorted detection events;
//   2. processing-cluster hierarchy (Methods, Algorithm "Clustering");
//   3. hierarchical execution (Methods, hierarchical execution rule and
//      Algorithm "Parallel sparse blossom"): level by level, the detection
//      events of that level seed growing regions at t = 0 while every stopped
//      lower-level configuration stays in place; a lower-level configuration
//      that a collision touches joins the running dynamics;
//   4. sparse blossom itself (Supplementary S1): graph-fill regions with
//      growth rate +1/0/-1, flooder events ARRIVE / LEAVE / COLLIDE /
//      IMPLODE and matcher events (a)-(g) on matches, alternating trees and
//      blossoms;
//   5. fuse: expand blossoms of the terminal configuration into matched
//      pairs, trace their paths through the arrival log, XOR them into the
//      edge set, and sum weights / XOR observable masks.
//
// All arithmetic is integer.  Times and radii are 128-bit integers in units
// of the tie-broken even weights, so every event happens at an integer time.
//
// State.  Only detectors that a region has reached ("explored" nodes, the
// detection events first, in ascending order) carry state; a direct map (or
// a hash, for graphs above 32,768 detectors) takes a detector id to its
// explored index, and in the wavefront tiers a neighbour table holds the
// explored index behind every adjacency slot of every explored node.
// Explored index i < nd is detection event i, whose detector region is
// region i and whose arrival record is record i.  The explored table, the
// region table and (per placement) the event cache, radius offsets and region
// bases form the StateLayout block, which lives in LDS for the wavefront
// tiers and in the slot's workspace for the lane tier; the rest of the
// per-shot state lives in the slot's workspace.
//
// Code style: every function is executed by all lanes of the wavefront with
// identical (uniform) values except inside the lane-parallel loops
// `for (i = lane(); i < n; i += PSB_WAVE)`.  Uniform stores of the same value
// by all lanes are intentional.
//
// The file is compiled twice: with the wavefront primitives of wave.h (one
// shot per wavefront, namespace psb::engine_wave, 64-entry event blocks) and
// with the single-lane primitives of lane_wave.h (one shot per lane, namespace
// psb::engine_lane, smaller event blocks).
#pragma once

#ifndef PSB_ENGINE_NS
#define PSB_ENGINE_NS engine_wave
#endif

#ifdef PSB_CHECK_INVARIANTS
// Host builds only (the harness defines the handler): checks of properties the
// paper proves about the dynamics.  Never compiled into a device build.
void psb_invariant_failed(const char* what, int64_t shot, int level);
#define PSB_INVARIANT(c, cond, what) \
  do { if (!(cond)) psb_invariant_failed((what), (c).dbg_shot, (c).dbg_lvl); } while (0)
#endif

namespace psb {
namespace PSB_ENGINE_NS {


#define T_INF (((i128)1) << 124)

// LDS scalars of one wavefront.
struct Lds {
  int x_n;              // explored-node count
  int fin_n;            // final compressed edges
  int stk_n;            // expansion stack
  int rel_n;            // nodes released by a shatter
  int pad[3];
};

struct Ctx {
  const Params* P;
  Lds* S;
  // graph
  const int32_t* nbr; const int32_t* eid; const i128* wt; const int32_t* w; const uint64_t* obs;
  int deg, n_det;
  // per-shot state (StateLayout)
  int32_t* x_node; int16_t *x_top, *x_reg, *x_src, *x_rec; i128 *x_wr, *x_ev;
  int16_t* x_nb;                     // [xcap][deg] explored index of each adjacency slot's neighbour (global)
  int32_t *h_key, *h_val; uint32_t hmask; int hshift;
  int16_t* dmap;                     // direct detector -> explored index map (global), or null
  i128* r_base; int16_t* r_f16; int32_t* r_f32; int rcap, xcap;
  // pools (global)
  int32_t *ce, *bc, *lg;
  int8_t* level;
  int32_t *uf, *cl_a, *cl_b, *cl_c, *cl_d, *bdl, *hit;
  int32_t* cid;                      // processing cluster (root event) of each detection event
  NearEntry* near;                   // clustering near-list entries, or null (WsLayout::near)
  int32_t* ehead;                    // near-list head of each detection event
  int32_t *shr, *chg, *stk, *fin; uint32_t* ebits;
  // uniform scalars
  int nd, n_regions, n_ce, n_bc, n_log, n_shr, n_chg, stamp, status;
  i128 now;
  int64_t n_ev;
  int n_visit;                       // clustering search visits (statistics)
  uint64_t t0, t_cl, t_dyn, t_fuse;  // device clock marks (statistics)
  char* acct;                        // event-accounting block, or null
#ifdef PSB_CHECK_INVARIANTS
  int64_t dbg_shot; int dbg_lvl;
  int32_t* dbg_cfg;                  // [rcap] processing cluster whose stopped configuration holds the region
  int32_t* dbg_touch;                // [dcap] per cluster: the cluster that touched its configuration at dbg_touch_lvl
  int32_t* dbg_touch_lvl;            // [dcap]
#endif
};

// Region field f of region r: int16 storage for ids, rates and flags, int32
// for the two stamps.
template <int F> struct RFType { typedef int16_t T; };
template <> struct RFType<RF_MARK> { typedef int32_t T; };
template <> struct RFType<RF_CHGM> { typedef int32_t T; };
template <int F> PSB_DEV typename RFType<F>::T& rf_ref(const Ctx& c, int r) {
  if constexpr (F >= RF_N16) return c.r_f32[(int64_t)(F - RF_N16) * c.rcap + r];
  else return c.r_f16[(int64_t)F * c.rcap + r];
}
#define RF(c, r, f) (rf_ref<(f)>((c), (r)))
#define CEF(c, i, f) ((c).ce[(int64_t)(i) * CE_COUNT + (f)])

// rate * t for a region rate in {-1, 0, +1}, as a select rather than a
// 128-bit multiply.
PSB_DEV i128 rate_times(int rate, i128 t) { return rate > 0 ? t : (rate < 0 ? -t : (i128)0); }

PSB_DEV i128 yrad(const Ctx& c, int r, i128 t) { return c.r_base[r] + rate_times(RF(c, r, RF_RATE), t); }

// ---------------------------------------------------------------------------
// parallel event count (Methods, numerical evaluation: the critical-path event
// count of hierarchical execution, E_ideal).  Every applied event is charged
// to the processing cluster whose alternating tree drives it; at the end of
// each level the clusters of that level are rolled up into the critical-path
// stopping time t_<k+1 and event count E_<k+1.
// ---------------------------------------------------------------------------
PSB_DEV int32_t* acct_hdr(const Ctx& c) { return (int32_t*)c.acct; }
PSB_DEV i128* acct_tlt(const Ctx& c) { return (i128*)(c.acct + ACCT_TLT); }
PSB_DEV int32_t* acct_cid(const Ctx& c) { return (int32_t*)(c.acct + ACCT_CID); }
PSB_DEV int32_t* acct_cnt(const Ctx& c) { return (int32_t*)(c.acct + acct_n(c.P->cap.dcap)); }
PSB_DEV int32_t* acct_early_n(const Ctx& c) { return (int32_t*)(c.acct + acct_early(c.P->cap.dcap)); }
PSB_DEV i128* acct_lastt(const Ctx& c) { return (i128*)(c.acct + acct_last(c.P->cap.dcap)); }

// Charges one applied event at time t to the cluster of tree `tid` (uniform).
PSB_DEV void account_event(Ctx& c, int tid, i128 t) {
  wave_sync();
  int32_t* h = acct_hdr(c);
  h[0] = uni(h[0]) + 1;
  if (tid >= 0) {
    const int cl = uni(acct_cid(c)[tid]);
    acct_cnt(c)[cl] = uni(acct_cnt(c)[cl]) + 1;
    if (t <= uni128(*acct_tlt(c))) acct_early_n(c)[cl] = uni(acct_early_n(c)[cl]) + 1;
    acct_lastt(c)[cl] = t;
  }
  wave_sync();
}

// A capacity of this tier is exhausted: the fast tier hands the shot to the
// overflow tier, the overflow tier reports it.
PSB_DEV void cap_fail(Ctx& c) { c.status = (c.P->tier == 0) ? S_OVERFLOW : S_CAPACITY; }

// ---------------------------------------------------------------------------
// detector id -> explored index (open addressing, linear probing)
// ---------------------------------------------------------------------------
PSB_DEV uint32_t hpos(const Ctx& c, int v) { return ((uint32_t)v * 2654435761u) >> c.hshift; }

PSB_DEV int node_idx(const Ctx& c, int v) {
  if (c.dmap) return c.dmap[v];
  uint32_t s = hpos(c, v);
  for (uint32_t k = 0; k <= c.hmask; ++k) {
    const int key = c.h_key[s];
    if (key == v) return c.h_val[s];
    if (key < 0) return -1;
    s = (s + 1) & c.hmask;
  }
  return -1;
}

// The same lookup for a uniform detector id, with a uniform result.
PSB_DEV int node_idx_u(const Ctx& c, int v) {
  if (c.dmap) return uni(c.dmap[v]);
  uint32_t s = hpos(c, v);
  for (uint32_t k = 0; k <= c.hmask; ++k) {
    const int key = uni(c.h_key[s]);
    if (key == v) return uni(c.h_val[s]);
    if (key < 0) return -1;
    s = (s + 1) & c.hmask;
  }
  return -1;
}

// Uniform insert of a detector that is not present (the table is sized at
// twice the explored capacity, so a free slot exists; the probe is bounded
// regardless).
PSB_DEV bool hash_put(Ctx& c, int v, int idx) {
  if (c.dmap) { c.dmap[v] = (int16_t)idx; return true; }
  uint32_t s = hpos(c, v);
  for (uint32_t k = 0; k <= c.hmask; ++k) {
    if (uni(c.h_key[s]) < 0) { c.h_key[s] = v; c.h_val[s] = idx; return true; }
    s = (s + 1) & c.hmask;
  }
  return false;
}

// Lane-parallel insert (distinct keys).
PSB_DEV void hash_put_atomic(Ctx& c, int v, int idx) {
  if (c.dmap) { c.dmap[v] = (int16_t)idx; return; }
  uint32_t s = hpos(c, v);
  for (uint32_t k = 0; k <= c.hmask; ++k) {
    if (atom_cas(&c.h_key[s], -1, v) == -1) { c.h_val[s] = idx; return; }
    s = (s + 1) & c.hmask;
  }
}

// ---------------------------------------------------------------------------
// event cache: the earliest event of every explored node, x_ev[i]
// ---------------------------------------------------------------------------
PSB_DEV void set_event(Ctx& c, int ix, i128 t) { c.x_ev[ix] = t; }

// Region codes rank before node codes at equal time (a region event is
// handled first); within a kind the smaller index wins.
constexpr int EV_NODE = 1 << 24;

// Next event of the dynamics: the earliest cached node event and the earliest
// shrinking top-level region reaching radius zero (y(t) = base - t is zero at
// t = base), in one scan and one reduction.  code < EV_NODE: region code;
// otherwise explored index code - EV_NODE.
PSB_DEV void next_event(Ctx& c, i128& t, int& code) {
  wave_sync();
  const int xn = uni(c.S->x_n);
  i128 key = T_INF; int arg = 0x7fffffff;
  // up to four entries per lane loaded before any is compared (one round trip
  // for up to 4 * PSB_WAVE explored nodes); each lane still takes its entries
  // in ascending index order, so ties go to the smaller index as before
  for (int i0 = 0; i0 < xn; i0 += 4 * PSB_WAVE) {
    i128 k[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + u * PSB_WAVE + lane();
      k[u] = i < xn ? c.x_ev[i] : T_INF;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (k[u] < key) { key = k[u]; arg = EV_NODE + i0 + u * PSB_WAVE + lane(); }
  }
  // regions: only once some region has been inner in this shot
  for (int x = lane(); c.n_shr > 0 && x < c.n_regions; x += PSB_WAVE) {
    if (RF(c, x, RF_RATE) < 0 && RF(c, x, RF_BPAR) < 0 && RF(c, x, RF_ALIVE)) {
      const i128 k = c.r_base[x];
      if (k < key || (k == key && x < arg)) { key = k; arg = x; }
    }
  }
  wave_argmin(key, arg);
  t = key; code = arg;
}

// ---------------------------------------------------------------------------
// node-level events (flooder): ARRIVE / COLLIDE / LEAVE times at node i
// ---------------------------------------------------------------------------
// The wavefront tiers keep a neighbour table per explored node (the explored
// index behind each adjacency slot); the lane tier looks neighbours up in the
// detector map instead (with the table, lane-tier shots on the hash-map path
// came back wrong on the device while the same code was correct on the CPU;
// the lane tier keeps the lookups until that is explained).
#ifndef PSB_NB_TABLE
#define PSB_NB_TABLE (PSB_WAVE > 1)
#endif
constexpr bool kNbTable = PSB_NB_TABLE;

// Explored index of the neighbour behind adjacency slot j of explored node i,
// or an XNB_* code.
PSB_DEV int nb_index(const Ctx& c, int i, int64_t row, int j);

// Earliest event seen from explored node i: returns time (T_INF = none) and
// kind (edge slot 0..deg-1 or K_LEAVE).  The local radius of an owned node
// is l(t) = y_top(t) + wr; an edge of weight W is crossed by one fill when
// l = W (ARRIVE at an empty neighbour, COLLIDE with the boundary) and two
// fills meet when l_u + l_v = W, provided their rates add up to > 0.
// Time of the event through adjacency slot j of explored node i (owned by
// top region `top` with rate ra > 0 or 0 and l_u(t) = bu + ra * t); T_INF if
// the slot gives none.
// (k: the slot's neighbour-table entry, already loaded)
PSB_DEV i128 slot_event_k(const Ctx& c, int top, int ra, i128 bu, int64_t row, int j, int k) {
  if (k == XNB_PAD) return T_INF;
  const i128 W = c.wt[row + j];
  if (k == XNB_BOUNDARY) return (ra > 0) ? W - bu : T_INF;
  const int vt = (k >= 0) ? c.x_top[k] : -1;
  if (vt < 0) return (ra > 0) ? W - bu : T_INF;      // ARRIVE
  if (vt == top) return T_INF;
  const int rs = ra + RF(c, vt, RF_RATE);
  if (rs <= 0) return T_INF;
  const i128 num = W - bu - (c.r_base[vt] + c.x_wr[k]);
  return (rs == 1) ? num : (num >> 1);               // COLLIDE (num even when rs == 2)
}

PSB_DEV i128 slot_event(const Ctx& c, int i, int top, int ra, i128 bu, int64_t row, int j) {
  return slot_event_k(c, top, ra, bu, row, j, nb_index(c, i, row, j));
}

// Earliest event seen from explored node i, evaluated by one lane.
PSB_DEV void node_event(const Ctx& c, int i, i128& tbest, int& kbest) {
  tbest = T_INF; kbest = K_NONE;
  const int top = c.x_top[i];
  if (top < 0) return;
  const int ra = RF(c, top, RF_RATE);
  const i128 bu = c.r_base[top] + c.x_wr[i];       // l_u(t) = bu + ra * t
  if (ra < 0) {
    // the detection event of a detector region is its own source: it never
    // leaves (explored index i < nd is detection event i, region i)
    if (c.x_reg[i] == top && !(i < c.nd && i == top)) { tbest = bu; kbest = K_LEAVE; }
    return;   // a shrinking fill cannot gain on any neighbour
  }
  const int deg = c.deg;
  const int64_t row = (int64_t)c.x_node[i] * deg;
  // four slots at a time: their neighbour entries are loaded before any slot
  // is evaluated (slots still taken in order, ties to the smaller slot)
  for (int j0 = 0; j0 < deg; j0 += 4) {
    int ks[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) ks[u] = j0 + u < deg ? nb_index(c, i, row, j0 + u) : XNB_PAD;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const i128 t = slot_event_k(c, top, ra, bu, row, j0 + u, ks[u]);
      if (t < tbest) { tbest = t; kbest = j0 + u; }
    }
  }
}

#if PSB_WAVE > 1
// The same event with the adjacency slots of node i spread over a group of G
// lanes (G a power of two >= deg, groups aligned to G): lane q of the group
// evaluates slot q, a butterfly over the group keeps the earliest (ties to
// the smaller slot, as the serial scan does).  i < 0 marks an idle group.
// Every lane of the wavefront must call this; each receives its group's result.
PSB_DEV void node_event_group(const Ctx& c, int i, int G, i128& tbest, int& kbest) {
  const int q = lane() & (G - 1);
  i128 t = T_INF; int k = 0x7fffffff;
  if (i >= 0) {
    const int top = c.x_top[i];
    if (top >= 0) {
      const int ra = RF(c, top, RF_RATE);
      const i128 bu = c.r_base[top] + c.x_wr[i];
      if (ra < 0) {
        if (q == 0 && c.x_reg[i] == top && !(i < c.nd && i == top)) { t = bu; k = K_LEAVE; }
      } else if (q < c.deg) {
        t = slot_event(c, i, top, ra, bu, (int64_t)c.x_node[i] * c.deg, q);
        k = q;
      }
    }
  }
  group_argmin(t, k, G);
  tbest = t; kbest = (t < T_INF) ? k : K_NONE;
}

PSB_DEV int slot_group(const Ctx& c) { int G = 1; while (G < c.deg) G <<= 1; return G; }
#endif

// Earliest event of explored node i for uniform code (uniform result).
PSB_DEV void node_event_u(const Ctx& c, int i, i128& t, int& k) {
#if PSB_WAVE > 1
  node_event_group(c, i, slot_group(c), t, k);
  t = uni128(t); k = uni(k);
#else
  node_event(c, i, t, k);
#endif
}

// Refresh of explored node i and all of its explored neighbours: the deg+1
// nodes are spread over groups of lanes, each group evaluating one node's
// adjacency slots.
PSB_DEV void refresh_star(Ctx& c, int i) {
  wave_sync();
  const int deg = c.deg;
#if PSB_WAVE > 1
  const int16_t* nb = c.x_nb + (int64_t)i * deg;
  const int G = slot_group(c), per = PSB_WAVE / G;
  for (int j0 = 0; j0 <= deg; j0 += per) {
    const int j = j0 + lane() / G;
    int x = -1;
    if (j < deg) {
      const int k = nb[j];
      if (k >= 0) x = k;
    } else if (j == deg) {
      x = i;
    }
    i128 t; int k;
    node_event_group(c, x, G, t, k);
    if (x >= 0 && (lane() & (G - 1)) == 0) set_event(c, x, t);
  }
#else
  const int64_t row = (int64_t)c.x_node[i] * deg;
  for (int j = 0; j <= deg; ++j) {
    int x = i;
    if (j < deg) {
      x = nb_index(c, i, row, j);
      if (x < 0) continue;
    }
    i128 t; int k;
    node_event(c, x, t, k);
    set_event(c, x, t);
  }
#endif
  wave_sync();
}

// Neighbour-table entry of an adjacency slot holding detector nbv.
PSB_DEV int xnb_code(const Ctx& c, int nbv) {
  if (nbv == NB_PAD) return XNB_PAD;
  if (nbv == NB_BOUNDARY) return XNB_BOUNDARY;
  return node_idx(c, nbv);
}

PSB_DEV int nb_index(const Ctx& c, int i, int64_t row, int j) {
  if constexpr (kNbTable) return c.x_nb[(int64_t)i * c.deg + j];
  else return xnb_code(c, c.nbr[row + j]);
}

// Fills the neighbour table of explored node ix (detector v) and points the
// slots of its explored neighbours that hold v at ix (every such slot: a
// graph may join two detectors by several edges).  Slots are spread over lanes.
PSB_DEV void link_neighbours(Ctx& c, int ix, int v) {
  const int deg = c.deg;
  for (int j = lane(); j < deg; j += PSB_WAVE) {
    const int nbv = c.nbr[(int64_t)v * deg + j];
    const int k = xnb_code(c, nbv);
    c.x_nb[(int64_t)ix * deg + j] = (int16_t)k;
    if (k >= 0) {
      // the neighbour's row four slots at a time, loaded before any is tested
      const int64_t r2 = (int64_t)nbv * deg;
      for (int j0 = 0; j0 < deg; j0 += 4) {
        int n4[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) n4[u] = j0 + u < deg ? c.nbr[r2 + j0 + u] : NB_PAD;
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (n4[u] == v) c.x_nb[(int64_t)k * deg + j0 + u] = (int16_t)ix;
      }
    }
  }
}

// Append detector v to the explored table (uniform); returns its index.
PSB_DEV int explore(Ctx& c, int v) {
  const int ix = uni(c.S->x_n);
  if (ix >= c.xcap) { cap_fail(c); return -1; }
  c.x_node[ix] = v; c.x_top[ix] = -1; c.x_reg[ix] = -1; c.x_src[ix] = -1; c.x_rec[ix] = -1;
  c.x_wr[ix] = 0; c.x_ev[ix] = T_INF;
  if (!hash_put(c, v, ix)) { cap_fail(c); return -1; }
  wave_sync();
  if constexpr (kNbTable) {
    link_neighbours(c, ix, v);
    wave_sync();
  }
  c.S->x_n = ix + 1;
  wave_sync();
  return ix;
}

// ---------------------------------------------------------------------------
// regions, compressed edges, tree bookkeeping
// ---------------------------------------------------------------------------
PSB_DEV void region_init(Ctx& c, int r, int rate, i128 base, int tid) {
  c.r_base[r] = base;
  RF(c, r, RF_RATE) = rate; RF(c, r, RF_BPAR) = -1; RF(c, r, RF_TPAR) = -1; RF(c, r, RF_TPE) = -1;
  RF(c, r, RF_TID) = tid; RF(c, r, RF_MATE) = -1; RF(c, r, RF_ME) = -1; RF(c, r, RF_BCO) = 0;
  RF(c, r, RF_BCN) = 0; RF(c, r, RF_ALIVE) = 1; RF(c, r, RF_MARK) = 0; RF(c, r, RF_INSHR) = 0;
  RF(c, r, RF_CHGM) = 0;
}

// Marks region r: the events of every node of its area must be recomputed.
PSB_DEV void note_change(Ctx& c, int r) {
  if (uni(RF(c, r, RF_CHGM)) == c.stamp) return;
  RF(c, r, RF_CHGM) = c.stamp;
  ++c.n_chg;
}

PSB_DEV void set_rate(Ctx& c, int r, int rate) {
  const i128 y = yrad(c, r, c.now);
  c.r_base[r] = y - rate_times(rate, c.now);
  RF(c, r, RF_RATE) = rate;
  if (rate < 0) c.n_shr = 1;                 // region events are possible from now on
  note_change(c, r);
}

PSB_DEV int ce_leaf(Ctx& c, int e, int rec_a, int rec_b, int sa, int sb) {
  if (c.n_ce >= c.P->cecap) { cap_fail(c); return -1; }
  const int i = c.n_ce++;
  CEF(c, i, CE_E) = e; CEF(c, i, CE_A) = rec_a; CEF(c, i, CE_B) = rec_b;
  CEF(c, i, CE_SA) = sa; CEF(c, i, CE_SB) = sb;
  return i;
}

PSB_DEV int ce_concat(Ctx& c, int a, int b, int sa, int sb) {
  if (c.n_ce >= c.P->cecap) { cap_fail(c); return -1; }
  const int i = c.n_ce++;
  CEF(c, i, CE_E) = -1; CEF(c, i, CE_A) = a; CEF(c, i, CE_B) = b;
  CEF(c, i, CE_SA) = sa; CEF(c, i, CE_SB) = sb;
  return i;
}

// The end of compressed edge `ce` that is not detection event `s`.
PSB_DEV int ce_other(const Ctx& c, int ce, int s) {
  const int a = uni(CEF(c, ce, CE_SA)), b = uni(CEF(c, ce, CE_SB));
  return a == s ? b : a;
}

// Child of blossom `b` containing region (or detection event) x (uniform).
PSB_DEV int child_containing(const Ctx& c, int x, int b) {
  int guard = 0;
  while (x >= 0) {
    const int p = uni(RF(c, x, RF_BPAR));
    if (p == b || ++guard > c.n_regions) break;
    x = p;
  }
  return x;
}

// Is detection event s inside region r (r itself or a descendant)?  Uniform
// version and per-lane version.
PSB_DEV bool inside(const Ctx& c, int s, int r) {
  int x = s, guard = 0;
  while (x >= 0 && guard++ <= c.n_regions) { if (x == r) return true; x = uni(RF(c, x, RF_BPAR)); }
  return false;
}
PSB_DEV bool inside_lane(const Ctx& c, int s, int r) {
  int x = s, guard = 0;
  while (x >= 0 && guard++ <= c.n_regions) { if (x == r) return true; x = RF(c, x, RF_BPAR); }
  return false;
}

// Augment from outer region x up to its tree root: every inner region on the
// path is re-matched to its tree parent (Supplementary S1: AUGMENT).
PSB_DEV void augment_to_root(Ctx& c, int x) {
  int cur = x;
  int guard = 0;
  while (uni(RF(c, cur, RF_TPAR)) >= 0) {
    const int in = uni(RF(c, cur, RF_TPAR));
    const int out = uni(RF(c, in, RF_TPAR));
    const int e = uni(RF(c, in, RF_TPE));
    RF(c, in, RF_MATE) = out; RF(c, in, RF_ME) = e;
    RF(c, out, RF_MATE) = in; RF(c, out, RF_ME) = e;
    cur = out;
    if (++guard > c.n_regions) { c.status = S_INTERNAL; return; }
  }
}

// All regions of tree `tid` become frozen and leave the tree.
PSB_DEV void dissolve_tree(Ctx& c, int tid) {
  const int nr = c.n_regions;
  int n = 0;
  wave_sync();
  for (int i0 = 0; i0 < nr; i0 += PSB_WAVE) {
    const int r = i0 + lane();
    const int take = (r < nr && RF(c, r, RF_ALIVE) && RF(c, r, RF_BPAR) < 0 && RF(c, r, RF_TID) == tid) ? 1 : 0;
    const uint64_t mask = ballot(take);
    if (take) c.stk[n + __builtin_popcountll(mask & lanemask_lt())] = r;
    n += __builtin_popcountll(mask);
  }
  wave_sync();
  for (int q = 0; q < n; ++q) {
    const int r = uni(c.stk[q]);
    RF(c, r, RF_TID) = -1;
    RF(c, r, RF_TPAR) = -1;
    set_rate(c, r, 0);
#ifdef PSB_CHECK_INVARIANTS
    if (c.acct) c.dbg_cfg[r] = acct_cid(c)[tid];
#endif
  }
}

// ---------------------------------------------------------------------------
// matcher events
// ---------------------------------------------------------------------------

// (c) tree hits itself / (e) after an implode: outer regions a and b of the
// same tree touch through compressed edge ce -> blossom (SHRINK).
PSB_DEV void form_blossom(Ctx& c, int a, int b, int ce) {
  // lowest common outer ancestor
  ++c.stamp;
  const int st = c.stamp;
  int x = a, guard = 0;
  RF(c, x, RF_MARK) = st;
  while (uni(RF(c, x, RF_TPAR)) >= 0) {
    x = uni(RF(c, uni(RF(c, x, RF_TPAR)), RF_TPAR));
    RF(c, x, RF_MARK) = st;
    if (++guard > c.n_regions) { c.status = S_INTERNAL; return; }
  }
  int y = b; guard = 0;
  while (uni(RF(c, y, RF_MARK)) != st) {
    const int yp = uni(RF(c, y, RF_TPAR));
    if (yp < 0) { c.status = S_INTERNAL; return; }
    y = uni(RF(c, yp, RF_TPAR));
    if (++guard > c.n_regions) { c.status = S_INTERNAL; return; }
  }
  const int lca = y;
  ++c.stamp;   // fresh stamp for cycle membership
  const int cs = c.stamp;
  // cycle = [lca] + reverse(path a->lca) + path b->lca  (paths exclude lca)
  int ma = 0, mb = 0;
  const int cap = c.P->stkcap;
  for (x = a; x != lca; x = uni(RF(c, uni(RF(c, x, RF_TPAR)), RF_TPAR))) {
    if (ma + 2 > cap) { cap_fail(c); return; }
    c.stk[ma++] = x; c.stk[ma++] = uni(RF(c, x, RF_TPAR));
  }
  for (x = b; x != lca; x = uni(RF(c, uni(RF(c, x, RF_TPAR)), RF_TPAR))) {
    if (ma + mb + 2 > cap) { cap_fail(c); return; }
    c.stk[ma + mb++] = x; c.stk[ma + mb++] = uni(RF(c, x, RF_TPAR));
  }
  const int m = 1 + ma + mb;
  if (c.n_bc + m > c.P->bccap || c.n_regions >= c.rcap) { cap_fail(c); return; }
  const int bo = c.n_bc;
  c.n_bc += m;
  int* cyc = c.bc + 2 * bo;   // pairs (child, edge to next)
  cyc[0] = lca;
  for (int i = 0; i < ma; ++i) cyc[2 * (1 + i)] = uni(c.stk[ma - 1 - i]);
  for (int i = 0; i < mb; ++i) cyc[2 * (1 + ma + i)] = uni(c.stk[ma + i]);
  for (int i = 0; i < m; ++i) {
    int e;
    if (i < ma) e = RF(c, uni(cyc[2 * (i + 1)]), RF_TPE);  // parent -> child: child's tree edge
    else if (i == ma) e = ce;                              // a -> b
    else e = RF(c, uni(cyc[2 * i]), RF_TPE);               // child -> parent
    cyc[2 * i + 1] = e;
  }
  wave_sync();
  // new blossom region
  const int X = c.n_regions++;
  const int tid = uni(RF(c, lca, RF_TID));
  const int lca_par = uni(RF(c, lca, RF_TPAR));
  region_init(c, X, 1, -c.now, tid);
  RF(c, X, RF_TPAR) = lca_par;
  RF(c, X, RF_TPE) = RF(c, lca, RF_TPE);
  RF(c, X, RF_MATE) = RF(c, lca, RF_MATE);
  RF(c, X, RF_ME) = RF(c, lca, RF_ME);
  RF(c, X, RF_BCO) = bo; RF(c, X, RF_BCN) = m;
  if (lca_par >= 0) RF(c, lca_par, RF_MATE) = X;
  for (int i = 0; i < m; ++i) RF(c, uni(cyc[2 * i]), RF_MARK) = cs;
  wave_sync();
  // tree children of cycle members that are not on the cycle hang from X
  for (int r = lane(); r < c.n_regions; r += PSB_WAVE) {
    if (r == X || !RF(c, r, RF_ALIVE) || RF(c, r, RF_BPAR) >= 0 || RF(c, r, RF_TID) != tid) continue;
    if (RF(c, r, RF_MARK) == cs) continue;
    const int p = RF(c, r, RF_TPAR);
    if (p >= 0 && RF(c, p, RF_MARK) == cs) RF(c, r, RF_TPAR) = X;
  }
  // nodes of the members now belong to X: l = y_member(now) + wr = y_X(now) + wr'
  // with y_X(now) = 0, so wr' = wr + y_member(now)
  const int xn = uni(c.S->x_n);
  for (int i = lane(); i < xn; i += PSB_WAVE) {
    const int t = c.x_top[i];
    if (t < 0 || RF(c, t, RF_MARK) != cs) continue;
    c.x_wr[i] = c.x_wr[i] + yrad(c, t, c.now);
    c.x_top[i] = X;
  }
  wave_sync();
  // freeze the cycle members inside X
  for (int i = 0; i < m; ++i) {
    const int ch = uni(cyc[2 * i]);
    c.r_base[ch] = yrad(c, ch, c.now);
    RF(c, ch, RF_RATE) = 0;
    RF(c, ch, RF_BPAR) = X;
    RF(c, ch, RF_TID) = -1; RF(c, ch, RF_TPAR) = -1; RF(c, ch, RF_MATE) = -1;
  }
  note_change(c, X);
}

// (d) an inner blossom's radius reaches zero: it shatters (EXPAND).
PSB_DEV void shatter(Ctx& c, int B) {
  const int m = uni(RF(c, B, RF_BCN));
  const int bo = uni(RF(c, B, RF_BCO));
  const int* cyc = c.bc + 2 * bo;
  const int P_ = uni(RF(c, B, RF_TPAR));
  const int ce_p = uni(RF(c, B, RF_TPE));
  const int C = uni(RF(c, B, RF_MATE));
  const int ce_c = uni(RF(c, B, RF_ME));
  const int tid = uni(RF(c, B, RF_TID));
  if (P_ < 0 || C < 0) { c.status = S_INTERNAL; return; }
  const int p_sa = uni(CEF(c, ce_p, CE_SA)), p_sb = uni(CEF(c, ce_p, CE_SB));
  const int c_sa = uni(CEF(c, ce_c, CE_SA)), c_sb = uni(CEF(c, ce_c, CE_SB));
  const int s_in = inside(c, p_sa, B) ? p_sa : p_sb;
  const int s_out = inside(c, c_sa, B) ? c_sa : c_sb;
  const int c_in = child_containing(c, s_in, B), c_out = child_containing(c, s_out, B);
  int i_in = -1, i_out = -1;
  for (int i = 0; i < m; ++i) { const int ch = uni(cyc[2 * i]); if (ch == c_in) i_in = i; if (ch == c_out) i_out = i; }
  if (i_in < 0 || i_out < 0) { c.status = S_INTERNAL; return; }
  const int fwd = ((i_out - i_in) % m + m) % m;
  const int dir = (fwd % 2 == 0) ? 1 : -1;
  const int L = (dir == 1) ? fwd : m - fwd;
  // children become top level; nodes of B's area move to the child holding
  // their shell region: l = y_B(now) + wr = y_child + (wr - y_child).
  // Nodes still in B's own shell sit exactly on its boundary and leave.
  for (int i = 0; i < m; ++i) RF(c, uni(cyc[2 * i]), RF_BPAR) = -1;
  wave_sync();
  c.S->rel_n = 0;
  wave_sync();
  const int xn = uni(c.S->x_n);
  for (int i = lane(); i < xn; i += PSB_WAVE) {
    if (c.x_top[i] != B) continue;
    const int reg = c.x_reg[i];
    if (reg == B) {
      c.x_top[i] = -1; c.x_reg[i] = -1; c.x_src[i] = -1; c.x_rec[i] = -1;
      const int k = atom_add(&c.S->rel_n, 1);
      c.stk[k] = i;
      continue;
    }
    int ch = reg;
    while (RF(c, ch, RF_BPAR) >= 0 && RF(c, ch, RF_BPAR) != B) ch = RF(c, ch, RF_BPAR);
    c.x_top[i] = ch;
    c.x_wr[i] = c.x_wr[i] - c.r_base[ch];   // frozen child: y = base
  }
  wave_sync();
  // the even path from c_in to c_out stays in the tree
  int prev = P_;
  for (int j = 0; j <= L; ++j) {
    const int idx = ((i_in + dir * j) % m + m) % m;
    const int ch = uni(cyc[2 * idx]);
    int e;
    if (j == 0) e = ce_p;
    else {
      const int pidx = ((i_in + dir * (j - 1)) % m + m) % m;
      e = uni((dir == 1) ? cyc[2 * pidx + 1] : cyc[2 * idx + 1]);
    }
    RF(c, ch, RF_TID) = tid;
    RF(c, ch, RF_TPAR) = prev;
    RF(c, ch, RF_TPE) = e;
    if (j % 2 == 1) {        // outer: matched to the inner before it
      RF(c, ch, RF_MATE) = prev; RF(c, ch, RF_ME) = e;
      RF(c, prev, RF_MATE) = ch; RF(c, prev, RF_ME) = e;
      set_rate(c, ch, 1);
    } else {
      set_rate(c, ch, -1);
    }
    prev = ch;
  }
  RF(c, prev, RF_MATE) = C; RF(c, prev, RF_ME) = ce_c;
  RF(c, C, RF_TPAR) = prev; RF(c, C, RF_MATE) = prev;
  // the remaining arc pairs up along the cycle
  const int rest = m - L - 1;
  for (int j = 1; j <= rest; j += 2) {
    const int ia = ((i_out + dir * j) % m + m) % m;
    const int ib = ((i_out + dir * (j + 1)) % m + m) % m;
    const int ca = uni(cyc[2 * ia]), cb = uni(cyc[2 * ib]);
    const int e = uni((dir == 1) ? cyc[2 * ia + 1] : cyc[2 * ib + 1]);
    RF(c, ca, RF_MATE) = cb; RF(c, ca, RF_ME) = e; RF(c, ca, RF_TID) = -1; RF(c, ca, RF_TPAR) = -1;
    RF(c, cb, RF_MATE) = ca; RF(c, cb, RF_ME) = e; RF(c, cb, RF_TID) = -1; RF(c, cb, RF_TPAR) = -1;
    set_rate(c, ca, 0); set_rate(c, cb, 0);
  }
  RF(c, B, RF_ALIVE) = 0;
  RF(c, B, RF_TID) = -1;
  const int nrel = uni(c.S->rel_n);
  for (int q = 0; q < nrel; ++q) refresh_star(c, uni(c.stk[q]));
}

// (e) an inner detector region shrinks to radius zero: its tree parent and
// child touch at its detection event and form a blossom with it.
PSB_DEV void implode(Ctx& c, int s) {
  const int P_ = uni(RF(c, s, RF_TPAR)), C = uni(RF(c, s, RF_MATE));
  if (P_ < 0 || C < 0) { c.status = S_INTERNAL; return; }
  const int e_c = uni(RF(c, s, RF_ME)), e_p = uni(RF(c, s, RF_TPE));
  const int ce = ce_concat(c, e_c, e_p, ce_other(c, e_c, s), ce_other(c, e_p, s));
  if (ce < 0) return;
  form_blossom(c, C, P_, ce);
}

// Growing region a (tree) touches region b (or the boundary when b < 0).
PSB_DEV void collide(Ctx& c, int a, int b, int ce) {
  const int ta = uni(RF(c, a, RF_TID));
  if (uni(RF(c, a, RF_RATE)) != 1 || ta < 0) { c.status = S_INTERNAL; return; }
  if (b < 0) {                                     // (f) tree hits boundary
    augment_to_root(c, a);
    RF(c, a, RF_MATE) = MATE_BOUNDARY; RF(c, a, RF_ME) = ce;
    dissolve_tree(c, ta);
    return;
  }
  const int rb = uni(RF(c, b, RF_RATE));
  if (rb == 1) {
    const int tb = uni(RF(c, b, RF_TID));
    if (tb == ta) { form_blossom(c, a, b, ce); return; }   // (c)
    augment_to_root(c, a);                                   // (b) tree hits tree
    augment_to_root(c, b);
    RF(c, a, RF_MATE) = b; RF(c, a, RF_ME) = ce;
    RF(c, b, RF_MATE) = a; RF(c, b, RF_ME) = ce;
    dissolve_tree(c, ta);
    dissolve_tree(c, tb);
    return;
  }
  if (rb != 0) { c.status = S_INTERNAL; return; }
#ifdef PSB_CHECK_INVARIANTS
  // Supplementary, unique touching of inherited matching configurations: a
  // configuration stopped at a lower level is touched by at most one
  // processing cluster of the running level
  if (c.acct && c.dbg_cfg[b] >= 0 && c.level[c.dbg_cfg[b]] < c.dbg_lvl) {
    const int owner = c.dbg_cfg[b], toucher = acct_cid(c)[ta];
    PSB_INVARIANT(c, !(c.dbg_touch_lvl[owner] == c.dbg_lvl && c.dbg_touch[owner] != toucher),
                  "an inherited configuration touched by two clusters of one level");
    c.dbg_touch[owner] = toucher; c.dbg_touch_lvl[owner] = c.dbg_lvl;
  }
#endif
  const int mb = uni(RF(c, b, RF_MATE));
  if (mb == MATE_BOUNDARY) {                                 // (g) tree hits boundary match
    augment_to_root(c, a);
    RF(c, a, RF_MATE) = b; RF(c, a, RF_ME) = ce;
    RF(c, b, RF_MATE) = a; RF(c, b, RF_ME) = ce;
    dissolve_tree(c, ta);
    return;
  }
  if (mb < 0) { c.status = S_INTERNAL; return; }
  // (a) tree hits match: b joins as inner, its partner as outer (GROW)
  RF(c, b, RF_TID) = ta; RF(c, b, RF_TPAR) = a; RF(c, b, RF_TPE) = ce;
  RF(c, mb, RF_TID) = ta; RF(c, mb, RF_TPAR) = b; RF(c, mb, RF_TPE) = RF(c, b, RF_ME);
  set_rate(c, b, -1);
  set_rate(c, mb, 1);
}

// ---------------------------------------------------------------------------
// flooder events
// ---------------------------------------------------------------------------
PSB_DEV void arrive(Ctx& c, int iu, int v, int e) {
  int k = node_idx_u(c, v);
  if (k >= 0 && k < c.nd) { c.status = S_INTERNAL; return; }   // an unseeded detection event was reached
  if (k < 0) { k = explore(c, v); if (k < 0) return; }
  const int a = uni(c.x_top[iu]);
  if (c.n_log >= c.P->lcap) { cap_fail(c); return; }
  const int rec = c.n_log++;
  c.lg[3 * rec] = v; c.lg[3 * rec + 1] = c.x_rec[iu]; c.lg[3 * rec + 2] = e;
  c.x_top[k] = a; c.x_reg[k] = a; c.x_src[k] = c.x_src[iu]; c.x_wr[k] = -yrad(c, a, c.now);
  c.x_rec[k] = rec;
  refresh_star(c, k);
}

PSB_DEV void leave(Ctx& c, int i) {
  c.x_top[i] = -1; c.x_reg[i] = -1; c.x_src[i] = -1; c.x_rec[i] = -1;
  refresh_star(c, i);
}

// Recompute the events of every node whose top region was marked changed.
PSB_DEV void flush_changes(Ctx& c) {
  if (c.n_chg > 0) {
    wave_sync();
    const int xn = uni(c.S->x_n);
    const int st = c.stamp;
#if PSB_WAVE > 1
    // compact the changed nodes into the change list, then evaluate them a
    // group of lanes per node
    int n = 0;
    for (int i0 = 0; i0 < xn; i0 += PSB_WAVE) {
      const int i = i0 + lane();
      int take = 0;
      if (i < xn) { const int t = c.x_top[i]; take = (t >= 0 && RF(c, t, RF_CHGM) == st) ? 1 : 0; }
      const uint64_t mask = ballot(take);
      if (take) c.chg[n + __builtin_popcountll(mask & lanemask_lt())] = i;
      n += __builtin_popcountll(mask);
    }
    wave_sync();
    const int G = slot_group(c), per = PSB_WAVE / G;
    for (int j0 = 0; j0 < n; j0 += per) {
      const int j = j0 + lane() / G;
      const int x = (j < n) ? c.chg[j] : -1;
      i128 tt; int k;
      node_event_group(c, x, G, tt, k);
      if (x >= 0 && (lane() & (G - 1)) == 0) set_event(c, x, tt);
    }
#else
    for (int i = 0; i < xn; ++i) {
      const int t = c.x_top[i];
      if (t < 0 || RF(c, t, RF_CHGM) != st) continue;
      i128 tt; int k;
      node_event(c, i, tt, k);
      set_event(c, i, tt);
    }
#endif
    wave_sync();
  }
  c.n_chg = 0;
  ++c.stamp;
}

PSB_DEV void node_event_apply(Ctx& c, int iu, int kind) {
  if (kind == K_LEAVE) { leave(c, iu); return; }
  const int deg = c.deg;
  const int64_t slot = (int64_t)uni(c.x_node[iu]) * deg + kind;
  const int v = uni(c.nbr[slot]);
  const int e = uni(c.eid[slot]);
  const int a = uni(c.x_top[iu]);
  if (v == NB_BOUNDARY) {
    const int ce = ce_leaf(c, e, c.x_rec[iu], -1, c.x_src[iu], -1);
    if (ce < 0) return;
    collide(c, a, -1, ce);
  } else {
    const int kv = kNbTable ? uni(c.x_nb[(int64_t)iu * deg + kind]) : node_idx_u(c, v);
    const int b = (kv >= 0) ? uni(c.x_top[kv]) : -1;
    if (b < 0) {
      arrive(c, iu, v, e);
    } else {
      int ce;
      if (uni(RF(c, a, RF_RATE)) >= uni(RF(c, b, RF_RATE))) {
        ce = ce_leaf(c, e, c.x_rec[iu], c.x_rec[kv], c.x_src[iu], c.x_src[kv]);
        if (ce < 0) return;
        collide(c, a, b, ce);
      } else {
        ce = ce_leaf(c, e, c.x_rec[kv], c.x_rec[iu], c.x_src[kv], c.x_src[iu]);
        if (ce < 0) return;
        collide(c, b, a, ce);
      }
    }
  }
  flush_changes(c);
}

// Run the dynamics until no alternating tree is left.
PSB_DEV void run_dynamics(Ctx& c) {
  const int64_t max_ev = c.P->max_events;
  for (;;) {
    if (c.status) return;
    if (++c.n_ev > max_ev) { c.status = S_INTERNAL; return; }
    i128 tn; int code;
    next_event(c, tn, code);
    if (tn >= T_INF) return;
    if (code < EV_NODE) {
      const int r = code;
      if (tn < c.now) { c.status = S_INTERNAL; return; }
      c.now = tn;
      if (c.acct) account_event(c, uni(RF(c, r, RF_TID)), tn);
      if (uni(RF(c, r, RF_BCN)) > 0) shatter(c, r); else implode(c, r);
      if (c.status) return;
      flush_changes(c);
      continue;
    }
    const int ix = code - EV_NODE;
#ifdef PSB_CHECK_INVARIANTS
    // Supplementary, persistent root: every alternating tree keeps a growing (outer) root
    for (int r = 0; r < c.n_regions; ++r)
      if (RF(c, r, RF_ALIVE) && RF(c, r, RF_BPAR) < 0 && RF(c, r, RF_TID) >= 0 && RF(c, r, RF_TPAR) < 0)
        PSB_INVARIANT(c, RF(c, r, RF_RATE) == 1, "a tree root that is not growing");
#endif
    i128 tf; int kf;
    node_event_u(c, ix, tf, kf);
    if (tf != tn) { wave_sync(); set_event(c, ix, tf); continue; }
    if (tf < c.now) { c.status = S_INTERNAL; return; }
    c.now = tf;
    if (c.acct) {
      // the event is driven by the tree of the node's region, or else (a
      // growing region reaching a frozen one) by the tree across the edge
      int tid = uni(RF(c, uni(c.x_top[ix]), RF_TID));
      if (tid < 0 && kf != K_LEAVE) {
        const int v = uni(c.nbr[(int64_t)uni(c.x_node[ix]) * c.deg + kf]);
        const int kv = v >= 0 ? node_idx_u(c, v) : -1;
        const int b = kv >= 0 ? uni(c.x_top[kv]) : -1;
        if (b >= 0) tid = uni(RF(c, b, RF_TID));
      }
      account_event(c, tid, tf);
    }
    node_event_apply(c, ix, kf);
  }
}

// ---------------------------------------------------------------------------
// syndrome intake: detection events become explored nodes 0..nd-1
// ---------------------------------------------------------------------------
PSB_DEV void load_defects(Ctx& c, const uint8_t* row) {
  const int nb = c.P->nbytes;
  const int lim = c.xcap < c.P->cap.dcap ? c.xcap : c.P->cap.dcap;
  int total = 0;
  // eight bytes per lane loaded before any is used; bytes are still taken in
  // ascending order, a wavefront-wide chunk at a time, skipping empty chunks
  constexpr int PER = 8;
  for (int b0 = 0; b0 < nb; b0 += PER * PSB_WAVE) {
    int bytes[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int i = b0 + u * PSB_WAVE + lane();
      bytes[u] = i < nb ? row[i] : 0;
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int i = b0 + u * PSB_WAVE + lane();
      const int byte = bytes[u];
      const int cnt = __builtin_popcount(byte);
      if (ballot(cnt != 0) == 0) continue;
      int pos = total + wave_prefix(cnt);
      for (int k = 0; k < 8; ++k) if (byte >> k & 1) {
        const int d = 8 * i + k;
        if (d < c.n_det && pos < lim) c.x_node[pos] = d;
        ++pos;
      }
      total += wave_sum(cnt);
    }
  }
  wave_sync();
  c.nd = total;
  if (total > lim) { cap_fail(c); return; }
  for (int i = lane(); i < total; i += PSB_WAVE) {
    c.x_top[i] = -1; c.x_reg[i] = -1; c.x_src[i] = -1; c.x_rec[i] = -1; c.x_wr[i] = 0; c.x_ev[i] = T_INF;
    c.level[i] = 0;
    hash_put_atomic(c, c.x_node[i], i);
  }
  wave_sync();
  // neighbour tables of the detection events (each other's entries included)
  // (a row's neighbours four at a time, their lookups issued together)
  for (int i = lane(); kNbTable && i < total; i += PSB_WAVE) {
    const int deg = c.deg;
    const int64_t row = (int64_t)c.x_node[i] * deg;
    for (int j0 = 0; j0 < deg; j0 += 4) {
      int nb4[4], k4[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) nb4[u] = j0 + u < deg ? c.nbr[row + j0 + u] : NB_PAD;
#pragma unroll
      for (int u = 0; u < 4; ++u) k4[u] = xnb_code(c, nb4[u]);
#pragma unroll
      for (int u = 0; u < 4; ++u) if (j0 + u < deg) c.x_nb[(int64_t)i * deg + j0 + u] = (int16_t)k4[u];
    }
  }
  wave_sync();
  c.S->x_n = total;
  wave_sync();
}

// ---------------------------------------------------------------------------
// processing-cluster hierarchy (Methods, Algorithm "Clustering")
// ---------------------------------------------------------------------------
PSB_DEV int uf_find(Ctx& c, int x) {
  while (true) { const int p = atom_load(&c.uf[x]); if (p == x) return x; x = p; }
}

PSB_DEV void uf_union(Ctx& c, int a, int b) {
  for (int guard = 0; guard < 1 << 20; ++guard) {
    a = uf_find(c, a); b = uf_find(c, b);
    if (a == b) return;
    if (a < b) { const int t = a; a = b; b = t; }
    if (atom_cas(&c.uf[a], a, b) == a) return;
  }
}

// Near lists of the clustering search (direct detector map only).  For a
// level's search every unresolved detection event i puts, for each adjacency
// slot j of its row that leads to a detector x, the entry i * deg + j on x's
// list: x's detector-map cell holds -2 - (head entry) while the search runs
// (-1 stays "no list"), and an event's own list head is ehead[i].  A path of
// the search whose last edge leaves detector x then reaches exactly the
// unresolved events on x's list (with the weight of that edge) and the
// boundary edges of x, so the last hop reads the list and, only if x has a
// boundary edge, x's row for its boundary slots.  Entries of one event never
// move; heads are swapped in with a compare-and-swap on the 32-bit word that
// holds the 16-bit cell.
PSB_DEV void near_push_cell(Ctx& c, int x, int e) {
  int16_t* cell = c.dmap + x;
  int* word = (int*)((uintptr_t)cell & ~(uintptr_t)3);
  const int sh = ((uintptr_t)cell & 2) ? 16 : 0;
  for (int guard = 0; guard < 1 << 20; ++guard) {
    const int old = atom_load(word);
    const int cur = (int)(int16_t)(uint16_t)((uint32_t)old >> sh);
    c.near[e].next = (int16_t)(cur <= -2 ? -2 - cur : -1);
    const uint32_t code = (uint32_t)(uint16_t)(int16_t)(-2 - e);
    const int nw = (int)(((uint32_t)old & ~(0xffffu << sh)) | (code << sh));
    if (atom_cas(word, old, nw) == old) return;
  }
}

// set = 1: builds the level's near lists (event heads already -1); set = 0:
// takes them out of the detector map again (before anything else reads it).
PSB_DEV void near_lists(Ctx& c, int set) {
  const int deg = c.deg;
  for (int i = lane(); i < c.nd; i += PSB_WAVE) {
    if (c.level[i] != 0) continue;
    const int64_t r0 = (int64_t)c.x_node[i] * deg;
    for (int j = 0; j < deg; ++j) {
      const int y = c.nbr[r0 + j];
      if (y == NB_PAD) break;
      if (y < 0) continue;
      if (!set) {
        if (c.dmap[y] <= -2) c.dmap[y] = -1;
        continue;
      }
      const int e = i * deg + j;
      c.near[e].widx = (int32_t)(r0 + j);
      c.near[e].ev = (int16_t)i;
      const int rj = c.dmap[y];
      if (rj >= 0) {
        c.near[e].next = (int16_t)atom_xchg((unsigned*)&c.ehead[rj], (unsigned)e);
      } else {
        near_push_cell(c, y, e);
      }
    }
  }
}

PSB_DEV bool has_boundary_edge(const Ctx& c, int x) { return (c.P->bndb[x >> 5] >> (x & 31)) & 1u; }

// Level of every detection event.  For each level k with b_k below the graph's
// diameter bound, the exploring region of radius b_k/2 around event u touches
// that of event v iff d(u, v) <= b_k; all such pairs are found by enumerating
// paths of at most H_k = floor(b_k / w_min) edges.  A component is accepted if
// every pair in it is within d_k (its diameter) and it has an even number of
// events or satisfies the boundary condition.  At the first level whose b_k
// exceeds the diameter bound, every remaining event is in the component of
// its connected part of the graph: these form the final clusters.  A level
// with a ball table (built with the decoder) reads each event's partners and
// boundary edges from it instead of walking the paths.
// DEEP, the deepest walk compiled in (the deeper ones hold registers that
// make the whole kernel spill more, so the host picks the least that the
// levels without a table need): 0 = paths of up to two edges; 1 = up to
// three, with near lists; 2 = the generic walk of up to MAXH edges as well.
template <int DEEP = 2>
PSB_DEV void cluster_levels(Ctx& c) {
  const int nd = c.nd;
  const int deg = c.deg;
  const int hitcap = c.P->hitcap, bdc = c.P->bdc;
  int32_t* close_cnt = c.cl_a;   // per event: close partners with larger index
  int32_t* bcount = c.cl_b;      // per event: boundary edges within d_k (loose flag in bit 30)
  int32_t* csize = c.cl_c;       // per root: size
  int32_t* cclose = c.cl_d;      // per root: close pairs
  for (int k = 0; k < c.P->n_levels; ++k) {
    int nres = 0;
    for (int i = lane(); i < nd; i += PSB_WAVE) nres += (c.level[i] == 0);
    nres = wave_sum(nres);
    if (nres == 0) return;
    const int H = uni(c.P->shmax[k]);
    if (H < 0) {
      // the final level: the remaining events form one processing cluster
      // (the detector graphs here are connected), rooted at the first of them
      int first = nd;
      for (int i = lane(); i < nd; i += PSB_WAVE) if (c.level[i] == 0 && i < first) first = i;
      first = -wave_max(-first);
      for (int i = lane(); i < nd; i += PSB_WAVE)
        if (c.level[i] == 0) { c.level[i] = (int8_t)(k + 1); c.cid[i] = first; if (c.acct) acct_cid(c)[i] = first; }
      wave_sync();
      return;
    }
    const i128 bk = uni128(c.P->sb[k]), dk = uni128(c.P->sd[k]);
    int visits = 0;
    // near lists pay from three edges on: shallower searches read each last
    // hop's row in chunks of independent loads, which is faster than a chain
    // of list entries
    const bool use_near = DEEP >= 1 && c.near && H >= 3;
    // the level's ball table, if the decoder built one (else it walks)
    const int bt = c.P->ball_slot ? uni(c.P->ball_slot[k]) : -1;
    for (int i = lane(); i < nd; i += PSB_WAVE) {
      c.uf[i] = i; close_cnt[i] = 0; bcount[i] = 0; csize[i] = 0; cclose[i] = 0;
      if (use_near) c.ehead[i] = -1;
    }
    if (use_near) {
      wave_sync();
      near_lists(c, 1);
    }
    wave_sync();
    for (int i = lane(); i < nd; i += PSB_WAVE) {
      if (c.level[i] != 0) continue;
      const int u = c.x_node[i];
      int32_t* hits = c.hit + (int64_t)(lane() % PSB_WAVE) * hitcap * 2;
      int nh = 0, nbd = 0, loose = 0, overflow = 0;
      int nvis = 0;
      // record one path of length nd_ from u ending at y (boundary: y < 0, edge e)
      // (rj_pre: the detector map's entry for y when already loaded, else -2)
      auto visit = [&](int y, int e, i128 nd_, int rj_pre = -2) {
        ++nvis;
        if (nd_ > bk) return;
        if (y == NB_BOUNDARY) {
          if (nd_ <= dk) {
            bool dup = false;
            for (int q = 0; q < nbd && q < bdc; ++q) dup |= (c.bdl[(int64_t)i * bdc + q] == e);
            if (!dup) { if (nbd < bdc) c.bdl[(int64_t)i * bdc + nbd] = e; ++nbd; }
          }
          if (2 * nd_ <= bk) loose = 1;
          return;
        }
        if (y == u) return;
        const int rj = rj_pre != -2 ? rj_pre : node_idx(c, y);
        if (rj >= 0 && rj < nd && c.level[rj] == 0) {
          const int cl = (nd_ <= dk) ? 1 : 0;
          int q = 0;
          for (; q < nh; ++q) if (hits[2 * q] == rj) { hits[2 * q + 1] |= cl; break; }
          if (q == nh) { if (nh < hitcap) { hits[2 * nh] = rj; hits[2 * nh + 1] = cl; ++nh; } else overflow = 1; }
        }
      };
      // the last hop of a path: the adjacency row of x (reached at distance
      // base) in chunks of four, each chunk's neighbours and their
      // detector-map entries loaded before any of them is visited (visit
      // order unchanged)
      // (hpre: x's detector-map cell when the caller has loaded it, else -3)
      auto leaf_row = [&](int x, i128 base, int hpre = -3) {
        const int64_t r0 = (int64_t)x * deg;
        if (use_near) {
          // the events next to x, from its near list, then x's boundary slots
          const int h = hpre != -3 ? hpre : c.dmap[x];
          int e = h >= 0 ? c.ehead[h] : (h <= -2 ? -2 - h : -1);
          while (e >= 0) {
            const NearEntry ne = c.near[e];
            e = ne.next;
            if (ne.ev == i) { ++nvis; continue; }
            visit(c.x_node[ne.ev], -1, base + c.wt[ne.widx], ne.ev);
          }
          if (!has_boundary_edge(c, x)) return;
          for (int k0 = 0; k0 < deg; ++k0) {
            const int z = c.nbr[r0 + k0];
            if (z == NB_PAD) return;
            if (z == NB_BOUNDARY) visit(NB_BOUNDARY, c.eid[r0 + k0], base + c.wt[r0 + k0]);
          }
          return;
        }
        for (int k0 = 0; k0 < deg; k0 += 4) {
          int zs[4], ix[4];
#pragma unroll
          for (int t = 0; t < 4; ++t) zs[t] = k0 + t < deg ? c.nbr[r0 + k0 + t] : NB_PAD;
#pragma unroll
          for (int t = 0; t < 4; ++t) ix[t] = (c.dmap && zs[t] >= 0) ? (int)c.dmap[zs[t]] : -2;
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            if (zs[t] == NB_PAD) return;
            visit(zs[t], c.eid[r0 + k0 + t], base + c.wt[r0 + k0 + t], ix[t]);
          }
        }
      };
      if (bt >= 0) {
        // the detectors and boundary edges that the level's paths reach, with
        // the flags their least distances decide; partners eight at a time, all
        // loads of a chunk issued before any of them is used
        const int32_t* row = c.P->ball_off + (int64_t)bt * (2 * (int64_t)c.n_det + 1) + 2 * (int64_t)u;
        const int a0 = row[0], a1 = row[1], a2 = row[2];
        const int32_t* ent = c.P->ball_ent;
        nvis += a2 - a0;
        for (int q0 = a0; q0 < a1; q0 += 8) {
          int ys[8], ix[8], lv[8];
#pragma unroll
          for (int t = 0; t < 8; ++t) ys[t] = q0 + t < a1 ? ent[q0 + t] : -1;
#pragma unroll
          for (int t = 0; t < 8; ++t) ix[t] = ys[t] >= 0 ? node_idx(c, ys[t] & BALL_ID) : -1;
#pragma unroll
          for (int t = 0; t < 8; ++t) lv[t] = (ix[t] >= 0 && ix[t] < nd) ? (int)c.level[ix[t]] : 1;
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            if (lv[t] != 0) continue;
            // the row's detectors are distinct: no partner repeats
            if (nh < hitcap) { hits[2 * nh] = ix[t]; hits[2 * nh + 1] = (ys[t] & BALL_CLOSE) ? 1 : 0; ++nh; }
            else overflow = 1;
          }
        }
        for (int q0 = a1; q0 < a2; ++q0) {
          const int v = ent[q0];
          if (v & BALL_LOOSE) loose = 1;
          if (v & BALL_CLOSE) { if (nbd < bdc) c.bdl[(int64_t)i * bdc + nbd] = v & BALL_ID; ++nbd; }
        }
      } else if (H <= (DEEP >= 1 ? 3 : 2)) {
        // up to three rounds of independent adjacency-row loads instead of a
        // serial walk over a stack in scratch memory
        if (H == 1) {
          leaf_row(u, 0);
        } else if (H >= 2) {
          for (int j = 0; j < deg; ++j) {
            const int y = c.nbr[(int64_t)u * deg + j];
            if (y == NB_PAD) break;
            const i128 d1 = c.wt[(int64_t)u * deg + j];
            visit(y, c.eid[(int64_t)u * deg + j], d1);
            if (y < 0 || d1 >= bk) continue;
            if (DEEP == 0 || H == 2) { leaf_row(y, d1); continue; }
            if (use_near) {
              // the second hop four neighbours at a time: their ids, detector-map
              // cells (event index, or near-list head) and weights are loaded
              // before any of them is visited (visit order unchanged); an edge
              // id is read only for a boundary slot
              const int64_t r1 = (int64_t)y * deg;
              for (int k0 = 0; k0 < deg; k0 += 4) {
                int zs[4], hs[4];
                i128 ds[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) zs[t] = k0 + t < deg ? c.nbr[r1 + k0 + t] : NB_PAD;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                  hs[t] = zs[t] >= 0 ? (int)c.dmap[zs[t]] : -1;
                  ds[t] = zs[t] != NB_PAD ? d1 + c.wt[r1 + k0 + t] : (i128)0;
                }
                bool end = false;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                  if (end || zs[t] == NB_PAD) { end = true; continue; }
                  visit(zs[t], zs[t] == NB_BOUNDARY ? c.eid[r1 + k0 + t] : -1, ds[t], hs[t] >= 0 ? hs[t] : -1);
                  if (zs[t] < 0 || ds[t] >= bk) continue;
                  leaf_row(zs[t], ds[t], hs[t]);
                }
                if (end) break;
              }
              continue;
            }
            for (int k2 = 0; k2 < deg; ++k2) {
              const int z = c.nbr[(int64_t)y * deg + k2];
              if (z == NB_PAD) break;
              const i128 d2 = d1 + c.wt[(int64_t)y * deg + k2];
              visit(z, c.eid[(int64_t)y * deg + k2], d2);
              if (z < 0 || d2 >= bk) continue;
              leaf_row(z, d2);
            }
          }
        }
      } else if constexpr (DEEP < 2) {
        overflow = 1;                    // never reached: the host builds deeper kernels for such graphs
        c.status = S_INTERNAL;
      } else {
        int st_node[MAXH + 1], st_slot[MAXH + 1];
        i128 st_dist[MAXH + 1];
        int dep = 0;
        st_node[0] = u; st_slot[0] = 0; st_dist[0] = 0;
        while (dep >= 0) {
          if (st_slot[dep] >= deg || dep >= H) { --dep; continue; }
          const int x = st_node[dep];
          if (dep == H - 1 && use_near) { leaf_row(x, st_dist[dep]); --dep; continue; }
          const int j = st_slot[dep]++;
          const int y = c.nbr[(int64_t)x * deg + j];
          if (y == NB_PAD) { st_slot[dep] = deg; continue; }
          const i128 nd_ = st_dist[dep] + c.wt[(int64_t)x * deg + j];
          visit(y, c.eid[(int64_t)x * deg + j], nd_);
          if (y < 0 || nd_ > bk) continue;
          if (dep + 1 < H) { ++dep; st_node[dep] = y; st_slot[dep] = 0; st_dist[dep] = nd_; }
        }
      }
      visits += nvis;
      int cc = 0;
      for (int q = 0; q < nh; ++q) {
        const int rj = hits[2 * q];
        uf_union(c, i, rj);
        if (rj > i && hits[2 * q + 1]) ++cc;
      }
      close_cnt[i] = overflow ? -(1 << 20) : cc;
      bcount[i] = (nbd > bdc ? bdc + 1 : nbd) | (loose << 30);
    }
    c.n_visit += wave_sum(visits);
    wave_sync();
    if (use_near) {
      near_lists(c, 0);
      wave_sync();
    }
    for (int i = lane(); i < nd; i += PSB_WAVE) {
      if (c.level[i] != 0) continue;
      const int r = uf_find(c, i);
      atom_add(&csize[r], 1);
      atom_add(&cclose[r], close_cnt[i]);
    }
    wave_sync();
    // acceptance, root by root
    for (int i = lane(); i < nd; i += PSB_WAVE) {
      if (c.level[i] != 0 || atom_load(&c.uf[i]) != i) continue;
      const int s = atom_load(&csize[i]);
      bool ok = (int64_t)atom_load(&cclose[i]) == (int64_t)s * (s - 1) / 2;
      if (ok && (s & 1)) {
        if (c.P->reading == 1) {
          int lo = 0;
          for (int j = 0; j < nd; ++j) if (c.level[j] == 0 && uf_find(c, j) == i) lo |= (bcount[j] >> 30) & 1;
          ok = lo != 0;
        } else if (s == 1) {
          ok = (bcount[i] & 0x3fffffff) > 0;
        } else {
          // some boundary edge (vertex) within d_k of every member
          bool any = false;
          const int nb0 = bcount[i] & 0x3fffffff;
          for (int q = 0; q < nb0 && q < bdc && !any; ++q) {
            const int e = c.bdl[(int64_t)i * bdc + q];
            bool all = true;
            for (int j = 0; j < nd && all; ++j) {
              if (c.level[j] != 0 || uf_find(c, j) != i || j == i) continue;
              const int nbj = bcount[j] & 0x3fffffff;
              bool has = false;
              for (int t2 = 0; t2 < nbj && t2 < bdc; ++t2) has |= (c.bdl[(int64_t)j * bdc + t2] == e);
              all = has;
            }
            any = all;
          }
          ok = any;
        }
      }
      atom_xchg((unsigned*)&csize[i], ok ? 0xffffffffu : 0u);   // reuse as accept flag
    }
    wave_sync();
    for (int i = lane(); i < nd; i += PSB_WAVE) {
      if (c.level[i] != 0) continue;
      const int r = uf_find(c, i);
      if (atom_load(&csize[r]) == -1) {
        c.level[i] = (int8_t)(k + 1);
        c.cid[i] = r;
        if (c.acct) acct_cid(c)[i] = r;
      }
    }
    wave_sync();
  }
}

// The clustering's union-find and per-root sizes use the two int32 region
// stamp arrays (in the state block: LDS on the wavefront tiers) instead of the
// workspace, so that its chains of atomics stay on chip: the stamps are not
// read before the dynamics, and the detection-event regions' stamps are set
// back to zero (region_init's value) afterwards.
template <int DEEP = 2>
PSB_DEV void cluster(Ctx& c) {
  int32_t* const uf_ws = c.uf;
  int32_t* const size_ws = c.cl_c;
  c.uf = &rf_ref<RF_MARK>(c, 0);
  c.cl_c = &rf_ref<RF_CHGM>(c, 0);
  wave_sync();
  cluster_levels<DEEP>(c);
  wave_sync();
  for (int i = lane(); i < c.nd; i += PSB_WAVE) { RF(c, i, RF_MARK) = 0; RF(c, i, RF_CHGM) = 0; }
  wave_sync();
  c.uf = uf_ws;
  c.cl_c = size_ws;
}

// ---------------------------------------------------------------------------
// fuse: terminal configuration -> edges, weight, observables
// ---------------------------------------------------------------------------
PSB_DEV void push_expand(Ctx& c, int region, int s) {
  if (uni(RF(c, region, RF_BCN)) == 0) return;
  const int n = uni(c.S->stk_n);
  if (n + 2 > c.P->stkcap) { c.status = S_CAPACITY; return; }
  c.stk[n] = region; c.stk[n + 1] = s;
  c.S->stk_n = n + 2;
}

PSB_DEV void add_fin(Ctx& c, int ce) {
  const int n = uni(c.S->fin_n);
  if (n >= c.P->fincap) { c.status = S_CAPACITY; return; }
  c.fin[n] = ce;
  c.S->fin_n = n + 1;
}

PSB_DEV void collect_final(Ctx& c) {
  c.S->fin_n = 0; c.S->stk_n = 0;
  wave_sync();
  int bad = 0;
  for (int r = lane(); r < c.n_regions; r += PSB_WAVE) {
    if (!RF(c, r, RF_ALIVE) || RF(c, r, RF_BPAR) >= 0) continue;
    const int mt = RF(c, r, RF_MATE);
    const int ce = RF(c, r, RF_ME);
    if (mt == -1 || ce < 0) { bad |= 1; continue; }
    if (mt != MATE_BOUNDARY && mt < r) continue;   // each pair once, from the smaller id
    const int k = atom_add(&c.S->fin_n, 1);
    if (k < c.P->fincap) c.fin[k] = ce; else bad |= 2;
    const int sa = CEF(c, ce, CE_SA), sb = CEF(c, ce, CE_SB);
    const int s_r = inside_lane(c, sa, r) ? sa : sb;
    if (RF(c, r, RF_BCN) > 0) {
      const int q = atom_add(&c.S->stk_n, 2);
      if (q + 2 <= c.P->stkcap) { c.stk[q] = r; c.stk[q + 1] = s_r; } else bad |= 2;
    }
    if (mt != MATE_BOUNDARY && RF(c, mt, RF_BCN) > 0) {
      const int q = atom_add(&c.S->stk_n, 2);
      if (q + 2 <= c.P->stkcap) { c.stk[q] = mt; c.stk[q + 1] = (s_r == sa ? sb : sa); } else bad |= 2;
    }
  }
  bad = wave_or(bad);
  wave_sync();
  if (bad & 1) { c.status = S_INFEASIBLE; return; }
  if (bad & 2) { c.status = S_CAPACITY; return; }
  for (;;) {
    const int n = uni(c.S->stk_n);
    if (n <= 0 || c.status) break;
    c.S->stk_n = n - 2;
    const int X = uni(c.stk[n - 2]), s = uni(c.stk[n - 1]);
    const int m = uni(RF(c, X, RF_BCN)), bo = uni(RF(c, X, RF_BCO));
    const int* cyc = c.bc + 2 * bo;
    const int ch = child_containing(c, s, X);
    int p = -1;
    for (int i = 0; i < m; ++i) if (uni(cyc[2 * i]) == ch) p = i;
    if (p < 0) { c.status = S_INTERNAL; return; }
    push_expand(c, ch, s);
    for (int j = 1; j < m; j += 2) {
      const int ia = (p + j) % m, ib = (p + j + 1) % m;
      const int ca = uni(cyc[2 * ia]), cb = uni(cyc[2 * ib]);
      const int ce = uni(cyc[2 * ia + 1]);
      add_fin(c, ce);
      const int sa = uni(CEF(c, ce, CE_SA)), sb = uni(CEF(c, ce, CE_SB));
      const bool a_has_sa = inside(c, sa, ca);
      push_expand(c, ca, a_has_sa ? sa : sb);
      push_expand(c, cb, a_has_sa ? sb : sa);
    }
  }
}

PSB_DEV void fuse_and_write(Ctx& c, int64_t shot) {
  collect_final(c);
  wave_sync();
  if (c.status) return;
  const int nf = uni(c.S->fin_n);
  // lane-parallel tracing; each lane flattens its compressed edges with a private stack
  int bad = 0;
  for (int i = lane(); i < nf; i += PSB_WAVE) {
    int* st = c.hit + (int64_t)(lane() % PSB_WAVE) * c.P->hitcap * 2;
    const int cap = c.P->hitcap * 2;
    int n = 0;
    st[n++] = c.fin[i];
    while (n > 0) {
      const int ce = st[--n];
      const int e = CEF(c, ce, CE_E);
      if (e >= 0) {
        atom_xor(&c.ebits[e >> 5], 1u << (e & 31));
        for (int side = 0; side < 2; ++side) {
          int rec = CEF(c, ce, side ? CE_B : CE_A), guard = 0;
          while (rec >= 0) {
            const int ee = c.lg[3 * rec + 2];
            if (ee >= 0) atom_xor(&c.ebits[ee >> 5], 1u << (ee & 31));
            rec = c.lg[3 * rec + 1];
            if (++guard > c.n_det + 1) { bad = 1; break; }
          }
        }
      } else {
        if (n + 2 > cap) { bad = 1; break; }
        st[n++] = CEF(c, ce, CE_A);
        st[n++] = CEF(c, ce, CE_B);
      }
    }
  }
  if (wave_or(bad)) c.status = S_INTERNAL;
  wave_sync();
  // scan the edge bitmap in ascending order (read-and-clear)
  const int64_t nwords = (c.P->n_edges + 31) / 32;
  int32_t* out = c.P->out_edges + shot * (int64_t)c.P->edge_stride;
  const int stride = c.P->edge_stride;
  int64_t wsum = 0; uint64_t ob = 0;
  int count = 0;
  for (int64_t w0 = 0; w0 < nwords; w0 += PSB_WAVE) {
    unsigned bits = 0;
    const int64_t wi = w0 + lane();
    if (wi < nwords) bits = atom_xchg(&c.ebits[wi], 0u);
    const int pc = __builtin_popcount(bits);
    int pos = count + wave_prefix(pc);
    for (int k = 0; k < 32; ++k) if (bits >> k & 1) {
      const int e = (int)(wi * 32 + k);
      if (pos < stride) out[pos] = e;
      ++pos; wsum += c.w[e]; ob ^= c.obs[e];
    }
    count += wave_sum(pc);
  }
  for (int m = PSB_WAVE / 2; m >= 1; m >>= 1) {
    const int lo = shfl_xor_i32((int)(uint32_t)(wsum & 0xffffffff), m);
    const int hi = shfl_xor_i32((int)(wsum >> 32), m);
    wsum += ((int64_t)hi << 32) | (uint32_t)lo;
    const int olo = shfl_xor_i32((int)(uint32_t)(ob & 0xffffffff), m);
    const int ohi = shfl_xor_i32((int)(ob >> 32), m);
    ob ^= ((uint64_t)(uint32_t)ohi << 32) | (uint32_t)olo;
  }
  if (c.status == S_OK && count > stride) c.status = S_TRUNC;
  // every lane holds the totals; all lanes store the same values
  c.P->out_nedges[shot] = count < stride ? count : stride;
  c.P->out_weight[shot] = wsum;
  c.P->out_obs[shot] = ob;
}

// ---------------------------------------------------------------------------
// level-1 clusters run concurrently (Methods, Algorithm "Parallel sparse
// blossom": the active clusters of a level execute in parallel), one lane per
// cluster, when the cluster's own dynamics is known to be a single event:
//  - two detection events whose joining edge e is lighter than twice every
//    other edge at either end: the two regions (radius t at time t, no
//    lower-level configuration exists yet) meet halfway, at t = W_e / 2,
//    before either could enter another detector or reach the boundary, and
//    the collision matches them (event (b)) and freezes both;
//  - one detection event whose lightest boundary edge b is lighter than
//    every other edge at it: the region meets the boundary at t = W_b first
//    (event (f)) and freezes.
// No other cluster can reach them before they stop (the clusters of a level
// are separated by more than b_1, and a level-1 cluster stops by d_1).  The
// pass leaves exactly the state the event loop would leave: radii, matches,
// one leaf compressed edge, empty event caches; its event is charged to the
// cluster.  Every other level-1 cluster stays in the event loop.
// ---------------------------------------------------------------------------
PSB_DEV void level_one_direct(Ctx& c) {
  const int nd = c.nd, deg = c.deg;
  int32_t* size = c.cl_c;      // per cluster root: level-1 members
  int32_t* other = c.cl_d;     // per cluster root: a member other than the root
  wave_sync();
  for (int i = lane(); i < nd; i += PSB_WAVE) { size[i] = 0; other[i] = -1; }
  wave_sync();
  for (int i = lane(); i < nd; i += PSB_WAVE) {
    if (c.level[i] != 1) continue;
    atom_add(&size[c.cid[i]], 1);
    if (c.cid[i] != i) atom_xchg((unsigned*)&other[c.cid[i]], (unsigned)i);
  }
  wave_sync();
  const int ce0 = c.n_ce;
  int n_new = 0;
  for (int i0 = 0; i0 < nd; i0 += PSB_WAVE) {
    const int r = i0 + lane();
    int kind = 0, v = -1, e = -1;     // kind 1: pair (r, v) through edge e; kind 2: boundary edge e
    i128 t = 0;
    if (r < nd && c.level[r] == 1 && c.cid[r] == r) {
      const int64_t ru = (int64_t)c.x_node[r] * deg;
      // the rows are read in chunks whose loads are all issued before any
      // value is tested (no early exit: every slot is checked)
      const int target = size[r] == 2 ? c.x_node[other[r]] : NB_BOUNDARY;
      int jm = -1;                     // lightest slot of r's row to the partner (or the boundary)
      i128 Wm = 0;
      if (size[r] == 1 || size[r] == 2) {
        for (int j0 = 0; j0 < deg; j0 += 4) {
          int nb4[4];
          i128 w4[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int j = j0 + u < deg ? j0 + u : deg - 1;
            nb4[u] = c.nbr[ru + j]; w4[u] = c.wt[ru + j];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (j0 + u < deg && nb4[u] == target && (jm < 0 || w4[u] < Wm)) { jm = j0 + u; Wm = w4[u]; }
        }
      }
      if (size[r] == 2 && jm >= 0) {
        // an adjacent pair meets halfway (at W/2) before either reaches
        // anything else: every other slot of both rows is heavier than W/2
        v = other[r];
        const int64_t rv = (int64_t)target * deg;
        const int em = c.eid[ru + jm];
        bool ok = true;
        for (int j0 = 0; j0 < deg; j0 += 2) {
          int na[2], nv[2], ev[2];
          i128 wa[2], wv[2];
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const int j = j0 + u < deg ? j0 + u : deg - 1;
            na[u] = c.nbr[ru + j]; wa[u] = c.wt[ru + j];
            nv[u] = c.nbr[rv + j]; wv[u] = c.wt[rv + j]; ev[u] = c.eid[rv + j];
          }
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            if (j0 + u >= deg) continue;
            if (j0 + u != jm && na[u] != NB_PAD && 2 * wa[u] <= Wm) ok = false;
            if (nv[u] != NB_PAD && ev[u] != em && 2 * wv[u] <= Wm) ok = false;
          }
        }
        if (ok) { kind = 1; e = em; t = Wm >> 1; }
      } else if (size[r] == 1 && jm >= 0) {
        // a lone event reaches its lightest boundary edge before any neighbour
        bool ok = true;
        for (int j0 = 0; j0 < deg; j0 += 4) {
          int nb4[4];
          i128 w4[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int j = j0 + u < deg ? j0 + u : deg - 1;
            nb4[u] = c.nbr[ru + j]; w4[u] = c.wt[ru + j];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (j0 + u < deg && nb4[u] >= 0 && w4[u] <= Wm) ok = false;
        }
        if (ok) { kind = 2; e = c.eid[ru + jm]; t = Wm; }
      }
    }
    const uint64_t mask = ballot(kind != 0);
    if (kind) {
      const int ce = ce0 + n_new + (int)__builtin_popcountll(mask & lanemask_lt());
      if (ce < c.P->cecap) {
        CEF(c, ce, CE_E) = e; CEF(c, ce, CE_A) = c.x_rec[r]; CEF(c, ce, CE_SA) = r;
        CEF(c, ce, CE_B) = kind == 1 ? c.x_rec[v] : -1; CEF(c, ce, CE_SB) = kind == 1 ? v : -1;
        c.r_base[r] = t; RF(c, r, RF_RATE) = 0; RF(c, r, RF_TID) = -1; RF(c, r, RF_TPAR) = -1;
        RF(c, r, RF_MATE) = kind == 1 ? v : MATE_BOUNDARY; RF(c, r, RF_ME) = ce;
        c.x_ev[r] = T_INF;
        if (kind == 1) {
          c.r_base[v] = t; RF(c, v, RF_RATE) = 0; RF(c, v, RF_TID) = -1; RF(c, v, RF_TPAR) = -1;
          RF(c, v, RF_MATE) = r; RF(c, v, RF_ME) = ce;
          c.x_ev[v] = T_INF;
        }
        if (c.acct) {
          // one event of cluster r at time t > 0 = t_<1
          acct_cnt(c)[r] = 1; acct_early_n(c)[r] = 0; acct_lastt(c)[r] = t;
        }
      }
    }
    n_new += (int)__builtin_popcountll(mask);
  }
  n_new = uni(n_new);
  wave_sync();
  if (ce0 + n_new > c.P->cecap) { cap_fail(c); return; }
  c.n_ce = ce0 + n_new;
  if (c.acct) acct_hdr(c)[0] = uni(acct_hdr(c)[0]) + n_new;
  wave_sync();
}

// ---------------------------------------------------------------------------
// one shot
// ---------------------------------------------------------------------------
PSB_DEV void seed_level(Ctx& c, int lvl) {
  // detector regions of this level start growing at t = 0 (one tree each)
  for (int i = lane(); i < c.nd; i += PSB_WAVE) {
    if (c.level[i] != lvl) continue;
    const int u = c.x_node[i];
    c.lg[3 * i] = u; c.lg[3 * i + 1] = -1; c.lg[3 * i + 2] = -1;
    c.x_top[i] = i; c.x_reg[i] = i; c.x_src[i] = i; c.x_wr[i] = 0; c.x_rec[i] = i;
    RF(c, i, RF_RATE) = 1; c.r_base[i] = 0; RF(c, i, RF_TID) = i;
  }
  wave_sync();
  for (int i = lane(); i < c.nd; i += PSB_WAVE) {
    if (c.level[i] != lvl) continue;
    i128 t; int k;
    node_event(c, i, t, k);
    set_event(c, i, t);
  }
  wave_sync();
}

// Clears the counters of the clusters of level lvl.
PSB_DEV void account_level_start(Ctx& c, int lvl) {
  wave_sync();
  for (int i = lane(); i < c.nd; i += PSB_WAVE) {
    if (c.level[i] != lvl) continue;
    acct_cnt(c)[i] = 0; acct_early_n(c)[i] = 0; acct_lastt(c)[i] = 0;
  }
  wave_sync();
}

// Rolls the clusters of level lvl into the critical path: for cluster C with
// stopping time s(C) (its last event) and E_C(t) events up to t,
//   t(C) = max(t_<k, s(C)),  E(C) = max(E_<k, E_C(t_<k)) + E_C(s(C)) - E_C(t_<k),
// then t_<k+1 and E_<k+1 are the maxima over the level's clusters.
PSB_DEV void account_level_end(Ctx& c, int lvl) {
  wave_sync();
  const i128 tlt = uni128(*acct_tlt(c));
  const int elt = uni(acct_hdr(c)[1]);
  i128 neg_t = -tlt; int arg = 0;
  int emax = elt, ncl = 0;
  for (int i = lane(); i < c.nd; i += PSB_WAVE) {
    if (c.level[i] != lvl || acct_cid(c)[i] != i) continue;
    const i128 sC = acct_lastt(c)[i];
    const int n = acct_cnt(c)[i], e = acct_early_n(c)[i];
    const i128 tC = sC > tlt ? sC : tlt;
    const int EC = (e > elt ? e : elt) + n - e;
    if (-tC < neg_t) neg_t = -tC;
    if (EC > emax) emax = EC;
    ++ncl;
  }
  wave_argmin(neg_t, arg);
  emax = wave_max(emax);
  ncl = wave_sum(ncl);
  wave_sync();
  *acct_tlt(c) = -neg_t;
  acct_hdr(c)[1] = emax;
  acct_hdr(c)[2] = uni(acct_hdr(c)[2]) + ncl;
  acct_hdr(c)[3] = lvl;
  wave_sync();
}

// Single-value outputs are stored by every lane with the same value: the
// persistent loop then has no lane-dependent branches.
PSB_DEV void write_empty(Ctx& c, int64_t shot, int status) {
  c.P->out_nedges[shot] = 0; c.P->out_weight[shot] = 0; c.P->out_obs[shot] = 0;
  c.P->out_status[shot] = status;
}

PSB_DEV void cleanup(Ctx& c, int64_t shot) {
  wave_sync();
  if (c.P->out_stats && c.status != S_OVERFLOW) {
    int32_t* st = c.P->out_stats + (int64_t)c.P->stats_stride * shot;
    if (c.acct) {
      // applied events, E_ideal, processing clusters, highest level (zeros for a shot without events)
      const bool ran = c.nd > 0 && (c.status == S_OK || c.status == S_TRUNC);
      for (int q = 0; q < 4; ++q) st[8 + q] = ran ? uni(acct_hdr(c)[q]) : 0;
    }
    const uint64_t t_end = dev_clock();
    st[0] = (int32_t)c.n_ev; st[1] = uni(c.S->x_n); st[2] = c.n_visit; st[3] = c.n_log;
    st[4] = (int32_t)(c.t_cl - c.t0); st[5] = (int32_t)(c.t_dyn - c.t_cl);
    st[6] = (int32_t)(c.t_fuse - c.t_dyn); st[7] = (int32_t)(t_end - c.t0);
  }
  // clear the hash slots of every explored node; a probe run that touched a
  // slot of one of them is cleared to its end so no stale key survives
  const int xn = uni(c.S->x_n);
  if (c.dmap) {
    for (int i = lane(); i < xn; i += PSB_WAVE) c.dmap[c.x_node[i]] = -1;
  } else if (4 * xn < (int)c.hmask) {
    for (int i = lane(); i < xn; i += PSB_WAVE) {
      uint32_t s = hpos(c, c.x_node[i]);
      for (uint32_t k = 0; k <= c.hmask; ++k) {
        if (c.h_key[s] == -1) break;
        c.h_key[s] = -3;                 // cleared below; keeps other runs intact meanwhile
        s = (s + 1) & c.hmask;
      }
    }
    wave_sync();
    for (int i = lane(); i < xn; i += PSB_WAVE) {
      uint32_t s = hpos(c, c.x_node[i]);
      for (uint32_t k = 0; k <= c.hmask; ++k) {
        if (c.h_key[s] == -1) break;
        c.h_key[s] = -1;
        s = (s + 1) & c.hmask;
      }
    }
  } else {
    for (uint32_t i = lane(); i <= c.hmask; i += PSB_WAVE) c.h_key[i] = -1;
  }
  const int64_t nwords = (c.P->n_edges + 31) / 32;
  if (c.status) for (int64_t i = lane(); i < nwords; i += PSB_WAVE) c.ebits[i] = 0;
  wave_sync();
  c.S->x_n = 0; c.S->fin_n = 0; c.S->stk_n = 0; c.S->rel_n = 0;
  wave_sync();
}

// Decodes one shot.  Returns the status; S_OVERFLOW means nothing was
// written and the shot must be decoded by the overflow tier.
template <int DEEP = 2>
PSB_DEV int decode_shot(Ctx& c, int64_t shot) {
#ifdef PSB_CHECK_INVARIANTS
  c.dbg_shot = shot; c.dbg_lvl = 0;
  for (int i = 0; i < c.rcap; ++i) c.dbg_cfg[i] = -1;
  for (int i = 0; i < c.P->cap.dcap; ++i) { c.dbg_touch[i] = -1; c.dbg_touch_lvl[i] = -1; }
#endif
  c.status = S_OK; c.n_ce = 0; c.n_bc = 0; c.n_shr = 0; c.n_chg = 0; c.stamp = 1; c.n_ev = 0;
  c.now = 0; c.n_visit = 0; c.nd = 0; c.n_log = 0; c.n_regions = 0;
  c.t0 = dev_clock(); c.t_cl = c.t0; c.t_dyn = c.t0; c.t_fuse = c.t0;
  const uint8_t* row = c.P->synd + shot * (int64_t)c.P->nbytes;
  load_defects(c, row);
  const int nd = c.nd;
  if (!c.status && nd > c.rcap) cap_fail(c);
  if (c.status || nd == 0) {
    const int st = c.status;
    if (st != S_OVERFLOW) write_empty(c, shot, st);
    cleanup(c, shot);
    return st;
  }
  c.n_regions = nd; c.n_log = nd;
  for (int i = lane(); i < nd; i += PSB_WAVE) region_init(c, i, 0, 0, -1);
  wave_sync();
  int max_level = 1;
  if (c.P->mode == 1) {
    for (int i = lane(); i < nd; i += PSB_WAVE) c.level[i] = 1;
    wave_sync();
  } else {
    cluster<DEEP>(c);
    int mx = 0, miss = 0;
    for (int i = lane(); i < nd; i += PSB_WAVE) { mx = c.level[i] > mx ? c.level[i] : mx; miss |= (c.level[i] == 0); }
    max_level = wave_max(mx);
    if (wave_or(miss)) c.status = S_INTERNAL;
  }
  c.t_cl = dev_clock();
  if (c.acct) {
    wave_sync();
    if (c.P->mode == 1) for (int i = lane(); i < nd; i += PSB_WAVE) acct_cid(c)[i] = 0;
    acct_hdr(c)[0] = 0; acct_hdr(c)[1] = 0; acct_hdr(c)[2] = 0; acct_hdr(c)[3] = 0;
    *acct_tlt(c) = 0;
    wave_sync();
  }
  for (int lvl = 1; lvl <= max_level && !c.status; ++lvl) {
    int present = 0;
    for (int i = lane(); i < nd; i += PSB_WAVE) present |= (c.level[i] == lvl);
    if (!wave_or(present)) continue;
    c.now = 0;       // every level starts its clock at zero; stopped regions are frozen
    if (c.acct) account_level_start(c, lvl);
    seed_level(c, lvl);
    if (lvl == 1 && c.P->mode == 0 && c.P->direct1) level_one_direct(c);
#ifdef PSB_CHECK_INVARIANTS
    c.dbg_lvl = lvl;
#endif
    run_dynamics(c);
#ifdef PSB_CHECK_INVARIANTS
    // Supplementary, stopping guarantee: below the final level a level-k
    // cluster has stopped by time d_k (its diameter bound)
    if (!c.status && c.P->shmax[lvl - 1] >= 0)
      PSB_INVARIANT(c, c.now <= c.P->sd[lvl - 1], "a cluster ran past d_k");
#endif
    if (c.acct && !c.status) account_level_end(c, lvl);
    if (!c.status) {
      int open = 0;
      for (int r = lane(); r < c.n_regions; r += PSB_WAVE)
        open |= (RF(c, r, RF_ALIVE) && RF(c, r, RF_BPAR) < 0 && RF(c, r, RF_TID) >= 0);
      if (wave_or(open)) c.status = S_INFEASIBLE;
    }
  }
  c.t_dyn = dev_clock(); c.t_fuse = c.t_dyn;
  if (c.status == S_OVERFLOW) { cleanup(c, shot); return S_OVERFLOW; }
  if (c.P->out_levels) {
    int8_t* lv = c.P->out_levels + shot * (int64_t)c.P->level_stride;
    const int nl = nd < c.P->level_stride ? nd : c.P->level_stride;
    for (int i = lane(); i < nl; i += PSB_WAVE) lv[i] = (c.P->mode == 1) ? 0 : c.level[i];
  }
  if (!c.status) {
    fuse_and_write(c, shot);
    c.t_fuse = dev_clock();
  }
  if (c.status == S_OVERFLOW) { cleanup(c, shot); return S_OVERFLOW; }
  if (c.status && c.status != S_TRUNC) write_empty(c, shot, c.status);
  else c.P->out_status[shot] = c.status;
  const int st = c.status;
  cleanup(c, shot);
  return st;
}

// Per-shot state pointers (base = LDS block or the slot's global state block)
// and global pool pointers of slot `slot`.
PSB_DEV void ctx_init(Ctx& c, const Params* P, Lds* S, char* state, int64_t slot) {
  c.P = P; c.S = S;
  c.nbr = P->nbr; c.eid = P->eid; c.wt = P->wt; c.w = P->w; c.obs = P->obs;
  c.deg = P->deg; c.n_det = P->n_det;
  c.rcap = P->cap.rcap; c.xcap = P->cap.xcap;
  c.hmask = P->cap.hcap > 0 ? (uint32_t)P->cap.hcap - 1 : 0;
  int lg = 0; while ((1 << lg) < P->cap.hcap) ++lg;
  c.hshift = 32 - lg;
  const StateLayout& SL = P->SL;
  c.x_node = (int32_t*)(state + SL.x_node); c.x_top = (int16_t*)(state + SL.x_top);
  c.x_reg = (int16_t*)(state + SL.x_reg); c.x_src = (int16_t*)(state + SL.x_src);
  c.x_rec = (int16_t*)(state + SL.x_rec);
  c.h_key = (int32_t*)(state + SL.h_key); c.h_val = (int32_t*)(state + SL.h_val);
  char* base = P->ws + slot * P->L.total;
  const WsLayout& L = P->L;
  c.x_ev = SL.x_ev >= 0 ? (i128*)(state + SL.x_ev) : (i128*)(base + L.x_ev);
  c.x_wr = SL.x_wr >= 0 ? (i128*)(state + SL.x_wr) : (i128*)(base + L.x_wr);
  c.r_base = SL.r_base >= 0 ? (i128*)(state + SL.r_base) : (i128*)(base + L.r_base);
  c.r_f16 = (int16_t*)(state + SL.r_f16); c.r_f32 = (int32_t*)(state + SL.r_f32);
  c.ce = (int32_t*)(base + L.ce); c.bc = (int32_t*)(base + L.bc); c.lg = (int32_t*)(base + L.lg);
  c.level = (int8_t*)(base + L.level);
  c.uf = (int32_t*)(base + L.uf); c.cl_a = (int32_t*)(base + L.cl_a); c.cl_b = (int32_t*)(base + L.cl_b);
  c.cl_c = (int32_t*)(base + L.cl_c); c.cl_d = (int32_t*)(base + L.cl_d);
  c.cid = (int32_t*)(base + L.cid);
  c.near = P->near_on ? (NearEntry*)(base + L.near) : nullptr;
  c.ehead = (int32_t*)(base + L.ehead);
  c.bdl = (int32_t*)(base + L.bdl); c.hit = (int32_t*)(base + L.hit);
  c.shr = (int32_t*)(base + L.shr); c.chg = (int32_t*)(base + L.chg); c.stk = (int32_t*)(base + L.stk);
  c.fin = (int32_t*)(base + L.fin); c.ebits = (uint32_t*)(base + L.ebits);
  c.dmap = P->cap.hcap == 0 ? (int16_t*)(base + L.dmap) : nullptr;
  c.x_nb = L.x_nb >= 0 ? (int16_t*)(base + L.x_nb) : nullptr;
  c.acct = (P->eacct && P->out_stats) ? base + L.acct : nullptr;
}

// Fresh state block: empty detector map or hash, zero scalars.
PSB_DEV void state_init(Ctx& c) {
  if (c.dmap) {
    for (int i = lane(); i < c.n_det; i += PSB_WAVE) c.dmap[i] = -1;
  } else {
    for (uint32_t i = lane(); i <= c.hmask; i += PSB_WAVE) c.h_key[i] = -1;
  }
  c.S->x_n = 0; c.S->fin_n = 0; c.S->stk_n = 0; c.S->rel_n = 0;
  wave_sync();
}

}  // namespace PSB_ENGINE_NS
}  // namespace psb
