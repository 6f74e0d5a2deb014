// Plain-data structures shared by the host library and the device engine.
#pragma once
#include <stdint.h>

namespace psb {

constexpr int K_NONE = -1;
constexpr int K_LEAVE = 1000;
constexpr int NB_BOUNDARY = -1;
constexpr int NB_PAD = -2;
// Neighbour-table codes of an adjacency slot without an explored neighbour.
constexpr int XNB_NONE = -1, XNB_BOUNDARY = -2, XNB_PAD = -3;
constexpr int MATE_BOUNDARY = -2;
// Deepest path walk of the clustering search.  The hop bound floor(b_k/w_min)
// assumes every edge is the lightest; the walk itself is cut by distance, so
// even graphs whose light edges allow 7-9 hops (timelike q = 0.2 against
// spatial p = 0.001-0.005) walk only a few hundred paths per event.
constexpr int MAXH = 16;
// Ball-table entry flags: within d_k of the detector (a close partner, or a
// boundary edge for the boundary condition), within b_k / 2 (a boundary edge
// for the loose reading); the id sits in the low 29 bits.
constexpr int BALL_CLOSE = 1 << 30, BALL_LOOSE = 1 << 29, BALL_ID = (1 << 29) - 1;
constexpr int S_OK = 0, S_CAPACITY = 1, S_INFEASIBLE = 2, S_TRUNC = 3, S_INTERNAL = 4, S_OVERFLOW = 5;

// Byte offsets of the per-shot state that the event loop touches on every
// event.  For the wavefront tiers the block lives in LDS; for the lane tier
// (one shot per lane) it lives in the lane's global workspace slot.
struct StateLayout {
  int64_t x_node;                                // explored nodes [xcap]: detector id, int32
  int64_t x_top, x_reg, x_src, x_rec;            // [xcap], int16 (region, region, event, log record)
  int64_t x_wr, x_ev;                            // [xcap], int128 (x_ev -1: in the workspace)
  int64_t h_key, h_val;                          // detector -> explored index hash [hcap], int32 (hcap 0:
                                                 // the direct map of the workspace is used instead)
  int64_t r_base, r_f16, r_f32;                  // regions: base [rcap] int128 (-1: in the workspace),
                                                 // fields [RF_N16][rcap] int16
                                                 // and [RF_COUNT - RF_N16][rcap] int32
  int64_t total;
};

// Byte offsets of the per-slot global workspace (pools touched per matcher
// event or once per shot).
struct WsLayout {
  int64_t state;                                 // lane tier, or a wavefront tier with Params::state_ws: Lds
                                                 // header + StateLayout block; else unused
  int64_t ce, bc, lg;                            // compressed edges, blossom cycles, arrival log
  int64_t level, uf, cl_a, cl_b, cl_c, cl_d, bdl, hit;   // clustering
  int64_t cid;                                   // processing cluster of each detection event (its root event)
  int64_t shr, chg, stk, fin, ebits;             // scratch lists, edge bitmap
  int64_t dmap;                                  // detector -> explored index [n_det] int16, -1 absent
                                                 // (only when the state block has no hash)
  int64_t x_ev, r_base, x_wr;                    // event cache, region bases, radius offsets, when the state block
                                                 // leaves them out (else unused)
  int64_t x_nb;                                  // [xcap][deg] int16: explored index of each adjacency slot's
                                                 // neighbour (XNB_* codes when it has none); -1: no table
  int64_t acct;                                  // per-cluster event accounting block (event_accounting only)
  int64_t near, ehead;                           // clustering search, direct detector map only: near-list
                                                 // entries [dcap*deg] (NearEntry) and the list head of each
                                                 // detection event [dcap] int32 (-1 empty)
  int64_t total;                                 // bytes per slot (multiple of 256)
};

// Region int-field indices (structure of arrays: field * rcap + region).
enum RegionField {
  RF_RATE = 0,   // +1 growing (outer), 0 frozen, -1 shrinking (inner)
  RF_BPAR,       // blossom parent, -1 if top level
  RF_TPAR,       // alternating-tree parent (top-level region), -1 for roots / no tree
  RF_TPE,        // compressed edge to the tree parent
  RF_TID,        // tree id (root detection event), -1 if not in a tree
  RF_MATE,       // matched region, -2 boundary, -1 none
  RF_ME,         // compressed edge of the match
  RF_BCO,        // blossom cycle offset into the cycle pool
  RF_BCN,        // blossom cycle length (0 = detector region)
  RF_ALIVE,
  RF_INSHR,      // present in the shrinking-region list
  RF_N16,        // fields above are int16, fields below int32
  RF_MARK = RF_N16,   // scratch stamp
  RF_CHGM,       // change-list stamp
  RF_COUNT
};

// Compressed-edge fields ([cecap][CE_COUNT]).
// Leaf: e >= 0 is a graph edge joining the nodes of arrival records a and b
// (b = -1 for a boundary edge).  Internal (e == -1): concatenation of the
// compressed edges a and b.  sa/sb: the detection events (defect indices) at
// the two ends, -1 for the boundary.
enum CeField { CE_E = 0, CE_A, CE_B, CE_SA, CE_SB, CE_COUNT };

// Event-accounting block of a slot (dcap = d): a header (applied events,
// critical-path event count so far, processing clusters, highest level), the
// critical-path stopping time so far, then per detection event: its
// processing cluster (the cluster's root event), and per cluster root: event
// count, events up to the lower levels' critical-path time, last event time.
constexpr int64_t ACCT_TLT = 16, ACCT_CID = 32;
constexpr int64_t acct_n(int64_t d) { return ACCT_CID + 4 * d; }
constexpr int64_t acct_early(int64_t d) { return ACCT_CID + 8 * d; }
constexpr int64_t acct_last(int64_t d) { return (ACCT_CID + 12 * d + 15) & ~(int64_t)15; }
constexpr int64_t acct_bytes(int64_t d) { return acct_last(d) + 16 * d; }

// Near-list entry of the clustering search: the adjacency slot (row * deg +
// slot, so the weight is wt[widx]) joining a detector to the unresolved
// detection event ev, and the next entry of the detector's list (-1 ends it).
struct NearEntry {
  int32_t widx;
  int16_t ev, next;
};

struct Caps {
  int32_t xcap, hcap, rcap, dcap;                // explored nodes, hash slots (power of 2), regions, events
};

struct Params {
  // graph (device pointers)
  int32_t n_det, deg, nbytes;
  int32_t state_ws;       // wavefront tier: the Lds header and state block sit in the slot's workspace (at L.state)
  int64_t n_edges;
  const int32_t* nbr;     // [n_det*deg]: neighbour detector, -1 boundary, -2 padding
  const int32_t* eid;     // [n_det*deg]: edge id
  const __int128* wt;     // [n_det*deg]: tie-broken even weight of each adjacency slot
  const int32_t* w;       // [n_edges]: caller weights
  const uint64_t* obs;    // [n_edges]
  const uint32_t* bndb;   // [ceil(n_det/32)]: detector has a boundary edge
  // schedule
  int32_t n_levels, reading, mode, tier;         // tier: 0 first tier (wave or lane), 1 overflow tier
  const __int128* sd;     // [n_levels] d_k
  const __int128* sb;     // [n_levels] b_k
  const int32_t* shmax;   // [n_levels] path-enumeration depth, -1 = final level
  // ball tables of the clustering levels (those that have one): level k
  // reads table ball_slot[k] (-1: it walks its paths), whose row for detector
  // u is ball_ent[off[2u] .. off[2u+1]) = the detectors within b_k of u, then
  // [off[2u+1] .. off[2u+2]) = the boundary edges that matter (off = ball_off +
  // table * (2 n_det + 1)); flags in the high bits of each entry (BALL_*)
  const int32_t* ball_slot;
  const int32_t* ball_off;
  const int32_t* ball_ent;
  // capacities (this tier)
  Caps cap;
  int32_t cecap, bccap, lcap, shrcap, stkcap, fincap, hitcap, bdc;
  int64_t max_events;
  int32_t direct1;                               // level-1 clusters of one known event applied directly
  int32_t near_on;                               // clustering search ends paths through near lists (needs the
                                                 // direct detector map and dcap*deg <= 32766)
  // batch
  int64_t n_shots;
  const uint8_t* synd;
  int32_t* out_edges;
  int32_t edge_stride, stats_stride;             // stats_stride: 8, or 12 with event accounting
  int32_t* out_nedges;
  int64_t* out_weight;
  uint64_t* out_obs;
  int32_t* out_status;
  int8_t* out_levels;
  int32_t level_stride, eacct;                   // eacct: per-cluster event accounting on
  uint64_t* out_tdone;
  int32_t* out_stats;     // [n][stats_stride] or null
  int32_t* counter;       // [0] first-tier work head, [1] overflow count, [2] overflow head
  int32_t* ovf_list;      // [n_shots] shots handed to the overflow tier
  const int32_t* order;   // [n_shots] the order in which the first tier takes shots (null: 0, 1, 2, ...)
  // workspace
  char* ws;
  WsLayout L;
  StateLayout SL;
};

}  // namespace psb
