// Plain-data structures shared by the host library and the device engine.
#pragma once
#include <stdint.h>

namespace psb {

// Byte offsets of the per-slot workspace arrays (one slot = one shot in flight).
struct WsLayout {
  // per detector [n_det]
  int64_t n_top, n_reg, n_src, n_eix, n_rec, n_pos, n_did, n_wr;
  // explored-node event cache [n_det] and its block minima [n_blk]
  int64_t x_node, x_ev, blk_min, blk_arg;
  // regions [rcap]: radius base (i128) and int fields [RF_COUNT][rcap]
  int64_t r_base, r_f;
  // shell chunks [ckcap] (+ 64 node ids each)
  int64_t ck_next, ck_prev, ck_nodes;
  // compressed edges [cecap][CE_COUNT], blossom cycles [bccap][2], arrival log [lcap][3]
  int64_t ce, bc, lg;
  // defects and clustering [dcap]
  int64_t defects, level, uf, cl_a, cl_b, cl_c, cl_d, bdl, hit;
  // scratch lists
  int64_t shr, chg, stk, fin, ebits;
  int64_t total;  // bytes per slot (multiple of 256)
};

// Region int-field indices (structure of arrays: field * rcap + region).
enum RegionField {
  RF_RATE = 0,   // +1 growing (outer), 0 frozen, -1 shrinking (inner)
  RF_BPAR,       // blossom parent, -1 if top level
  RF_TPAR,       // alternating-tree parent (top-level region), -1 for roots / no tree
  RF_TPE,        // compressed edge to the tree parent
  RF_TID,        // tree id (root detector region), -1 if not in a tree
  RF_MATE,       // matched region, -2 boundary, -1 none
  RF_ME,         // compressed edge of the match
  RF_BCO,        // blossom cycle offset into the cycle pool
  RF_BCN,        // blossom cycle length (0 = detector region)
  RF_ALIVE,
  RF_CKH,        // shell: first chunk
  RF_CKT,        // shell: last chunk
  RF_CNT,        // shell: number of nodes
  RF_MARK,       // scratch stamp
  RF_INSHR,      // present in the shrinking-region list
  RF_CHGM,       // change-list stamp
  RF_COUNT
};

// Compressed-edge fields ([cecap][CE_COUNT]).
// Leaf: e >= 0 is a graph edge joining the nodes of arrival records a and b
// (b = -1 for a boundary edge).  Internal (e == -1): concatenation of the
// compressed edges a and b.  sa/sb: the detection events (defect indices) at
// the two ends, -1 for the boundary.
enum CeField { CE_E = 0, CE_A, CE_B, CE_SA, CE_SB, CE_COUNT };

struct Params {
  // graph (device pointers)
  int32_t n_det, deg, nbytes, pad0;
  int64_t n_edges;
  const int32_t* nbr;     // [n_det*deg]: neighbour detector, -1 boundary, -2 padding
  const int32_t* eid;     // [n_det*deg]: edge id
  const __int128* wt;     // [n_edges]: tie-broken even weights
  const int32_t* w;       // [n_edges]: caller weights
  const uint64_t* obs;    // [n_edges]
  // schedule
  int32_t n_levels, reading, mode, pad1;
  const __int128* sd;     // [n_levels] d_k
  const __int128* sb;     // [n_levels] b_k
  const int32_t* shmax;   // [n_levels] path-enumeration depth, -1 = final level
  // capacities
  int32_t dcap, rcap, cecap, bccap, lcap, ckcap, shrcap, stkcap, fincap, hitcap, bdc, pad2;
  int64_t max_events;
  // batch
  int64_t n_shots;
  const uint8_t* synd;
  int32_t* out_edges;
  int32_t edge_stride, pad3;
  int32_t* out_nedges;
  int64_t* out_weight;
  uint64_t* out_obs;
  int32_t* out_status;
  int8_t* out_levels;
  uint64_t* out_tdone;
  int32_t* out_stats;     // [n][4] or null
  int32_t* counter;       // work queue head
  // workspace
  char* ws;
  WsLayout L;
};

}  // namespace psb
