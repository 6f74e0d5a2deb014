// Host-side setup shared by the HIP library and tooling: exact level
// schedule (big-integer rationals), tie-broken weights, diameter bound and
// the per-slot workspace layout.  Plain C++ (no HIP).
#pragma once
#include <stdint.h>
#include <algorithm>
#include <queue>
#include <string>
#include <vector>

#include "../../include/psb.h"
#include "psb_types.h"

namespace psb_host {
typedef unsigned __int128 u128;
using psb::WsLayout;
using psb::Params;

// Provided by the including translation unit.
int32_t fail(int32_t code, const std::string& msg);

// Graph topology in fixed-width adjacency form.
struct Ell {
  int32_t n_det = 0, deg = 0;
  int64_t n_edges = 0;
  std::vector<int32_t> nbr, eid;
};

// ---------------------------------------------------------------------------
// exact level schedule (Methods, Algorithm "Parameter schedule"), unsigned
// big integers so that the rationals phi_k are handled without rounding
// ---------------------------------------------------------------------------
struct Big {
  std::vector<uint32_t> d;  // little endian, no leading zeros
  static Big of(u128 x) { Big b; while (x) { b.d.push_back((uint32_t)x); x >>= 32; } return b; }
  void trim() { while (!d.empty() && d.back() == 0) d.pop_back(); }
};
static Big badd(const Big& a, const Big& b) {
  Big r; r.d.resize(std::max(a.d.size(), b.d.size()) + 1, 0);
  uint64_t carry = 0;
  for (size_t i = 0; i < r.d.size(); ++i) {
    uint64_t s = carry + (i < a.d.size() ? a.d[i] : 0) + (i < b.d.size() ? b.d[i] : 0);
    r.d[i] = (uint32_t)s; carry = s >> 32;
  }
  r.trim(); return r;
}
static Big bsub(const Big& a, const Big& b) {   // requires a >= b
  Big r; r.d.resize(a.d.size(), 0);
  int64_t borrow = 0;
  for (size_t i = 0; i < a.d.size(); ++i) {
    int64_t s = (int64_t)a.d[i] - borrow - (i < b.d.size() ? b.d[i] : 0);
    borrow = s < 0; if (s < 0) s += (1LL << 32);
    r.d[i] = (uint32_t)s;
  }
  r.trim(); return r;
}
static Big bmul(const Big& a, const Big& b) {
  Big r; if (a.d.empty() || b.d.empty()) return r;
  std::vector<uint64_t> t(a.d.size() + b.d.size() + 1, 0);
  for (size_t i = 0; i < a.d.size(); ++i) {
    uint64_t carry = 0;
    for (size_t j = 0; j < b.d.size(); ++j) {
      uint64_t cur = t[i + j] + (uint64_t)a.d[i] * b.d[j] + carry;
      t[i + j] = cur & 0xffffffffu; carry = cur >> 32;
    }
    size_t k = i + b.d.size();
    while (carry) { uint64_t cur = t[k] + carry; t[k] = cur & 0xffffffffu; carry = cur >> 32; ++k; }
  }
  r.d.resize(t.size()); for (size_t i = 0; i < t.size(); ++i) r.d[i] = (uint32_t)t[i];
  r.trim(); return r;
}
static int bcmp(const Big& a, const Big& b) {
  if (a.d.size() != b.d.size()) return a.d.size() < b.d.size() ? -1 : 1;
  for (size_t i = a.d.size(); i-- > 0;) if (a.d[i] != b.d[i]) return a.d[i] < b.d[i] ? -1 : 1;
  return 0;
}

struct LevelSchedule { std::vector<u128> d, b; std::vector<int> final_level; };

// phi = n/m; target = P/Q; admissibility of an integer b (Algorithm "Parameter schedule"):
// b >= d, phi > 2 d / b, Phi_{k+1}(b) = phi - (phi+2) d / ((phi+1) d + phi b) >= target.
static bool admissible(u128 b, u128 d, const Big& n, const Big& m, const Big& P, const Big& Q) {
  if (b < d) return false;
  const Big B = Big::of(b), D_ = Big::of(d);
  if (bcmp(bmul(n, B), bmul(Big::of(2), bmul(D_, m))) <= 0) return false;
  const Big Dn = badd(bmul(badd(n, m), D_), bmul(n, B));               // (n+m) d + n b
  const Big lhs = bmul(bmul(n, Dn), Q);
  const Big rhs = badd(bmul(bmul(P, m), Dn), bmul(bmul(m, badd(n, bmul(Big::of(2), m))), bmul(D_, Q)));
  return bcmp(lhs, rhs) >= 0;
}

static int32_t build_schedule(u128 wmax, u128 diam, int64_t qn, int64_t qd, int64_t pn, int64_t pd,
                              LevelSchedule& out) {
  const u128 LIM = ((u128)1) << 123;
  u128 d = wmax + 1;
  Big n = Big::of(1), m = Big::of(1);
  Big qn_pow = Big::of(1), qd_pow = Big::of(1);
  for (int k = 1; k <= 32; ++k) {
    qn_pow = bmul(qn_pow, Big::of((u128)qn)); qd_pow = bmul(qd_pow, Big::of((u128)qd));
    // target phi_bar_{k+1} = phi_min + (1 - phi_min) q^k = [pn qd^k + (pd - pn) qn^k] / (pd qd^k)
    const Big P = badd(bmul(Big::of((u128)pn), qd_pow), bmul(Big::of((u128)(pd - pn)), qn_pow));
    const Big Q = bmul(Big::of((u128)pd), qd_pow);
    u128 b;
    if (admissible(d, d, n, m, P, Q)) b = d;
    else {
      u128 lo = d, hi = d * 2;
      while (!admissible(hi, d, n, m, P, Q)) {
        if (hi > LIM) return fail(PSB_E_UNSUPPORTED, "level parameters exceed 2^123");
        lo = hi; hi *= 2;
      }
      while (hi - lo > 1) { u128 mid = lo + (hi - lo) / 2; if (admissible(mid, d, n, m, P, Q)) hi = mid; else lo = mid; }
      b = hi;
    }
    out.d.push_back(d); out.b.push_back(b);
    const bool fin = b >= diam;
    out.final_level.push_back(fin ? 1 : 0);
    if (fin) return PSB_OK;
    // phi_{k+1} = (n Dn - m (n + 2m) d) / (m Dn)
    const Big D_ = Big::of(d), B = Big::of(b);
    const Big Dn = badd(bmul(badd(n, m), D_), bmul(n, B));
    const Big num = bsub(bmul(n, Dn), bmul(bmul(m, badd(n, bmul(Big::of(2), m))), D_));
    const Big den = bmul(m, Dn);
    n = num; m = den;
    const u128 dn = 3 * d + 4 * b + 2 * wmax;
    if (dn > LIM) return fail(PSB_E_UNSUPPORTED, "level parameters exceed 2^123");
    d = dn;
  }
  return fail(PSB_E_UNSUPPORTED, "schedule did not reach the graph diameter within 32 levels");
}

static uint64_t lib_splitmix(uint64_t seed, uint64_t k) {
  uint64_t z = seed + k * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// Upper bound on the tie-broken distance between any two vertices (detectors
// or boundary vertices) of one connected component: twice the eccentricity
// of a detector plus the heaviest edge, maximised over components.
static u128 diameter_bound(const Ell* g, const std::vector<__int128>& wt) {
  const int32_t n = g->n_det, deg = g->deg;
  std::vector<__int128> dist(n, -1);
  __int128 wmax = 0;
  for (auto x : wt) wmax = std::max(wmax, x);
  __int128 best = 0;
  typedef std::pair<__int128, int32_t> item;
  for (int32_t s = 0; s < n; ++s) {
    if (dist[s] >= 0) continue;
    std::priority_queue<item, std::vector<item>, std::greater<item>> pq;
    dist[s] = 0; pq.push({0, s});
    __int128 ecc = 0;
    while (!pq.empty()) {
      auto [dd, x] = pq.top(); pq.pop();
      if (dd != dist[x]) continue;
      ecc = std::max(ecc, dd);
      for (int j = 0; j < deg; ++j) {
        const int32_t y = g->nbr[(size_t)x * deg + j];
        if (y < 0) continue;
        const __int128 nd = dd + wt[g->eid[(size_t)x * deg + j]];
        if (dist[y] < 0 || nd < dist[y]) { dist[y] = nd; pq.push({nd, y}); }
      }
    }
    best = std::max(best, 2 * (ecc + wmax));
  }
  return (u128)best;
}

static int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }


// Tie-broken even weights wt(e) = 2 w(e) 2^64 + 2 h(e), h = SplitMix64 output (e+1) >> 24.
static void tiebroken_weights(const int32_t* w, int64_t m, uint64_t seed, std::vector<__int128>& wt,
                              __int128& wmax, __int128& wmin) {
  wt.resize(m);
  wmax = 0; wmin = 0;
  for (int64_t e = 0; e < m; ++e) {
    const uint64_t h = lib_splitmix(seed, (uint64_t)e + 1) >> 24;
    wt[e] = ((__int128)(2 * (int64_t)w[e]) << 64) + (__int128)(2 * h);
    wmax = std::max(wmax, wt[e]);
    wmin = (e == 0) ? wt[e] : std::min(wmin, wt[e]);
  }
  if (m == 0) { wmax = 2; wmin = 2; }
}



// Layout of the per-shot state block for the given capacities.
// lean >= 1: the event cache and the region bases go to the workspace;
// lean >= 2: the explored nodes' radius offsets too.  Each shrinks the LDS
// block by 16 bytes per node or region.
static void plan_state(psb::StateLayout& SL, const psb::Caps& cap, int lean) {
  int64_t off = 0;
  auto take = [&](int64_t bytes) { int64_t o = off; off += (bytes + 15) & ~(int64_t)15; return o; };
  const int64_t x = cap.xcap, h = cap.hcap, r = cap.rcap;
  SL.x_wr = lean >= 2 ? -1 : take(16 * x);
  SL.x_ev = lean >= 1 ? -1 : take(16 * x);
  SL.r_base = lean >= 1 ? -1 : take(16 * r);
  SL.x_node = take(4 * x); SL.x_top = take(2 * x); SL.x_reg = take(2 * x); SL.x_src = take(2 * x); SL.x_rec = take(2 * x);
  SL.h_key = take(4 * h); SL.h_val = take(4 * h);
  SL.r_f32 = take(4LL * (psb::RF_COUNT - psb::RF_N16) * r);
  SL.r_f16 = take(2LL * psb::RF_N16 * r);
  SL.total = off;
}

static int32_t next_pow2(int64_t x) { int32_t p = 1; while (p < x) p <<= 1; return p; }

// Capacities and global workspace layout for one slot of a tier.  lean >= 3
// (wavefront tiers): as lean 2, and the state block itself in the workspace.  A slot is
// one wavefront (wavefront tiers: per-shot state in LDS, 64 lanes share the
// clustering hit buffers) or one lane (lane tier: the Lds header and the state
// block sit at the start of the slot, pools are sized more tightly and a shot
// that exceeds them is handed on).
static void plan_tier(Params& P, int32_t n, int32_t deg, int64_t n_edges, const psb::Caps& cap, bool lane_slot,
                      int lean = 0, bool acct = false, bool lane_nb_table = false) {
  P.n_det = n; P.deg = deg; P.nbytes = (n + 7) / 8; P.n_edges = n_edges;
  P.cap = cap;
  const int32_t d = cap.dcap;
  P.cecap = lane_slot ? 4 * d + 128 : 8 * d + 256;
  P.bccap = lane_slot ? 4 * d + 128 : 8 * d + 256;
  P.lcap = std::min<int64_t>(2LL * n + 4 * d + 64, 2LL * cap.xcap + 4 * d + 64);
  P.shrcap = cap.rcap;
  P.stkcap = std::max(4 * cap.rcap + 64, cap.xcap + 64);
  P.fincap = 2 * d + 64;
  P.hitcap = 32;
  P.bdc = 8;
  P.max_events = (int64_t)64 * ((int64_t)cap.xcap + 64 * (int64_t)d);
  plan_state(P.SL, cap, lean >= 3 ? 2 : lean);
  P.state_ws = (!lane_slot && lean >= 3) ? 1 : 0;
  WsLayout& L = P.L;
  int64_t off = 0;
  auto take = [&](int64_t bytes) { int64_t o = off; off = align256(off + bytes); return o; };
  L.state = (lane_slot || P.state_ws) ? take(64 + P.SL.total) : 0;
  L.ce = take(4LL * psb::CE_COUNT * P.cecap); L.bc = take(8LL * P.bccap); L.lg = take(12LL * P.lcap);
  L.level = take(d); L.uf = take(4LL * d);
  L.cl_a = take(4LL * d); L.cl_b = take(4LL * d); L.cl_c = take(4LL * d); L.cl_d = take(4LL * d);
  L.cid = take(4LL * d);
  L.bdl = take(4LL * d * P.bdc); L.hit = take(4LL * (lane_slot ? 1 : 64) * P.hitcap * 2);
  L.shr = take(4LL * P.shrcap); L.chg = take(4LL * cap.xcap); L.stk = take(4LL * P.stkcap);
  L.fin = take(4LL * P.fincap); L.ebits = take(4 * ((n_edges + 31) / 32 + 1));
  L.dmap = cap.hcap == 0 ? take(2LL * n) : 0;
  L.x_ev = lean >= 1 ? take(16LL * cap.xcap) : 0;
  L.r_base = lean >= 1 ? take(16LL * cap.rcap) : 0;
  L.x_wr = lean >= 2 ? take(16LL * cap.xcap) : 0;
  // the lane tier keeps no neighbour table (-1: none; only a host build of the engine can ask for one)
  L.x_nb = (lane_slot && !lane_nb_table) ? -1 : take(2LL * cap.xcap * deg);
  L.acct = acct ? take(psb::acct_bytes(d)) : 0;
  P.near_on = (cap.hcap == 0 && (int64_t)d * deg <= 32766) ? 1 : 0;
  L.near = P.near_on ? take((int64_t)sizeof(psb::NearEntry) * d * deg) : 0;
  L.ehead = P.near_on ? take(4LL * d) : 0;
  P.eacct = acct ? 1 : 0;
  L.total = off;
}

// Path-enumeration depth per level (-1 = final level); returns false if a
// level would need deeper enumeration than the clustering kernel supports.
static bool level_depths(const LevelSchedule& S, __int128 wmin, std::vector<int32_t>& hmax, int& bad_level) {
  hmax.clear();
  for (size_t k = 0; k < S.d.size(); ++k) {
    int h = -1;
    if (!S.final_level[k]) {
      const u128 H = S.b[k] / (u128)wmin;
      if (H > (u128)psb::MAXH) { bad_level = (int)k + 1; return false; }
      h = (int)H;
    }
    hmax.push_back(h);
  }
  return true;
}

// Ball tables of the clustering levels below the final one (shmax >= 1): the
// search walks paths of at most shmax edges, each cut at length b_k and
// extended only while shorter than b_k.  Row u of a level's table lists every detector x != u
// at the end of such a path, flagged BALL_CLOSE when its least such length is
// at most d_k, then every boundary edge ending such a path whose least length
// is at most d_k (BALL_CLOSE) or at most b_k / 2 (BALL_LOOSE).  Reading the row
// gives the search exactly the partners, close pairs, boundary edges within d_k
// and loose flag that walking the paths gives, in one pass of independent
// loads.  A level whose walks, replayed here for every detector, take more
// than max_paths steps in all (default 2048 per detector) gets no table (its
// search walks on the device).
// Returns false (and no tables) when ids do not fit the entries or the tables
// would exceed max_entries.
struct BallTables {
  std::vector<int32_t> slot, off, ent;
};

static bool build_ball_tables(const Ell& g, const std::vector<__int128>& ell_w, const std::vector<__int128>& sb,
                              const std::vector<__int128>& sd, const std::vector<int32_t>& hmax, int64_t max_entries,
                              BallTables& T, int64_t max_paths = -1) {
  const int32_t n = g.n_det, deg = g.deg;
  if (max_paths < 0) max_paths = 2048 * (int64_t)n + (1 << 20);
  T.slot.assign(hmax.size(), -1); T.off.clear(); T.ent.clear();
  if (n > psb::BALL_ID || g.n_edges > psb::BALL_ID) return false;
  std::vector<std::pair<int32_t, __int128>> cand, bc;
  int32_t tables = 0;
  for (size_t k = 0; k < hmax.size(); ++k) {
    const int hops = hmax[k];
    if (hops < 1) continue;
    const __int128 b = sb[k], d = sd[k];
    const size_t base = T.off.size(), ebase = T.ent.size();
    T.off.resize(base + 2 * (size_t)n + 1);
    int64_t steps = 0;
    bool over = false;
    for (int32_t u = 0; u < n && !over; ++u) {
      cand.clear(); bc.clear();
      // the paths in the walk's order (depth first, adjacency slots in row
      // order), returns to u included: the order decides which boundary edges
      // a full list keeps
      auto walk = [&](auto&& self, int32_t x, __int128 base_w, int depth) -> void {
        for (int32_t j = 0; j < deg && !over; ++j) {
          if (++steps > max_paths) { over = true; return; }
          const int64_t a = (int64_t)x * deg + j;
          const int32_t y = g.nbr[a];
          if (y == psb::NB_PAD) break;
          const __int128 w = base_w + ell_w[a];
          if (w > b) continue;
          if (y == psb::NB_BOUNDARY) { bc.push_back({g.eid[a], w}); continue; }
          if (y != u) cand.push_back({y, w});
          if (depth + 1 < hops && w < b) self(self, y, w, depth + 1);
        }
      };
      walk(walk, u, 0, 0);
      std::sort(cand.begin(), cand.end());
      T.off[base + 2 * (size_t)u] = (int32_t)T.ent.size();
      for (size_t q = 0; q < cand.size(); ++q)
        if (q == 0 || cand[q - 1].first != cand[q].first)   // least length of each detector
          T.ent.push_back(cand[q].first | (cand[q].second <= d ? psb::BALL_CLOSE : 0));
      T.off[base + 2 * (size_t)u + 1] = (int32_t)T.ent.size();
      // boundary edges: those within d_k in the order of the walk's first path
      // within d_k (the order in which the walk lists them), then those only
      // within b_k / 2
      for (int pass = 0; pass < 2; ++pass)
        for (size_t k2 = 0; k2 < bc.size(); ++k2) {
          const int32_t e = bc[k2].first;
          bool seen = false;
          __int128 least = bc[k2].second;
          for (size_t k3 = 0; k3 < bc.size(); ++k3) {
            if (bc[k3].first != e) continue;
            if (k3 < k2 && (pass == 1 || bc[k3].second <= d)) seen = true;
            if (bc[k3].second < least) least = bc[k3].second;
          }
          if (seen) continue;
          if (pass == 0 && bc[k2].second <= d)
            T.ent.push_back(e | psb::BALL_CLOSE | (2 * least <= b ? psb::BALL_LOOSE : 0));
          else if (pass == 1 && least > d && 2 * least <= b)
            T.ent.push_back(e | psb::BALL_LOOSE);
        }
      if ((int64_t)T.ent.size() > max_entries) { T.slot.assign(hmax.size(), -1); T.off.clear(); T.ent.clear(); return false; }
    }
    if (over) {                          // this level walks: drop its partial table
      T.off.resize(base);
      T.ent.resize(ebase);
      continue;
    }
    T.off[base + 2 * (size_t)n] = (int32_t)T.ent.size();
    T.slot[k] = tables++;
  }
  return true;
}

}  // namespace psb_host
