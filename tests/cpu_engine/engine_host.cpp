// CPU build of the decoder engine for tests: the engine of the HIP library
// compiled with the single-lane host primitives (one shot at a time), the
// library's own host-side set-up (tie-broken weights, level schedule,
// workspace layout), and the invariant checks.  Built by the tests with
// g++ and the address / undefined-behaviour sanitizers; not part of the
// library.
//
// usage: engine_host <dir> <seed> <mode> <reading> <xcap> <rcap> <dcap> <hash> <direct1> [<walk>]
//   (walk = 1: the clustering search walks its paths at every level; 0, the
//   default: levels of at most two edges read the library's ball tables)
//   <dir>/graph.bin : int32 n, int64 m, int32 u[m], int32 v[m], int32 w[m], uint64 obs[m]
//   <dir>/synd.bin  : int64 shots, int32 bytes per row, uint8 rows[shots][bytes]
// writes <dir>/out.bin: per shot int32 status, int32 n_edges, int64 weight,
//   uint64 obs, int32 stats[12], int32 edges[edge_stride]  (edge_stride first, as int32)
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>
#include <vector>

#include "../../paper_2609_12262_amd/csrc/psb_types.h"
#include "../../paper_2609_12262_amd/csrc/host_wave.h"
#define PSB_ENGINE_NS engine_host
#include "../../paper_2609_12262_amd/csrc/engine.h"
#include "../../paper_2609_12262_amd/csrc/host_setup.h"

namespace psb_host {
int32_t fail(int32_t code, const std::string& msg) {
  fprintf(stderr, "setup failed (%d): %s\n", code, msg.c_str());
  return code;
}
}  // namespace psb_host

void psb_invariant_failed(const char* what, int64_t shot, int level) {
  fprintf(stderr, "INVARIANT: %s (shot %lld, level %d)\n", what, (long long)shot, level);
  abort();
}

template <class T> static bool rd(FILE* f, T* p, size_t n) { return fread(p, sizeof(T), n, f) == n; }

int main(int argc, char** argv) {
  if (argc != 10 && argc != 11) {
    fprintf(stderr, "usage: engine_host dir seed mode reading xcap rcap dcap hash direct1 [walk]\n");
    return 2;
  }
  const int walk = argc == 11 ? atoi(argv[10]) : 0;
  const std::string dir = argv[1];
  const uint64_t seed = strtoull(argv[2], nullptr, 0);
  const int mode = atoi(argv[3]), reading = atoi(argv[4]);
  const int xcap_in = atoi(argv[5]), rcap_in = atoi(argv[6]), dcap_in = atoi(argv[7]), force_hash = atoi(argv[8]);
  FILE* fg = fopen((dir + "/graph.bin").c_str(), "rb");
  if (!fg) return 2;
  int32_t n; int64_t m;
  if (!rd(fg, &n, 1) || !rd(fg, &m, 1)) return 2;
  std::vector<int32_t> u(m), v(m), w(m);
  std::vector<uint64_t> obs(m);
  if (!rd(fg, u.data(), m) || !rd(fg, v.data(), m) || !rd(fg, w.data(), m) || !rd(fg, obs.data(), m)) return 2;
  fclose(fg);
  // fixed-width adjacency, in edge order (as the library lays it out)
  std::vector<int32_t> degree(n, 0);
  for (int64_t e = 0; e < m; ++e) { ++degree[u[e]]; if (v[e] >= 0) ++degree[v[e]]; }
  int32_t deg = 1;
  for (int32_t x : degree) deg = std::max(deg, x);
  psb_host::Ell ell;
  ell.n_det = n; ell.deg = deg; ell.n_edges = m;
  ell.nbr.assign((size_t)n * deg, psb::NB_PAD);
  ell.eid.assign((size_t)n * deg, -1);
  std::vector<int32_t> fill(n, 0);
  for (int64_t e = 0; e < m; ++e) {
    ell.nbr[(size_t)u[e] * deg + fill[u[e]]] = v[e] >= 0 ? v[e] : psb::NB_BOUNDARY;
    ell.eid[(size_t)u[e] * deg + fill[u[e]]++] = (int32_t)e;
    if (v[e] >= 0) { ell.nbr[(size_t)v[e] * deg + fill[v[e]]] = u[e]; ell.eid[(size_t)v[e] * deg + fill[v[e]]++] = (int32_t)e; }
  }
  std::vector<__int128> wt;
  __int128 wmax, wmin;
  psb_host::tiebroken_weights(w.data(), m, seed, wt, wmax, wmin);
  psb_host::LevelSchedule S;
  if (psb_host::build_schedule((psb_host::u128)wmax, psb_host::diameter_bound(&ell, wt), 1, 10, 1, 100, S) != PSB_OK) return 3;
  std::vector<int32_t> hmax;
  int bad_level = 0;
  if (mode == 1) hmax.assign(S.d.size(), -1);
  else if (!psb_host::level_depths(S, wmin, hmax, bad_level)) return 4;
  std::vector<__int128> ell_w((size_t)n * deg, 0), sd(S.d.size()), sb(S.d.size());
  for (size_t k = 0; k < ell_w.size(); ++k) if (ell.eid[k] >= 0) ell_w[k] = wt[ell.eid[k]];
  for (size_t k = 0; k < S.d.size(); ++k) { sd[k] = (__int128)S.d[k]; sb[k] = (__int128)S.b[k]; }

  psb::Caps cap;
  cap.dcap = std::max(1, std::min(dcap_in, n));
  cap.xcap = std::min(n, xcap_in);
  cap.rcap = rcap_in;
  cap.dcap = std::min(std::min(cap.xcap, cap.rcap), cap.dcap);
  cap.hcap = (force_hash || n > 32768) ? psb_host::next_pow2(2LL * cap.xcap) : 0;
  psb::Params P;
  memset(&P, 0, sizeof(P));
  psb_host::plan_tier(P, n, deg, m, cap, /*lane_slot=*/true, 0, /*acct=*/true, /*lane_nb_table=*/PSB_NB_TABLE);
  std::vector<uint32_t> bndb(((size_t)n + 31) / 32, 0u);
  for (size_t k = 0; k < ell.nbr.size(); ++k)
    if (ell.nbr[k] == psb::NB_BOUNDARY) bndb[(k / deg) >> 5] |= 1u << ((k / deg) & 31);
  P.nbr = ell.nbr.data(); P.eid = ell.eid.data(); P.wt = ell_w.data(); P.w = w.data(); P.obs = obs.data();
  P.bndb = bndb.data();
  P.n_levels = (int32_t)S.d.size(); P.reading = reading; P.mode = mode; P.tier = 1; P.direct1 = atoi(argv[9]);
  P.sd = sd.data(); P.sb = sb.data(); P.shmax = hmax.data();
  psb_host::BallTables balls;
  if (!walk && mode == 0 && psb_host::build_ball_tables(ell, ell_w, sb, sd, hmax, (int64_t)1 << 28, balls) &&
      !balls.off.empty()) {
    P.ball_slot = balls.slot.data(); P.ball_off = balls.off.data(); P.ball_ent = balls.ent.data();
  }

  FILE* fs = fopen((dir + "/synd.bin").c_str(), "rb");
  if (!fs) return 2;
  int64_t shots; int32_t nbytes;
  if (!rd(fs, &shots, 1) || !rd(fs, &nbytes, 1) || nbytes != P.nbytes) return 2;
  std::vector<uint8_t> synd((size_t)shots * nbytes);
  if (!rd(fs, synd.data(), synd.size())) return 2;
  fclose(fs);
  const int32_t stride = std::max(64, cap.dcap * 8);
  std::vector<int32_t> edges((size_t)shots * stride), nedges(shots), status(shots), stats((size_t)shots * 12);
  std::vector<int64_t> weight(shots);
  std::vector<uint64_t> ob(shots);
  std::vector<int8_t> levels((size_t)shots * cap.dcap);
  P.n_shots = shots; P.synd = synd.data(); P.out_edges = edges.data(); P.edge_stride = stride;
  P.out_nedges = nedges.data(); P.out_weight = weight.data(); P.out_obs = ob.data(); P.out_status = status.data();
  P.out_levels = levels.data(); P.level_stride = cap.dcap; P.out_stats = stats.data(); P.stats_stride = 12;

  // one lane slot: Lds header and state block at its start, then the pools
  std::vector<char> ws((size_t)P.L.total + 256, 0);
  char* slot = (char*)(((uintptr_t)ws.data() + 255) & ~(uintptr_t)255);
  P.ws = slot;
  namespace eh = psb::engine_host;
  eh::Ctx c;
  eh::ctx_init(c, &P, (eh::Lds*)(slot + P.L.state), slot + P.L.state + 64, 0);
  std::vector<int32_t> dbg_cfg(cap.rcap), dbg_touch(cap.dcap), dbg_touch_lvl(cap.dcap);
  c.dbg_cfg = dbg_cfg.data(); c.dbg_touch = dbg_touch.data(); c.dbg_touch_lvl = dbg_touch_lvl.data();
  eh::state_init(c);
  for (int64_t k = 0; k < shots; ++k) eh::decode_shot(c, k);

  FILE* fo = fopen((dir + "/out.bin").c_str(), "wb");
  fwrite(&stride, 4, 1, fo);
  for (int64_t k = 0; k < shots; ++k) {
    fwrite(&status[k], 4, 1, fo); fwrite(&nedges[k], 4, 1, fo); fwrite(&weight[k], 8, 1, fo); fwrite(&ob[k], 8, 1, fo);
    fwrite(&stats[(size_t)k * 12], 4, 12, fo); fwrite(&edges[(size_t)k * stride], 4, stride, fo);
  }
  fclose(fo);
  return 0;
}
