// libpsb: host side of the decoder (graph upload, level schedule, workspace,
// launch) and the persistent decode kernel.  See include/psb.h for the ABI.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <queue>
#include <string>
#include <vector>

#include "../../include/psb.h"
#include "psb_types.h"
#include "wave.h"
#include "engine.h"
#include "host_setup.h"
#include "lane_launch.h"

using namespace psb_host;

using psb::Params;
namespace ew = psb::engine_wave;
using psb::WsLayout;
typedef unsigned __int128 u128;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;
namespace psb_host { int32_t fail(int32_t code, const std::string& msg) { g_err = msg; return code; } }
using psb_host::fail;
extern "C" const char* psb_last_error(void) { return g_err.c_str(); }

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess) return fail(PSB_E_DEVICE, std::string(#expr " failed: ") + hipGetErrorString(_e)); \
  } while (0)

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
__global__ void psb_zero_kernel(int32_t* p, int n, uint64_t* t_start) {
  // resets the work counters (fill kernel rather than a memset node, so the
  // launch sequence stays valid under stream capture)
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
  if (i == 0 && t_start) *t_start = wall_clock64();
}

// Largest shots first: the first tier takes shots in descending order of
// their detection-event counts (a count predicts a shot's decode time), so
// the shots left when wavefronts start to run out of work are the short ones
// and the launch's idle tail shrinks.  Counts above kOrderBuckets - 1 share
// the first bucket; order within a bucket is whatever the atomics give (the
// results do not depend on the order).  Three kernels, no memset: count and
// bucket every shot, scan the bucket sizes, scatter.  The count and scatter
// kernels run kOrderBlocks blocks of 1,024 threads over contiguous chunks of
// shots with histograms in LDS, so each block adds to a global bucket once
// (thousands of shots in a handful of buckets would otherwise queue on the
// same few atomic counters).
constexpr int kOrderBuckets = 1024;
constexpr int kOrderBlocks = 256;

__global__ __launch_bounds__(1024) void psb_order_count(const uint8_t* synd, int32_t nbytes, int64_t n,
                                                        int32_t* bkt, int32_t* hist) {
  __shared__ int32_t lh[kOrderBuckets];
  for (int b = threadIdx.x; b < kOrderBuckets; b += blockDim.x) lh[b] = 0;
  __syncthreads();
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min(n, lo + chunk);
  const int wave = threadIdx.x >> 6, ln = threadIdx.x & 63, waves = blockDim.x >> 6;
  for (int64_t i = lo + wave; i < hi; i += waves) {           // one wavefront per shot, lanes over its bytes
    const uint8_t* row = synd + i * (int64_t)nbytes;
    int cnt = 0;
    for (int b = ln; b < nbytes; b += 64) cnt += __builtin_popcount((unsigned)row[b]);
    for (int m = 32; m >= 1; m >>= 1) cnt += __shfl_xor(cnt, m, 64);
    if (ln == 0) {
      const int b = kOrderBuckets - 1 - min(cnt, kOrderBuckets - 1);
      bkt[i] = b;
      atomicAdd(&lh[b], 1);
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kOrderBuckets; b += blockDim.x)
    if (lh[b]) atomicAdd(&hist[b], lh[b]);
}

// hist[b] -> the first position of bucket b (exclusive prefix sum), one block
// of kOrderBuckets threads
__global__ __launch_bounds__(kOrderBuckets) void psb_order_scan(int32_t* hist) {
  __shared__ int32_t buf[kOrderBuckets];
  const int t = threadIdx.x;
  const int32_t v = hist[t];
  buf[t] = v;
  __syncthreads();
  for (int off = 1; off < kOrderBuckets; off <<= 1) {
    const int32_t add = t >= off ? buf[t - off] : 0;
    __syncthreads();
    buf[t] += add;
    __syncthreads();
  }
  hist[t] = buf[t] - v;
}

// Each block reserves, per bucket, a range for its chunk's shots (one global
// atomic per bucket it uses), then places them with LDS atomics.
__global__ __launch_bounds__(1024) void psb_order_scatter(int64_t n, const int32_t* bkt, int32_t* hist,
                                                          int32_t* order) {
  __shared__ int32_t cnt[kOrderBuckets], base[kOrderBuckets];
  for (int b = threadIdx.x; b < kOrderBuckets; b += blockDim.x) cnt[b] = 0;
  __syncthreads();
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min(n, lo + chunk);
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) atomicAdd(&cnt[bkt[i]], 1);
  __syncthreads();
  for (int b = threadIdx.x; b < kOrderBuckets; b += blockDim.x) {
    base[b] = cnt[b] ? atomicAdd(&hist[b], cnt[b]) : 0;
    cnt[b] = 0;
  }
  __syncthreads();
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    const int b = bkt[i];
    order[base[b] + atomicAdd(&cnt[b], 1)] = (int32_t)i;
  }
}

// Persistent decode kernel, one wavefront per shot, per-shot state in LDS.
// TIER 0 (small capacities, many waves per CU) hands shots that exceed its
// capacities to the overflow list; TIER 1 (large capacities, a few waves
// per CU) decodes either that list (ovf_list != null) or every shot directly.
// At most 128 VGPRs, so that four wavefronts share a SIMD (the per-shot
// event loop is latency-bound: throughput grows with resident wavefronts).
// ACCT: per-cluster event accounting compiled in (ACCT = 0 removes it).
// DEEP: the clustering search's generic walk for paths of more than three
// edges compiled in (only graphs whose levels need it get it).
// WS: the Lds header and state block sit in the slot's workspace instead of
// LDS (first tier only, Params::state_ws).
template <int TIER, int ACCT, int DEEP, int WS = 0>
__global__ __launch_bounds__(64, 4) void psb_decode_kernel(Params P) {
  extern __shared__ __align__(16) char psb_dyn_lds[];
  char* base = WS ? P.ws + (int64_t)blockIdx.x * P.L.total + P.L.state : psb_dyn_lds;
  ew::Lds* S = (ew::Lds*)base;
  char* state = base + 64;
  ew::Ctx c;
  ew::ctx_init(c, &P, S, state, blockIdx.x);
  if (!ACCT) c.acct = nullptr;
  ew::state_init(c);
  for (;;) {
    // every lane takes part in the counter update (lane 0 adds 1, the others
    // add 0) and lane 0's old value is broadcast: no lane-dependent branch
    // and no per-lane constant feeds the broadcast
    const int k = lane0(atomicAdd(TIER == 0 ? &P.counter[0] : &P.counter[2], lane() == 0 ? 1 : 0));
    int64_t shot;
    if (TIER == 0 || P.ovf_list == nullptr) {
      if (k >= P.n_shots) break;
      shot = (TIER == 0 && P.order) ? uni(P.order[k]) : k;
    } else {
      const int lim = uni(__hip_atomic_load(&P.counter[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      if (k >= lim) break;
      shot = uni(P.ovf_list[k]);
    }
    const int st = ew::decode_shot<DEEP>(c, shot);
    if (st == psb::S_OVERFLOW) {
      const int q = lane0(atomicAdd(&P.counter[1], lane() == 0 ? 1 : 0));
      P.ovf_list[q] = (int32_t)shot;               // same value from every lane
    } else if (P.out_tdone) {
      P.out_tdone[shot] = wall_clock64();
    }
  }
}

// The decode kernel instantiation for a tier, accounting and search depth
// class of the walking levels (0: paths of up to two edges, 1: three, 2: the
// generic walk).
static const void* decode_kernel_fn(int tier, bool acct, int deep, bool ws = false) {
  if (ws) {                                       // first tier without accounting only (host-checked)
    const void* kw[3] = {(const void*)psb_decode_kernel<0, 0, 0, 1>, (const void*)psb_decode_kernel<0, 0, 1, 1>,
                         (const void*)psb_decode_kernel<0, 0, 2, 1>};
    return kw[deep];
  }
  const void* k[2][2][3] = {
      {{(const void*)psb_decode_kernel<0, 0, 0>, (const void*)psb_decode_kernel<0, 0, 1>,
        (const void*)psb_decode_kernel<0, 0, 2>},
       {(const void*)psb_decode_kernel<0, 1, 0>, (const void*)psb_decode_kernel<0, 1, 1>,
        (const void*)psb_decode_kernel<0, 1, 2>}},
      {{(const void*)psb_decode_kernel<1, 0, 0>, (const void*)psb_decode_kernel<1, 0, 1>,
        (const void*)psb_decode_kernel<1, 0, 2>},
       {(const void*)psb_decode_kernel<1, 1, 0>, (const void*)psb_decode_kernel<1, 1, 1>,
        (const void*)psb_decode_kernel<1, 1, 2>}}};
  return k[tier][acct ? 1 : 0][deep];
}

static hipError_t launch_decode_kernel(int tier, bool acct, int deep, unsigned grid, size_t lds, hipStream_t s,
                                       const Params& P) {
  void* args[] = {(void*)&P};
  return hipLaunchKernel(decode_kernel_fn(tier, acct, deep, P.state_ws != 0), dim3(grid), dim3(64), args, lds, s);
}

// ---------------------------------------------------------------------------
// allocation-free batches: the work counters and the overflow list live in
// `scratch`, one copy per device, instead of the decoder's own buffers
// ---------------------------------------------------------------------------
constexpr int64_t kScratchHeader = 64;   // int32 slots before the overflow list (counters in [0..2])
static __device__ __align__(256) int32_t scratch[kScratchHeader + PSB_NOALLOC_MAX_SHOTS];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static int32_t* g_scratch_ptr[kMaxDevices];   // device address of `scratch`, per device

// Called by psb_decoder_create with the decoder's device current: the device
// address of this device's copy of `scratch` (the array's name in host code is
// only a host-side stand-in).
static int32_t scratch_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return fail(PSB_E_UNSUPPORTED, "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev]) return PSB_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) return fail(PSB_E_DEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") +
                                                         hipGetErrorString(e));
  g_scratch_ptr[dev] = (int32_t*)ptr;
  return PSB_OK;
}

// ---------------------------------------------------------------------------
// graph
// ---------------------------------------------------------------------------
struct psb_graph {
  int32_t n_det = 0, deg = 0;
  int64_t n_edges = 0;
  std::vector<int32_t> u, v, w;
  std::vector<uint64_t> obs;
  std::vector<int32_t> nbr, eid;     // host ELL
  int32_t *d_nbr = nullptr, *d_eid = nullptr, *d_w = nullptr;
  uint64_t* d_obs = nullptr;
  uint32_t* d_bndb = nullptr;        // bit per detector: it has a boundary edge
};

extern "C" int32_t psb_graph_create(const psb_graph_desc* desc, psb_graph** out) {
  if (!desc || !out) return fail(PSB_E_INVALID, "null argument");
  *out = nullptr;
  const int32_t n = desc->num_detectors;
  const int64_t m = desc->num_edges;
  if (n <= 0 || m < 0 || m >= (1LL << 23)) return fail(PSB_E_INVALID, "num_detectors must be > 0 and num_edges in [0, 2^23)");
  if (m > 0 && (!desc->u || !desc->v || !desc->w || !desc->obs_mask)) return fail(PSB_E_INVALID, "null edge array");
  std::vector<int32_t> degree(n, 0);
  for (int64_t e = 0; e < m; ++e) {
    const int32_t a = desc->u[e], b = desc->v[e];
    if (a < 0 || a >= n || b < PSB_BOUNDARY || b >= n || a == b)
      return fail(PSB_E_INVALID, "edge " + std::to_string(e) + " has an endpoint out of range or is a self loop");
    if (desc->w[e] <= 0) return fail(PSB_E_INVALID, "edge " + std::to_string(e) + " has a non-positive weight");
    ++degree[a];
    if (b >= 0) ++degree[b];
  }
  int32_t deg = 1;
  for (int32_t x : degree) deg = std::max(deg, x);
  if (deg > 16) return fail(PSB_E_INVALID, "a detector has degree > 16");
  psb_graph* g = new psb_graph();
  g->n_det = n; g->n_edges = m; g->deg = deg;
  g->u.assign(desc->u, desc->u + m); g->v.assign(desc->v, desc->v + m);
  g->w.assign(desc->w, desc->w + m); g->obs.assign(desc->obs_mask, desc->obs_mask + m);
  g->nbr.assign((size_t)n * deg, psb::NB_PAD);
  g->eid.assign((size_t)n * deg, -1);
  std::vector<int32_t> fill(n, 0);
  for (int64_t e = 0; e < m; ++e) {
    const int32_t a = g->u[e], b = g->v[e];
    g->nbr[(size_t)a * deg + fill[a]] = (b >= 0) ? b : psb::NB_BOUNDARY;
    g->eid[(size_t)a * deg + fill[a]++] = (int32_t)e;
    if (b >= 0) {
      g->nbr[(size_t)b * deg + fill[b]] = a;
      g->eid[(size_t)b * deg + fill[b]++] = (int32_t)e;
    }
  }
  auto up = [&](void** dst, const void* src, size_t bytes) -> hipError_t {
    hipError_t e = hipMalloc(dst, bytes ? bytes : 16);
    if (e != hipSuccess) return e;
    return bytes ? hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) : hipSuccess;
  };
  hipError_t e1 = up((void**)&g->d_nbr, g->nbr.data(), g->nbr.size() * 4);
  hipError_t e2 = up((void**)&g->d_eid, g->eid.data(), g->eid.size() * 4);
  hipError_t e3 = up((void**)&g->d_w, g->w.data(), g->w.size() * 4);
  hipError_t e4 = up((void**)&g->d_obs, g->obs.data(), g->obs.size() * 8);
  std::vector<uint32_t> bndb(((size_t)n + 31) / 32, 0u);
  for (int64_t k = 0; k < (int64_t)g->nbr.size(); ++k)
    if (g->nbr[k] == psb::NB_BOUNDARY) bndb[(size_t)(k / deg) >> 5] |= 1u << ((k / deg) & 31);
  hipError_t e5 = up((void**)&g->d_bndb, bndb.data(), bndb.size() * 4);
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess || e5 != hipSuccess) {
    psb_graph_destroy(g);
    return fail(PSB_E_DEVICE, "graph upload failed");
  }
  *out = g;
  return PSB_OK;
}

extern "C" int32_t psb_graph_destroy(psb_graph* g) {
  if (!g) return PSB_OK;
  if (g->d_nbr) (void)hipFree(g->d_nbr);
  if (g->d_eid) (void)hipFree(g->d_eid);
  if (g->d_w) (void)hipFree(g->d_w);
  if (g->d_obs) (void)hipFree(g->d_obs);
  if (g->d_bndb) (void)hipFree(g->d_bndb);
  delete g;
  return PSB_OK;
}

extern "C" int32_t psb_graph_syndrome_bytes(const psb_graph* g) { return g ? (g->n_det + 7) / 8 : -1; }

// For the serving runtime: the same graph with every weight 1 (requests with
// one uniform weight decode on it; their reported weight is scaled), and the
// edge count.
int32_t psb_graph_unit_copy(const psb_graph* g, psb_graph** out) {
  std::vector<int32_t> w1(g->n_edges, 1);
  psb_graph_desc d{};
  d.num_detectors = g->n_det; d.num_edges = g->n_edges;
  d.u = g->u.data(); d.v = g->v.data(); d.w = w1.data(); d.obs_mask = g->obs.data();
  return psb_graph_create(&d, out);
}
int64_t psb_graph_edges(const psb_graph* g) { return g->n_edges; }

// ---------------------------------------------------------------------------
// decoder
// ---------------------------------------------------------------------------
struct psb_decoder {
  const psb_graph* g = nullptr;
  psb_decoder_opts opts{};
  int32_t edge_stride = 0, dcap = 0;
  int32_t slots_fast = 0, slots_ovf = 0;
  bool acct = false;                 // per-cluster event accounting (kernel variant)
  int deep = 0;                      // search depth class the levels need: 0 (<= 2 edges), 1 (3), 2 (deeper)
  size_t lds_fast = 0, lds_ovf = 0;
  bool fast_enabled = true;
  bool first_lane = true;          // first tier: one shot per lane (else one per wavefront)
  __int128* d_wt = nullptr;
  __int128* d_sd = nullptr; __int128* d_sb = nullptr; int32_t* d_shmax = nullptr;
  int32_t* d_ball = nullptr;         // ball tables: [levels] slot, then the offsets, then the entries
  int64_t ball_bytes = 0;
  int32_t* d_counter = nullptr;
  char* d_ws_fast = nullptr;
  char* d_ws_ovf = nullptr;
  int32_t* d_ovf_list = nullptr;     // [cap] overflow list, then [2 cap + kOrderBuckets] the shot order's buffers
  int64_t ovf_list_cap = 0;
  int32_t n_graphs = 0;              // captured batch graphs whose kernel arguments hold d_ovf_list
  int32_t* last_counter = nullptr;   // work counters of the most recent launch
  int32_t device = 0;
  Params P_fast{}, P_ovf{};
  LevelSchedule sched;
  std::vector<int32_t> hmax;
};

extern "C" int32_t psb_decoder_create(const psb_graph* g, const psb_decoder_opts* o, psb_decoder** out) {
  if (!g || !out) return fail(PSB_E_INVALID, "null argument");
  *out = nullptr;
  psb_decoder_opts opts = o ? *o : psb_decoder_opts{};
  if (opts.q_num == 0 && opts.q_den == 0) { opts.q_num = 1; opts.q_den = 10; }
  if (opts.phi_min_num == 0 && opts.phi_min_den == 0) { opts.phi_min_num = 1; opts.phi_min_den = 100; }
  if (opts.q_num <= 0 || opts.q_den <= opts.q_num || opts.phi_min_num <= 0 || opts.phi_min_den <= opts.phi_min_num)
    return fail(PSB_E_INVALID, "q and phi_min must lie in (0, 1)");
  if (opts.mode != 0 && opts.mode != 1) return fail(PSB_E_INVALID, "mode must be 0 or 1");
  if (opts.boundary_reading != 0 && opts.boundary_reading != 1) return fail(PSB_E_INVALID, "boundary_reading must be 0 or 1");
  const int32_t n = g->n_det;
  int32_t dcap = opts.max_defects_per_shot > 0 ? opts.max_defects_per_shot : std::min(n, n > 20000 ? 1024 : 512);
  dcap = std::max(1, std::min(dcap, n));
  const int32_t stride = opts.edges_per_shot > 0 ? opts.edges_per_shot : std::max(64, dcap * 8);

  psb_decoder* D = new psb_decoder();
  D->g = g; D->opts = opts; D->dcap = dcap; D->edge_stride = stride;
  std::vector<__int128> wt;
  __int128 wmax, wmin;
  tiebroken_weights(g->w.data(), g->n_edges, opts.tiebreak_seed, wt, wmax, wmin);
  Ell ell; ell.n_det = g->n_det; ell.deg = g->deg; ell.n_edges = g->n_edges; ell.nbr = g->nbr; ell.eid = g->eid;
  const u128 diam = diameter_bound(&ell, wt);
  int32_t rc = build_schedule((u128)wmax, diam, opts.q_num, opts.q_den, opts.phi_min_num, opts.phi_min_den, D->sched);
  if (rc != PSB_OK) { delete D; return rc; }
  int bad_level = 0;
  if (opts.mode == 1) {
    // global sparse blossom runs no clustering: no path enumeration depth applies
    D->hmax.assign(D->sched.d.size(), -1);
  } else if (!level_depths(D->sched, wmin, D->hmax, bad_level)) {
    delete D;
    return fail(PSB_E_UNSUPPORTED, "level " + std::to_string(bad_level) + " needs paths of more than " +
                                       std::to_string(psb::MAXH) + " edges; the clustering kernel enumerates at most that");
  }
  // weights laid out like the adjacency rows, so a row is read in one pass
  std::vector<__int128> ell_w((size_t)n * g->deg, 0);
  for (size_t k = 0; k < ell_w.size(); ++k) if (g->eid[k] >= 0) ell_w[k] = wt[g->eid[k]];
  const size_t nl = D->sched.d.size();
  std::vector<__int128> sd(nl), sb(nl);
  for (size_t k = 0; k < nl; ++k) { sd[k] = (__int128)D->sched.d[k]; sb[k] = (__int128)D->sched.b[k]; }
  // the levels below the final one read ball tables instead of walking (at most
  // 2^28 entries in all and about 2048 replayed walk steps per detector and
  // level; beyond that, or with cluster_walk, they walk)
  BallTables balls;
  const bool use_balls = opts.cluster_walk == 0 && opts.mode == 0 &&
                         build_ball_tables(ell, ell_w, sb, sd, D->hmax, (int64_t)1 << 28, balls) && !balls.off.empty();
  // the search depth class that the walking levels need
  for (size_t k = 0; k < nl; ++k) {
    const int32_t h = D->hmax[k];
    if (use_balls && balls.slot[k] >= 0) continue;
    D->deep = std::max(D->deep, h > 3 ? 2 : h == 3 ? 1 : 0);
  }
  // tier capacities: the first tier (one shot per lane, state in its global
  // workspace slot; or one shot per wavefront, state in LDS) and the
  // overflow tier (one shot per wavefront, large LDS state)
  if (opts.first_tier != 0 && opts.first_tier != 1) { delete D; return fail(PSB_E_INVALID, "first_tier must be 0 or 1"); }
  if (opts.fast_lds_state < 0 || opts.fast_lds_state > 4) { delete D; return fail(PSB_E_INVALID, "fast_lds_state must be 0..4"); }
  if (opts.fast_lds_state == 4 && opts.event_accounting) {
    delete D;
    return fail(PSB_E_UNSUPPORTED, "fast_lds_state 4 has no event-accounting kernel");
  }
  if (opts.event_accounting != 0 && opts.event_accounting != 1) { delete D; return fail(PSB_E_INVALID, "event_accounting must be 0 or 1"); }
  if (opts.serial_level_one != 0 && opts.serial_level_one != 1) { delete D; return fail(PSB_E_INVALID, "serial_level_one must be 0 or 1"); }
  if (opts.cluster_walk != 0 && opts.cluster_walk != 1) { delete D; return fail(PSB_E_INVALID, "cluster_walk must be 0 or 1"); }
  const bool acct = opts.event_accounting == 1;
  D->acct = acct;
  D->first_lane = opts.first_tier == 1;
  psb::Caps cf, co;
  co.xcap = std::min(n, 1024); co.rcap = std::min(4 * dcap + 64, 768);
  // detector -> explored index: a direct int16 map in the slot's workspace
  // when the graph is small enough (2 bytes per detector), else a hash in the
  // state block
  const bool direct = n <= 32768;
  co.dcap = std::min(std::min(co.xcap, co.rcap), dcap); co.hcap = direct ? 0 : next_pow2(2LL * co.xcap);
  D->fast_enabled = opts.fast_max_nodes >= 0;
  cf.xcap = std::min(n, opts.fast_max_nodes > 0 ? opts.fast_max_nodes : 320);
  cf.rcap = opts.fast_max_regions > 0 ? opts.fast_max_regions : (D->first_lane ? 256 : 208);
  cf.dcap = std::min(std::min(cf.xcap, cf.rcap), dcap);
  cf.hcap = direct ? 0 : next_pow2(2LL * cf.xcap);
  Params& PF = D->P_fast;
  Params& PO = D->P_ovf;
  // by default the wavefront first tier keeps its event cache, region bases
  // and radius offsets in the workspace: its LDS block (about 10 KB at the
  // default capacities) lets 16 wavefronts share a CU.  fast_lds_state moves
  // them into LDS (fewer wavefronts per CU, shorter dependent-load chains).
  static const int kLean[5] = {2, 2, 1, 0, 3};
  plan_tier(PF, n, g->deg, g->n_edges, cf, D->first_lane, D->first_lane ? 0 : kLean[opts.fast_lds_state], acct);
  plan_tier(PO, n, g->deg, g->n_edges, co, false, 0, acct);
  for (Params* P : {&PF, &PO}) {
    P->n_levels = (int32_t)D->sched.d.size(); P->reading = opts.boundary_reading; P->mode = opts.mode;
    P->edge_stride = stride;
    P->direct1 = opts.serial_level_one ? 0 : 1;
  }
  PF.tier = 0; PO.tier = 1;
  for (const Params* P : {&PF, &PO}) {
    // region ids, log records and pool offsets are stored as int16
    const int64_t widest = std::max<int64_t>({P->cap.rcap, P->cap.xcap, P->cecap, P->bccap, P->lcap});
    if (widest >= 32767) {
      delete D;
      return fail(PSB_E_UNSUPPORTED, "tier capacities exceed the 16-bit state indices (lower fast_max_nodes / "
                                     "fast_max_regions / max_defects_per_shot)");
    }
  }
  D->lds_fast = (D->first_lane || PF.state_ws) ? 0 : 64 + (size_t)PF.SL.total;
  D->lds_ovf = 64 + (size_t)PO.SL.total;
  if (D->lds_ovf > 160 * 1024) {
    delete D;
    return fail(PSB_E_UNSUPPORTED, "per-shot state of the overflow tier exceeds 160 KB of LDS");
  }
  // occupancy-derived slot counts
  int dev = 0, cus = 256;
  HIP_TRY(hipGetDevice(&dev));
  D->device = dev;
  {
    const int32_t src = scratch_setup(dev);
    if (src != PSB_OK) { delete D; return src; }
  }
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  int per_cu = 0, per_cu_o = 0;
  if (D->lds_fast > 160 * 1024) D->fast_enabled = false;
  if (D->fast_enabled && D->first_lane) {
    HIP_TRY(psb_lane_occupancy(&per_cu));
    if (per_cu < 1) D->fast_enabled = false;
  } else if (D->fast_enabled) {
    const void* kf = decode_kernel_fn(0, D->acct, D->deep, PF.state_ws != 0);
    HIP_TRY(hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)D->lds_fast));
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kf, 64, D->lds_fast));
    if (per_cu < 1) D->fast_enabled = false;
  }
  HIP_TRY(hipFuncSetAttribute(decode_kernel_fn(1, D->acct, D->deep), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)D->lds_ovf));
  HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_o, decode_kernel_fn(1, D->acct, D->deep), 64, D->lds_ovf));
  if (per_cu_o < 1) { delete D; return fail(PSB_E_UNSUPPORTED, "overflow tier does not fit on a compute unit"); }
  if (D->first_lane) {
    // lanes in flight: every wave the chip holds, at most 65536 lanes
    const int64_t lanes = opts.num_slots > 0 ? opts.num_slots : std::min<int64_t>(65536, 64LL * std::max(1, per_cu) * cus);
    D->slots_fast = (int32_t)((lanes + 63) / 64 * 64);
  } else {
    D->slots_fast = opts.num_slots > 0 ? opts.num_slots : std::max(1, per_cu) * cus;
  }
  D->slots_ovf = opts.overflow_slots > 0 ? opts.overflow_slots : per_cu_o * cus;
  // device buffers
  auto fail_dev = [&](const char* what) { psb_decoder_destroy(D); return fail(PSB_E_NOMEM, std::string("device allocation failed: ") + what); };
  {
    if (hipMalloc((void**)&D->d_wt, 16 * ell_w.size()) != hipSuccess) return fail_dev("weights");
    HIP_TRY(hipMemcpy(D->d_wt, ell_w.data(), 16 * ell_w.size(), hipMemcpyHostToDevice));
    if (use_balls) {
      BallTables& T = balls;
      const size_t words = T.slot.size() + T.off.size() + T.ent.size();
      T.slot.insert(T.slot.end(), T.off.begin(), T.off.end());
      T.slot.insert(T.slot.end(), T.ent.begin(), T.ent.end());
      if (hipMalloc((void**)&D->d_ball, 4 * words) != hipSuccess) return fail_dev("ball tables");
      HIP_TRY(hipMemcpy(D->d_ball, T.slot.data(), 4 * words, hipMemcpyHostToDevice));
      D->ball_bytes = 4 * (int64_t)words;
      for (Params* P : {&PF, &PO}) {
        P->ball_slot = D->d_ball;
        P->ball_off = D->d_ball + nl;
        P->ball_ent = D->d_ball + nl + T.off.size();
      }
    }
  }
  if (hipMalloc((void**)&D->d_sd, 16 * nl) != hipSuccess || hipMalloc((void**)&D->d_sb, 16 * nl) != hipSuccess ||
      hipMalloc((void**)&D->d_shmax, 4 * nl) != hipSuccess || hipMalloc((void**)&D->d_counter, 256) != hipSuccess)
    return fail_dev("schedule");
  HIP_TRY(hipMemcpy(D->d_sd, sd.data(), 16 * nl, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(D->d_sb, sb.data(), 16 * nl, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(D->d_shmax, D->hmax.data(), 4 * nl, hipMemcpyHostToDevice));
  if (D->fast_enabled) {
    if (hipMalloc((void**)&D->d_ws_fast, (size_t)PF.L.total * D->slots_fast) != hipSuccess) return fail_dev("workspace");
    HIP_TRY(hipMemset(D->d_ws_fast, 0, (size_t)PF.L.total * D->slots_fast));
  }
  if (hipMalloc((void**)&D->d_ws_ovf, (size_t)PO.L.total * D->slots_ovf) != hipSuccess) return fail_dev("overflow workspace");
  HIP_TRY(hipMemset(D->d_ws_ovf, 0, (size_t)PO.L.total * D->slots_ovf));
  HIP_TRY(hipDeviceSynchronize());
  for (Params* P : {&PF, &PO}) {
    P->nbr = g->d_nbr; P->eid = g->d_eid; P->wt = D->d_wt; P->w = g->d_w; P->obs = g->d_obs; P->bndb = g->d_bndb;
    P->sd = D->d_sd; P->sb = D->d_sb; P->shmax = D->d_shmax;
    P->counter = D->d_counter;
  }
  PF.ws = D->d_ws_fast; PO.ws = D->d_ws_ovf;
  *out = D;
  return PSB_OK;
}

extern "C" int32_t psb_decoder_destroy(psb_decoder* D) {
  if (!D) return PSB_OK;
  if (D->d_wt) (void)hipFree(D->d_wt);
  if (D->d_sd) (void)hipFree(D->d_sd);
  if (D->d_sb) (void)hipFree(D->d_sb);
  if (D->d_shmax) (void)hipFree(D->d_shmax);
  if (D->d_ball) (void)hipFree(D->d_ball);
  if (D->d_counter) (void)hipFree(D->d_counter);
  if (D->d_ws_fast) (void)hipFree(D->d_ws_fast);
  if (D->d_ws_ovf) (void)hipFree(D->d_ws_ovf);
  if (D->d_ovf_list) (void)hipFree(D->d_ovf_list);
  delete D;
  return PSB_OK;
}

extern "C" int32_t psb_decoder_levels(const psb_decoder* D, int32_t max_levels, int64_t* d_hi, uint64_t* d_lo,
                                      int64_t* b_hi, uint64_t* b_lo, int32_t* final_level) {
  if (!D) return fail(PSB_E_INVALID, "null decoder");
  const int32_t nl = (int32_t)std::min<size_t>(D->sched.d.size(), (size_t)std::max(0, max_levels));
  for (int32_t k = 0; k < nl; ++k) {
    if (d_hi) d_hi[k] = (int64_t)(D->sched.d[k] >> 64);
    if (d_lo) d_lo[k] = (uint64_t)D->sched.d[k];
    if (b_hi) b_hi[k] = (int64_t)(D->sched.b[k] >> 64);
    if (b_lo) b_lo[k] = (uint64_t)D->sched.b[k];
    if (final_level) final_level[k] = D->sched.final_level[k];
  }
  return nl;
}

extern "C" int32_t psb_decoder_edges_per_shot(const psb_decoder* D) { return D ? D->edge_stride : -1; }

extern "C" int32_t psb_decoder_device_bytes(const psb_decoder* D, int64_t* bytes) {
  if (!D || !bytes) return fail(PSB_E_INVALID, "null argument");
  int64_t b = (int64_t)D->P_ovf.L.total * D->slots_ovf + 16LL * D->g->n_det * D->g->deg + 256;
  if (D->fast_enabled) b += (int64_t)D->P_fast.L.total * D->slots_fast;
  if (D->ovf_list_cap > 0) b += 4 * (3 * D->ovf_list_cap + kOrderBuckets);
  b += D->ball_bytes;
  *bytes = b;
  return PSB_OK;
}
extern "C" int32_t psb_decoder_max_defects(const psb_decoder* D) { return D ? D->dcap : -1; }

extern "C" int32_t psb_decoder_reserve(psb_decoder* D, int64_t max_batch) {
  if (!D) return fail(PSB_E_INVALID, "null decoder");
  if (max_batch < 0 || max_batch > (int64_t)INT32_MAX) return fail(PSB_E_INVALID, "max_batch out of range");
  if (!D->fast_enabled || D->ovf_list_cap >= max_batch) return PSB_OK;
  if (D->n_graphs > 0)
    return fail(PSB_E_INVALID, "a captured batch graph of this decoder holds its overflow list; reserve the "
                               "largest batch before capturing, or destroy the graphs first");
  HIP_TRY(hipDeviceSynchronize());
  if (D->d_ovf_list) (void)hipFree(D->d_ovf_list);
  D->d_ovf_list = nullptr;
  D->ovf_list_cap = 0;
  if (hipMalloc((void**)&D->d_ovf_list, 4 * (3 * (size_t)std::max<int64_t>(max_batch, 1) + kOrderBuckets)) != hipSuccess)
    return fail(PSB_E_NOMEM, "overflow list");
  D->ovf_list_cap = max_batch;
  return PSB_OK;
}

// For the slot-level server (psb_slots.hip): the wavefront first tier's
// parameters (graph, schedule, capacities, state layout, workspace of its
// slots), its LDS bytes per wavefront and its slot count.  PSB_E_UNSUPPORTED
// when the decoder has no wavefront first tier or keeps a hash in LDS.
int32_t psb_decoder_first_tier(const psb_decoder* D, psb::Params* P, int32_t* lds_bytes, int32_t* slots) {
  if (!D || !P || !lds_bytes || !slots) return fail(PSB_E_INVALID, "null argument");
  if (!D->fast_enabled || D->first_lane || D->P_fast.cap.hcap != 0 || D->P_fast.state_ws)
    return fail(PSB_E_UNSUPPORTED, "slot-level serving needs a wavefront first tier with its state in LDS and a "
                                   "direct detector map");
  *P = D->P_fast;
  *lds_bytes = (int32_t)D->lds_fast;
  *slots = D->slots_fast;
  return PSB_OK;
}

extern "C" int32_t psb_decoder_slots(const psb_decoder* D, int32_t* fast_slots, int32_t* overflow_slots,
                                     int32_t* fast_lds_bytes) {
  if (!D) return fail(PSB_E_INVALID, "null decoder");
  if (fast_slots) *fast_slots = D->fast_enabled ? D->slots_fast : 0;
  if (overflow_slots) *overflow_slots = D->slots_ovf;
  if (fast_lds_bytes) *fast_lds_bytes = D->fast_enabled ? (int32_t)D->lds_fast : 0;
  return PSB_OK;
}

// Launches one batch: the counter reset, the first tier and the overflow tier,
// with the given work counters ([0] first-tier head, [1] overflow count, [2]
// overflow head) and overflow list (room for n shots).
// order_buf (room for 2 n + kOrderBuckets int32, or null for the identity
// order): the largest-first shot order is built there first.
static int32_t launch_batch(psb_decoder* D, const uint8_t* syndromes, int64_t n, int32_t* edges, int32_t* n_edges,
                            int64_t* weight, uint64_t* obs, int32_t* status, int8_t* levels, uint64_t* t_done,
                            int32_t* stats, int32_t* counter, int32_t* ovf_list, int32_t* order_buf,
                            hipStream_t s) {
  Params* tiers[2] = {&D->P_fast, &D->P_ovf};
  for (Params* P : tiers) {
    P->n_shots = n; P->synd = syndromes; P->out_edges = edges; P->out_nedges = n_edges; P->out_weight = weight;
    P->out_obs = obs; P->out_status = status; P->out_levels = levels; P->out_tdone = t_done; P->out_stats = stats;
    P->stats_stride = P->eacct ? 12 : 8;
    P->level_stride = D->dcap;
    P->counter = counter;
    P->ovf_list = D->fast_enabled ? ovf_list : nullptr;
  }
  D->last_counter = counter;
  psb_zero_kernel<<<1, 64, 0, s>>>(counter, 3, t_done ? t_done + n : nullptr);
  HIP_TRY(hipGetLastError());
  D->P_fast.order = nullptr; D->P_ovf.order = nullptr;
  if (order_buf && D->fast_enabled && n > 1) {
    int32_t* order = order_buf;
    int32_t* bkt = order_buf + n;
    int32_t* hist = order_buf + 2 * n;
    psb_zero_kernel<<<kOrderBuckets / 64, 64, 0, s>>>(hist, kOrderBuckets, nullptr);
    const unsigned blocks = (unsigned)std::min<int64_t>(kOrderBlocks, (n + 63) / 64);
    psb_order_count<<<blocks, 1024, 0, s>>>(syndromes, D->P_fast.nbytes, n, bkt, hist);
    psb_order_scan<<<1, kOrderBuckets, 0, s>>>(hist);
    psb_order_scatter<<<blocks, 1024, 0, s>>>(n, bkt, hist, order);
    HIP_TRY(hipGetLastError());
    D->P_fast.order = order;
  }
  if (D->fast_enabled && D->first_lane) {
    const int64_t waves = std::min<int64_t>((n + 63) / 64, D->slots_fast / 64);
    HIP_TRY(psb_lane_launch(D->P_fast, (unsigned)waves, s));
  } else if (D->fast_enabled) {
    const int64_t grid = std::min<int64_t>(n, D->slots_fast);
    HIP_TRY(launch_decode_kernel(0, D->acct, D->deep, (unsigned)grid, D->lds_fast, s, D->P_fast));
  }
  const int64_t grid_o = D->fast_enabled ? D->slots_ovf : std::min<int64_t>(n, D->slots_ovf);
  HIP_TRY(launch_decode_kernel(1, D->acct, D->deep, (unsigned)grid_o, D->lds_ovf, s, D->P_ovf));
  return PSB_OK;
}

static int32_t check_batch_args(psb_decoder* D, const uint8_t* syndromes, int64_t n, int32_t* edges,
                                int32_t* n_edges, int64_t* weight, uint64_t* obs, int32_t* status) {
  if (!D) return fail(PSB_E_INVALID, "null decoder");
  if (n < 0) return fail(PSB_E_INVALID, "negative batch size");
  if (n > (int64_t)INT32_MAX) return fail(PSB_E_INVALID, "batch too large");
  if (n > 0 && (!syndromes || !edges || !n_edges || !weight || !obs || !status)) return fail(PSB_E_INVALID, "null output");
  return PSB_OK;
}

extern "C" int32_t psb_decode_batch(psb_decoder* D, const uint8_t* syndromes, int64_t n, int32_t* edges,
                                    int32_t* n_edges, int64_t* weight, uint64_t* obs, int32_t* status,
                                    int8_t* levels, uint64_t* t_done, int32_t* stats, void* stream) {
  const int32_t rc = check_batch_args(D, syndromes, n, edges, n_edges, weight, obs, status);
  if (rc != PSB_OK || n == 0) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (D->fast_enabled && D->ovf_list_cap < n) {
    // a captured graph's kernel arguments point at the current list: it must not move
    if (D->n_graphs > 0)
      return fail(PSB_E_INVALID, "batch larger than the overflow list that a captured batch graph of this decoder "
                                 "holds; reserve the largest batch before capturing");
    // grows only between launches; the caller's stream is synchronised first
    HIP_TRY(hipStreamSynchronize(s));
    if (D->d_ovf_list) (void)hipFree(D->d_ovf_list);
    D->d_ovf_list = nullptr;
    D->ovf_list_cap = 0;
    if (hipMalloc((void**)&D->d_ovf_list, 4 * (3 * (size_t)n + kOrderBuckets)) != hipSuccess)
      return fail(PSB_E_NOMEM, "overflow list");
    D->ovf_list_cap = n;
  }
  return launch_batch(D, syndromes, n, edges, n_edges, weight, obs, status, levels, t_done, stats, D->d_counter,
                      D->d_ovf_list, D->fast_enabled ? D->d_ovf_list + D->ovf_list_cap : nullptr, s);
}

extern "C" int32_t psb_decode_batch_noalloc(psb_decoder* D, const uint8_t* syndromes, int64_t n, int32_t* edges,
                                            int32_t* n_edges, int64_t* weight, uint64_t* obs, int32_t* status,
                                            int8_t* levels, uint64_t* t_done, int32_t* stats, void* stream) {
  const int32_t rc = check_batch_args(D, syndromes, n, edges, n_edges, weight, obs, status);
  if (rc != PSB_OK || n == 0) return rc;
  if (n > PSB_NOALLOC_MAX_SHOTS)
    return fail(PSB_E_INVALID, "batch of " + std::to_string(n) + " shots exceeds the allocation-free limit of " +
                               std::to_string((long long)PSB_NOALLOC_MAX_SHOTS));
  int32_t* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    base = g_scratch_ptr[D->device];
  }
  if (!base) return fail(PSB_E_INTERNAL, "no scratch address for the decoder's device");
  // the fill kernel at the head of the launch clears the counters; the list
  // is written before it is read
  return launch_batch(D, syndromes, n, edges, n_edges, weight, obs, status, levels, t_done, stats, base,
                      base + kScratchHeader, nullptr, (hipStream_t)stream);
}

struct psb_batch_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  psb_decoder* dec = nullptr;        // its overflow list must not move while the graph exists
};

extern "C" int32_t psb_batch_graph_destroy(psb_batch_graph* B) {
  if (!B) return PSB_OK;
  if (B->dec) --B->dec->n_graphs;
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  delete B;
  return PSB_OK;
}

extern "C" int32_t psb_batch_graph_create(psb_decoder* D, const uint8_t* syndromes, int64_t n, int32_t* edges,
                                          int32_t* n_edges, int64_t* weight, uint64_t* obs, int32_t* status,
                                          int8_t* levels, uint64_t* t_done, int32_t* stats,
                                          psb_batch_graph** out) {
  if (!D || !out) return fail(PSB_E_INVALID, "null argument");
  *out = nullptr;
  if (n <= 0) return fail(PSB_E_INVALID, "a captured batch needs at least one shot");
  // per-batch storage sized before capture: nothing is allocated or synchronised inside it
  int32_t rc = psb_decoder_reserve(D, n);
  if (rc != PSB_OK) return rc;
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return fail(PSB_E_DEVICE, "capture stream");
  auto* B = new psb_batch_graph();
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipStreamDestroy(cs); delete B;
    return fail(PSB_E_DEVICE, "hipStreamBeginCapture");
  }
  rc = psb_decode_batch(D, syndromes, n, edges, n_edges, weight, obs, status, levels, t_done, stats, cs);
  const hipError_t e = hipStreamEndCapture(cs, &B->graph);
  B->dec = D;
  ++D->n_graphs;
  (void)hipStreamDestroy(cs);
  if (rc != PSB_OK || e != hipSuccess) {
    psb_batch_graph_destroy(B);
    return rc != PSB_OK ? rc : fail(PSB_E_DEVICE, "hipStreamEndCapture");
  }
  if (hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0) != hipSuccess) {
    psb_batch_graph_destroy(B);
    return fail(PSB_E_DEVICE, "hipGraphInstantiate");
  }
  *out = B;
  return PSB_OK;
}

extern "C" int32_t psb_batch_graph_launch(psb_batch_graph* B, void* stream) {
  if (!B || !B->exec) return fail(PSB_E_INVALID, "null batch graph");
  HIP_TRY(hipGraphLaunch(B->exec, (hipStream_t)stream));
  return PSB_OK;
}

extern "C" int32_t psb_schedule_levels(uint64_t wmax_hi, uint64_t wmax_lo, uint64_t diam_hi, uint64_t diam_lo,
                                       int64_t q_num, int64_t q_den, int64_t phi_min_num, int64_t phi_min_den,
                                       int32_t max_levels, uint64_t* d_hi, uint64_t* d_lo, uint64_t* b_hi,
                                       uint64_t* b_lo, int32_t* final_level) {
  if (q_num <= 0 || q_den <= q_num || phi_min_num <= 0 || phi_min_den <= phi_min_num)
    return fail(PSB_E_INVALID, "q and phi_min must lie in (0, 1)");
  const u128 wmax = ((u128)wmax_hi << 64) | wmax_lo, diam = ((u128)diam_hi << 64) | diam_lo;
  if (wmax == 0) return fail(PSB_E_INVALID, "w_max must be positive");
  LevelSchedule S;
  const int32_t rc = build_schedule(wmax, diam, q_num, q_den, phi_min_num, phi_min_den, S);
  if (rc != PSB_OK) return rc;
  const int32_t nl = (int32_t)std::min<size_t>(S.d.size(), (size_t)std::max(0, max_levels));
  for (int32_t k = 0; k < nl; ++k) {
    d_hi[k] = (uint64_t)(S.d[k] >> 64); d_lo[k] = (uint64_t)S.d[k];
    b_hi[k] = (uint64_t)(S.b[k] >> 64); b_lo[k] = (uint64_t)S.b[k];
    final_level[k] = S.final_level[k];
  }
  return nl;
}

extern "C" int32_t psb_decoder_last_overflow(psb_decoder* D, void* stream, int32_t* n_overflow) {
  if (!D || !n_overflow) return fail(PSB_E_INVALID, "null argument");
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  int32_t v[3] = {0, 0, 0};
  HIP_TRY(hipMemcpy(v, D->last_counter ? D->last_counter : D->d_counter, sizeof(v), hipMemcpyDeviceToHost));
  *n_overflow = D->fast_enabled ? v[1] : 0;
  return PSB_OK;
}
