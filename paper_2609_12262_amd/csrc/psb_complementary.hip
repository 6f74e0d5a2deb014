// Complementary-gap decoding: the MWEM under each value of one logical
// observable, and their weight difference (Introduction: the gap between the
// best correction and the best one that flips the logical observable is a
// measure of confidence; the MWEM is the problem of Results, "Decoding
// task").
//
// Requires every edge carrying observable bit b to be a boundary edge (the
// observable is a cut through the boundary).  The graph is rewritten:
//   * each such edge j ends at a new detector x_j instead of the boundary;
//   * consecutive x_j are joined by chain edges of weight 1;
//   * every original weight is multiplied by S, the smallest power of two
//     >= the number m of such edges.
// In an edge set with odd degree exactly at the active detectors, the chain
// edges add an even amount to the degrees of the x_j, so the number of
// observable edges has the parity of the number of active x_j: activating
// only x_1 forces observable bit b to 1, activating none forces it to 0.
// The chain edges used weigh at most m - 1 < S, so the original weight of each
// constrained optimum is its decoded weight divided by S (integer division).
// One side is the MWEM itself: each shot is decoded once on the original graph
// and once on the rewritten graph, with the other value of the bit forced.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <memory>
#include <string>
#include <vector>

#include "../../include/psb.h"

namespace psb_host { int32_t fail(int32_t code, const std::string& msg); }
using psb_host::fail;

namespace {

// Row i: the original syndrome, with x_1 (detector n_orig) active exactly
// when the MWEM of shot i has observable bit 0, so that the rewritten graph's
// decode returns the minimum with the other value of the bit.  One thread per
// output byte.
__global__ void comp_expand(const uint8_t* syn, int64_t n, int32_t in_bytes, int32_t n_orig, const uint64_t* mwem_obs,
                            uint64_t obs_bit_mask, uint8_t* out, int32_t out_bytes) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * out_bytes) return;
  const int64_t i = t / out_bytes;
  const int32_t k = (int32_t)(t % out_bytes);
  uint32_t v = 0;
  if (k < in_bytes) {
    v = syn[i * in_bytes + k];
    if (k == in_bytes - 1 && (n_orig & 7)) v &= (1u << (n_orig & 7)) - 1u;   // bits past the original detectors
  }
  if (k == (n_orig >> 3) && (mwem_obs[i] & obs_bit_mask) == 0) v |= 1u << (n_orig & 7);
  out[i * out_bytes + k] = (uint8_t)v;
}

// a = the MWEM (original graph), b = the constrained minimum with the other
// value of the bit (rewritten graph, scaled weights).
__global__ void comp_gap(int64_t n, const int64_t* wa, const uint64_t* oa, const int32_t* sa, const int64_t* wb,
                         const uint64_t* ob, const int32_t* sb, int64_t scale, uint64_t obs_bit_mask, int64_t* w0,
                         int64_t* w1, int64_t* gap, uint64_t* obs_best, int32_t* status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t s = sa[i] != PSB_S_OK ? sa[i] : sb[i];
  if (s == PSB_S_EDGES_TRUNCATED) s = PSB_S_OK;        // weights and observables stay valid
  status[i] = s;
  const int64_t a = wa[i], b = wb[i] / scale;
  const bool mwem_one = (oa[i] & obs_bit_mask) != 0;
  w0[i] = mwem_one ? b : a;
  w1[i] = mwem_one ? a : b;
  gap[i] = b - a;                                      // a is the minimum over both values
  // the lighter side's observables; on a tie, the side with the bit at 0
  obs_best[i] = (mwem_one && b == a) ? (ob[i] & ~obs_bit_mask) : oa[i];
}

}  // namespace

struct psb_comp_plan {
  psb_graph *g = nullptr, *g0 = nullptr;        // rewritten graph, original graph
  psb_decoder *d = nullptr, *d0 = nullptr;
  int32_t n_orig = 0, in_bytes = 0, out_bytes = 0, stride = 0, stride0 = 0, obs_bit = 0;
  int64_t scale = 1;
  int64_t cap = 0;
  uint8_t* d_syn = nullptr;
  int32_t *d_edges = nullptr, *d_ne = nullptr, *d_st = nullptr;      // rewritten-graph decode
  int64_t* d_wt = nullptr;
  uint64_t* d_ob = nullptr;
  int32_t *d_edges0 = nullptr, *d_ne0 = nullptr, *d_st0 = nullptr;   // MWEM decode
  int64_t* d_wt0 = nullptr;
  uint64_t* d_ob0 = nullptr;
};

static void comp_free_buffers(psb_comp_plan* P) {
  for (void* p : {(void*)P->d_syn, (void*)P->d_edges, (void*)P->d_ne, (void*)P->d_st, (void*)P->d_wt, (void*)P->d_ob,
                  (void*)P->d_edges0, (void*)P->d_ne0, (void*)P->d_st0, (void*)P->d_wt0, (void*)P->d_ob0})
    if (p) (void)hipFree(p);
  P->d_syn = nullptr; P->d_edges = P->d_ne = P->d_st = nullptr; P->d_wt = nullptr; P->d_ob = nullptr;
  P->d_edges0 = P->d_ne0 = P->d_st0 = nullptr; P->d_wt0 = nullptr; P->d_ob0 = nullptr;
  P->cap = 0;
}

extern "C" int32_t psb_comp_plan_destroy(psb_comp_plan* P) {
  if (!P) return PSB_OK;
  (void)hipDeviceSynchronize();
  comp_free_buffers(P);
  if (P->d) psb_decoder_destroy(P->d);
  if (P->g) psb_graph_destroy(P->g);
  if (P->d0) psb_decoder_destroy(P->d0);
  if (P->g0) psb_graph_destroy(P->g0);
  delete P;
  return PSB_OK;
}

extern "C" int32_t psb_comp_plan_create(const psb_graph_desc* desc, int32_t obs_bit, const psb_decoder_opts* opts,
                                        psb_comp_plan** out) {
  if (!desc || !out) return fail(PSB_E_INVALID, "null argument");
  *out = nullptr;
  if (obs_bit < 0 || obs_bit > 63) return fail(PSB_E_INVALID, "obs_bit must be 0..63");
  const int32_t n = desc->num_detectors;
  const int64_t m = desc->num_edges;
  if (n <= 0 || m < 0) return fail(PSB_E_INVALID, "empty graph");
  if (m > 0 && (!desc->u || !desc->v || !desc->w || !desc->obs_mask)) return fail(PSB_E_INVALID, "null edge array");
  const uint64_t bit = 1ull << obs_bit;
  std::vector<int64_t> cut;
  int64_t wmax = 0;
  for (int64_t e = 0; e < m; ++e) {
    if (desc->w[e] <= 0) return fail(PSB_E_INVALID, "weights must be positive");
    wmax = std::max<int64_t>(wmax, desc->w[e]);
    if (desc->obs_mask[e] & bit) {
      if (desc->v[e] != PSB_BOUNDARY)
        return fail(PSB_E_UNSUPPORTED, "an edge carrying the observable is not a boundary edge");
      cut.push_back(e);
    }
  }
  if (cut.empty()) return fail(PSB_E_UNSUPPORTED, "no edge carries the observable");
  int64_t S = 1;
  while (S < (int64_t)cut.size()) S <<= 1;
  if (wmax * S >= (1LL << 31)) return fail(PSB_E_UNSUPPORTED, "scaled weights exceed int32");
  const int64_t nx = (int64_t)cut.size();
  if ((int64_t)n + nx >= (1LL << 31)) return fail(PSB_E_UNSUPPORTED, "too many detectors");
  std::vector<int32_t> u(desc->u, desc->u + m), v(desc->v, desc->v + m), w(m);
  std::vector<uint64_t> ob(desc->obs_mask, desc->obs_mask + m);
  for (int64_t e = 0; e < m; ++e) w[e] = (int32_t)(desc->w[e] * S);
  for (int64_t j = 0; j < nx; ++j) v[cut[j]] = n + (int32_t)j;          // observable edge j ends at x_j
  for (int64_t j = 0; j + 1 < nx; ++j) {                               // chain x_j - x_{j+1}
    u.push_back(n + (int32_t)j); v.push_back(n + (int32_t)j + 1); w.push_back(1); ob.push_back(0);
  }
  auto P = std::unique_ptr<psb_comp_plan, int32_t (*)(psb_comp_plan*)>(new psb_comp_plan(), psb_comp_plan_destroy);
  psb_graph_desc cd{};
  cd.num_detectors = n + (int32_t)nx; cd.num_edges = (int64_t)u.size();
  cd.u = u.data(); cd.v = v.data(); cd.w = w.data(); cd.obs_mask = ob.data();
  // the weight-1 chain makes the clustering's path depth (b_k / w_min) unbounded: the rewritten graph is
  // decoded by global sparse blossom, whose result is the same MWEM (Theorem 1)
  psb_decoder_opts o{};
  if (opts) o = *opts;
  o.mode = 1;
  // once a region reaches an x_j the whole chain and the observable boundary
  // of every round are explored, and at d = 21 most of the graph.  Unless the
  // caller chose otherwise, the first tier is a wavefront tier sized to the
  // whole rewritten graph (up to 8,192 detectors).  Graphs the overflow tier
  // holds whole (1,024 detectors) keep 208 regions per shot and the usual
  // placement (event cache, region bases and radius offsets in the workspace,
  // the rest in LDS); larger ones get 512 regions (at most 512 detection
  // events) and keep the whole per-shot state in the workspace: in LDS it
  // would take about 79 KB at d = 21 and leave room for two wavefronts per
  // compute unit instead of sixteen
  const bool caller_chose = opts && (opts->fast_max_nodes != 0 || opts->fast_max_regions != 0 ||
                                     opts->first_tier != 0 || opts->fast_lds_state != 0);
  if (!caller_chose) {
    o.first_tier = 0;
    o.fast_max_nodes = (int32_t)std::min<int64_t>(n + nx, 8192);
    o.fast_max_regions = n + nx > 1024 ? 512 : 208;
    if (n + nx > 1024) o.fast_lds_state = 4;
  }
  int32_t rc = psb_graph_create(&cd, &P->g);
  if (rc == PSB_OK) rc = psb_decoder_create(P->g, &o, &P->d);
  // the MWEM itself comes from the original graph, with the library's
  // default decoder (partition-and-fuse; the tie-break seed of opts).  A
  // graph whose weight spread needs deeper clustering paths than the kernel
  // enumerates falls back to global sparse blossom: the same MWEM (Theorem 1)
  psb_decoder_opts o0{};
  if (opts) { o0.tiebreak_seed = opts->tiebreak_seed; o0.boundary_reading = opts->boundary_reading; }
  if (rc == PSB_OK) rc = psb_graph_create(desc, &P->g0);
  if (rc == PSB_OK) {
    rc = psb_decoder_create(P->g0, &o0, &P->d0);
    if (rc == PSB_E_UNSUPPORTED) {
      o0.mode = 1;
      rc = psb_decoder_create(P->g0, &o0, &P->d0);
    }
  }
  if (rc != PSB_OK) return rc;
  P->n_orig = n; P->in_bytes = (n + 7) / 8; P->out_bytes = psb_graph_syndrome_bytes(P->g);
  P->stride = psb_decoder_edges_per_shot(P->d); P->stride0 = psb_decoder_edges_per_shot(P->d0);
  P->obs_bit = obs_bit; P->scale = S;
  *out = P.release();
  return PSB_OK;
}

extern "C" int32_t psb_comp_decode(psb_comp_plan* P, const uint8_t* syndromes, int64_t n, int64_t* weight0,
                                   int64_t* weight1, int64_t* gap, uint64_t* obs, int32_t* status, void* stream) {
  if (!P) return fail(PSB_E_INVALID, "null plan");
  if (n < 0) return fail(PSB_E_INVALID, "negative batch size");
  if (n == 0) return PSB_OK;
  if (!syndromes || !weight0 || !weight1 || !gap || !obs || !status) return fail(PSB_E_INVALID, "null argument");
  hipStream_t s = (hipStream_t)stream;
  if (n > P->cap) {
    if (hipStreamSynchronize(s) != hipSuccess) return fail(PSB_E_DEVICE, "hipStreamSynchronize");
    comp_free_buffers(P);
    bool ok = hipMalloc((void**)&P->d_syn, (size_t)n * P->out_bytes) == hipSuccess &&
              hipMalloc((void**)&P->d_edges, (size_t)n * P->stride * 4) == hipSuccess &&
              hipMalloc((void**)&P->d_ne, (size_t)n * 4) == hipSuccess &&
              hipMalloc((void**)&P->d_st, (size_t)n * 4) == hipSuccess &&
              hipMalloc((void**)&P->d_wt, (size_t)n * 8) == hipSuccess &&
              hipMalloc((void**)&P->d_ob, (size_t)n * 8) == hipSuccess &&
              hipMalloc((void**)&P->d_edges0, (size_t)n * P->stride0 * 4) == hipSuccess &&
              hipMalloc((void**)&P->d_ne0, (size_t)n * 4) == hipSuccess &&
              hipMalloc((void**)&P->d_st0, (size_t)n * 4) == hipSuccess &&
              hipMalloc((void**)&P->d_wt0, (size_t)n * 8) == hipSuccess &&
              hipMalloc((void**)&P->d_ob0, (size_t)n * 8) == hipSuccess;
    if (!ok) { comp_free_buffers(P); return fail(PSB_E_NOMEM, "complementary batch buffers"); }
    P->cap = n;
  }
  // 1. the MWEM of every shot on the original graph
  int32_t rc = psb_decode_batch(P->d0, syndromes, n, P->d_edges0, P->d_ne0, P->d_wt0, P->d_ob0, P->d_st0, nullptr,
                                nullptr, nullptr, stream);
  if (rc != PSB_OK) return rc;
  // 2. the rewritten graph with the other value of the observable bit
  const unsigned tb = 256;
  const uint64_t mask = 1ull << P->obs_bit;
  const int64_t nb = n * P->out_bytes;
  comp_expand<<<(unsigned)((nb + tb - 1) / tb), tb, 0, s>>>(syndromes, n, P->in_bytes, P->n_orig, P->d_ob0, mask,
                                                            P->d_syn, P->out_bytes);
  if (hipGetLastError() != hipSuccess) return fail(PSB_E_DEVICE, "complementary kernel launch");
  rc = psb_decode_batch(P->d, P->d_syn, n, P->d_edges, P->d_ne, P->d_wt, P->d_ob, P->d_st, nullptr, nullptr, nullptr,
                        stream);
  if (rc != PSB_OK) return rc;
  comp_gap<<<(unsigned)((n + tb - 1) / tb), tb, 0, s>>>(n, P->d_wt0, P->d_ob0, P->d_st0, P->d_wt, P->d_ob, P->d_st,
                                                        P->scale, mask, weight0, weight1, gap, obs, status);
  if (hipGetLastError() != hipSuccess) return fail(PSB_E_DEVICE, "complementary kernel launch");
  return PSB_OK;
}
