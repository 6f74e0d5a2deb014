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

// Rows [0, n): the original syndrome with no x_j active; rows [n, 2n): the
// same with x_1 (detector n_orig) active.  One thread per output byte.
__global__ void comp_expand(const uint8_t* syn, int64_t n, int32_t in_bytes, int32_t n_orig, uint8_t* out,
                            int32_t out_bytes) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * n * out_bytes) return;
  const int64_t row = t / out_bytes;
  const int32_t k = (int32_t)(t % out_bytes);
  const int64_t i = row < n ? row : row - n;
  uint32_t v = 0;
  if (k < in_bytes) {
    v = syn[i * in_bytes + k];
    if (k == in_bytes - 1 && (n_orig & 7)) v &= (1u << (n_orig & 7)) - 1u;   // bits past the original detectors
  }
  if (row >= n && k == (n_orig >> 3)) v |= 1u << (n_orig & 7);
  out[row * out_bytes + k] = (uint8_t)v;
}

__global__ void comp_gap(int64_t n, const int64_t* wt, const uint64_t* ob, const int32_t* st, int64_t scale,
                         uint64_t obs_bit_mask, int64_t* w0, int64_t* w1, int64_t* gap, uint64_t* obs_best,
                         int32_t* status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t s = st[i] != PSB_S_OK ? st[i] : st[n + i];
  if (s == PSB_S_EDGES_TRUNCATED) s = PSB_S_OK;        // weights and observables stay valid
  status[i] = s;
  const int64_t a = wt[i] / scale, b = wt[n + i] / scale;
  w0[i] = a; w1[i] = b;
  gap[i] = a > b ? a - b : b - a;
  // the unconstrained optimum: the lighter side (ties to observable 0), with
  // the other observable bits of that side
  obs_best[i] = (b < a) ? ((ob[n + i] & ~obs_bit_mask) | obs_bit_mask) : (ob[i] & ~obs_bit_mask);
}

}  // namespace

struct psb_comp_plan {
  psb_graph* g = nullptr;
  psb_decoder* d = nullptr;
  int32_t n_orig = 0, in_bytes = 0, out_bytes = 0, stride = 0, obs_bit = 0;
  int64_t scale = 1;
  int64_t cap = 0;
  uint8_t* d_syn = nullptr;
  int32_t *d_edges = nullptr, *d_ne = nullptr, *d_st = nullptr;
  int64_t* d_wt = nullptr;
  uint64_t* d_ob = nullptr;
};

static void comp_free_buffers(psb_comp_plan* P) {
  for (void* p : {(void*)P->d_syn, (void*)P->d_edges, (void*)P->d_ne, (void*)P->d_st, (void*)P->d_wt, (void*)P->d_ob})
    if (p) (void)hipFree(p);
  P->d_syn = nullptr; P->d_edges = P->d_ne = P->d_st = nullptr; P->d_wt = nullptr; P->d_ob = nullptr;
  P->cap = 0;
}

extern "C" int32_t psb_comp_plan_destroy(psb_comp_plan* P) {
  if (!P) return PSB_OK;
  (void)hipDeviceSynchronize();
  comp_free_buffers(P);
  if (P->d) psb_decoder_destroy(P->d);
  if (P->g) psb_graph_destroy(P->g);
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
  // of every round are explored, and at d = 21 most of the graph.  Graphs the
  // wavefront overflow tier holds whole (1,024 detectors) keep the default
  // tiers; larger ones, unless the caller chose otherwise, decode in a
  // wavefront first tier sized to the whole rewritten graph (up to 8,192
  // detectors) with 1,024 regions per shot: its per-shot LDS block is then
  // about 128 KB, one wavefront per compute unit, with the event cache,
  // region bases and radius offsets in the workspace
  const bool caller_chose = opts && (opts->fast_max_nodes != 0 || opts->fast_max_regions != 0 || opts->first_tier != 0);
  if (!caller_chose && n + nx > 1024) {
    o.first_tier = 0;
    o.fast_max_nodes = (int32_t)std::min<int64_t>(n + nx, 8192);
    o.fast_max_regions = 1024;
  }
  int32_t rc = psb_graph_create(&cd, &P->g);
  if (rc == PSB_OK) rc = psb_decoder_create(P->g, &o, &P->d);
  if (rc != PSB_OK) return rc;
  P->n_orig = n; P->in_bytes = (n + 7) / 8; P->out_bytes = psb_graph_syndrome_bytes(P->g);
  P->stride = psb_decoder_edges_per_shot(P->d); P->obs_bit = obs_bit; P->scale = S;
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
    const int64_t r = 2 * n;
    bool ok = hipMalloc((void**)&P->d_syn, (size_t)r * P->out_bytes) == hipSuccess &&
              hipMalloc((void**)&P->d_edges, (size_t)r * P->stride * 4) == hipSuccess &&
              hipMalloc((void**)&P->d_ne, (size_t)r * 4) == hipSuccess &&
              hipMalloc((void**)&P->d_st, (size_t)r * 4) == hipSuccess &&
              hipMalloc((void**)&P->d_wt, (size_t)r * 8) == hipSuccess &&
              hipMalloc((void**)&P->d_ob, (size_t)r * 8) == hipSuccess;
    if (!ok) { comp_free_buffers(P); return fail(PSB_E_NOMEM, "complementary batch buffers"); }
    P->cap = n;
  }
  const unsigned tb = 256;
  const int64_t nb = 2 * n * P->out_bytes;
  comp_expand<<<(unsigned)((nb + tb - 1) / tb), tb, 0, s>>>(syndromes, n, P->in_bytes, P->n_orig, P->d_syn,
                                                            P->out_bytes);
  int32_t rc = psb_decode_batch(P->d, P->d_syn, 2 * n, P->d_edges, P->d_ne, P->d_wt, P->d_ob, P->d_st, nullptr,
                                nullptr, nullptr, stream);
  if (rc != PSB_OK) return rc;
  comp_gap<<<(unsigned)((n + tb - 1) / tb), tb, 0, s>>>(n, P->d_wt, P->d_ob, P->d_st, P->scale, 1ull << P->obs_bit,
                                                        weight0, weight1, gap, obs, status);
  if (hipGetLastError() != hipSuccess) return fail(PSB_E_DEVICE, "complementary kernel launch");
  return PSB_OK;
}
