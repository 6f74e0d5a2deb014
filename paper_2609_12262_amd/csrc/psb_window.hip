// Sliding-window decoding of a batch of layered detector graphs' syndrome
// streams (Introduction: decoding a stream of syndrome-extraction rounds in
// overlapping windows, committing the corrections of the oldest rounds).  The
// window rule is in window_rule.h.  Each window's MWEM is decoded with
// psb_decode_batch; its committed edges' weights and observable masks are
// accumulated and both of their endpoints are flipped in the running
// syndrome, which resolves every detector of the committed layers and carries
// the flips of edges into the next window's first layer.  The last window
// reaches the final layer and commits everything; afterwards the running
// syndrome must be empty.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/psb.h"
#include "window_rule.h"

namespace psb_host { int32_t fail(int32_t code, const std::string& msg); }
using psb_host::fail;

namespace {

// One window shape: its graph, decoder and per-edge commit flags; windows of
// equal shape share them.
struct Shape {
  psb_graph* g = nullptr;
  psb_decoder* d = nullptr;
  int32_t n_det = 0, nbytes = 0, stride = 0;
  int64_t m = 0;
  uint8_t* d_commit = nullptr;     // [m] 1 = committed when matched
};

struct Window {
  int32_t first_layer = 0, shape = 0;
  int32_t* d_map = nullptr;        // [m] local edge -> edge of the full graph
};

// Copies bits [lo, lo + nbits) of each running row into a packed window row;
// bits past nbits in the last byte stay zero.  One thread per output byte.
__global__ void window_extract(const uint8_t* run, int32_t run_bytes, int64_t n, int64_t lo, int32_t nbits,
                               uint8_t* out, int32_t out_bytes) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * out_bytes) return;
  const int64_t i = t / out_bytes;
  const int32_t k = (int32_t)(t % out_bytes);
  const uint8_t* row = run + i * run_bytes;
  uint32_t v = 0;
  for (int b = 0; b < 8; ++b) {
    const int64_t j = 8LL * k + b;
    if (j >= nbits) break;
    const int64_t p = lo + j;
    v |= (uint32_t)((row[p >> 3] >> (p & 7)) & 1) << b;
  }
  out[i * out_bytes + k] = (uint8_t)v;
}

// Commits the matched edges of one window for shot i (one thread per shot).
__global__ void window_commit(int64_t n, const int32_t* edges, int32_t stride, const int32_t* n_edges,
                              const int32_t* st, const uint8_t* commit, const int32_t* map, const int32_t* u,
                              const int32_t* v, const int32_t* w, const uint64_t* obs, uint8_t* run,
                              int32_t run_bytes, int64_t* weight, uint64_t* obs_out, int32_t* status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (status[i] != PSB_S_OK) return;
  if (st[i] != PSB_S_OK || n_edges[i] > stride) {
    status[i] = st[i] != PSB_S_OK ? st[i] : PSB_S_EDGES_TRUNCATED;
    return;
  }
  uint8_t* row = run + i * run_bytes;
  int64_t wsum = 0;
  uint64_t o = 0;
  for (int32_t j = 0; j < n_edges[i]; ++j) {
    const int32_t e = edges[i * (int64_t)stride + j];
    if (!commit[e]) continue;
    const int32_t g = map[e];
    wsum += w[g];
    o ^= obs[g];
    row[u[g] >> 3] ^= (uint8_t)(1u << (u[g] & 7));
    if (v[g] >= 0) row[v[g] >> 3] ^= (uint8_t)(1u << (v[g] & 7));
  }
  weight[i] += wsum;
  obs_out[i] ^= o;
}

// After the last window every detection event must be resolved.
__global__ void window_check(int64_t n, const uint8_t* run, int32_t run_bytes, int32_t* status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || status[i] != PSB_S_OK) return;
  const uint8_t* row = run + i * run_bytes;
  for (int32_t k = 0; k < run_bytes; ++k)
    if (row[k]) { status[i] = PSB_S_INTERNAL; return; }
}

__global__ void window_init(int64_t n, int64_t* weight, uint64_t* obs, int32_t* status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  weight[i] = 0; obs[i] = 0; status[i] = PSB_S_OK;
}

template <typename T> bool dev_copy(T** dst, const std::vector<T>& src) {
  if (hipMalloc((void**)dst, std::max<size_t>(1, src.size()) * sizeof(T)) != hipSuccess) return false;
  return src.empty() || hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice) == hipSuccess;
}

}  // namespace

struct psb_window_plan {
  int32_t n_det = 0, layer = 0, n_layers = 0, W = 0, C = 0, run_bytes = 0;
  int64_t m = 0;
  std::vector<Shape> shapes;
  std::vector<Window> windows;
  int32_t *d_u = nullptr, *d_v = nullptr, *d_w = nullptr;
  uint64_t* d_obs = nullptr;
  // batch buffers, grown to the largest batch seen
  int64_t cap = 0;
  int32_t max_win_bytes = 0, max_stride = 0;
  uint8_t *d_run = nullptr, *d_win = nullptr;
  int32_t *d_edges = nullptr, *d_ne = nullptr, *d_st = nullptr;
  int64_t* d_wt = nullptr;
  uint64_t* d_ob = nullptr;
};

static void free_buffers(psb_window_plan* P) {
  for (void* p : {(void*)P->d_run, (void*)P->d_win, (void*)P->d_edges, (void*)P->d_ne, (void*)P->d_st,
                  (void*)P->d_wt, (void*)P->d_ob})
    if (p) (void)hipFree(p);
  P->d_run = P->d_win = nullptr; P->d_edges = P->d_ne = P->d_st = nullptr; P->d_wt = nullptr; P->d_ob = nullptr;
  P->cap = 0;
}

extern "C" int32_t psb_window_plan_destroy(psb_window_plan* P) {
  if (!P) return PSB_OK;
  (void)hipDeviceSynchronize();
  free_buffers(P);
  for (Window& w : P->windows) if (w.d_map) (void)hipFree(w.d_map);
  for (Shape& s : P->shapes) {
    if (s.d) psb_decoder_destroy(s.d);
    if (s.g) psb_graph_destroy(s.g);
    if (s.d_commit) (void)hipFree(s.d_commit);
  }
  for (void* p : {(void*)P->d_u, (void*)P->d_v, (void*)P->d_w, (void*)P->d_obs}) if (p) (void)hipFree(p);
  delete P;
  return PSB_OK;
}

extern "C" int32_t psb_window_plan_create(const psb_graph_desc* desc, int32_t layer_size, int32_t window_layers,
                                          int32_t commit_layers, const psb_decoder_opts* opts,
                                          psb_window_plan** out) {
  if (!desc || !out) return fail(PSB_E_INVALID, "null argument");
  *out = nullptr;
  const int32_t n = desc->num_detectors;
  const int64_t m = desc->num_edges;
  if (layer_size <= 0 || n <= 0 || n % layer_size != 0)
    return fail(PSB_E_INVALID, "num_detectors must be a positive multiple of layer_size");
  if (commit_layers <= 0 || window_layers <= commit_layers)
    return fail(PSB_E_INVALID, "need 0 < commit_layers < window_layers");
  if (m > 0 && (!desc->u || !desc->v || !desc->w || !desc->obs_mask)) return fail(PSB_E_INVALID, "null edge array");
  for (int64_t e = 0; e < m; ++e)
    if (desc->u[e] < 0 || desc->u[e] >= n || desc->v[e] < PSB_BOUNDARY || desc->v[e] >= n)
      return fail(PSB_E_INVALID, "edge endpoint out of range");
  auto P = std::unique_ptr<psb_window_plan, int32_t (*)(psb_window_plan*)>(new psb_window_plan(), psb_window_plan_destroy);
  P->n_det = n; P->layer = layer_size; P->n_layers = n / layer_size; P->W = window_layers; P->C = commit_layers;
  P->m = m; P->run_bytes = (n + 7) / 8;
  std::vector<psb_host::WindowShape> hs;
  std::vector<psb_host::WindowSpan> spans;
  psb_host::build_windows(desc, layer_size, window_layers, commit_layers, hs, spans);
  for (const psb_host::WindowShape& H : hs) {
    Shape S;
    psb_graph_desc wd{};
    wd.num_detectors = H.n_det; wd.num_edges = (int64_t)H.u.size();
    wd.u = H.u.data(); wd.v = H.v.data(); wd.w = H.w.data(); wd.obs_mask = H.obs.data();
    int32_t rc = psb_graph_create(&wd, &S.g);
    if (rc == PSB_OK) rc = psb_decoder_create(S.g, opts, &S.d);
    if (rc == PSB_OK && !dev_copy(&S.d_commit, H.commit)) rc = fail(PSB_E_NOMEM, "commit flags");
    if (rc != PSB_OK) {
      if (S.d) psb_decoder_destroy(S.d);
      if (S.g) psb_graph_destroy(S.g);
      if (S.d_commit) (void)hipFree(S.d_commit);
      return rc;
    }
    S.n_det = wd.num_detectors; S.nbytes = psb_graph_syndrome_bytes(S.g); S.m = wd.num_edges;
    S.stride = psb_decoder_edges_per_shot(S.d);
    P->shapes.push_back(S);
    P->max_win_bytes = std::max(P->max_win_bytes, S.nbytes);
    P->max_stride = std::max(P->max_stride, S.stride);
  }
  for (const psb_host::WindowSpan& sp : spans) {
    Window w;
    w.first_layer = sp.first_layer; w.shape = sp.shape;
    if (!dev_copy(&w.d_map, sp.map)) return fail(PSB_E_NOMEM, "edge map");
    P->windows.push_back(w);
  }
  std::vector<int32_t> u(desc->u, desc->u + m), v(desc->v, desc->v + m), wv(desc->w, desc->w + m);
  std::vector<uint64_t> ob(desc->obs_mask, desc->obs_mask + m);
  if (!dev_copy(&P->d_u, u) || !dev_copy(&P->d_v, v) || !dev_copy(&P->d_w, wv) || !dev_copy(&P->d_obs, ob))
    return fail(PSB_E_NOMEM, "graph arrays");
  *out = P.release();
  return PSB_OK;
}

extern "C" int32_t psb_window_plan_info(const psb_window_plan* P, int32_t* n_windows, int32_t* n_shapes) {
  if (!P) return fail(PSB_E_INVALID, "null plan");
  if (n_windows) *n_windows = (int32_t)P->windows.size();
  if (n_shapes) *n_shapes = (int32_t)P->shapes.size();
  return PSB_OK;
}

extern "C" int32_t psb_window_decode(psb_window_plan* P, const uint8_t* syndromes, int64_t n, int64_t* weight,
                                     uint64_t* obs, int32_t* status, void* stream) {
  if (!P) return fail(PSB_E_INVALID, "null plan");
  if (n < 0) return fail(PSB_E_INVALID, "negative batch size");
  if (n == 0) return PSB_OK;
  if (!syndromes || !weight || !obs || !status) return fail(PSB_E_INVALID, "null argument");
  hipStream_t s = (hipStream_t)stream;
  if (n > P->cap) {
    // grows between calls only: the stream is synchronised first
    if (hipStreamSynchronize(s) != hipSuccess) return fail(PSB_E_DEVICE, "hipStreamSynchronize");
    free_buffers(P);
    bool ok = hipMalloc((void**)&P->d_run, (size_t)n * P->run_bytes) == hipSuccess &&
              hipMalloc((void**)&P->d_win, (size_t)n * P->max_win_bytes) == hipSuccess &&
              hipMalloc((void**)&P->d_edges, (size_t)n * P->max_stride * 4) == hipSuccess &&
              hipMalloc((void**)&P->d_ne, (size_t)n * 4) == hipSuccess &&
              hipMalloc((void**)&P->d_st, (size_t)n * 4) == hipSuccess &&
              hipMalloc((void**)&P->d_wt, (size_t)n * 8) == hipSuccess &&
              hipMalloc((void**)&P->d_ob, (size_t)n * 8) == hipSuccess;
    if (!ok) { free_buffers(P); return fail(PSB_E_NOMEM, "window batch buffers"); }
    P->cap = n;
  }
  const unsigned tb = 256;
  const unsigned gs = (unsigned)((n + tb - 1) / tb);
  if (hipMemcpyAsync(P->d_run, syndromes, (size_t)n * P->run_bytes, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return fail(PSB_E_DEVICE, "syndrome copy");
  window_init<<<gs, tb, 0, s>>>(n, weight, obs, status);
  for (const Window& w : P->windows) {
    const Shape& S = P->shapes[w.shape];
    const int64_t lo = (int64_t)w.first_layer * P->layer;
    const int64_t nb = n * S.nbytes;
    window_extract<<<(unsigned)((nb + tb - 1) / tb), tb, 0, s>>>(P->d_run, P->run_bytes, n, lo, S.n_det, P->d_win,
                                                                  S.nbytes);
    int32_t rc = psb_decode_batch(S.d, P->d_win, n, P->d_edges, P->d_ne, P->d_wt, P->d_ob, P->d_st, nullptr, nullptr,
                                  nullptr, stream);
    if (rc != PSB_OK) return rc;
    window_commit<<<gs, tb, 0, s>>>(n, P->d_edges, S.stride, P->d_ne, P->d_st, S.d_commit, w.d_map, P->d_u, P->d_v,
                                    P->d_w, P->d_obs, P->d_run, P->run_bytes, weight, obs, status);
  }
  window_check<<<gs, tb, 0, s>>>(n, P->d_run, P->run_bytes, status);
  if (hipGetLastError() != hipSuccess) return fail(PSB_E_DEVICE, "window kernel launch");
  return PSB_OK;
}
