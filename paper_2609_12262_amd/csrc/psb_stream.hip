// Streaming sliding-window decoding fed by the serving loop (Introduction:
// decoding a live stream of syndrome-extraction rounds in overlapping
// windows).  Each stream is one run of a layered detector graph (one layer of
// detectors per round) whose layers arrive over time.  The window rule is the
// one of window_rule.h; window k of a stream is decoded as soon as its last
// layer has arrived and window k - 1 has committed, by the slot server (one
// persistent kernel whose wavefronts take windows as they free up), so the
// windows of many streams share the GPU while each stream's windows stay in
// order.  A host thread collects finished windows with their edges and
// commits them on the stream's running syndrome: the committed edges' weights
// and observable masks are accumulated and both of their endpoints flipped,
// which resolves the committed layers and carries into the next window.  The
// result of a stream is the one psb_window_decode gives for it.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/psb.h"
#include "window_rule.h"

namespace psb_host { int32_t fail(int32_t code, const std::string& msg); }
using psb_host::fail;

namespace {

using Clock = std::chrono::steady_clock;

struct StreamState {
  std::vector<uint8_t> run;                   // running syndrome over the whole graph, packed LSB-first
  int32_t layers = 0;                         // layers arrived
  int32_t next = 0;                           // next window to decode
  bool in_flight = false, done = false;
  int64_t weight = 0;
  uint64_t obs = 0;
  int32_t status = PSB_S_OK;
  std::vector<Clock::time_point> layer_t;     // arrival time of each layer
  std::vector<int64_t> lat_ns;                // per committed window: commit minus its last layer's arrival
  std::vector<int64_t> dec_ns;                // per committed window: slot-server submit to decoded
};

}  // namespace

struct psb_stream_server {
  int32_t L = 0, n_layers = 0, W = 0, C = 0, n_det = 0, run_bytes = 0, stride = 0;
  std::vector<psb_host::WindowShape> shapes;
  std::vector<psb_host::WindowSpan> spans;
  std::vector<int32_t> gu, gv, gw;            // the whole graph's edges
  std::vector<uint64_t> gobs;
  std::vector<psb_graph*> graphs;             // one per window shape
  psb_slot_server* ss = nullptr;
  std::mutex mu;
  std::condition_variable cv;                 // wakes an idle worker when a window is submitted
  std::vector<StreamState> streams;
  std::unordered_map<uint64_t, std::pair<int32_t, int32_t>> tickets;   // ticket -> (stream, window)
  int64_t in_flight = 0;
  bool stop = false;
  std::thread worker;
  std::string error;
};

static void stream_free(psb_stream_server* S) {
  if (S->ss) psb_slot_server_destroy(S->ss);
  for (psb_graph* g : S->graphs) if (g) psb_graph_destroy(g);
}

// Submits the stream's next window if it is due (lock held): its layers have
// arrived and no window of the stream is in flight.
static void maybe_submit(psb_stream_server* S, int32_t i) {
  StreamState& T = S->streams[i];
  if (T.in_flight || T.done || T.next >= (int32_t)S->spans.size()) return;
  const psb_host::WindowSpan& sp = S->spans[T.next];
  if (T.layers < sp.end_layer) return;
  const psb_host::WindowShape& sh = S->shapes[sp.shape];
  // the window's bits [lo, lo + n_det) of the running syndrome, a byte at a time
  const int32_t nb = (sh.n_det + 7) / 8;
  std::vector<uint8_t> row(nb, 0);
  const int64_t lo = (int64_t)sp.first_layer * S->L;
  const int64_t b0 = lo >> 3;
  const int sh8 = (int)(lo & 7);
  for (int32_t j = 0; j < nb; ++j) {
    const uint32_t a = T.run[b0 + j];
    const uint32_t b = b0 + j + 1 < (int64_t)T.run.size() ? T.run[b0 + j + 1] : 0u;
    row[j] = (uint8_t)((a >> sh8) | (b << (8 - sh8)));
  }
  if (sh.n_det & 7) row[nb - 1] &= (uint8_t)((1u << (sh.n_det & 7)) - 1);
  const uint8_t* rp = row.data();
  const int32_t g = sp.shape;
  uint64_t ticket = 0;
  if (psb_slot_server_submit_many(S->ss, 1, &g, &rp, nullptr, &ticket) != PSB_OK) {
    T.status = PSB_S_INTERNAL; T.done = true;
    S->error = "window submission failed";
    return;
  }
  S->tickets[ticket] = {i, T.next};
  T.in_flight = true;
  ++S->in_flight;
  S->cv.notify_one();
}

// Commits window k of stream i from its decoded edges (lock held).
static void commit_window(psb_stream_server* S, int32_t i, int32_t k, int32_t status, const int32_t* edges,
                          int64_t n_edges, int64_t decode_ns) {
  StreamState& T = S->streams[i];
  T.in_flight = false;
  --S->in_flight;
  if (T.done) return;
  if (status != PSB_S_OK) { T.status = status; T.done = true; return; }
  const psb_host::WindowSpan& sp = S->spans[k];
  const psb_host::WindowShape& sh = S->shapes[sp.shape];
  for (int64_t j = 0; j < n_edges; ++j) {
    const int32_t e = edges[j];
    if (e < 0 || e >= (int32_t)sh.commit.size()) { T.status = PSB_S_INTERNAL; T.done = true; return; }
    if (!sh.commit[e]) continue;
    const int32_t g = sp.map[e];
    T.weight += S->gw[g];
    T.obs ^= S->gobs[g];
    T.run[S->gu[g] >> 3] ^= (uint8_t)(1u << (S->gu[g] & 7));
    if (S->gv[g] >= 0) T.run[S->gv[g] >> 3] ^= (uint8_t)(1u << (S->gv[g] & 7));
  }
  T.lat_ns.push_back(std::chrono::duration_cast<std::chrono::nanoseconds>(
                         Clock::now() - T.layer_t[sp.end_layer - 1]).count());
  T.dec_ns.push_back(decode_ns);
  T.next = k + 1;
  if (T.next == (int32_t)S->spans.size()) {
    for (uint8_t b : T.run) if (b) { T.status = PSB_S_INTERNAL; break; }   // every detection event resolved
    T.done = true;
    return;
  }
  maybe_submit(S, i);
}

static void worker_main(psb_stream_server* S) {
  const int32_t cap = 256;
  std::vector<uint64_t> t(cap);
  std::vector<int32_t> st(cap);
  std::vector<int64_t> lat(cap);
  std::vector<int32_t> edges((size_t)cap * S->stride);
  std::vector<int64_t> ne(cap);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(S->mu);
      if (S->in_flight == 0) {
        if (S->stop) return;
        S->cv.wait_for(lk, std::chrono::milliseconds(1));
        continue;
      }
    }
    const int32_t k = psb_slot_server_collect_edges(S->ss, cap, t.data(), nullptr, nullptr, st.data(), lat.data(),
                                                    edges.data(), S->stride, ne.data());
    if (k <= 0) {
      if (k < 0) { std::lock_guard<std::mutex> lk(S->mu); S->error = "collect failed"; }
      std::this_thread::yield();
      continue;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    for (int32_t q = 0; q < k; ++q) {
      auto it = S->tickets.find(t[q]);
      if (it == S->tickets.end()) continue;
      const auto iw = it->second;
      S->tickets.erase(it);
      commit_window(S, iw.first, iw.second, st[q], edges.data() + (int64_t)q * S->stride,
                    std::min<int64_t>(ne[q], S->stride), lat[q]);
    }
  }
}

extern "C" int32_t psb_stream_server_create(const psb_graph_desc* desc, int32_t layer_size, int32_t window_layers,
                                            int32_t commit_layers, const psb_decoder_opts* opts, int32_t n_streams,
                                            int32_t slots, psb_stream_server** out) {
  if (!desc || !out) return fail(PSB_E_INVALID, "null argument");
  *out = nullptr;
  const int32_t n = desc->num_detectors;
  const int64_t m = desc->num_edges;
  if (layer_size <= 0 || n <= 0 || n % layer_size != 0)
    return fail(PSB_E_INVALID, "num_detectors must be a positive multiple of layer_size");
  if (commit_layers <= 0 || window_layers <= commit_layers)
    return fail(PSB_E_INVALID, "need 0 < commit_layers < window_layers");
  if (n_streams <= 0 || slots < 0) return fail(PSB_E_INVALID, "need n_streams > 0 and slots >= 0");
  if (m > 0 && (!desc->u || !desc->v || !desc->w || !desc->obs_mask)) return fail(PSB_E_INVALID, "null edge array");
  for (int64_t e = 0; e < m; ++e)
    if (desc->u[e] < 0 || desc->u[e] >= n || desc->v[e] < PSB_BOUNDARY || desc->v[e] >= n)
      return fail(PSB_E_INVALID, "edge endpoint out of range");
  auto S = std::make_unique<psb_stream_server>();
  S->L = layer_size; S->n_layers = n / layer_size; S->W = window_layers; S->C = commit_layers; S->n_det = n;
  S->run_bytes = (n + 7) / 8;
  psb_host::build_windows(desc, layer_size, window_layers, commit_layers, S->shapes, S->spans);
  S->gu.assign(desc->u, desc->u + m); S->gv.assign(desc->v, desc->v + m); S->gw.assign(desc->w, desc->w + m);
  S->gobs.assign(desc->obs_mask, desc->obs_mask + m);
  int32_t rc = PSB_OK;
  for (const psb_host::WindowShape& H : S->shapes) {
    psb_graph_desc wd{};
    wd.num_detectors = H.n_det; wd.num_edges = (int64_t)H.u.size();
    wd.u = H.u.data(); wd.v = H.v.data(); wd.w = H.w.data(); wd.obs_mask = H.obs.data();
    psb_graph* g = nullptr;
    rc = psb_graph_create(&wd, &g);
    if (rc != PSB_OK) break;
    S->graphs.push_back(g);
  }
  std::vector<psb_decoder_opts> o(S->graphs.size(), opts ? *opts : psb_decoder_opts{});
  if (rc == PSB_OK)
    rc = psb_slot_server_create(S->graphs.data(), (int32_t)S->graphs.size(), o.data(), slots, 0, &S->ss);
  if (rc != PSB_OK) { stream_free(S.get()); return rc; }
  S->stride = std::max(1, o[0].edges_per_shot > 0 ? o[0].edges_per_shot : 1024);
  S->streams.resize(n_streams);
  for (StreamState& T : S->streams) {
    T.run.assign(S->run_bytes, 0);
    T.layer_t.resize(S->n_layers);
  }
  psb_stream_server* raw = S.release();
  raw->worker = std::thread(worker_main, raw);
  *out = raw;
  return PSB_OK;
}

// Takes layers [first_layer, first_layer + n_layers) of one stream (lock held).
static int32_t push_locked(psb_stream_server* S, int32_t stream, int32_t first_layer, int32_t n_layers,
                           const uint8_t* bits, Clock::time_point now) {
  if (!bits) return fail(PSB_E_INVALID, "null syndrome row");
  if (stream < 0 || stream >= (int32_t)S->streams.size()) return fail(PSB_E_INVALID, "stream out of range");
  StreamState& T = S->streams[stream];
  if (first_layer != T.layers) return fail(PSB_E_INVALID, "layers must arrive in order, each once");
  if (n_layers <= 0 || first_layer + n_layers > S->n_layers) return fail(PSB_E_INVALID, "layer range out of bounds");
  // XOR bits [lo, hi) of the row into the running syndrome, a byte at a time
  const int64_t lo = (int64_t)first_layer * S->L, hi = (int64_t)(first_layer + n_layers) * S->L;
  const int64_t b_lo = lo >> 3, b_hi = (hi - 1) >> 3;
  for (int64_t b = b_lo; b <= b_hi; ++b) {
    uint32_t mask = 0xffu;
    if (b == b_lo) mask &= 0xffu << (lo & 7);
    if (b == b_hi) mask &= 0xffu >> (7 - ((hi - 1) & 7));
    T.run[b] ^= (uint8_t)(bits[b] & mask);
  }
  for (int32_t l = first_layer; l < first_layer + n_layers; ++l) T.layer_t[l] = now;
  T.layers += n_layers;
  maybe_submit(S, stream);
  return PSB_OK;
}

extern "C" int32_t psb_stream_push(psb_stream_server* S, int32_t stream, int32_t first_layer, int32_t n_layers,
                                   const uint8_t* bits) {
  if (!S || !bits) return fail(PSB_E_INVALID, "null argument");
  const auto now = Clock::now();
  std::lock_guard<std::mutex> lk(S->mu);
  return push_locked(S, stream, first_layer, n_layers, bits, now);
}

extern "C" int32_t psb_stream_push_many(psb_stream_server* S, int32_t n, const int32_t* streams, int32_t first_layer,
                                        int32_t n_layers, const uint8_t* const* rows) {
  if (!S || n < 0 || (n > 0 && (!streams || !rows))) return fail(PSB_E_INVALID, "null argument");
  const auto now = Clock::now();
  std::lock_guard<std::mutex> lk(S->mu);
  for (int32_t i = 0; i < n; ++i) {
    const int32_t rc = push_locked(S, streams[i], first_layer, n_layers, rows[i], now);
    if (rc != PSB_OK) return rc;
  }
  return PSB_OK;
}

extern "C" int32_t psb_stream_poll(psb_stream_server* S, int32_t stream, int32_t* done, int32_t* committed_layers,
                                   int64_t* weight, uint64_t* obs, int32_t* status) {
  if (!S || !done) return fail(PSB_E_INVALID, "null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  if (stream < 0 || stream >= (int32_t)S->streams.size()) return fail(PSB_E_INVALID, "stream out of range");
  const StreamState& T = S->streams[stream];
  *done = T.done ? 1 : 0;
  if (committed_layers)
    *committed_layers = T.next == (int32_t)S->spans.size() ? S->n_layers
                        : T.next == 0 ? 0 : S->spans[T.next - 1].first_layer + S->C;
  if (weight) *weight = T.weight;
  if (obs) *obs = T.obs;
  if (status) *status = T.status;
  return PSB_OK;
}

extern "C" int32_t psb_stream_latencies(psb_stream_server* S, int32_t stream, int32_t max, int64_t* ns,
                                        int64_t* decode_ns, int32_t* n) {
  if (!S || !n || (max > 0 && !ns) || max < 0) return fail(PSB_E_INVALID, "null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  if (stream < 0 || stream >= (int32_t)S->streams.size()) return fail(PSB_E_INVALID, "stream out of range");
  const StreamState& T = S->streams[stream];
  *n = (int32_t)T.lat_ns.size();
  for (int32_t k = 0; k < std::min<int32_t>(max, *n); ++k) {
    ns[k] = T.lat_ns[k];
    if (decode_ns) decode_ns[k] = T.dec_ns[k];
  }
  return PSB_OK;
}

extern "C" int32_t psb_stream_reset(psb_stream_server* S, int32_t stream) {
  if (!S) return fail(PSB_E_INVALID, "null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  if (stream < 0 || stream >= (int32_t)S->streams.size()) return fail(PSB_E_INVALID, "stream out of range");
  StreamState& T = S->streams[stream];
  if (T.in_flight) return fail(PSB_E_INVALID, "a window of the stream is still decoding");
  std::fill(T.run.begin(), T.run.end(), 0);
  T.layers = 0; T.next = 0; T.done = false; T.weight = 0; T.obs = 0; T.status = PSB_S_OK;
  T.lat_ns.clear(); T.dec_ns.clear();
  return PSB_OK;
}

extern "C" int32_t psb_stream_server_info(const psb_stream_server* S, int32_t* n_windows, int32_t* n_shapes,
                                          int32_t* n_layers) {
  if (!S) return fail(PSB_E_INVALID, "null argument");
  if (n_windows) *n_windows = (int32_t)S->spans.size();
  if (n_shapes) *n_shapes = (int32_t)S->shapes.size();
  if (n_layers) *n_layers = S->n_layers;
  return PSB_OK;
}

extern "C" int32_t psb_stream_server_destroy(psb_stream_server* S) {
  if (!S) return PSB_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;                           // windows in flight finish first
    S->cv.notify_one();
  }
  if (S->worker.joinable()) S->worker.join();
  stream_free(S);
  delete S;
  return PSB_OK;
}
