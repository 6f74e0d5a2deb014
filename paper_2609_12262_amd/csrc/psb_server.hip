// Serving runtime: windows (shots) submitted one at a time from host threads
// while earlier ones decode.  A worker thread groups pending requests per
// (graph, weight class) into batches, runs each batch as one psb_decode_batch
// launch on that group's stream (groups of different graphs run
// concurrently), copies the results to pinned host memory and completes the
// tickets.  A result is identical to decoding the same syndrome alone with
// psb_decode_batch: the decoder is per graph and per weight set, and a shot's
// result does not depend on the other shots of its batch.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/psb.h"

namespace psb_host { int32_t fail(int32_t code, const std::string& msg); }
using psb_host::fail;

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  int32_t group = 0;
  int64_t scale = 1;                 // weight multiplier (uniform-weight requests decode on unit weights)
  std::vector<uint8_t> synd;
  bool done = false;
  int32_t status = 0;
  int64_t weight = 0;
  uint64_t obs = 0;
  std::vector<int32_t> edges;        // first min(n_edges, edges_per_shot) edge ids
  int64_t n_edges = 0;
  Clock::time_point t_submit, t_done;
};

// One decoder (graph x weight set) with its stream and batch buffers.
struct Group {
  psb_graph* own_graph = nullptr;    // unit-weight copy owned by the server, else null
  psb_decoder* dec = nullptr;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int64_t max_batch = 0;
  int32_t nbytes = 0, stride = 0;
  uint8_t *h_synd = nullptr, *d_synd = nullptr;
  int32_t *d_edges = nullptr, *d_ne = nullptr, *d_st = nullptr;
  int64_t* d_w = nullptr; uint64_t* d_obs = nullptr;
  int32_t *h_edges = nullptr, *h_ne = nullptr, *h_st = nullptr;
  int64_t* h_w = nullptr; uint64_t* h_obs = nullptr;
  hipEvent_t done_ev = nullptr;
  std::deque<uint64_t> pending;
  std::vector<uint64_t> inflight;
  bool busy = false;
};

}  // namespace

struct psb_server {
  int device = 0;
  std::vector<const psb_graph*> graphs;
  psb_decoder_opts opts{};
  int64_t budget = 0, used = 0;
  hipStream_t user_stream = nullptr;
  std::vector<std::unique_ptr<Group>> groups;    // [2 * graph + (unit weights ? 1 : 0)]
  std::unordered_map<uint64_t, Request> reqs;
  std::mutex mu;
  std::condition_variable cv;
  std::thread worker;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::string worker_error;
};

// graph accessors implemented in psb_lib.hip
extern "C" int32_t psb_graph_syndrome_bytes(const psb_graph* g);
int32_t psb_graph_unit_copy(const psb_graph* g, psb_graph** out);
int64_t psb_graph_edges(const psb_graph* g);

static void free_group(Group* G) {
  if (!G) return;
  if (G->done_ev) (void)hipEventDestroy(G->done_ev);
  for (void* p : {(void*)G->d_synd, (void*)G->d_edges, (void*)G->d_ne, (void*)G->d_st, (void*)G->d_w, (void*)G->d_obs})
    if (p) (void)hipFree(p);
  for (void* p : {(void*)G->h_synd, (void*)G->h_edges, (void*)G->h_ne, (void*)G->h_st, (void*)G->h_w, (void*)G->h_obs})
    if (p) (void)hipHostFree(p);
  if (G->dec) psb_decoder_destroy(G->dec);
  if (G->own_graph) psb_graph_destroy(G->own_graph);
  if (G->own_stream && G->stream) (void)hipStreamDestroy(G->stream);
}

// Builds the decoder and buffers of group `gi`; called with the lock held or
// before the worker starts.
static int32_t make_group(psb_server* S, int gi) {
  const int graph = gi / 2;
  const bool unit = gi % 2 == 1;
  auto G = std::make_unique<Group>();
  const psb_graph* g = S->graphs[graph];
  if (unit) {
    const int32_t rc = psb_graph_unit_copy(g, &G->own_graph);
    if (rc != PSB_OK) return rc;
    g = G->own_graph;
  }
  int32_t rc = psb_decoder_create(g, &S->opts, &G->dec);
  if (rc != PSB_OK) { free_group(G.get()); return rc; }
  G->nbytes = psb_graph_syndrome_bytes(g);
  G->stride = psb_decoder_edges_per_shot(G->dec);
  int32_t fs = 0, os = 0, lds = 0;
  psb_decoder_slots(G->dec, &fs, &os, &lds);
  int64_t ws = 0;
  psb_decoder_device_bytes(G->dec, &ws);
  G->max_batch = std::max<int64_t>(64, (int64_t)fs * 4);
  const int64_t per_shot = G->nbytes + 4LL * G->stride + 4 + 8 + 8 + 4;
  if (S->budget > 0) {
    const int64_t left = S->budget - S->used - ws;
    if (left < 64 * per_shot) {
      free_group(G.get());
      return fail(PSB_E_NOMEM, "device_mem_budget too small for another decoder and a 64-shot batch");
    }
    G->max_batch = std::min<int64_t>(G->max_batch, left / per_shot);
  }
  const int64_t B = G->max_batch;
  bool ok = hipMalloc((void**)&G->d_synd, (size_t)B * G->nbytes) == hipSuccess &&
            hipMalloc((void**)&G->d_edges, (size_t)B * G->stride * 4) == hipSuccess &&
            hipMalloc((void**)&G->d_ne, (size_t)B * 4) == hipSuccess &&
            hipMalloc((void**)&G->d_st, (size_t)B * 4) == hipSuccess &&
            hipMalloc((void**)&G->d_w, (size_t)B * 8) == hipSuccess &&
            hipMalloc((void**)&G->d_obs, (size_t)B * 8) == hipSuccess &&
            hipHostMalloc((void**)&G->h_synd, (size_t)B * G->nbytes, hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void**)&G->h_edges, (size_t)B * G->stride * 4, hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void**)&G->h_ne, (size_t)B * 4, hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void**)&G->h_st, (size_t)B * 4, hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void**)&G->h_w, (size_t)B * 8, hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void**)&G->h_obs, (size_t)B * 8, hipHostMallocDefault) == hipSuccess &&
            hipEventCreateWithFlags(&G->done_ev, hipEventDisableTiming) == hipSuccess;
  if (ok && S->user_stream) {
    G->stream = S->user_stream;
  } else if (ok) {
    ok = hipStreamCreateWithFlags(&G->stream, hipStreamNonBlocking) == hipSuccess;
    G->own_stream = ok;
  }
  if (!ok) { free_group(G.get()); return fail(PSB_E_NOMEM, "server batch buffers"); }
  S->used += ws + B * per_shot;
  S->groups[gi] = std::move(G);
  return PSB_OK;
}

// Launches the next batch of group G (lock held).
static void launch(psb_server* S, Group* G) {
  const int64_t k = std::min<int64_t>((int64_t)G->pending.size(), G->max_batch);
  G->inflight.clear();
  for (int64_t i = 0; i < k; ++i) {
    const uint64_t t = G->pending.front();
    G->pending.pop_front();
    G->inflight.push_back(t);
    memcpy(G->h_synd + i * G->nbytes, S->reqs[t].synd.data(), G->nbytes);
  }
  hipError_t e = hipMemcpyAsync(G->d_synd, G->h_synd, (size_t)k * G->nbytes, hipMemcpyHostToDevice, G->stream);
  int32_t rc = e == hipSuccess ? psb_decode_batch(G->dec, G->d_synd, k, G->d_edges, G->d_ne, G->d_w, G->d_obs,
                                                  G->d_st, nullptr, nullptr, nullptr, G->stream)
                               : PSB_E_DEVICE;
  if (rc == PSB_OK) {
    e = hipMemcpyAsync(G->h_ne, G->d_ne, (size_t)k * 4, hipMemcpyDeviceToHost, G->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(G->h_st, G->d_st, (size_t)k * 4, hipMemcpyDeviceToHost, G->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(G->h_w, G->d_w, (size_t)k * 8, hipMemcpyDeviceToHost, G->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(G->h_obs, G->d_obs, (size_t)k * 8, hipMemcpyDeviceToHost, G->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(G->h_edges, G->d_edges, (size_t)k * G->stride * 4, hipMemcpyDeviceToHost, G->stream);
    if (e == hipSuccess) e = hipEventRecord(G->done_ev, G->stream);
    if (e != hipSuccess) rc = PSB_E_DEVICE;
  }
  if (rc != PSB_OK) {
    // the batch cannot run: its requests complete with an internal status
    const auto now = Clock::now();
    for (uint64_t t : G->inflight) { Request& R = S->reqs[t]; R.done = true; R.status = PSB_S_INTERNAL; R.t_done = now; }
    G->inflight.clear();
    S->worker_error = "batch launch failed";
    S->cv.notify_all();
    return;
  }
  G->busy = true;
}

// Scatters a finished batch into its requests (lock held).
static void complete(psb_server* S, Group* G) {
  const auto now = Clock::now();
  for (size_t i = 0; i < G->inflight.size(); ++i) {
    Request& R = S->reqs[G->inflight[i]];
    R.status = G->h_st[i];
    R.weight = G->h_w[i] * R.scale;
    R.obs = G->h_obs[i];
    R.n_edges = G->h_ne[i];
    const int64_t m = std::min<int64_t>(R.n_edges, G->stride);
    R.edges.assign(G->h_edges + i * (int64_t)G->stride, G->h_edges + i * (int64_t)G->stride + m);
    R.synd.clear(); R.synd.shrink_to_fit();
    R.done = true;
    R.t_done = now;
  }
  G->inflight.clear();
  G->busy = false;
  S->cv.notify_all();
}

static void worker_main(psb_server* S) {
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  while (!S->stop) {
    bool busy = false, work = false;
    for (auto& up : S->groups) {
      Group* G = up.get();
      if (!G) continue;
      if (G->busy) {
        const hipError_t q = hipEventQuery(G->done_ev);
        if (q == hipSuccess) complete(S, G);
        else if (q != hipErrorNotReady) { S->worker_error = "device error while a batch ran"; complete(S, G); }
      }
      if (!G->busy && !G->pending.empty()) launch(S, G);
      busy |= G->busy;
      work |= !G->pending.empty();
    }
    if (busy || work) {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    } else {
      S->cv.wait(lk);
    }
  }
}

extern "C" int32_t psb_server_create(const psb_graph* const* graphs, int32_t n_graphs, const psb_decoder_opts* opts,
                                     int64_t device_mem_budget, void* stream, psb_server** out) {
  if (!graphs || n_graphs <= 0 || !out) return fail(PSB_E_INVALID, "null argument or no graphs");
  *out = nullptr;
  for (int32_t i = 0; i < n_graphs; ++i) if (!graphs[i]) return fail(PSB_E_INVALID, "null graph");
  if (device_mem_budget < 0) return fail(PSB_E_INVALID, "negative device_mem_budget");
  auto S = std::make_unique<psb_server>();
  if (hipGetDevice(&S->device) != hipSuccess) return fail(PSB_E_DEVICE, "hipGetDevice");
  S->graphs.assign(graphs, graphs + n_graphs);
  if (opts) S->opts = *opts;
  if (S->opts.edges_per_shot == 0) S->opts.edges_per_shot = 1024;   // results are copied per request
  S->budget = device_mem_budget;
  S->user_stream = (hipStream_t)stream;
  S->groups.resize(2 * (size_t)n_graphs);
  for (int32_t i = 0; i < n_graphs; ++i) {
    const int32_t rc = make_group(S.get(), 2 * i);
    if (rc != PSB_OK) { for (auto& G : S->groups) free_group(G.get()); return rc; }
  }
  psb_server* raw = S.release();
  raw->worker = std::thread(worker_main, raw);
  *out = raw;
  return PSB_OK;
}

extern "C" int32_t psb_server_submit(psb_server* S, int32_t graph_idx, const uint8_t* syndrome_host,
                                     const int32_t* w_override, uint64_t* ticket) {
  if (!S || !syndrome_host || !ticket) return fail(PSB_E_INVALID, "null argument");
  if (graph_idx < 0 || graph_idx >= (int32_t)S->graphs.size()) return fail(PSB_E_INVALID, "graph_idx out of range");
  int64_t scale = 1;
  int gi = 2 * graph_idx;
  if (w_override) {
    const int64_t m = psb_graph_edges(S->graphs[graph_idx]);
    const int32_t w0 = w_override[0];
    for (int64_t e = 1; e < m; ++e)
      if (w_override[e] != w0) return fail(PSB_E_UNSUPPORTED, "per-request weights must be uniform (one weight for every edge)");
    if (w0 <= 0) return fail(PSB_E_INVALID, "weights must be positive");
    scale = w0;
    gi += 1;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  if (!S->groups[gi]) {
    const int32_t rc = make_group(S, gi);
    if (rc != PSB_OK) return rc;
  }
  Group* G = S->groups[gi].get();
  const uint64_t t = S->next_ticket++;
  Request& R = S->reqs[t];
  R.group = gi;
  R.scale = scale;
  R.synd.assign(syndrome_host, syndrome_host + G->nbytes);
  R.t_submit = Clock::now();
  G->pending.push_back(t);
  *ticket = t;
  S->cv.notify_all();
  return PSB_OK;
}

extern "C" int32_t psb_server_poll(psb_server* S, uint64_t ticket, int32_t* done, int64_t* weight, uint64_t* obs,
                                   int32_t* edges, int64_t edges_cap, int64_t* n_edges, int32_t* status,
                                   int64_t* latency_ns) {
  if (!S || !done) return fail(PSB_E_INVALID, "null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return fail(PSB_E_INVALID, "unknown or already collected ticket");
  Request& R = it->second;
  *done = R.done ? 1 : 0;
  if (!R.done) return PSB_OK;
  if (weight) *weight = R.weight;
  if (obs) *obs = R.obs;
  if (n_edges) *n_edges = R.n_edges;
  if (status) *status = (R.n_edges > edges_cap && R.status == PSB_S_OK) ? PSB_S_EDGES_TRUNCATED : R.status;
  if (edges) {
    const int64_t m = std::min<int64_t>((int64_t)R.edges.size(), std::max<int64_t>(edges_cap, 0));
    if (m > 0) memcpy(edges, R.edges.data(), (size_t)m * 4);
  }
  if (latency_ns)
    *latency_ns = std::chrono::duration_cast<std::chrono::nanoseconds>(R.t_done - R.t_submit).count();
  S->reqs.erase(it);
  return PSB_OK;
}

extern "C" int32_t psb_server_destroy(psb_server* S) {
  if (!S) return PSB_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    S->cv.notify_all();
  }
  if (S->worker.joinable()) S->worker.join();
  for (auto& G : S->groups) {
    if (G && G->stream) (void)hipStreamSynchronize(G->stream);
    free_group(G.get());
  }
  delete S;
  return PSB_OK;
}
