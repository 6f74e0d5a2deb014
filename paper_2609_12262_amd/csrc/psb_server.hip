// Serving runtime: windows (shots) submitted from host threads while earlier
// ones decode.  Requests are grouped per (graph, weight class).  A small pool
// of pipes (a stream, pinned and device batch buffers, and one decoder per
// group) runs batches: whenever a pipe is idle the worker thread gives it the
// group whose oldest waiting window is oldest, as one psb_decode_batch launch,
// copies the results to pinned host memory and completes the tickets.  A pipe
// only ever receives work while idle, so no batch waits behind another on a
// stream or hardware queue.  A result is identical to decoding the same
// syndrome alone with psb_decode_batch: the decoder is per graph and per
// weight set, and a shot's result does not depend on the other shots of its
// batch.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
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

// Pipes (streams with batch buffers).  One per hardware queue of the default
// HIP configuration: every pipe's stream then has a queue of its own.
constexpr int kPipes = 4;

// One stream and its batch buffers; it runs one batch at a time, of any
// group, on that group's decoder for this pipe (two batches of one decoder
// would share its per-slot workspaces).
struct Pipe {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int64_t cap = 0;                   // shots the buffers hold
  uint8_t *h_synd = nullptr, *d_synd = nullptr;
  int32_t *d_edges = nullptr, *d_ne = nullptr, *d_st = nullptr;
  int64_t* d_w = nullptr; uint64_t* d_obs = nullptr;
  int32_t *h_edges = nullptr, *h_ne = nullptr, *h_st = nullptr;
  int64_t* h_w = nullptr; uint64_t* h_obs = nullptr;
  hipEvent_t done_ev = nullptr;
  std::vector<uint64_t> inflight;
  int group = -1;                    // group of the batch in flight, -1 = idle
  Clock::time_point t_launch;
};

// Requests of one (graph, weight set): a FIFO and one decoder per pipe, all
// made with the group (decoder set-up synchronises the device, so making one
// while batches run would stall them).
struct Group {
  int32_t graph_idx = 0;
  const psb_graph* graph = nullptr;
  psb_graph* own_graph = nullptr;    // unit-weight copy owned by the server, else null
  int32_t nbytes = 0, stride = 0;
  int64_t max_batch = 0;             // shots per launch: one per first-tier slot
  std::deque<uint64_t> pending;
  std::vector<psb_decoder*> dec;     // [kPipes]
};

}  // namespace

struct psb_server {
  int device = 0;
  std::vector<const psb_graph*> graphs;
  std::vector<psb_decoder_opts> opts;            // per graph
  int64_t budget = 0, used = 0;
  hipStream_t user_stream = nullptr;
  int32_t max_nbytes = 0, max_stride = 0;
  std::vector<std::unique_ptr<Pipe>> pipes;
  std::vector<std::unique_ptr<Group>> groups;    // [2 * graph + (unit weights ? 1 : 0)]
  std::unordered_map<uint64_t, Request> reqs;
  std::deque<uint64_t> finished;                 // completion order, for psb_server_collect
  std::mutex mu;
  std::condition_variable cv;
  std::thread worker;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::string worker_error;
  // running totals reported by psb_server_stats
  int64_t n_batches = 0, n_windows = 0, queue_ns = 0, run_ns = 0, launch_ns = 0;
};

static int64_t ns_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(b - a).count();
}

// graph accessors implemented in psb_lib.hip
extern "C" int32_t psb_graph_syndrome_bytes(const psb_graph* g);
int32_t psb_graph_unit_copy(const psb_graph* g, psb_graph** out);
int64_t psb_graph_edges(const psb_graph* g);

static void free_pipe(Pipe* P) {
  if (!P) return;
  if (P->stream) (void)hipStreamSynchronize(P->stream);
  if (P->done_ev) (void)hipEventDestroy(P->done_ev);
  for (void* p : {(void*)P->d_synd, (void*)P->d_edges, (void*)P->d_ne, (void*)P->d_st, (void*)P->d_w, (void*)P->d_obs})
    if (p) (void)hipFree(p);
  for (void* p : {(void*)P->h_synd, (void*)P->h_edges, (void*)P->h_ne, (void*)P->h_st, (void*)P->h_w, (void*)P->h_obs})
    if (p) (void)hipHostFree(p);
  if (P->own_stream && P->stream) (void)hipStreamDestroy(P->stream);
}

static void free_group(Group* G) {
  if (!G) return;
  for (psb_decoder* D : G->dec) if (D) psb_decoder_destroy(D);
  G->dec.clear();
  if (G->own_graph) psb_graph_destroy(G->own_graph);
  G->own_graph = nullptr;
}

// Per-shot bytes of a pipe's buffers.
static int64_t pipe_shot_bytes(const psb_server* S) { return S->max_nbytes + 4LL * S->max_stride + 4 + 8 + 8 + 4; }

// The pipes; their buffers hold `cap` shots of the largest graph.
static int32_t make_pipes(psb_server* S, int64_t cap) {
  for (int i = 0; i < kPipes; ++i) {
    auto P = std::make_unique<Pipe>();
    P->cap = cap;
    const int64_t B = cap;
    bool ok = hipMalloc((void**)&P->d_synd, (size_t)B * S->max_nbytes) == hipSuccess &&
              hipMalloc((void**)&P->d_edges, (size_t)B * S->max_stride * 4) == hipSuccess &&
              hipMalloc((void**)&P->d_ne, (size_t)B * 4) == hipSuccess &&
              hipMalloc((void**)&P->d_st, (size_t)B * 4) == hipSuccess &&
              hipMalloc((void**)&P->d_w, (size_t)B * 8) == hipSuccess &&
              hipMalloc((void**)&P->d_obs, (size_t)B * 8) == hipSuccess &&
              hipHostMalloc((void**)&P->h_synd, (size_t)B * S->max_nbytes, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc((void**)&P->h_edges, (size_t)B * S->max_stride * 4, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc((void**)&P->h_ne, (size_t)B * 4, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc((void**)&P->h_st, (size_t)B * 4, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc((void**)&P->h_w, (size_t)B * 8, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc((void**)&P->h_obs, (size_t)B * 8, hipHostMallocDefault) == hipSuccess &&
              hipEventCreateWithFlags(&P->done_ev, hipEventDisableTiming) == hipSuccess;
    if (ok && S->user_stream) {
      P->stream = S->user_stream;
    } else if (ok) {
      ok = hipStreamCreateWithFlags(&P->stream, hipStreamNonBlocking) == hipSuccess;
      P->own_stream = ok;
    }
    if (!ok) { free_pipe(P.get()); return fail(PSB_E_NOMEM, "server batch buffers"); }
    S->used += B * pipe_shot_bytes(S);
    S->pipes.push_back(std::move(P));
  }
  return PSB_OK;
}

static int32_t make_group(psb_server* S, int gi) {
  auto G = std::make_unique<Group>();
  G->graph_idx = gi / 2;
  G->graph = S->graphs[gi / 2];
  if (gi % 2 == 1) {
    const int32_t rc = psb_graph_unit_copy(G->graph, &G->own_graph);
    if (rc != PSB_OK) return rc;
    G->graph = G->own_graph;
  }
  G->nbytes = psb_graph_syndrome_bytes(G->graph);
  G->max_batch = S->pipes.empty() ? 0 : S->pipes[0]->cap;
  int64_t added = 0;
  for (int i = 0; i < kPipes; ++i) {
    psb_decoder* D = nullptr;
    int32_t rc = psb_decoder_create(G->graph, &S->opts[G->graph_idx], &D);
    if (rc == PSB_OK) {
      G->dec.push_back(D);
      G->stride = psb_decoder_edges_per_shot(D);
      int32_t fs = 0, os = 0, lds = 0;
      psb_decoder_slots(D, &fs, &os, &lds);
      if (fs > 0) G->max_batch = std::min<int64_t>(G->max_batch, fs);
      int64_t ws = 0;
      psb_decoder_device_bytes(D, &ws);
      added += ws;
      if (S->budget > 0 && S->used + added > S->budget)
        rc = fail(PSB_E_NOMEM, "device_mem_budget too small for this group's decoders");
      else if (G->stride > S->max_stride)
        rc = fail(PSB_E_INTERNAL, "decoder output stride exceeds the pipe buffers");
      else
        rc = psb_decoder_reserve(D, std::max<int64_t>(1, S->pipes[0]->cap));
    }
    if (rc != PSB_OK) { free_group(G.get()); return rc; }
  }
  G->max_batch = std::max<int64_t>(1, G->max_batch);
  S->used += added;
  S->groups[gi] = std::move(G);
  return PSB_OK;
}

// Launches the next batch of group gi on idle pipe P (lock held).
static void launch(psb_server* S, int gi, int pipe_idx) {
  Group* G = S->groups[gi].get();
  Pipe* P = S->pipes[pipe_idx].get();
  const int64_t k = std::min<int64_t>((int64_t)G->pending.size(), G->max_batch);
  const auto t0 = Clock::now();
  P->inflight.clear();
  for (int64_t i = 0; i < k; ++i) {
    const uint64_t t = G->pending.front();
    G->pending.pop_front();
    P->inflight.push_back(t);
    const Request& R = S->reqs[t];
    memcpy(P->h_synd + i * G->nbytes, R.synd.data(), G->nbytes);
    S->queue_ns += ns_between(R.t_submit, t0);
  }
  hipError_t e = hipMemcpyAsync(P->d_synd, P->h_synd, (size_t)k * G->nbytes, hipMemcpyHostToDevice, P->stream);
  int32_t rc = e == hipSuccess ? psb_decode_batch(G->dec[pipe_idx], P->d_synd, k, P->d_edges, P->d_ne, P->d_w,
                                                  P->d_obs, P->d_st, nullptr, nullptr, nullptr, P->stream)
                               : PSB_E_DEVICE;
  if (rc == PSB_OK) {
    e = hipMemcpyAsync(P->h_ne, P->d_ne, (size_t)k * 4, hipMemcpyDeviceToHost, P->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(P->h_st, P->d_st, (size_t)k * 4, hipMemcpyDeviceToHost, P->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(P->h_w, P->d_w, (size_t)k * 8, hipMemcpyDeviceToHost, P->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(P->h_obs, P->d_obs, (size_t)k * 8, hipMemcpyDeviceToHost, P->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(P->h_edges, P->d_edges, (size_t)k * G->stride * 4, hipMemcpyDeviceToHost, P->stream);
    if (e == hipSuccess) e = hipEventRecord(P->done_ev, P->stream);
    if (e != hipSuccess) rc = PSB_E_DEVICE;
  }
  if (rc != PSB_OK) {
    // the batch cannot run: its requests complete with an internal status
    const auto now = Clock::now();
    for (uint64_t t : P->inflight) {
      Request& R = S->reqs[t]; R.done = true; R.status = PSB_S_INTERNAL; R.t_done = now;
      S->finished.push_back(t);
    }
    P->inflight.clear();
    S->worker_error = "batch launch failed";
    S->cv.notify_all();
    return;
  }
  P->group = gi;
  P->t_launch = Clock::now();
  S->n_batches += 1;
  S->n_windows += k;
  S->launch_ns += ns_between(t0, P->t_launch);
}

// Scatters pipe P's finished batch into its requests (lock held); a batch
// whose device work failed completes with an internal status.
static void complete(psb_server* S, Pipe* P, bool ok) {
  const Group* G = S->groups[P->group].get();
  const auto now = Clock::now();
  S->run_ns += ns_between(P->t_launch, now);
  for (size_t i = 0; i < P->inflight.size(); ++i) {
    Request& R = S->reqs[P->inflight[i]];
    R.status = ok ? P->h_st[i] : PSB_S_INTERNAL;
    R.weight = P->h_w[i] * R.scale;
    R.obs = P->h_obs[i];
    R.n_edges = P->h_ne[i];
    const int64_t m = std::min<int64_t>(R.n_edges, G->stride);
    R.edges.assign(P->h_edges + i * (int64_t)G->stride, P->h_edges + i * (int64_t)G->stride + m);
    R.synd.clear(); R.synd.shrink_to_fit();
    R.done = true;
    R.t_done = now;
    S->finished.push_back(P->inflight[i]);
  }
  P->inflight.clear();
  P->group = -1;
  // tickets already taken by psb_server_poll stay in the completion list
  // until psb_server_collect passes them; drop them once they dominate it
  if (S->finished.size() > 2 * S->reqs.size() + 4096) {
    std::deque<uint64_t> keep;
    for (uint64_t t : S->finished) if (S->reqs.count(t)) keep.push_back(t);
    S->finished.swap(keep);
  }
  S->cv.notify_all();
}

// Group whose oldest waiting window is oldest, or -1 (lock held).
static int oldest_group(const psb_server* S) {
  int best = -1;
  Clock::time_point tb;
  for (size_t gi = 0; gi < S->groups.size(); ++gi) {
    const Group* G = S->groups[gi].get();
    if (!G || G->pending.empty()) continue;
    const Clock::time_point t = S->reqs.at(G->pending.front()).t_submit;
    if (best < 0 || t < tb) { best = (int)gi; tb = t; }
  }
  return best;
}

static void worker_main(psb_server* S) {
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  while (!S->stop) {
    bool busy = false;
    for (auto& up : S->pipes) {
      Pipe* P = up.get();
      if (P->group < 0) continue;
      const hipError_t q = hipEventQuery(P->done_ev);
      if (q == hipSuccess) complete(S, P, true);
      else if (q != hipErrorNotReady) { S->worker_error = "device error while a batch ran"; complete(S, P, false); }
    }
    for (size_t i = 0; i < S->pipes.size(); ++i) {
      if (S->pipes[i]->group >= 0) continue;
      const int gi = oldest_group(S);
      if (gi < 0) break;
      launch(S, gi, (int)i);
    }
    for (auto& up : S->pipes) busy |= up->group >= 0;
    const bool work = oldest_group(S) >= 0;
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
  S->opts.assign(n_graphs, psb_decoder_opts{});
  int64_t cap = 64;
  for (int32_t i = 0; i < n_graphs; ++i) {
    psb_decoder_opts& o = S->opts[i];
    if (opts) o = opts[i];
    if (o.edges_per_shot < 0 || o.num_slots < 0) return fail(PSB_E_INVALID, "negative edges_per_shot or num_slots");
    if (o.edges_per_shot == 0) o.edges_per_shot = 1024;       // results are copied per request
    if (o.num_slots == 0) o.num_slots = 1024;                 // one batch = one shot per slot
    if (o.overflow_slots == 0) o.overflow_slots = 256;
    S->max_nbytes = std::max(S->max_nbytes, psb_graph_syndrome_bytes(graphs[i]));
    S->max_stride = std::max(S->max_stride, o.edges_per_shot);
    cap = std::max<int64_t>(cap, o.num_slots);
  }
  S->budget = device_mem_budget;
  S->user_stream = (hipStream_t)stream;
  if (S->budget > 0) {
    // pipes take at most half the budget; the decoders the rest
    const int64_t fit = S->budget / 2 / (kPipes * pipe_shot_bytes(S.get()));
    if (fit < 64) return fail(PSB_E_NOMEM, "device_mem_budget too small for 64-shot batches");
    cap = std::min(cap, fit);
  }
  int32_t rc = make_pipes(S.get(), cap);
  S->groups.resize(2 * (size_t)n_graphs);
  for (int32_t i = 0; i < n_graphs && rc == PSB_OK; ++i) rc = make_group(S.get(), 2 * i);
  if (rc != PSB_OK) {
    for (auto& G : S->groups) free_group(G.get());
    for (auto& P : S->pipes) free_pipe(P.get());
    return rc;
  }
  psb_server* raw = S.release();
  raw->worker = std::thread(worker_main, raw);
  *out = raw;
  return PSB_OK;
}

// Queues one window (lock held): gi = group index, scale = weight multiplier.
static int32_t enqueue(psb_server* S, int gi, int64_t scale, const uint8_t* syndrome_host, Clock::time_point t_submit,
                       uint64_t* ticket) {
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
  R.t_submit = t_submit;
  G->pending.push_back(t);
  *ticket = t;
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
  const auto t_submit = Clock::now();
  std::lock_guard<std::mutex> lk(S->mu);
  const int32_t rc = enqueue(S, gi, scale, syndrome_host, t_submit, ticket);
  if (rc == PSB_OK) S->cv.notify_all();
  return rc;
}

extern "C" int32_t psb_server_submit_many(psb_server* S, int32_t n, const int32_t* graph_idx,
                                          const uint8_t* const* syndromes, const int32_t* uniform_weight,
                                          uint64_t* tickets) {
  if (!S || n < 0 || (n > 0 && (!graph_idx || !syndromes || !tickets))) return fail(PSB_E_INVALID, "null argument");
  for (int32_t i = 0; i < n; ++i) {
    if (graph_idx[i] < 0 || graph_idx[i] >= (int32_t)S->graphs.size()) return fail(PSB_E_INVALID, "graph_idx out of range");
    if (!syndromes[i]) return fail(PSB_E_INVALID, "null syndrome");
    if (uniform_weight && uniform_weight[i] < 0) return fail(PSB_E_INVALID, "weights must be positive");
  }
  const auto t_submit = Clock::now();
  std::lock_guard<std::mutex> lk(S->mu);
  for (int32_t i = 0; i < n; ++i) {
    const int32_t w = uniform_weight ? uniform_weight[i] : 0;
    const int32_t rc = enqueue(S, 2 * graph_idx[i] + (w > 0 ? 1 : 0), w > 0 ? w : 1, syndromes[i], t_submit, &tickets[i]);
    if (rc != PSB_OK) { S->cv.notify_all(); return rc; }      // windows 0..i-1 stay queued
  }
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

extern "C" int32_t psb_server_collect(psb_server* S, int32_t max, uint64_t* tickets, int64_t* weight, uint64_t* obs,
                                      int32_t* status, int64_t* latency_ns) {
  if (!S || max < 0 || (max > 0 && !tickets)) return fail(PSB_E_INVALID, "null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  int32_t k = 0;
  while (k < max && !S->finished.empty()) {
    const uint64_t t = S->finished.front();
    S->finished.pop_front();
    auto it = S->reqs.find(t);
    if (it == S->reqs.end()) continue;            // already collected by psb_server_poll
    const Request& R = it->second;
    tickets[k] = t;
    if (weight) weight[k] = R.weight;
    if (obs) obs[k] = R.obs;
    if (status) status[k] = R.status;
    if (latency_ns) latency_ns[k] = std::chrono::duration_cast<std::chrono::nanoseconds>(R.t_done - R.t_submit).count();
    S->reqs.erase(it);
    ++k;
  }
  return k;
}

extern "C" int32_t psb_server_cancel(psb_server* S, uint64_t ticket, int32_t* cancelled) {
  if (!S || !cancelled) return fail(PSB_E_INVALID, "null argument");
  *cancelled = 0;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return fail(PSB_E_INVALID, "unknown or already collected ticket");
  Request& R = it->second;
  if (R.done) return PSB_OK;                       // finished (or cancelled) already
  Group* G = S->groups[R.group].get();
  auto q = std::find(G->pending.begin(), G->pending.end(), ticket);
  if (q == G->pending.end()) return PSB_OK;        // on the device: it completes normally
  G->pending.erase(q);
  R.done = true;
  R.status = PSB_S_CANCELLED;
  R.t_done = Clock::now();
  R.synd.clear(); R.synd.shrink_to_fit();
  S->finished.push_back(ticket);
  *cancelled = 1;
  return PSB_OK;
}

extern "C" int32_t psb_server_wait(psb_server* S, uint64_t ticket, int64_t timeout_us, int32_t* done) {
  if (!S || !done || timeout_us < 0) return fail(PSB_E_INVALID, "null argument or negative timeout");
  std::unique_lock<std::mutex> lk(S->mu);
  auto ready = [&]() { auto it = S->reqs.find(ticket); return it == S->reqs.end() || it->second.done; };
  if (S->reqs.find(ticket) == S->reqs.end()) return fail(PSB_E_INVALID, "unknown or already collected ticket");
  *done = S->cv.wait_for(lk, std::chrono::microseconds(timeout_us), ready) ? 1 : 0;
  return PSB_OK;
}

extern "C" int32_t psb_server_stats(psb_server* S, int64_t* out5) {
  if (!S || !out5) return fail(PSB_E_INVALID, "null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  out5[0] = S->n_batches; out5[1] = S->n_windows; out5[2] = S->queue_ns; out5[3] = S->run_ns;
  out5[4] = S->launch_ns;
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
  for (auto& P : S->pipes) free_pipe(P.get());
  for (auto& G : S->groups) free_group(G.get());
  delete S;
  return PSB_OK;
}
