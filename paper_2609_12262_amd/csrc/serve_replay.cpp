// Load replay for the serving runtime (measurement tool, not on the decoding
// path): submits windows at given arrival times from a native thread while a
// second thread collects completions, so that the offered load is not
// limited by an interpreter; and the same stream decoded one window per
// launch, for comparison.  Built as libpsb_replay.so next to libpsb.so.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/psb.h"

// The two serving runtimes share the submit / collect calls' shape.
struct PipeServer {
  psb_server* s;
  int32_t submit_many(int32_t n, const int32_t* g, const uint8_t* const* syn, const int32_t* w, uint64_t* t) const {
    return psb_server_submit_many(s, n, g, syn, w, t);
  }
  int32_t collect(int32_t max, uint64_t* t, int32_t* st, int64_t* lat) const {
    return psb_server_collect(s, max, t, nullptr, nullptr, st, lat);
  }
};
struct SlotServer {
  psb_slot_server* s;
  int32_t submit_many(int32_t n, const int32_t* g, const uint8_t* const* syn, const int32_t* w, uint64_t* t) const {
    return psb_slot_server_submit_many(s, n, g, syn, w, t);
  }
  int32_t collect(int32_t max, uint64_t* t, int32_t* st, int64_t* lat) const {
    return psb_slot_server_collect(s, max, t, nullptr, nullptr, st, lat);
  }
};

template <class Srv>
static int32_t replay(const Srv& srv, int64_t n, const int32_t* graph_idx, const uint8_t* const* syndromes,
                      const int32_t* uniform_weight, const double* arrival_s, int64_t* latency_ns,
                      int32_t* status, double* submit_span_s, double* wall_s) {
  if (!srv.s || n <= 0 || !graph_idx || !syndromes || !latency_ns || !status) return -1;
  std::vector<uint64_t> tickets(n, 0);
  std::vector<int64_t> lag(n, 0);       // arrival to submission, added to the server's latency
  std::atomic<int64_t> submitted{0};
  std::atomic<int32_t> error{0};
  using Clock = std::chrono::steady_clock;
  const auto t0 = Clock::now();
  std::thread collector([&] {
    std::vector<uint64_t> t(4096);
    std::vector<int64_t> lat(4096);
    std::vector<int32_t> st(4096);
    std::unordered_map<uint64_t, int64_t> local;
    local.reserve((size_t)n * 2);
    int64_t got = 0, seen = 0;
    while (got < n && !error.load()) {
      const int32_t k = srv.collect(4096, t.data(), st.data(), lat.data());
      if (k < 0) { error = 1; break; }
      const int64_t sub = submitted.load(std::memory_order_acquire);
      for (; seen < sub; ++seen) local[tickets[seen]] = seen;
      for (int32_t j = 0; j < k; ++j) {
        auto it = local.find(t[j]);
        if (it == local.end()) {        // completed before its index was published: wait for it
          while (submitted.load(std::memory_order_acquire) == seen) std::this_thread::yield();
          const int64_t sub2 = submitted.load(std::memory_order_acquire);
          for (; seen < sub2; ++seen) local[tickets[seen]] = seen;
          it = local.find(t[j]);
          if (it == local.end()) { error = 2; break; }
        }
        latency_ns[it->second] = lat[j] + lag[it->second];
        status[it->second] = st[j];
        ++got;
      }
      if (k == 0) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
  });
  // windows whose arrival time has passed are submitted together (at most 1024 per call)
  constexpr int64_t kBurst = 1024;
  int64_t i = 0;
  while (i < n && !error.load()) {
    if (arrival_s) {
      while (std::chrono::duration<double>(Clock::now() - t0).count() < arrival_s[i]) {}
    }
    int64_t j = i + 1;
    if (arrival_s) {
      const double now = std::chrono::duration<double>(Clock::now() - t0).count();
      while (j < n && j - i < kBurst && arrival_s[j] <= now) ++j;
    } else {
      j = std::min<int64_t>(n, i + kBurst);
    }
    if (arrival_s) {
      const double now = std::chrono::duration<double>(Clock::now() - t0).count();
      for (int64_t k = i; k < j; ++k) lag[k] = (int64_t)((now - arrival_s[k]) * 1e9);
    }
    if (srv.submit_many((int32_t)(j - i), graph_idx + i, syndromes + i, uniform_weight ? uniform_weight + i : nullptr,
                        tickets.data() + i) != 0) {
      error = 3;
      break;
    }
    submitted.store(j, std::memory_order_release);
    i = j;
  }
  if (submit_span_s) *submit_span_s = std::chrono::duration<double>(Clock::now() - t0).count();
  collector.join();
  if (wall_s) *wall_s = std::chrono::duration<double>(Clock::now() - t0).count();
  return error.load() ? -error.load() : 0;
}

extern "C" int32_t psb_replay(psb_server* s, int64_t n, const int32_t* graph_idx, const uint8_t* const* syndromes,
                              const int32_t* uniform_weight, const double* arrival_s, int64_t* latency_ns,
                              int32_t* status, double* submit_span_s, double* wall_s) {
  return replay(PipeServer{s}, n, graph_idx, syndromes, uniform_weight, arrival_s, latency_ns, status, submit_span_s,
                wall_s);
}

extern "C" int32_t psb_replay_slots(psb_slot_server* s, int64_t n, const int32_t* graph_idx,
                                    const uint8_t* const* syndromes, const int32_t* uniform_weight,
                                    const double* arrival_s, int64_t* latency_ns, int32_t* status,
                                    double* submit_span_s, double* wall_s) {
  return replay(SlotServer{s}, n, graph_idx, syndromes, uniform_weight, arrival_s, latency_ns, status, submit_span_s,
                wall_s);
}

// The one-shot-per-launch form on the same stream of windows: one thread
// takes the windows in arrival order and decodes each alone (copy in, one
// psb_decode_batch of one shot, copy results out, wait), so a window that
// arrives while another decodes waits for it.  decs[dec_idx[i]] decodes
// window i; latency = completion minus arrival (minus the start of its own
// decode when arrival_s is NULL, i.e. back to back).
extern "C" int32_t psb_replay_oneshot(psb_decoder* const* decs, int32_t n_dec, int64_t n, const int32_t* dec_idx,
                                      const uint8_t* const* syndromes, const int32_t* syndrome_bytes,
                                      const double* arrival_s, int64_t* latency_ns, int32_t* status,
                                      double* wall_s) {
  if (!decs || n_dec <= 0 || n <= 0 || !dec_idx || !syndromes || !syndrome_bytes || !latency_ns || !status)
    return -1;
  int32_t max_bytes = 1, max_stride = 1;
  for (int32_t j = 0; j < n_dec; ++j) {
    max_bytes = std::max(max_bytes, syndrome_bytes[j]);
    max_stride = std::max(max_stride, psb_decoder_edges_per_shot(decs[j]));
  }
  hipStream_t s = nullptr;
  uint8_t *d_synd = nullptr, *h_synd = nullptr;
  int32_t *d_edges = nullptr, *d_small = nullptr, *h_edges = nullptr, *h_small = nullptr;
  int64_t* d_w = nullptr; uint64_t* d_obs = nullptr;
  int32_t rc = 0;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
      hipMalloc((void**)&d_synd, max_bytes) != hipSuccess ||
      hipMalloc((void**)&d_edges, 4 * (size_t)max_stride) != hipSuccess ||
      hipMalloc((void**)&d_small, 32) != hipSuccess || hipMalloc((void**)&d_w, 8) != hipSuccess ||
      hipMalloc((void**)&d_obs, 8) != hipSuccess ||
      hipHostMalloc((void**)&h_synd, max_bytes, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&h_edges, 4 * (size_t)max_stride + 64, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&h_small, 64, hipHostMallocDefault) != hipSuccess)
    rc = -2;
  using Clock = std::chrono::steady_clock;
  const auto t0 = Clock::now();
  for (int64_t i = 0; i < n && rc == 0; ++i) {
    const int32_t j = dec_idx[i];
    if (j < 0 || j >= n_dec) { rc = -1; break; }
    Clock::time_point t_arr;
    if (arrival_s) {
      t_arr = t0 + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(arrival_s[i]));
      while (Clock::now() < t_arr) {}
    } else {
      t_arr = Clock::now();
    }
    memcpy(h_synd, syndromes[i], syndrome_bytes[j]);
    const int32_t stride = psb_decoder_edges_per_shot(decs[j]);
    bool ok = hipMemcpyAsync(d_synd, h_synd, syndrome_bytes[j], hipMemcpyHostToDevice, s) == hipSuccess &&
              psb_decode_batch(decs[j], d_synd, 1, d_edges, d_small, d_w, d_obs, d_small + 1, nullptr, nullptr,
                               nullptr, s) == PSB_OK &&
              hipMemcpyAsync(h_small, d_small, 8, hipMemcpyDeviceToHost, s) == hipSuccess &&
              hipMemcpyAsync(h_small + 2, d_w, 8, hipMemcpyDeviceToHost, s) == hipSuccess &&
              hipMemcpyAsync(h_small + 4, d_obs, 8, hipMemcpyDeviceToHost, s) == hipSuccess &&
              hipMemcpyAsync(h_edges, d_edges, 4 * (size_t)stride, hipMemcpyDeviceToHost, s) == hipSuccess &&
              hipStreamSynchronize(s) == hipSuccess;
    if (!ok) { rc = -3; break; }
    latency_ns[i] = std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - t_arr).count();
    status[i] = h_small[1];
  }
  if (wall_s) *wall_s = std::chrono::duration<double>(Clock::now() - t0).count();
  if (s) (void)hipStreamSynchronize(s);
  for (void* p : {(void*)d_synd, (void*)d_edges, (void*)d_small, (void*)d_w, (void*)d_obs}) if (p) (void)hipFree(p);
  for (void* p : {(void*)h_synd, (void*)h_edges, (void*)h_small}) if (p) (void)hipHostFree(p);
  if (s) (void)hipStreamDestroy(s);
  return rc;
}

// Streaming windows at a syndrome rate: layer group g (layers_per_push layers)
// of every stream is pushed once its last round has been measured, at
// (g + 1) * layers_per_push * round_s after the start (round_s = 0: as fast as
// the pushes go), all streams in one call; then waits until every stream is done
// (at most timeout_s).  The server records each layer's actual arrival.
extern "C" int32_t psb_stream_replay(psb_stream_server* s, int32_t n_streams, const uint8_t* const* rows,
                                     int32_t n_layers, int32_t layers_per_push, double round_s, double timeout_s,
                                     double* wall_s, double* push_span_s) {
  if (!s || n_streams <= 0 || !rows || n_layers <= 0 || layers_per_push <= 0) return -1;
  using Clock = std::chrono::steady_clock;
  std::vector<int32_t> ids(n_streams);
  for (int32_t i = 0; i < n_streams; ++i) ids[i] = i;
  const auto t0 = Clock::now();
  auto since = [&] { return std::chrono::duration<double>(Clock::now() - t0).count(); };
  for (int32_t l0 = 0; l0 < n_layers; l0 += layers_per_push) {
    const int32_t n = std::min(layers_per_push, n_layers - l0);
    if (round_s > 0) {
      const double due = (l0 + n) * round_s;
      while (since() < due) {}
    }
    if (psb_stream_push_many(s, n_streams, ids.data(), l0, n, rows) != 0) return -2;
  }
  if (push_span_s) *push_span_s = since();
  for (;;) {
    bool all = true;
    for (int32_t i = 0; i < n_streams && all; ++i) {
      int32_t done = 0;
      if (psb_stream_poll(s, i, &done, nullptr, nullptr, nullptr, nullptr) != 0) return -3;
      all = done != 0;
    }
    if (all) break;
    if (since() > timeout_s) return -4;
    std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
  if (wall_s) *wall_s = since();
  return 0;
}
