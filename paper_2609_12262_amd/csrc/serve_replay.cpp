// Load replay for the serving runtime (measurement tool, not on the decoding
// path): submits windows at given arrival times from a native thread while a
// second thread collects completions, so that the offered load is not
// limited by an interpreter.  Built as libpsb_replay.so next to libpsb.so.
#include <stdint.h>

#include <atomic>
#include <chrono>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/psb.h"

extern "C" int32_t psb_replay(psb_server* s, int64_t n, const int32_t* graph_idx, const uint8_t* const* syndromes,
                              const int32_t* const* w_override, const double* arrival_s, int64_t* latency_ns,
                              int32_t* status, double* submit_span_s, double* wall_s) {
  if (!s || n <= 0 || !graph_idx || !syndromes || !latency_ns || !status) return -1;
  std::vector<uint64_t> tickets(n, 0);
  std::unordered_map<uint64_t, int64_t> index;
  index.reserve((size_t)n * 2);
  std::atomic<int64_t> submitted{0};
  std::atomic<int32_t> error{0};
  using Clock = std::chrono::steady_clock;
  const auto t0 = Clock::now();
  std::thread collector([&] {
    std::vector<uint64_t> t(4096);
    std::vector<int64_t> lat(4096);
    std::vector<int32_t> st(4096);
    std::unordered_map<uint64_t, int64_t> local;
    int64_t got = 0, seen = 0;
    while (got < n && !error.load()) {
      const int32_t k = psb_server_collect(s, 4096, t.data(), nullptr, nullptr, st.data(), lat.data());
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
        latency_ns[it->second] = lat[j];
        status[it->second] = st[j];
        ++got;
      }
      if (k == 0) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
  });
  for (int64_t i = 0; i < n && !error.load(); ++i) {
    if (arrival_s) {
      while (std::chrono::duration<double>(Clock::now() - t0).count() < arrival_s[i]) {}
    }
    uint64_t t = 0;
    if (psb_server_submit(s, graph_idx[i], syndromes[i], w_override ? w_override[i] : nullptr, &t) != 0) {
      error = 3;
      break;
    }
    tickets[i] = t;
    submitted.store(i + 1, std::memory_order_release);
  }
  if (submit_span_s) *submit_span_s = std::chrono::duration<double>(Clock::now() - t0).count();
  collector.join();
  if (wall_s) *wall_s = std::chrono::duration<double>(Clock::now() - t0).count();
  return error.load() ? -error.load() : 0;
}
