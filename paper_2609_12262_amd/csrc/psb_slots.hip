// Slot-level serving (continuous batching per slot): one persistent kernel
// whose wavefronts are decode slots.  The host publishes decode windows, as
// they arrive, into a ring in pinned host memory; one dispatcher wavefront
// watches the ring's tail and passes it on in device memory; every other
// wavefront takes the next window as soon as it is free, fetches that
// window's syndrome row across the bus itself (all of its loads in flight at
// once), decodes it with the same engine and the same per-slot state layout
// as psb_decode_batch (the first tier of the decoder of the window's graph
// and weight class), writes the result into pinned host memory and appends
// the window to a completion queue in pinned host memory, which the host
// reads in order.  A window therefore starts as soon as one slot is free and
// completes on its own, whatever else is in flight; its result is the one
// psb_decode_batch gives for it alone (Results, "Decoding task": every window
// is an independent MWEM).  Windows that exceed the first tier's per-shot
// capacities are decoded again, on the host's side stream, by an
// overflow-only decoder.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
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
#include "psb_types.h"
#include "wave.h"
#define PSB_ENGINE_NS engine_slots
#include "engine.h"

namespace psb_host { int32_t fail(int32_t code, const std::string& msg); }
using psb_host::fail;
namespace es = psb::engine_slots;

// implemented in psb_lib.hip
int32_t psb_decoder_first_tier(const psb_decoder* D, psb::Params* P, int32_t* lds_bytes, int32_t* slots);
int32_t psb_graph_unit_copy(const psb_graph* g, psb_graph** out);
int64_t psb_graph_edges(const psb_graph* g);

namespace {

// A completion queue entry: bit 63 = the first tier handed the window on,
// bits 32..62 = (completion number + 1) mod 2^31 (tells a fresh entry from
// the one a lap before), bits 0..31 = the window's ring entry.
constexpr uint64_t kOverflowFlag = 1ull << 63;
constexpr uint64_t kTagMask = 0x7fffffffull;

struct SlotArgs {
  const psb::Params* params;      // [n_groups] first-tier parameters of each group (device memory)
  int32_t n_groups, synd_words;   // synd_words: 32-bit words per ring syndrome row
  int64_t mask;                   // ring entries - 1 (a power of two)
  // pinned host memory written by the host
  const uint64_t* h_tail;         // windows published
  const uint32_t* h_stop;         // 1: stop once every published window is done
  const int32_t* h_group;         // [ring] group of each window
  const uint32_t* h_synd;         // [ring][synd_words] syndrome rows
  // pinned host memory written by the device
  uint64_t* h_cq;                 // [ring] completion queue
  // device memory
  uint64_t* d_ctl;                // [0] slots' reservations, [1] windows published, [2] stop, [3] completions
};

PSB_DEV uint64_t lane0_u64(uint64_t v) {
  const uint32_t lo = (uint32_t)lane0((int)(uint32_t)v), hi = (uint32_t)lane0((int)(uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

PSB_DEV uint64_t load_sys(const uint64_t* p) {
  return (uint64_t)uni64((int64_t)__hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM));
}

// The dispatcher: passes the host's count of published windows on to the
// slots in device memory.  On the stop request it reads the count once more
// (the host publishes before it asks to stop), passes that on, and only then
// raises the device stop flag, so that no published window is left behind.
// Every lane runs it with the same values.
PSB_DEV void dispatch(const SlotArgs& A) {
  uint64_t seen = load_sys(&A.d_ctl[1]);
  for (;;) {
    const uint64_t pub = load_sys(A.h_tail);
    if (pub > seen) {
      __hip_atomic_store(&A.d_ctl[1], pub, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      seen = pub;
      continue;
    }
    if (uni((int)__hip_atomic_load(A.h_stop, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM))) {
      const uint64_t last = load_sys(A.h_tail);
      __hip_atomic_store(&A.d_ctl[1], last, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&A.d_ctl[2], (uint64_t)1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    __builtin_amdgcn_s_sleep(16);
  }
}

// Copies ring row e (nb bytes, from pinned host memory) to dst in device
// memory: each lane issues up to four word loads before it stores any, so a
// row of up to 1 KiB costs one bus round trip.
PSB_DEV void fetch_row(const uint32_t* src, uint8_t* dst, int nb) {
  const int nw = (nb + 3) >> 2;
  for (int w0 = 0; w0 < nw; w0 += 4 * PSB_WAVE) {
    uint32_t x[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int w = w0 + j * PSB_WAVE + lane();
      x[j] = w < nw ? __hip_atomic_load(src + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) : 0u;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int w = w0 + j * PSB_WAVE + lane();
      for (int b = 0; b < 4; ++b)
        if (w < nw && 4 * w + b < nb) dst[4 * w + b] = (uint8_t)(x[j] >> (8 * b));
    }
  }
}

}  // namespace

// Block 0 dispatches; block s >= 1 is slot s - 1 of every group's first-tier
// workspace.  At most 128 VGPRs (four wavefronts per SIMD), as the batch
// kernel; DEEP as there (the search depth class compiled in).
// `params` (= A.params) is its own restrict argument: the table is written
// once before the launch and only read here, which lets the compiler keep the
// decode context built from it per window in scalar registers.
template <int DEEP>
__global__ __launch_bounds__(64, 4) void psb_slot_kernel(SlotArgs A, const psb::Params* __restrict__ params) {
  extern __shared__ __align__(16) char psb_dyn_lds[];
  if (blockIdx.x == 0) { dispatch(A); return; }
  es::Lds* S = (es::Lds*)psb_dyn_lds;
  char* state = psb_dyn_lds + 64;
  const int64_t slot = (int64_t)blockIdx.x - 1;
  for (int g = 0; g < A.n_groups; ++g) {          // every group's detector map of this slot starts empty
    es::Ctx c;
    es::ctx_init(c, params + g, S, state, slot);
    es::state_init(c);
  }
  for (;;) {
    // every lane takes part in the reservation (lane 0 adds 1); lane 0's old value is broadcast
    const uint64_t k = lane0_u64(atomicAdd((unsigned long long*)&A.d_ctl[0], lane() == 0 ? 1ull : 0ull));
    for (;;) {
      const uint64_t t = (uint64_t)uni64((int64_t)__hip_atomic_load(&A.d_ctl[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT));
      if (k < t) break;
      if (uni((int)__hip_atomic_load(&A.d_ctl[2], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT))) {
        // the final count was passed on before the stop flag: windows below it are still this slot's
        if (k < (uint64_t)uni64((int64_t)__hip_atomic_load(&A.d_ctl[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)))
          break;
        return;
      }
      // idle slots poll one counter: the slot next in line polls most often,
      // one m windows further back m + 1 times less often (at most 32 times),
      // so that the polling leaves the busy slots' memory traffic alone
      const int naps = (int)std::min<uint64_t>(k - t + 1, 32);
      for (int i = 0; i < naps; ++i) __builtin_amdgcn_s_sleep(8);
    }
    const int64_t e = (int64_t)(k & (uint64_t)A.mask);
    const int g = uni(__hip_atomic_load(&A.h_group[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM));
    const psb::Params* P = params + g;
    const int nb = uni(P->nbytes);
    fetch_row(A.h_synd + e * (int64_t)A.synd_words, const_cast<uint8_t*>(P->synd) + e * (int64_t)nb, nb);
    __threadfence();                              // the row is in device memory before the engine reads it
    es::Ctx c;
    es::ctx_init(c, P, S, state, slot);
    c.acct = nullptr;                             // no event accounting in serving
    const int st = es::decode_shot<DEEP>(c, e);
    __threadfence_system();                       // the result reaches host memory before its queue entry
    const uint64_t n = lane0_u64(atomicAdd((unsigned long long*)&A.d_ctl[3], lane() == 0 ? 1ull : 0ull));
    if (lane() == 0) {
      const uint64_t v = (((n + 1) & kTagMask) << 32) | (uint64_t)e | (st == psb::S_OVERFLOW ? kOverflowFlag : 0);
      __hip_atomic_store(&A.h_cq[n & (uint64_t)A.mask], v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

namespace {

using Clock = std::chrono::steady_clock;

struct SlotRequest {
  int32_t group = 0;
  int64_t scale = 1;
  uint64_t seq = 0;
  bool published = false, done = false;
  std::vector<uint8_t> synd;       // kept until published
  int32_t status = 0;
  int64_t weight = 0;
  uint64_t obs = 0;
  std::vector<int32_t> edges;
  int64_t n_edges = 0;
  Clock::time_point t_submit, t_done;
};

struct SlotGroup {
  const psb_graph* graph = nullptr;
  psb_graph* own_graph = nullptr;
  psb_decoder* dec = nullptr;      // first tier used by the slots
  psb_decoder* ovf = nullptr;      // overflow tier only, for windows the first tier hands on
  int32_t nbytes = 0;
};

}  // namespace

struct psb_slot_server {
  int device = 0;
  int32_t waves = 0, ring = 0, max_stride = 0, synd_words = 0, lds = 0;
  int deep = 0;                                     // search depth class the groups need (as psb_decode_kernel)
  std::vector<std::unique_ptr<SlotGroup>> groups;   // [2 * graph + (unit weights ? 1 : 0)]
  int32_t n_graphs = 0;
  hipStream_t stream = nullptr, side = nullptr;
  // pinned host memory
  uint64_t* h_tail = nullptr; uint32_t* h_stop = nullptr; int32_t* h_group = nullptr; uint32_t* h_synd = nullptr;
  uint64_t* h_cq = nullptr;
  int32_t *h_edges = nullptr, *h_ne = nullptr, *h_st = nullptr; int64_t* h_w = nullptr; uint64_t* h_obs = nullptr;
  // device memory
  psb::Params* d_params = nullptr; uint64_t* d_ctl = nullptr; uint8_t* d_synd = nullptr;
  uint8_t* d_ovf_synd = nullptr; int32_t *d_ovf_edges = nullptr, *d_ovf_small = nullptr; int64_t* d_ovf_w = nullptr;
  uint64_t* d_ovf_obs = nullptr;
  bool running = false;
  // host bookkeeping
  std::mutex mu;
  std::condition_variable cv;                       // wakes an idle completer when windows are published
  std::thread completer;
  bool stop = false;
  uint64_t next_ticket = 1, published = 0;          // ticket t has sequence number t - 1
  std::atomic<uint64_t> n_published{0};             // = published, read by the completer without the lock
  std::unordered_map<uint64_t, SlotRequest> reqs;
  std::vector<uint64_t> entry_ticket;               // [ring] ticket of the window published in each entry
  std::deque<uint64_t> waiting;                     // submitted, not yet published (ring full)
  std::deque<uint64_t> inflight;                    // published, in publication order
  std::deque<uint64_t> finished;
  int64_t n_windows = 0, n_overflow = 0;
  std::string error;
};

static void slot_free(psb_slot_server* S) {
  for (void* p : {(void*)S->h_tail, (void*)S->h_stop, (void*)S->h_group, (void*)S->h_synd, (void*)S->h_cq,
                  (void*)S->h_edges, (void*)S->h_ne, (void*)S->h_st, (void*)S->h_w, (void*)S->h_obs})
    if (p) (void)hipHostFree(p);
  for (void* p : {(void*)S->d_params, (void*)S->d_ctl, (void*)S->d_synd, (void*)S->d_ovf_synd,
                  (void*)S->d_ovf_edges, (void*)S->d_ovf_small, (void*)S->d_ovf_w, (void*)S->d_ovf_obs})
    if (p) (void)hipFree(p);
  for (auto& G : S->groups) {
    if (!G) continue;
    if (G->dec) psb_decoder_destroy(G->dec);
    if (G->ovf) psb_decoder_destroy(G->ovf);
    if (G->own_graph) psb_graph_destroy(G->own_graph);
  }
  if (S->stream) (void)hipStreamDestroy(S->stream);
  if (S->side) (void)hipStreamDestroy(S->side);
}

// Publishes waiting windows while the ring has room (lock held).  Window seq
// uses ring entry seq mod ring, free once window seq - ring is finished.
static void publish(psb_slot_server* S) {
  const uint64_t oldest = S->inflight.empty() ? S->published : S->inflight.front() - 1;   // seq = ticket - 1
  uint64_t n = 0;
  while (!S->waiting.empty()) {
    const uint64_t t = S->waiting.front();
    SlotRequest& R = S->reqs[t];
    if (R.seq >= oldest + (uint64_t)S->ring) break;
    const int64_t e = (int64_t)(R.seq & (uint64_t)(S->ring - 1));
    S->h_group[e] = R.group;
    memcpy(S->h_synd + e * S->synd_words, R.synd.data(), R.synd.size());
    S->entry_ticket[e] = t;
    R.synd.clear(); R.synd.shrink_to_fit();
    R.published = true;
    S->inflight.push_back(t);
    S->waiting.pop_front();
    ++n;
  }
  if (n) {
    S->published += n;
    S->n_published.store(S->published, std::memory_order_release);
    __atomic_store_n(S->h_tail, S->published, __ATOMIC_RELEASE);
    S->cv.notify_one();
  }
}

// Decodes the window in ring entry e again with its group's overflow-only
// decoder on the side stream; the results replace the first tier's in the
// entry's result rows.
static int32_t redo_overflow(psb_slot_server* S, int64_t e) {
  SlotGroup* G = S->groups[S->h_group[e]].get();
  const uint8_t* row = (const uint8_t*)(S->h_synd + e * S->synd_words);
  bool ok = hipMemcpyAsync(S->d_ovf_synd, row, (size_t)G->nbytes, hipMemcpyHostToDevice, S->side) == hipSuccess &&
            psb_decode_batch(G->ovf, S->d_ovf_synd, 1, S->d_ovf_edges, S->d_ovf_small, S->d_ovf_w, S->d_ovf_obs,
                             S->d_ovf_small + 1, nullptr, nullptr, nullptr, S->side) == PSB_OK &&
            hipMemcpyAsync(S->h_ne + e, S->d_ovf_small, 4, hipMemcpyDeviceToHost, S->side) == hipSuccess &&
            hipMemcpyAsync(S->h_st + e, S->d_ovf_small + 1, 4, hipMemcpyDeviceToHost, S->side) == hipSuccess &&
            hipMemcpyAsync(S->h_w + e, S->d_ovf_w, 8, hipMemcpyDeviceToHost, S->side) == hipSuccess &&
            hipMemcpyAsync(S->h_obs + e, S->d_ovf_obs, 8, hipMemcpyDeviceToHost, S->side) == hipSuccess &&
            hipMemcpyAsync(S->h_edges + e * S->max_stride, S->d_ovf_edges, 4 * (size_t)S->max_stride,
                           hipMemcpyDeviceToHost, S->side) == hipSuccess &&
            hipStreamSynchronize(S->side) == hipSuccess;
  return ok ? PSB_OK : PSB_E_DEVICE;
}

// The completer reads the completion queue in order.  While windows are in
// flight it polls closely (a window decodes in tens of microseconds); when
// none are, it waits for the next publication.
static void completer_main(psb_slot_server* S) {
  (void)hipSetDevice(S->device);
  struct Ready { int64_t e; bool ovf; };
  std::vector<Ready> ready;
  const uint64_t mask = (uint64_t)S->ring - 1;
  uint64_t next = 0;                                // completions read so far
  for (;;) {
    ready.clear();
    for (;;) {                                      // only this thread reads the queue: no lock needed
      const uint64_t v = __atomic_load_n(S->h_cq + (next & mask), __ATOMIC_ACQUIRE);
      if (((v >> 32) & kTagMask) != ((next + 1) & kTagMask)) break;
      ready.push_back({(int64_t)(v & 0xffffffffull), (v & kOverflowFlag) != 0});
      ++next;
    }
    if (ready.empty()) {
      if (next < S->n_published.load(std::memory_order_acquire)) {
        std::this_thread::yield();
        continue;
      }
      std::unique_lock<std::mutex> lk(S->mu);
      if (next >= S->published) {
        if (S->stop) return;
        S->cv.wait_for(lk, std::chrono::milliseconds(1));
      }
      continue;
    }
    // an entry stays its window's until that window is done, so the
    // overflow re-decode may run without the lock
    int32_t redo_rc = PSB_OK;
    for (const Ready& r : ready)
      if (r.ovf && redo_overflow(S, r.e) != PSB_OK) { S->h_st[r.e] = PSB_S_INTERNAL; redo_rc = PSB_E_DEVICE; }
    std::lock_guard<std::mutex> lk(S->mu);
    if (redo_rc != PSB_OK) S->error = "overflow re-decode failed";
    const auto now = Clock::now();
    for (const Ready& r : ready) {
      const int64_t e = r.e;
      const uint64_t t = S->entry_ticket[e];
      SlotRequest& R = S->reqs[t];
      S->n_overflow += r.ovf;
      R.status = S->h_st[e];
      R.weight = S->h_w[e] * R.scale;
      R.obs = S->h_obs[e];
      R.n_edges = S->h_ne[e];
      const int64_t m = std::min<int64_t>(R.n_edges, S->max_stride);
      R.edges.assign(S->h_edges + e * (int64_t)S->max_stride, S->h_edges + e * (int64_t)S->max_stride + m);
      R.done = true;
      R.t_done = now;
      S->finished.push_back(t);
      ++S->n_windows;
    }
    while (!S->inflight.empty()) {
      auto it = S->reqs.find(S->inflight.front());
      if (it != S->reqs.end() && !it->second.done) break;
      S->inflight.pop_front();
    }
    publish(S);
  }
}

extern "C" int32_t psb_slot_server_create(const psb_graph* const* graphs, int32_t n_graphs,
                                          const psb_decoder_opts* opts, int32_t waves, int32_t ring,
                                          psb_slot_server** out) {
  if (!graphs || n_graphs <= 0 || !out) return fail(PSB_E_INVALID, "null argument or no graphs");
  *out = nullptr;
  for (int32_t i = 0; i < n_graphs; ++i) if (!graphs[i]) return fail(PSB_E_INVALID, "null graph");
  if (waves < 0 || ring < 0) return fail(PSB_E_INVALID, "negative waves or ring");
  const bool auto_waves = waves == 0;
  if (auto_waves) waves = 1024;          // decoders are sized for this many; the launch may use fewer (below)
  if (ring == 0) ring = 8192;
  if (ring & (ring - 1)) return fail(PSB_E_INVALID, "ring entries must be a power of two");
  auto S = std::make_unique<psb_slot_server>();
  if (hipGetDevice(&S->device) != hipSuccess) return fail(PSB_E_DEVICE, "hipGetDevice");
  S->waves = waves; S->ring = ring; S->n_graphs = n_graphs;
  S->groups.resize(2 * (size_t)n_graphs);
  int32_t max_nbytes = 4;
  std::vector<psb::Params> params(2 * (size_t)n_graphs);
  int32_t rc = PSB_OK;
  for (int32_t gi = 0; gi < 2 * n_graphs && rc == PSB_OK; ++gi) {
    auto G = std::make_unique<SlotGroup>();
    G->graph = graphs[gi / 2];
    if (gi % 2 == 1) {
      rc = psb_graph_unit_copy(G->graph, &G->own_graph);
      if (rc != PSB_OK) break;
      G->graph = G->own_graph;
    }
    G->nbytes = psb_graph_syndrome_bytes(G->graph);
    psb_decoder_opts o = opts ? opts[gi / 2] : psb_decoder_opts{};
    if (o.edges_per_shot == 0) o.edges_per_shot = 1024;
    o.first_tier = 0;
    o.num_slots = waves;
    o.event_accounting = 0;
    rc = psb_decoder_create(G->graph, &o, &G->dec);
    int32_t lds = 0, slots = 0;
    if (rc == PSB_OK) rc = psb_decoder_first_tier(G->dec, &params[gi], &lds, &slots);
    if (rc == PSB_OK) {
      // the search depth of each level, and whether it reads a ball table,
      // are in the parameters' device copies; read them back once
      std::vector<int32_t> h(params[gi].n_levels), bt(params[gi].n_levels, -1);
      if (!h.empty() && hipMemcpy(h.data(), params[gi].shmax, 4 * h.size(), hipMemcpyDeviceToHost) != hipSuccess)
        rc = fail(PSB_E_DEVICE, "level depths");
      if (!bt.empty() && params[gi].ball_slot &&
          hipMemcpy(bt.data(), params[gi].ball_slot, 4 * bt.size(), hipMemcpyDeviceToHost) != hipSuccess)
        rc = fail(PSB_E_DEVICE, "ball tables");
      for (size_t k = 0; k < h.size(); ++k)
        if (bt[k] < 0) S->deep = std::max(S->deep, h[k] > 3 ? 2 : h[k] == 3 ? 1 : 0);
    }
    if (rc == PSB_OK && slots < waves) rc = fail(PSB_E_INTERNAL, "first tier has fewer slots than waves");
    psb_decoder_opts oo = o;
    oo.fast_max_nodes = -1;                         // overflow tier only
    oo.num_slots = 0;
    oo.overflow_slots = 1;
    if (rc == PSB_OK) rc = psb_decoder_create(G->graph, &oo, &G->ovf);
    if (rc == PSB_OK) {
      S->lds = std::max(S->lds, lds);
      S->max_stride = std::max(S->max_stride, psb_decoder_edges_per_shot(G->dec));
      max_nbytes = std::max(max_nbytes, G->nbytes);
    }
    S->groups[gi] = std::move(G);
  }
  if (rc != PSB_OK) { slot_free(S.get()); return rc; }
  // the slots leave at least half of every CU's LDS free, so that an
  // overflow re-decode (a kernel of its own on the side stream) always finds
  // room while the persistent kernel runs
  int cus = 256;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, S->device);
  if (auto_waves) {
    const int64_t fit = std::min<int64_t>(12LL * cus, (int64_t)cus * 80 * 1024 / std::max(1, S->lds));
    waves = (int32_t)std::max<int64_t>(1, std::min<int64_t>(waves, fit));
    S->waves = waves;
  }
  if ((int64_t)waves * S->lds > (int64_t)cus * 80 * 1024 || waves > 12 * cus) {
    slot_free(S.get());
    return fail(PSB_E_UNSUPPORTED, "too many slots: they must leave half of each compute unit's LDS free");
  }
  S->synd_words = (max_nbytes + 3) / 4;
  const size_t R = (size_t)ring, st = (size_t)S->max_stride;
  auto hm = [&](void** p, size_t bytes) { return hipHostMalloc(p, bytes, hipHostMallocCoherent) == hipSuccess; };
  bool ok = hm((void**)&S->h_tail, 64) && hm((void**)&S->h_stop, 64) && hm((void**)&S->h_group, 4 * R) &&
            hm((void**)&S->h_synd, 4 * R * S->synd_words) && hm((void**)&S->h_cq, 8 * R) &&
            hm((void**)&S->h_edges, 4 * R * st) && hm((void**)&S->h_ne, 4 * R) && hm((void**)&S->h_st, 4 * R) &&
            hm((void**)&S->h_w, 8 * R) && hm((void**)&S->h_obs, 8 * R);
  ok = ok && hipMalloc((void**)&S->d_params, sizeof(psb::Params) * params.size()) == hipSuccess &&
       hipMalloc((void**)&S->d_ctl, 64) == hipSuccess &&
       hipMalloc((void**)&S->d_synd, R * (size_t)max_nbytes * params.size()) == hipSuccess &&
       hipMalloc((void**)&S->d_ovf_synd, (size_t)max_nbytes) == hipSuccess &&
       hipMalloc((void**)&S->d_ovf_edges, 4 * st) == hipSuccess && hipMalloc((void**)&S->d_ovf_small, 16) == hipSuccess &&
       hipMalloc((void**)&S->d_ovf_w, 8) == hipSuccess && hipMalloc((void**)&S->d_ovf_obs, 8) == hipSuccess;
  if (!ok) { slot_free(S.get()); return fail(PSB_E_NOMEM, "slot server buffers"); }
  *S->h_tail = 0; *S->h_stop = 0;
  memset(S->h_cq, 0, 8 * R);
  S->entry_ticket.assign(R, 0);
  // every group reads its syndromes from its own device pool and writes the shared pinned result rows
  for (size_t gi = 0; gi < params.size(); ++gi) {
    psb::Params& P = params[gi];
    P.synd = S->d_synd + gi * R * (size_t)max_nbytes;
    P.n_shots = ring;
    P.out_edges = S->h_edges; P.edge_stride = S->max_stride;
    P.out_nedges = S->h_ne; P.out_weight = S->h_w; P.out_obs = S->h_obs; P.out_status = S->h_st;
    P.out_levels = nullptr; P.out_tdone = nullptr; P.out_stats = nullptr; P.stats_stride = 8;
    P.counter = nullptr; P.ovf_list = nullptr; P.tier = 0; P.eacct = 0;
  }
  if (hipMemcpy(S->d_params, params.data(), sizeof(psb::Params) * params.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(S->d_ctl, 0, 64) != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
      hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&S->side, hipStreamNonBlocking) != hipSuccess ||
      hipFuncSetAttribute(S->deep == 2 ? (const void*)psb_slot_kernel<2>
                          : S->deep == 1 ? (const void*)psb_slot_kernel<1> : (const void*)psb_slot_kernel<0>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, S->lds) != hipSuccess) {
    slot_free(S.get());
    return fail(PSB_E_DEVICE, "slot server set-up");
  }
  SlotArgs A{};
  A.params = S->d_params; A.n_groups = (int32_t)params.size(); A.synd_words = S->synd_words; A.mask = ring - 1;
  void* dp = nullptr;
  auto dev = [&](void* h) { dp = nullptr; (void)hipHostGetDevicePointer(&dp, h, 0); return dp; };
  A.h_tail = (const uint64_t*)dev(S->h_tail); A.h_stop = (const uint32_t*)dev(S->h_stop);
  A.h_group = (const int32_t*)dev(S->h_group); A.h_synd = (const uint32_t*)dev(S->h_synd);
  A.h_cq = (uint64_t*)dev(S->h_cq);
  A.d_ctl = S->d_ctl;
  if (!A.h_tail || !A.h_stop || !A.h_group || !A.h_synd || !A.h_cq) {
    slot_free(S.get());
    return fail(PSB_E_DEVICE, "device addresses of the pinned ring");
  }
  if (S->deep == 2) psb_slot_kernel<2><<<(unsigned)(waves + 1), 64, S->lds, S->stream>>>(A, A.params);
  else if (S->deep == 1) psb_slot_kernel<1><<<(unsigned)(waves + 1), 64, S->lds, S->stream>>>(A, A.params);
  else psb_slot_kernel<0><<<(unsigned)(waves + 1), 64, S->lds, S->stream>>>(A, A.params);
  if (hipGetLastError() != hipSuccess) { slot_free(S.get()); return fail(PSB_E_DEVICE, "slot kernel launch"); }
  S->running = true;
  psb_slot_server* raw = S.release();
  raw->completer = std::thread(completer_main, raw);
  *out = raw;
  return PSB_OK;
}

extern "C" int32_t psb_slot_server_submit_many(psb_slot_server* S, int32_t n, const int32_t* graph_idx,
                                               const uint8_t* const* syndromes, const int32_t* uniform_weight,
                                               uint64_t* tickets) {
  if (!S || n < 0 || (n > 0 && (!graph_idx || !syndromes || !tickets))) return fail(PSB_E_INVALID, "null argument");
  for (int32_t i = 0; i < n; ++i) {
    if (graph_idx[i] < 0 || graph_idx[i] >= S->n_graphs) return fail(PSB_E_INVALID, "graph_idx out of range");
    if (!syndromes[i]) return fail(PSB_E_INVALID, "null syndrome");
    if (uniform_weight && uniform_weight[i] < 0) return fail(PSB_E_INVALID, "weights must be positive");
  }
  const auto t_submit = Clock::now();
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->stop) return fail(PSB_E_INVALID, "server is stopping");
  for (int32_t i = 0; i < n; ++i) {
    const int32_t w = uniform_weight ? uniform_weight[i] : 0;
    const uint64_t t = S->next_ticket++;
    SlotRequest& R = S->reqs[t];
    R.group = 2 * graph_idx[i] + (w > 0 ? 1 : 0);
    R.scale = w > 0 ? w : 1;
    R.seq = t - 1;
    R.synd.assign(syndromes[i], syndromes[i] + S->groups[R.group]->nbytes);
    R.t_submit = t_submit;
    S->waiting.push_back(t);
    tickets[i] = t;
  }
  publish(S);
  return PSB_OK;
}

static int32_t collect_common(psb_slot_server* S, int32_t max, uint64_t* tickets, int64_t* weight, uint64_t* obs,
                              int32_t* status, int64_t* latency_ns, int32_t* edges, int64_t edges_stride,
                              int64_t* n_edges) {
  std::lock_guard<std::mutex> lk(S->mu);
  int32_t k = 0;
  while (k < max && !S->finished.empty()) {
    const uint64_t t = S->finished.front();
    S->finished.pop_front();
    auto it = S->reqs.find(t);
    if (it == S->reqs.end()) continue;
    const SlotRequest& R = it->second;
    tickets[k] = t;
    if (weight) weight[k] = R.weight;
    if (obs) obs[k] = R.obs;
    if (status) status[k] = (edges && R.n_edges > edges_stride && R.status == PSB_S_OK) ? PSB_S_EDGES_TRUNCATED : R.status;
    if (latency_ns) latency_ns[k] = std::chrono::duration_cast<std::chrono::nanoseconds>(R.t_done - R.t_submit).count();
    if (edges) {
      const int64_t m = std::min<int64_t>((int64_t)R.edges.size(), edges_stride);
      if (m > 0) memcpy(edges + (int64_t)k * edges_stride, R.edges.data(), (size_t)m * 4);
      n_edges[k] = R.n_edges;
    }
    S->reqs.erase(it);
    ++k;
  }
  return k;
}

extern "C" int32_t psb_slot_server_collect(psb_slot_server* S, int32_t max, uint64_t* tickets, int64_t* weight,
                                           uint64_t* obs, int32_t* status, int64_t* latency_ns) {
  if (!S || max < 0 || (max > 0 && !tickets)) return fail(PSB_E_INVALID, "null argument");
  return collect_common(S, max, tickets, weight, obs, status, latency_ns, nullptr, 0, nullptr);
}

extern "C" int32_t psb_slot_server_collect_edges(psb_slot_server* S, int32_t max, uint64_t* tickets, int64_t* weight,
                                                 uint64_t* obs, int32_t* status, int64_t* latency_ns, int32_t* edges,
                                                 int64_t edges_stride, int64_t* n_edges) {
  if (!S || max < 0 || edges_stride < 0 || (max > 0 && (!tickets || !edges || !n_edges)))
    return fail(PSB_E_INVALID, "null argument or negative stride");
  return collect_common(S, max, tickets, weight, obs, status, latency_ns, edges, edges_stride, n_edges);
}

extern "C" int32_t psb_slot_server_poll(psb_slot_server* S, uint64_t ticket, int32_t* done, int64_t* weight,
                                        uint64_t* obs, int32_t* edges, int64_t edges_cap, int64_t* n_edges,
                                        int32_t* status, int64_t* latency_ns) {
  if (!S || !done) return fail(PSB_E_INVALID, "null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return fail(PSB_E_INVALID, "unknown or already collected ticket");
  SlotRequest& R = it->second;
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
  if (latency_ns) *latency_ns = std::chrono::duration_cast<std::chrono::nanoseconds>(R.t_done - R.t_submit).count();
  // the ticket is released once collected from the completion list as well
  S->reqs.erase(it);
  return PSB_OK;
}

extern "C" int32_t psb_slot_server_stats(psb_slot_server* S, int64_t* out5) {
  if (!S || !out5) return fail(PSB_E_INVALID, "null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  out5[0] = S->n_windows; out5[1] = S->n_overflow; out5[2] = (int64_t)S->waiting.size();
  out5[3] = (int64_t)S->inflight.size(); out5[4] = S->waves;
  return PSB_OK;
}

extern "C" int32_t psb_slot_server_destroy(psb_slot_server* S) {
  if (!S) return PSB_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    // windows still waiting for a ring entry are dropped; everything published completes
    for (uint64_t t : S->waiting) S->reqs.erase(t);
    S->waiting.clear();
    __atomic_store_n(S->h_stop, 1u, __ATOMIC_RELEASE);
    S->cv.notify_one();
  }
  if (S->completer.joinable()) S->completer.join();
  if (S->running) (void)hipStreamSynchronize(S->stream);
  slot_free(S);
  delete S;
  return PSB_OK;
}
