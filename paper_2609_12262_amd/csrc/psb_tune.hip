// Autotuner: decodes a caller's sample batch with each candidate decoder
// configuration, times the launches with HIP events on the caller's stream
// and reports the fastest.  The candidates vary what changes speed but not
// results: the first tier's shape (one shot per wavefront with the hot state
// in LDS, or one shot per lane), its state capacity (detectors and regions
// per shot before a shot moves to the overflow tier), where its per-shot
// state lives (LDS or the global workspace slot) and the clustering
// schedule's ratio q (Methods, Algorithm "Parameter schedule"; the
// partition-and-fuse result equals the serial MWEM for every admissible
// schedule).  Every candidate's weights and observable flips are compared
// with the first candidate's, so a tuning run is also a consistency check.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/psb.h"

namespace psb_host { int32_t fail(int32_t code, const std::string& msg); }
using psb_host::fail;

namespace {

struct Candidate { int32_t first_tier, nodes, regions, lds_state; int64_t q_num, q_den; };

// wave tier: its state lives in LDS, so capacity and placement trade against
// wavefronts per CU
constexpr Candidate kCandidates[] = {
    {0, 320, 208, 0, 1, 10}, {0, 480, 320, 0, 1, 10}, {0, 640, 416, 0, 1, 10}, {0, 896, 560, 0, 1, 10},
    {0, 320, 208, 2, 1, 10}, {0, 320, 208, 3, 1, 10}, {0, 640, 416, 3, 1, 10}, {0, 1024, 768, 3, 1, 10},
    {0, 320, 208, 0, 1, 4},  {0, 640, 416, 0, 1, 4},
    {1, 320, 256, 0, 1, 10}, {1, 640, 512, 0, 1, 10},
};

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() { if (p) (void)hipFree(p); }
  bool alloc(size_t b) { return hipMalloc(&p, b ? b : 16) == hipSuccess; }
};

}  // namespace

extern "C" int32_t psb_autotune_candidates(void) { return (int32_t)(sizeof(kCandidates) / sizeof(kCandidates[0])); }

extern "C" int32_t psb_autotune(const psb_graph* g, const psb_decoder_opts* base, const uint8_t* syndromes,
                                int64_t n, int32_t reps, void* stream, psb_tune_entry* entries,
                                int32_t max_entries, int32_t* best_index) {
  if (!g || !syndromes || !entries || !best_index) return fail(PSB_E_INVALID, "null argument");
  if (n <= 0 || reps <= 0) return fail(PSB_E_INVALID, "sample size and repetitions must be positive");
  const int32_t nc = psb_autotune_candidates();
  if (max_entries < nc) return fail(PSB_E_INVALID, "entries must hold psb_autotune_candidates() records");
  hipStream_t s = (hipStream_t)stream;
  psb_decoder_opts b0{};
  if (base) b0 = *base;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(PSB_E_DEVICE, "hipEventCreate");
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return fail(PSB_E_DEVICE, "hipEventCreate"); }
  DevBuf d_ne, d_w, d_obs, d_st;
  if (!d_ne.alloc(4 * (size_t)n) || !d_w.alloc(8 * (size_t)n) || !d_obs.alloc(8 * (size_t)n) || !d_st.alloc(4 * (size_t)n)) {
    (void)hipEventDestroy(e0); (void)hipEventDestroy(e1);
    return fail(PSB_E_NOMEM, "tuning outputs");
  }
  std::vector<int64_t> w_ref, w_cur((size_t)n);
  std::vector<uint64_t> o_ref, o_cur((size_t)n);
  int32_t best = -1, rc_out = PSB_OK;
  std::string err;
  for (int32_t c = 0; c < nc && rc_out == PSB_OK; ++c) {
    psb_tune_entry& E = entries[c];
    E.opts = b0;
    E.opts.first_tier = kCandidates[c].first_tier;
    E.opts.fast_max_nodes = kCandidates[c].nodes;
    E.opts.fast_max_regions = kCandidates[c].regions;
    E.opts.fast_lds_state = kCandidates[c].lds_state;
    E.opts.q_num = kCandidates[c].q_num;
    E.opts.q_den = kCandidates[c].q_den;
    E.ms = -1.0f;
    psb_decoder* D = nullptr;
    // the lane tier is only offered on the direct detector-map path (graphs of at most 32,768 detectors):
    // on the hash-map path a lane-tier variant once gave wrong device results whose cause was not shown
    if (E.opts.first_tier == 1 && psb_graph_syndrome_bytes(g) > 32768 / 8) {
      E.status = PSB_E_UNSUPPORTED;
      continue;
    }
    E.status = psb_decoder_create(g, &E.opts, &D);
    if (E.status != PSB_OK) continue;        // outside this graph's limits: skipped
    DevBuf d_edges;
    const int32_t stride = psb_decoder_edges_per_shot(D);
    int32_t rc = d_edges.alloc((size_t)n * stride * 4) ? psb_decoder_reserve(D, n) : PSB_E_NOMEM;
    float best_ms = 0.0f;
    for (int32_t r = -1; r < reps && rc == PSB_OK; ++r) {   // r = -1: warm-up
      if (hipEventRecord(e0, s) != hipSuccess) { rc = PSB_E_DEVICE; break; }
      rc = psb_decode_batch(D, syndromes, n, (int32_t*)d_edges.p, (int32_t*)d_ne.p, (int64_t*)d_w.p,
                            (uint64_t*)d_obs.p, (int32_t*)d_st.p, nullptr, nullptr, nullptr, stream);
      if (rc != PSB_OK) break;
      float ms = 0.0f;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = PSB_E_DEVICE; break; }
      if (r == 0 || (r > 0 && ms < best_ms)) best_ms = ms;
    }
    if (rc == PSB_OK) {
      if (hipMemcpy(w_cur.data(), d_w.p, 8 * (size_t)n, hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(o_cur.data(), d_obs.p, 8 * (size_t)n, hipMemcpyDeviceToHost) != hipSuccess) {
        rc = PSB_E_DEVICE;
      } else if (w_ref.empty()) {
        w_ref = w_cur; o_ref = o_cur;
      } else if (w_cur != w_ref || o_cur != o_ref) {
        rc_out = PSB_E_INTERNAL;
        err = "autotune candidates disagree on the decoded weights or observables";
      }
    }
    psb_decoder_destroy(D);
    E.status = rc;
    if (rc != PSB_OK) {
      if (rc == PSB_E_DEVICE) { rc_out = rc; err = "device error while tuning"; }
      continue;
    }
    E.ms = best_ms;
    // a later candidate must be at least 2 % faster to replace an earlier one:
    // within timing noise the earlier (the library default comes first) stays
    if (best < 0 || best_ms < 0.98f * entries[best].ms) best = c;
  }
  (void)hipEventDestroy(e0); (void)hipEventDestroy(e1);
  if (rc_out != PSB_OK) return fail(rc_out, err);
  if (best < 0) return fail(PSB_E_UNSUPPORTED, "no candidate configuration fits this graph");
  *best_index = best;
  return nc;
}
