/* psb -- parallel sparse-blossom decoding on MI355X (gfx950).
 *
 * C ABI of the decoder library (libpsb.so).  The calls follow the decoding
 * task of the paper "Sparse-Blossom Decoding in o(1) Time" (Mikami &
 * Yamasaki): a detector graph with positive integer edge weights and a set of
 * active detectors go in; the minimum-weight embedded matching (MWEM: odd
 * degree at active detectors, even degree at the other detectors, any degree
 * at boundary vertices -- Results, "Decoding task"), its weight and the
 * predicted observable flips come out (Methods, Algorithm "Parallel sparse
 * blossom", last two steps).
 *
 * Conventions for every call:
 *   * return value 0 = PSB_OK, negative = error (PSB_E_*); psb_last_error()
 *     returns a thread-local message describing the last failure;
 *   * no call takes ownership of caller memory; objects created by the
 *     library are released by the matching *_destroy call;
 *   * a psb_decoder may be used by one host thread / one stream at a time.
 */
#ifndef PSB_H
#define PSB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PSB_OK 0
#define PSB_E_INVALID (-1)      /* bad argument: ids out of range, w <= 0, sizes */
#define PSB_E_NOMEM (-2)        /* host or device allocation failed */
#define PSB_E_DEVICE (-3)       /* HIP runtime error (launch, copy) */
#define PSB_E_UNSUPPORTED (-4)  /* graph/schedule combination outside the kernel's limits */
#define PSB_E_INTERNAL (-5)     /* an internal consistency check failed (autotune candidates disagree) */

/* Per-shot status codes written by psb_decode_batch. */
#define PSB_S_OK 0
#define PSB_S_CAPACITY 1        /* a per-shot workspace bound was exceeded; outputs invalid */
#define PSB_S_INFEASIBLE 2      /* odd number of active detectors in a component with no boundary */
#define PSB_S_EDGES_TRUNCATED 3 /* weight/obs valid, edge list cut at edges_per_shot */
#define PSB_S_INTERNAL 4        /* an internal consistency check failed */
#define PSB_S_CANCELLED 6       /* serving: the request was cancelled before it reached the device */

#define PSB_BOUNDARY (-1)

typedef struct psb_graph psb_graph;
typedef struct psb_decoder psb_decoder;

/* Detector graph (Results, "Decoding task"): vertices are detectors
 * 0..num_detectors-1 plus boundary vertices; edge i joins u[i] and v[i], or
 * u[i] and its own fresh boundary vertex when v[i] == PSB_BOUNDARY.
 * All pointers are HOST pointers, read during psb_graph_create only. */
typedef struct {
  int32_t num_detectors;
  int64_t num_edges;
  const int32_t* u;          /* [num_edges], 0 <= u < num_detectors */
  const int32_t* v;          /* [num_edges], PSB_BOUNDARY or 0 <= v < num_detectors, v != u */
  const int32_t* w;          /* [num_edges], > 0 */
  const uint64_t* obs_mask;  /* [num_edges], bit j = the edge flips observable j */
} psb_graph_desc;

/* Creates a device-resident copy of the graph (fixed-width adjacency).
 * Errors: PSB_E_INVALID (ids out of range, w <= 0, self loop, more than
 * 2^23 edges, a detector of degree > 16), PSB_E_NOMEM, PSB_E_DEVICE. */
int32_t psb_graph_create(const psb_graph_desc* desc, psb_graph** out);
int32_t psb_graph_destroy(psb_graph* g);

typedef struct {
  /* Finite-size parameter schedule (Methods, Algorithm "Parameter schedule"):
   * q = q_num/q_den and phi_min = phi_min_num/phi_min_den, both in (0, 1).
   * Zeros select the paper's numerical choice q = 1/10, phi_min = 1/100. */
  int64_t q_num, q_den, phi_min_num, phi_min_den;
  /* Tie-break seed: every weight is replaced by the even integer
   * 2*w*2^64 + 2*h(e), h(e) = (SplitMix64 output e+1 for this seed) >> 24,
   * so that the MWEM is unique with overwhelming probability. */
  uint64_t tiebreak_seed;
  /* 0 = partition-and-fuse (hierarchical execution over processing clusters,
   *     Methods, Algorithms "Clustering" and "Parallel sparse blossom");
   * 1 = global sparse blossom (every active detector in one execution). */
  int32_t mode;
  /* Boundary reading of the parity condition for odd clusters:
   * 0 = a boundary vertex lies within d_k of every member (default);
   * 1 = some member's exploring region of radius b_k/2 reaches the boundary. */
  int32_t boundary_reading;
  int32_t max_defects_per_shot;   /* 0 = choose from the graph */
  int32_t edges_per_shot;         /* output stride of psb_decode_batch; 0 = max_defects_per_shot*8 */
  int32_t num_slots;              /* first-tier shots in flight; 0 = as many as fit the device
                                     (lane tier: at most 65536 lanes) */
  /* First tier, for shots that reach at most fast_max_nodes detectors and
   * create at most fast_max_regions regions (fast_max_nodes < 0 disables the
   * tier).  first_tier = 0 (default): one shot per wavefront, the per-shot
   * state touched on every event in LDS, the rest in the wavefront's global
   * workspace slot (0 = 320 / 208); first_tier = 1: one shot per lane, the
   * per-shot state in the lane's global workspace slot (0 = 320 / 256).  Shots beyond these
   * bounds are decoded by the overflow tier (one shot per wavefront, up to
   * 1024 detectors and 768 regions per shot in LDS, overflow_slots shots in
   * flight, 0 = chosen from the device) within the same psb_decode_batch
   * call; results do not depend on the tier.  Shots beyond the overflow tier
   * report PSB_S_CAPACITY. */
  int32_t fast_max_nodes, fast_max_regions, overflow_slots;
  int32_t first_tier;
  /* Placement of the wavefront first tier's per-shot state (first_tier = 0):
   * 0 or 1 = event cache, region bases and radius offsets in the wavefront's
   * global workspace slot, the rest in LDS (default; most wavefronts per CU);
   * 2 = radius offsets in the workspace, event cache and region bases in LDS;
   * 3 = all per-shot state in LDS (fewest dependent global loads per event,
   * fewer wavefronts per CU); 4 = all per-shot state in the workspace, no LDS
   * (for whole-graph capacities, whose LDS block would allow few wavefronts
   * per CU; not with event_accounting, and not for the slot-level server).
   * Results do not depend on it. */
  int32_t fast_lds_state;
  /* 1 = per-cluster event accounting (Methods, numerical evaluation: the
   * parallel event count E_ideal of hierarchical execution): each applied
   * event is charged to the processing cluster whose alternating tree drives
   * it, and psb_decode_batch's stats rows grow to 12 fields (see there).
   * Slower; results do not depend on it.  0 = off (stats rows of 8). */
  int32_t event_accounting;
  /* Level-1 processing clusters whose own dynamics is a single event (an
   * adjacent pair meeting halfway before anything else, or one event meeting
   * its boundary first) are, by default, executed concurrently in one pass,
   * one lane per cluster, before the event loop runs the rest (Methods,
   * Algorithm "Parallel sparse blossom").  1 = send them through the event
   * loop one event at a time instead.  Results and event counts do not
   * depend on it. */
  int32_t serial_level_one;
  /* The clustering search of a level below the final one (Methods, Algorithm
   * "Clustering": paths of at most H_k = floor(b_k / w_min) edges within b_k)
   * reads, by default, a table built with the decoder: for every detector, the
   * detectors and boundary edges within b_k along such paths, flagged by
   * whether their least distance is within d_k (and, for boundary edges,
   * b_k / 2).  The tables take about 4 bytes per such pair of device memory; a
   * level whose paths are too many to replay on the host (more than about 2048
   * walk steps per detector) walks them on the device instead.  1 = walk the paths at every level.
   * Results do not depend on it. */
  int32_t cluster_walk;
} psb_decoder_opts;

/* Builds the decoder: tie-broken weights, level parameters d_k, b_k (exact
 * rational arithmetic) and per-slot device workspaces.
 * Errors: PSB_E_INVALID, PSB_E_NOMEM, PSB_E_DEVICE, PSB_E_UNSUPPORTED. */
int32_t psb_decoder_create(const psb_graph* g, const psb_decoder_opts* opts, psb_decoder** out);
int32_t psb_decoder_destroy(psb_decoder* d);

/* Level parameters in tie-broken weight units, each as two int64 halves
 * (value = hi * 2^64 + lo).  final_level[k] != 0 marks a level whose b_k
 * exceeds the graph's diameter bound, where every remaining detection event
 * forms the final clusters.  Returns the number of levels written. */
int32_t psb_decoder_levels(const psb_decoder* d, int32_t max_levels, int64_t* d_hi, uint64_t* d_lo,
                           int64_t* b_hi, uint64_t* b_lo, int32_t* final_level);

/* Decodes n shots in one persistent launch, asynchronously on `stream`
 * (a hipStream_t; NULL = the default stream).  The first tier takes the shots
 * in descending order of their detection-event counts (three small kernels
 * sort them first), so that short shots are the last ones; results do not
 * depend on the order.  All array arguments are DEVICE pointers owned by the
 * caller:
 *   syndromes  [n][ceil(num_detectors/8)] uint8, detector j = bit (j&7) of byte (j>>3);
 *   edges      [n][edges_per_shot] int32, MWEM edge ids in ascending order;
 *   n_edges    [n] int32;  weight [n] int64 (sum of caller weights);
 *   obs        [n] uint64 (XOR of observable masks);  status [n] int32 (PSB_S_*);
 *   levels     [n][max_defects_per_shot] int8 or NULL: processing-cluster level of
 *              each active detector in ascending detector order (0 = global mode);
 *   t_done     [n+1] uint64 or NULL: device clock (100 MHz) when shot i finished;
 *              t_done[n] receives the clock when the launch started;
 *   stats      [n][8] int32 or NULL ([n][12] with event_accounting): per-shot
 *              work counters (events processed, detectors reached by region
 *              growth, nodes visited by the clustering search, arrival-log
 *              records) and device-clock durations of clustering, dynamics,
 *              fuse and the whole shot; with event_accounting also the
 *              applied events, the parallel event count E_ideal (events on
 *              the critical path of hierarchical execution, with each
 *              cluster's stopping time taken as its last event), the number
 *              of processing clusters and the highest level (all 0 for a
 *              shot without detection events).
 * Errors: PSB_E_INVALID, PSB_E_DEVICE. */
int32_t psb_decode_batch(psb_decoder* d, const uint8_t* syndromes, int64_t n, int32_t* edges,
                         int32_t* n_edges, int64_t* weight, uint64_t* obs, int32_t* status,
                         int8_t* levels, uint64_t* t_done, int32_t* stats, void* stream);

/* psb_decode_batch for callers that cannot allocate device memory: code
 * being captured into a HIP graph, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, outputs and errors as psb_decode_batch; the
 * decoder itself is created beforehand (psb_decoder_create allocates).  The
 * call allocates nothing: the batch's work counters and the list of shots the
 * fast tier hands to the overflow tier live in a fixed device array of
 * (64 + PSB_NOALLOC_MAX_SHOTS) int32 (about 4 MiB) that each device holds
 * once until the process ends, so n may be at most PSB_NOALLOC_MAX_SHOTS
 * (PSB_E_INVALID beyond).  Every call on one device shares that array: calls
 * whose launches overlap on a device race (serialise them on one stream), and
 * psb_decoder_last_overflow reports the most recent launch of the decoder,
 * whichever entry point made it.  The counters are cleared by a fill kernel
 * at the head of each launch (no memset).  Its first tier takes the shots in
 * index order (no room for the largest-first ordering). */
#define PSB_NOALLOC_MAX_SHOTS (1 << 20)
int32_t psb_decode_batch_noalloc(psb_decoder* d, const uint8_t* syndromes, int64_t n, int32_t* edges,
                                 int32_t* n_edges, int64_t* weight, uint64_t* obs, int32_t* status,
                                 int8_t* levels, uint64_t* t_done, int32_t* stats, void* stream);

/* Host-only: the finite-size level schedule of Methods, Algorithm "Parameter
 * schedule" (Supplementary S11) for maximum edge weight w_max and target
 * diameter bound diam, both given as (hi, lo) halves of unsigned 128-bit
 * integers.  d_1 = w_max + 1, phi_1 = 1; b_k is the smallest integer with
 * b_k >= d_k, phi_k > 2 d_k / b_k and Phi_{k+1}(b_k) >= phi_bar_{k+1};
 * d_{k+1} = 3 d_k + 4 b_k + 2 w_max.  Generation stops at the first level
 * with b_k >= diam (marked final).  Exact rational arithmetic.  Returns the
 * number of levels written (<= max_levels) or a negative error. */
int32_t psb_schedule_levels(uint64_t wmax_hi, uint64_t wmax_lo, uint64_t diam_hi, uint64_t diam_lo,
                            int64_t q_num, int64_t q_den, int64_t phi_min_num, int64_t phi_min_den,
                            int32_t max_levels, uint64_t* d_hi, uint64_t* d_lo, uint64_t* b_hi,
                            uint64_t* b_lo, int32_t* final_level);

/* Device memory the decoder holds (workspaces, weights, schedule, ball tables, shot-order and overflow
 * buffers), in bytes. */
int32_t psb_decoder_device_bytes(const psb_decoder* d, int64_t* bytes);

/* A psb_decode_batch call captured once into a HIP graph and replayed with
 * one launch: the counter reset, the shot ordering and both tiers'
 * persistent kernels (fill kernels clear the counters, no memset node).  The arguments are those of
 * psb_decode_batch and are fixed at capture (the caller refills
 * `syndromes` in place between launches); all pointers are DEVICE memory
 * owned by the caller and must outlive the graph.  Creation reserves the
 * decoder's per-batch storage for n shots and captures on a stream of its
 * own; a replay may run on any stream.  A replay and any other batch of the
 * same decoder must not overlap (they share its workspaces and counters).
 * Errors: PSB_E_INVALID, PSB_E_NOMEM, PSB_E_DEVICE. */
typedef struct psb_batch_graph psb_batch_graph;
int32_t psb_batch_graph_create(psb_decoder* d, const uint8_t* syndromes, int64_t n, int32_t* edges,
                               int32_t* n_edges, int64_t* weight, uint64_t* obs, int32_t* status,
                               int8_t* levels, uint64_t* t_done, int32_t* stats, psb_batch_graph** out);
int32_t psb_batch_graph_launch(psb_batch_graph* g, void* stream);
int32_t psb_batch_graph_destroy(psb_batch_graph* g);

/* Sizes the decoder's internal per-batch storage (the list of shots the fast
 * tier hands to the overflow tier) for batches of up to `max_batch` shots.
 * psb_decode_batch grows that list by itself when a larger batch comes, which
 * synchronises the stream and frees device memory (a device-wide wait); a
 * caller that keeps several batches in flight reserves once up front.
 * Returns PSB_E_INVALID for max_batch < 0, PSB_E_NOMEM if allocation fails.
 * Not safe to call while a batch of this decoder is in flight. */
int32_t psb_decoder_reserve(psb_decoder* d, int64_t max_batch);

/* Autotuner.  Decodes a sample batch `syndromes` (DEVICE, [n][ceil(num_detectors/8)])
 * with each of psb_autotune_candidates() configurations built from `base`
 * (NULL = defaults) by overriding first_tier, fast_max_nodes,
 * fast_max_regions, fast_lds_state and the schedule ratio q; times `reps` launches of each
 * (after one warm-up) with HIP events on `stream` and writes one record per
 * candidate to entries[0 .. psb_autotune_candidates()-1]: its options, the
 * fastest launch in milliseconds (-1 if skipped) and its status (PSB_OK, or
 * the error that skipped it, e.g. PSB_E_UNSUPPORTED when its state does not
 * fit).  *best_index = the fastest candidate, where a later candidate must
 * be at least 2 % faster than an earlier one to replace it (within timing
 * noise the earlier stays; the library default comes first).  These options change speed
 * only: the partition-and-fuse result is the serial MWEM for every
 * admissible schedule (Methods, "Parallel sparse blossom"), and every
 * candidate's weights and observables are checked against the first one's
 * (PSB_E_INTERNAL if any differ).  Synchronises the device (decoders are
 * created and destroyed).  Returns the number of candidates, or an error:
 * PSB_E_INVALID, PSB_E_NOMEM, PSB_E_DEVICE, PSB_E_INTERNAL, PSB_E_UNSUPPORTED
 * (no candidate fits). */
typedef struct {
  psb_decoder_opts opts;
  float ms;
  int32_t status;
} psb_tune_entry;
int32_t psb_autotune_candidates(void);
int32_t psb_autotune(const psb_graph* g, const psb_decoder_opts* base, const uint8_t* syndromes, int64_t n,
                     int32_t reps, void* stream, psb_tune_entry* entries, int32_t max_entries,
                     int32_t* best_index);

/* Shots in flight per tier and the fast tier's LDS bytes per shot. */
int32_t psb_decoder_slots(const psb_decoder* d, int32_t* fast_slots, int32_t* overflow_slots,
                          int32_t* fast_lds_bytes);

/* Number of shots of the most recent psb_decode_batch call that the fast
 * tier handed to the overflow tier.  Synchronises `stream` first. */
int32_t psb_decoder_last_overflow(psb_decoder* d, void* stream, int32_t* n_overflow);

/* Sizes the caller needs to allocate outputs. */
int32_t psb_decoder_edges_per_shot(const psb_decoder* d);
int32_t psb_decoder_max_defects(const psb_decoder* d);
int32_t psb_graph_syndrome_bytes(const psb_graph* g);

/* ---------------------------------------------------------------------
 * Sliding-window decoding (Introduction: decoding a long stream of rounds
 * in overlapping windows; the MWEM of each window is the paper's problem).
 *
 * The graph's detectors come in num_detectors / layer_size layers (one per
 * round, layer t = detectors t*layer_size .. (t+1)*layer_size-1).  Window k
 * covers layers [k*commit_layers, k*commit_layers + window_layers): edges
 * inside it are kept, an edge to a later layer becomes a boundary edge at
 * its end in the window, an edge to an earlier layer is dropped.  Each
 * window's MWEM is decoded with psb_decode_batch (decoders built with `opts`,
 * NULL = defaults; windows of equal structure share one decoder); the
 * matched edges whose lower layer is among the window's first commit_layers
 * layers are committed (weight and observable accumulated, both endpoints
 * flipped in a running copy of the syndrome).  The window that reaches the
 * last layer commits everything, after which the running syndrome must be
 * empty.  The result is a valid correction (odd degree exactly at the
 * detection events); with window_layers >= the layer count it is the MWEM.
 * Errors: PSB_E_INVALID (layer_size does not divide num_detectors, not
 * 0 < commit_layers < window_layers, endpoints out of range), PSB_E_NOMEM,
 * PSB_E_DEVICE, PSB_E_UNSUPPORTED (a window graph outside the decoder's
 * limits). */
typedef struct psb_window_plan psb_window_plan;
int32_t psb_window_plan_create(const psb_graph_desc* desc, int32_t layer_size, int32_t window_layers,
                               int32_t commit_layers, const psb_decoder_opts* opts, psb_window_plan** out);
/* Number of windows and of distinct window graphs (decoders) of the plan. */
int32_t psb_window_plan_info(const psb_window_plan* p, int32_t* n_windows, int32_t* n_shapes);
/* Decodes n shots asynchronously on `stream`: syndromes [n][ceil(num_detectors/8)]
 * uint8 (DEVICE); outputs weight [n] int64 (sum of committed caller weights),
 * obs [n] uint64, status [n] int32 (PSB_S_OK, the first failing window's
 * status, or PSB_S_INTERNAL if detection events were left unresolved), all
 * DEVICE pointers owned by the caller.  Batch buffers are held by the plan
 * and grow (after synchronising the stream) when a larger batch comes; one
 * batch per plan at a time.  Errors: PSB_E_INVALID, PSB_E_NOMEM, PSB_E_DEVICE. */
int32_t psb_window_decode(psb_window_plan* p, const uint8_t* syndromes, int64_t n, int64_t* weight,
                          uint64_t* obs, int32_t* status, void* stream);
int32_t psb_window_plan_destroy(psb_window_plan* p);

/* ---------------------------------------------------------------------
 * Complementary-gap decoding (Introduction: the weight gap between the
 * best correction and the best one with the other value of a logical
 * observable, a confidence measure; each is an MWEM, Results "Decoding
 * task").  Every edge carrying observable bit `obs_bit` must be a boundary
 * edge.  The plan rewrites the graph: observable edge j ends at a new
 * detector x_j, consecutive x_j are joined by weight-1 chain edges, and all
 * original weights are multiplied by S = the smallest power of two >= the
 * number of observable edges.  Decoding with x_1 active forces the
 * observable bit to 1, with none active to 0 (chain edges add even degree to
 * the x_j); the chain weighs less than S, so each constrained optimum's
 * original weight is its decoded weight / S.  Each shot is decoded once on the
 * original graph (the MWEM: one of the two minima, with its observable; by
 * partition-and-fuse, or by global sparse blossom when the clustering cannot
 * search the graph's weight range) and once on the rewritten graph with the other value of the bit forced (x_1
 * active exactly when the MWEM's bit is 0).  The rewritten graph is decoded
 * in global mode (opts->mode is overridden to 1): the weight-1 chain leaves
 * the clustering no bounded path depth, and both modes return the MWEM.
 * Tiers: unless opts sets fast_max_nodes, fast_max_regions or first_tier,
 * the first tier is a wavefront tier holding the whole rewritten graph (up
 * to 8,192 detectors) with 208 regions per shot, or 512 above 1,024
 * detectors; a shot beyond it ends with PSB_S_CAPACITY unless the overflow
 * tier (1,024 detectors) holds it.
 * Errors: PSB_E_INVALID, PSB_E_UNSUPPORTED (an observable edge that is not a
 * boundary edge, no observable edge, scaled weights beyond int32),
 * PSB_E_NOMEM, PSB_E_DEVICE. */
typedef struct psb_comp_plan psb_comp_plan;
int32_t psb_comp_plan_create(const psb_graph_desc* desc, int32_t obs_bit, const psb_decoder_opts* opts,
                             psb_comp_plan** out);
/* n shots of the ORIGINAL graph, syndromes [n][ceil(num_detectors/8)] (DEVICE);
 * outputs (DEVICE, caller-owned, [n] each): weight0 / weight1 = minimum
 * weight with the observable bit 0 / 1; gap = |weight1 - weight0|; obs = the
 * observable mask of the lighter side (ties to bit 0), i.e. the MWEM's;
 * status (PSB_S_* of the two decodes, the MWEM's first).  Asynchronous on `stream`; batch
 * buffers are held by the plan (grown after synchronising the stream). */
int32_t psb_comp_decode(psb_comp_plan* p, const uint8_t* syndromes, int64_t n, int64_t* weight0, int64_t* weight1,
                        int64_t* gap, uint64_t* obs, int32_t* status, void* stream);
int32_t psb_comp_plan_destroy(psb_comp_plan* p);

/* ---------------------------------------------------------------------
 * Serving (windows arriving one at a time while others decode).
 *
 * Requests are grouped per (graph, weight set): the graph's own weights, or,
 * for requests that carry a uniform per-request weight, the graph with unit
 * weights (made on first use).  Batches run on a pool of 4 pipes, each a
 * stream (its own, or `stream` for all when it is not NULL) with pinned and
 * device batch buffers; every group holds one decoder per pipe, built with
 * that graph's options (`opts`: NULL, or an array of n_graphs records, one
 * per graph; zeros here select edges_per_shot 1024, num_slots 1024 and
 * overflow_slots 256).  Whenever a pipe is idle, a worker thread gives it
 * the group whose oldest waiting window is oldest, as one psb_decode_batch
 * launch of up to num_slots windows (one per first-tier slot), copies the
 * results to pinned host memory and completes the tickets.  Windows that
 * arrive meanwhile wait for the next idle pipe; no batch is queued behind
 * another on a stream.  Each result is identical to psb_decode_batch on that
 * window alone: a shot's decoding does not depend on the other shots of its
 * batch (Results, "Decoding task": every window is an independent MWEM).
 * device_mem_budget > 0 bounds the bytes of decoders and batch buffers
 * (pipe buffers take at most half and shrink to fit; PSB_E_NOMEM if 64-shot
 * batches or a group's decoders do not fit).
 * All calls are thread-safe; one server per device.
 * Errors: PSB_E_INVALID, PSB_E_NOMEM, PSB_E_DEVICE, PSB_E_UNSUPPORTED. */
typedef struct psb_server psb_server;
int32_t psb_server_create(const psb_graph* const* graphs, int32_t n_graphs, const psb_decoder_opts* opts,
                          int64_t device_mem_budget, void* stream, psb_server** out);
/* Queues one window: syndrome_host [ceil(num_detectors/8)] bytes (host
 * memory, copied before the call returns).  w_override: NULL (the graph's
 * weights) or [num_edges] int32 holding one positive weight for every edge
 * (the MWEM under a uniform weight does not depend on its value, so the
 * window decodes on the unit-weight decoder and its weight is scaled);
 * non-uniform overrides return PSB_E_UNSUPPORTED.  *ticket identifies the
 * request. */
int32_t psb_server_submit(psb_server* s, int32_t graph_idx, const uint8_t* syndrome_host,
                          const int32_t* w_override, uint64_t* ticket);
/* Queues n windows under one lock: window i decodes on graph graph_idx[i]
 * with syndrome syndromes[i] (host memory, copied before the call returns);
 * uniform_weight NULL or uniform_weight[i] == 0 = the graph's weights,
 * uniform_weight[i] > 0 = that weight on every edge (as a uniform
 * w_override in psb_server_submit).  tickets[n] receives the tickets.  On an
 * error in window i, windows before i stay queued (their tickets written).
 * Errors: PSB_E_INVALID (checked for every window before any is queued),
 * PSB_E_NOMEM, PSB_E_DEVICE, PSB_E_UNSUPPORTED. */
int32_t psb_server_submit_many(psb_server* s, int32_t n, const int32_t* graph_idx,
                               const uint8_t* const* syndromes, const int32_t* uniform_weight,
                               uint64_t* tickets);
/* Non-blocking: *done = 0 while the window is pending; once done, copies the
 * results to the host pointers (any may be NULL; edges gets at most
 * edges_cap ids, status PSB_S_EDGES_TRUNCATED if more exist), writes the
 * submit-to-completion time in nanoseconds to *latency_ns and releases the
 * ticket. */
int32_t psb_server_poll(psb_server* s, uint64_t ticket, int32_t* done, int64_t* weight, uint64_t* obs,
                        int32_t* edges, int64_t edges_cap, int64_t* n_edges, int32_t* status,
                        int64_t* latency_ns);
/* Collects up to `max` finished windows in completion order without their
 * edge lists: tickets, weights, observable masks, statuses and
 * submit-to-completion nanoseconds (any output but tickets may be NULL);
 * releases them and returns how many were written (0 if none is finished). */
int32_t psb_server_collect(psb_server* s, int32_t max, uint64_t* tickets, int64_t* weight, uint64_t* obs,
                           int32_t* status, int64_t* latency_ns);
/* Cancels a window that has not reached the device yet: it completes at
 * once with status PSB_S_CANCELLED (weight 0, no edges; poll or collect
 * releases it as usual) and *cancelled = 1.  A window already in a running
 * batch (or finished) is not affected: *cancelled = 0 and its result comes
 * as usual.  PSB_E_INVALID for an unknown or released ticket. */
int32_t psb_server_cancel(psb_server* s, uint64_t ticket, int32_t* cancelled);
/* Blocks until the window is done or timeout_us microseconds have passed:
 * *done = 1 if it is done (the ticket stays valid for poll or collect),
 * 0 on time-out.  PSB_E_INVALID for an unknown or released ticket. */
int32_t psb_server_wait(psb_server* s, uint64_t ticket, int64_t timeout_us, int32_t* done);
/* Running totals since creation, out5[5]: batches launched, windows in them,
 * summed submit-to-launch nanoseconds over windows, summed launch-to-
 * completion nanoseconds over batches, summed host nanoseconds spent
 * launching batches. */
int32_t psb_server_stats(psb_server* s, int64_t* out5);
/* Stops the worker after its running batches and frees everything;
 * uncollected tickets are dropped. */
int32_t psb_server_destroy(psb_server* s);

/* ---------------------------------------------------------------------
 * Slot-level serving (continuous batching at the granularity of one
 * window): one persistent kernel whose wavefronts are decode slots.  The
 * host publishes windows, as they are submitted, into a ring of `ring`
 * entries (a power of two; 0 = 8192) in pinned host memory; one dispatcher
 * wavefront copies new windows to the device; each of the `waves` slots
 * (at most 12 per compute unit and half of each unit's LDS, so that other
 * kernels keep room; 0 = as many as that allows, up to 1024) takes the next
 * window as soon as it is
 * free, decodes it with the first tier of the window's group decoder (the
 * same engine and per-shot state as psb_decode_batch), writes its result
 * into pinned host memory and appends the window to a completion queue
 * there, which a host thread reads in order to complete the tickets.  A window thus starts as soon as one slot is free and completes
 * on its own, whatever else is in flight, and its result is the one
 * psb_decode_batch gives for it alone (Results, "Decoding task").  Windows
 * beyond the first tier's capacities are decoded again by an overflow-tier
 * decoder on a side stream.  Groups: per graph its own weights, and unit
 * weights for windows that carry a uniform weight (the result's weight is
 * scaled); all decoders are made at creation (`opts`: NULL or one record per
 * graph; edges_per_shot 0 = 1024).  Windows that find the ring full wait on
 * the host and are published in submission order as entries free up.
 * Graphs must use the direct detector map (at most 32,768 detectors).
 * While the server exists its kernel occupies `waves` slots, and a
 * device-wide synchronisation in the process would wait for it: destroy the
 * server first.  Thread-safe.
 * Errors: PSB_E_INVALID, PSB_E_NOMEM, PSB_E_DEVICE, PSB_E_UNSUPPORTED. */
typedef struct psb_slot_server psb_slot_server;
int32_t psb_slot_server_create(const psb_graph* const* graphs, int32_t n_graphs, const psb_decoder_opts* opts,
                               int32_t waves, int32_t ring, psb_slot_server** out);
/* As psb_server_submit_many. */
int32_t psb_slot_server_submit_many(psb_slot_server* s, int32_t n, const int32_t* graph_idx,
                                    const uint8_t* const* syndromes, const int32_t* uniform_weight,
                                    uint64_t* tickets);
/* As psb_server_collect. */
int32_t psb_slot_server_collect(psb_slot_server* s, int32_t max, uint64_t* tickets, int64_t* weight, uint64_t* obs,
                                int32_t* status, int64_t* latency_ns);
/* As psb_slot_server_collect, also writing each window's matched edges:
 * edges[k * edges_stride ..] receives up to edges_stride edge ids of the k-th
 * ticket and n_edges[k] its edge count (status PSB_S_EDGES_TRUNCATED when
 * that exceeds edges_stride).  edges and n_edges are host arrays of at least
 * max * edges_stride and max entries. */
int32_t psb_slot_server_collect_edges(psb_slot_server* s, int32_t max, uint64_t* tickets, int64_t* weight,
                                      uint64_t* obs, int32_t* status, int64_t* latency_ns, int32_t* edges,
                                      int64_t edges_stride, int64_t* n_edges);
/* As psb_server_poll. */
int32_t psb_slot_server_poll(psb_slot_server* s, uint64_t ticket, int32_t* done, int64_t* weight, uint64_t* obs,
                             int32_t* edges, int64_t edges_cap, int64_t* n_edges, int32_t* status,
                             int64_t* latency_ns);
/* out5[5]: windows completed, windows decoded again by the overflow tier,
 * windows waiting for a ring entry, windows published and not yet done,
 * decode slots (wavefronts) of the kernel. */
int32_t psb_slot_server_stats(psb_slot_server* s, int64_t* out5);
/* Stops the kernel once every published window is done (windows still
 * waiting for a ring entry are dropped), then frees everything. */
int32_t psb_slot_server_destroy(psb_slot_server* s);

/* Streaming sliding-window decoding fed by the serving loop (Introduction:
 * streaming decoding of syndrome-extraction rounds; the window rule of
 * psb_window_plan_create).  `desc` is one run of a layered detector graph
 * (layers of layer_size detectors, one per round); the server keeps
 * n_streams independent streams of it.  Callers push each stream's layers as
 * they arrive; window k of a stream (layers [k*C, k*C + W), the last window to
 * the final layer) is decoded as soon as its last layer has arrived and
 * window k - 1 has committed, by a slot server (psb_slot_server_create with
 * `slots`, 0 = as many as fit) whose groups are the window shapes, so windows
 * of different streams share the GPU.  A host thread commits each decoded
 * window on its stream's running syndrome (weights and observable masks of the
 * committed edges accumulate; their endpoints flip).  A finished stream's
 * weight, observable and status are what psb_window_decode gives for its
 * syndrome; status PSB_S_INTERNAL if a detection event was left unresolved.
 * While the server exists its kernel occupies the slots (see
 * psb_slot_server_create).  Thread-safe.
 * Errors: PSB_E_INVALID, PSB_E_NOMEM, PSB_E_DEVICE, PSB_E_UNSUPPORTED. */
typedef struct psb_stream_server psb_stream_server;
int32_t psb_stream_server_create(const psb_graph_desc* desc, int32_t layer_size, int32_t window_layers,
                                 int32_t commit_layers, const psb_decoder_opts* opts, int32_t n_streams,
                                 int32_t slots, psb_stream_server** out);
/* Layers [first_layer, first_layer + n_layers) of `stream` have arrived.
 * bits: a host row packed LSB-first over the whole graph's detectors (as a
 * psb_decode_batch syndrome row); only the bits of those layers are read.
 * Layers arrive in order, each once (PSB_E_INVALID otherwise). */
int32_t psb_stream_push(psb_stream_server* s, int32_t stream, int32_t first_layer, int32_t n_layers,
                        const uint8_t* bits);
/* psb_stream_push for n streams (streams[i] with rows[i]) that all deliver
 * the same layer range, under one lock.  Stops at the first refused push
 * (the earlier ones stand). */
int32_t psb_stream_push_many(psb_stream_server* s, int32_t n, const int32_t* streams, int32_t first_layer,
                             int32_t n_layers, const uint8_t* const* rows);
/* *done = 1 once every window of the stream has committed (or one failed:
 * *status); committed_layers: layers whose corrections are final; weight and
 * obs: of the committed edges so far (any output but done may be NULL). */
int32_t psb_stream_poll(psb_stream_server* s, int32_t stream, int32_t* done, int32_t* committed_layers,
                        int64_t* weight, uint64_t* obs, int32_t* status);
/* Per committed window of the stream, in window order: ns = nanoseconds from
 * the arrival of the window's last layer to its commit (waiting for the
 * previous window included); decode_ns (may be NULL) = from its submission to
 * the slot server to its decoded result.  *n = windows committed; up to max
 * are written. */
int32_t psb_stream_latencies(psb_stream_server* s, int32_t stream, int32_t max, int64_t* ns, int64_t* decode_ns,
                             int32_t* n);
/* Clears a stream that has no window in flight, for a new run. */
int32_t psb_stream_reset(psb_stream_server* s, int32_t stream);
int32_t psb_stream_server_info(const psb_stream_server* s, int32_t* n_windows, int32_t* n_shapes, int32_t* n_layers);
/* Waits for the windows in flight, then frees everything. */
int32_t psb_stream_server_destroy(psb_stream_server* s);

const char* psb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PSB_H */
