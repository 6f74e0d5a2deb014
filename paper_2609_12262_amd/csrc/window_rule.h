// The sliding-window rule (Introduction: decoding a stream of syndrome
// rounds in overlapping windows, committing the oldest rounds' corrections)
// on the host: which edges of a layered detector graph each window keeps,
// turns into boundary edges or drops, and which of them it commits.  Used by
// the batch window plan and by the streaming server alike.
//
// The detectors come in layers of equal size L (one layer per round).
// Window k covers layers [a, b) with a = k*C and b = a + W (the last window
// ends at the final layer).  Inside it:
//   * edges with both ends in the window are kept;
//   * an edge from the window to a later layer becomes a boundary edge at its
//     window end (the future is open);
//   * an edge to an earlier layer is dropped (the past is committed; its
//     effect is already in the running syndrome).
// A matched edge is committed when its lower layer lies in the window's first
// C layers, or when the window is the last one.  Window detector j is
// detector a*L + j of the full graph.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <map>
#include <vector>

#include "../../include/psb.h"

namespace psb_host {

struct WindowShape {                       // a window structure: its graph and commit flags
  int32_t n_det = 0;
  std::vector<int32_t> u, v, w;
  std::vector<uint64_t> obs;
  std::vector<uint8_t> commit;             // [m] 1 = committed when matched
};

struct WindowSpan {
  int32_t first_layer = 0, end_layer = 0, shape = 0;
  std::vector<int32_t> map;                // [m of its shape] local edge -> edge of the full graph
};

// Splits the graph into windows; equal structures share one shape.  The
// caller has checked the arguments (layer_size divides the detector count,
// 0 < C < W, endpoints in range).
static void build_windows(const psb_graph_desc* desc, int32_t L, int32_t W, int32_t C,
                          std::vector<WindowShape>& shapes, std::vector<WindowSpan>& spans) {
  const int32_t n_layers = desc->num_detectors / L;
  const int64_t m = desc->num_edges;
  std::map<std::vector<int64_t>, int32_t> shape_of;
  for (int32_t a = 0;; a += C) {
    const bool last = a + W >= n_layers;
    const int32_t b = last ? n_layers : a + W;
    WindowShape S;
    WindowSpan span;
    S.n_det = (b - a) * L;
    for (int64_t e = 0; e < m; ++e) {
      const int32_t u = desc->u[e], v = desc->v[e];
      const int32_t la = u / L;
      const bool in_u = la >= a && la < b;
      int32_t x = -1, y = PSB_BOUNDARY, low = -1;
      if (v < 0) {
        if (!in_u) continue;
        x = u - a * L; low = la;
      } else {
        const int32_t lb = v / L;
        const bool in_v = lb >= a && lb < b;
        if (in_u && in_v) { x = u - a * L; y = v - a * L; low = std::min(la, lb); }
        else if (in_u && lb >= b) { x = u - a * L; low = la; }
        else if (in_v && la >= b) { x = v - a * L; low = lb; }
        else continue;                                   // outside, or reaching into the committed past
      }
      S.u.push_back(x); S.v.push_back(y); S.w.push_back(desc->w[e]); S.obs.push_back(desc->obs_mask[e]);
      S.commit.push_back((uint8_t)(last || low < a + C));
      span.map.push_back((int32_t)e);
    }
    std::vector<int64_t> key;
    key.reserve(5 * S.u.size() + 1);
    key.push_back(b - a);
    for (size_t k = 0; k < S.u.size(); ++k) {
      key.push_back(S.u[k]); key.push_back(S.v[k]); key.push_back(S.w[k]); key.push_back((int64_t)S.obs[k]);
      key.push_back(S.commit[k]);
    }
    auto it = shape_of.find(key);
    if (it != shape_of.end()) {
      span.shape = it->second;
    } else {
      span.shape = (int32_t)shapes.size();
      shapes.push_back(std::move(S));
      shape_of.emplace(std::move(key), span.shape);
    }
    span.first_layer = a; span.end_layer = b;
    spans.push_back(std::move(span));
    if (last) break;
  }
}

}  // namespace psb_host
