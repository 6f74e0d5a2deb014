// Lane tier: the decoding engine compiled with single-lane primitives, one
// shot per lane.  Each lane owns a workspace slot (Lds header, per-shot state
// block and pools) in global memory and takes shots from the batch counter on
// its own; a shot that exceeds the slot's capacities goes to the overflow
// list, which the wavefront overflow tier decodes afterwards.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "psb_types.h"
#include "lane_wave.h"
#define PSB_ENGINE_NS engine_lane
#include "engine.h"
#include "lane_launch.h"

namespace el = psb::engine_lane;

__global__ __launch_bounds__(64) void psb_lane_kernel(psb::Params P) {
  const int64_t slot = (int64_t)blockIdx.x * 64 + threadIdx.x;
  char* base = P.ws + slot * P.L.total + P.L.state;
  el::Lds* S = (el::Lds*)base;
  el::Ctx c;
  el::ctx_init(c, &P, S, base + 64, slot);
  el::state_init(c);
  for (;;) {
    const int j = atomicAdd(&P.counter[0], 1);
    if (j >= P.n_shots) break;
    const int k = P.order ? P.order[j] : j;
    const int st = el::decode_shot(c, k);
    if (st == psb::S_OVERFLOW) {
      const int q = atomicAdd(&P.counter[1], 1);
      P.ovf_list[q] = k;
    } else if (P.out_tdone) {
      P.out_tdone[k] = wall_clock64();
    }
  }
}

hipError_t psb_lane_launch(const psb::Params& P, unsigned waves, hipStream_t s) {
  psb_lane_kernel<<<waves, 64, 0, s>>>(P);
  return hipGetLastError();
}

hipError_t psb_lane_occupancy(int* waves_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(waves_per_cu, psb_lane_kernel, 64, 0);
}
