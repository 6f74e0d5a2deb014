// Host entry points of the lane tier (psb_lane.hip), used by the library.
#pragma once
#include <hip/hip_runtime.h>
#include "psb_types.h"

hipError_t psb_lane_launch(const psb::Params& P, unsigned waves, hipStream_t s);
hipError_t psb_lane_occupancy(int* waves_per_cu);
