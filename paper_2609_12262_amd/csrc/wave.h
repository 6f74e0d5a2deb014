// Wavefront primitives for CDNA4 (gfx950, wave64) used by the decoder engine.
//
// The engine is written as "uniform" code executed identically by all 64
// lanes of one wavefront (one shot per wavefront), with lane-parallel loops
// `for (i = lane(); i < n; i += WAVE)` whose results are combined with the
// reductions below.  Memory written in one lane-parallel phase and read by
// other lanes in the next is separated by wave_sync().
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define PSB_DEV __device__ __forceinline__
#define PSB_WAVE 64

typedef __int128 i128;

PSB_DEV int lane() { return (int)__lane_id(); }

// Orders this wave's LDS and global accesses (one wave per work-group).
PSB_DEV void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

PSB_DEV int shfl_xor_i32(int v, int m) { return __shfl_xor(v, m, PSB_WAVE); }
PSB_DEV int shfl_i32(int v, int src) { return __shfl(v, src, PSB_WAVE); }

PSB_DEV i128 shfl_xor_i128(i128 v, int m) {
  uint64_t lo = (uint64_t)v, hi = (uint64_t)(v >> 64);
  uint32_t a = __shfl_xor((unsigned)(lo & 0xffffffffu), m, PSB_WAVE);
  uint32_t b = __shfl_xor((unsigned)(lo >> 32), m, PSB_WAVE);
  uint32_t c = __shfl_xor((unsigned)(hi & 0xffffffffu), m, PSB_WAVE);
  uint32_t d = __shfl_xor((unsigned)(hi >> 32), m, PSB_WAVE);
  uint64_t nlo = ((uint64_t)b << 32) | a, nhi = ((uint64_t)d << 32) | c;
  return (i128)(((unsigned __int128)nhi << 64) | nlo);
}

// Wave-wide (key, arg) minimum; ties broken by the smaller arg.  All lanes
// receive the result.
PSB_DEV void wave_argmin(i128& key, int& arg) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    i128 k2 = shfl_xor_i128(key, m);
    int a2 = shfl_xor_i32(arg, m);
    if (k2 < key || (k2 == key && a2 < arg)) { key = k2; arg = a2; }
  }
}

// Minimum over groups of `g` consecutive lanes (g a power of two <= 64).
PSB_DEV void group_argmin(i128& key, int& arg, int g) {
  for (int m = g >> 1; m >= 1; m >>= 1) {
    i128 k2 = shfl_xor_i128(key, m);
    int a2 = shfl_xor_i32(arg, m);
    if (k2 < key || (k2 == key && a2 < arg)) { key = k2; arg = a2; }
  }
}

PSB_DEV int wave_sum(int v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += shfl_xor_i32(v, m);
  return v;
}

PSB_DEV int wave_max(int v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) { int o = shfl_xor_i32(v, m); v = o > v ? o : v; }
  return v;
}

PSB_DEV int wave_or(int v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v |= shfl_xor_i32(v, m);
  return v;
}

// Exclusive prefix sum across the wave.
PSB_DEV int wave_prefix(int v) {
  int x = v;
#pragma unroll
  for (int d = 1; d < PSB_WAVE; d <<= 1) {
    int y = __shfl_up(x, d, PSB_WAVE);
    if (lane() >= d) x += y;
  }
  return x - v;
}

PSB_DEV int atom_add(int* p, int v) { return atomicAdd(p, v); }
PSB_DEV int atom_or(int* p, int v) { return atomicOr(p, v); }
PSB_DEV unsigned atom_xor(unsigned* p, unsigned v) { return atomicXor(p, v); }
PSB_DEV int atom_cas(int* p, int cmp, int v) { return atomicCAS(p, cmp, v); }
PSB_DEV int atom_min(int* p, int v) { return atomicMin(p, v); }
PSB_DEV unsigned atom_xchg(unsigned* p, unsigned v) { return atomicExch(p, v); }
// Relaxed load at device scope: bypasses the CU's L1 so that values changed by
// atomics (which execute in L2) are observed.
PSB_DEV int atom_load(int* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

PSB_DEV uint64_t ballot(int pred) { return __ballot(pred); }
PSB_DEV uint64_t lanemask_lt() { return (lane() == 0) ? 0ull : (~0ull >> (64 - lane())); }
PSB_DEV uint64_t dev_clock() { return wall_clock64(); }
