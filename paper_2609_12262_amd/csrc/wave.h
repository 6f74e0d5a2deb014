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
#define T_INF_W (((i128)1) << 124)

PSB_DEV int lane() { return (int)__lane_id(); }

// Orders this wave's LDS and global accesses (one wave per work-group).
PSB_DEV void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// Every cross-lane operation takes its operand through an empty asm
// statement.  The optimizer then cannot evaluate the operand separately along
// each incoming control-flow edge: a value that is a constant on one edge (the
// initial 0 of lanes that skipped a branch or a loop) would otherwise let it
// fold the cross-lane operation for that edge alone and send those lanes
// around it, which breaks the wavefront's lockstep.
PSB_DEV int opq(int v) { asm volatile("" : "+v"(v)); return v; }

// A value that is identical in every active lane, made visibly uniform to the
// compiler (scalar register, scalar branches).  Uniform code reads every
// loaded value that steers control flow through these.
PSB_DEV int uni(int v) { return __builtin_amdgcn_readfirstlane(opq(v)); }
PSB_DEV int64_t uni64(int64_t v) {
  const int lo = uni((int)(uint32_t)(uint64_t)v);
  const int hi = uni((int)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
// Lane 0's value, for values that only lane 0 computed.
PSB_DEV int lane0(int v) { return __builtin_amdgcn_readlane(opq(v), 0); }
PSB_DEV i128 uni128(i128 v) {
  const uint64_t lo = (uint64_t)uni64((int64_t)(uint64_t)v);
  const uint64_t hi = (uint64_t)uni64((int64_t)(uint64_t)((unsigned __int128)v >> 64));
  return (i128)(((unsigned __int128)hi << 64) | lo);
}

PSB_DEV int shfl_xor_i32(int v, int m) { return __shfl_xor(opq(v), m, PSB_WAVE); }
PSB_DEV int shfl_i32(int v, int src) { return __shfl(opq(v), src, PSB_WAVE); }

PSB_DEV i128 shfl_xor_i128(i128 v, int m) {
  uint64_t lo = (uint64_t)v, hi = (uint64_t)(v >> 64);
  uint32_t a = (uint32_t)shfl_xor_i32((int)(uint32_t)(lo & 0xffffffffu), m);
  uint32_t b = (uint32_t)shfl_xor_i32((int)(uint32_t)(lo >> 32), m);
  uint32_t c = (uint32_t)shfl_xor_i32((int)(uint32_t)(hi & 0xffffffffu), m);
  uint32_t d = (uint32_t)shfl_xor_i32((int)(uint32_t)(hi >> 32), m);
  uint64_t nlo = ((uint64_t)b << 32) | a, nhi = ((uint64_t)d << 32) | c;
  return (i128)(((unsigned __int128)nhi << 64) | nlo);
}

// (key, arg) minimum steps over lane permutations inside a row of 16 lanes,
// done with DPP moves (a VALU operand modifier) rather than LDS-routed
// permutes.  Every pattern used here reads an active lane of the same row, so
// no lane reads an out-of-range source.
constexpr int DPP_QUAD_XOR1 = 0xB1;     // quad_perm [1,0,3,2]
constexpr int DPP_QUAD_XOR2 = 0x4E;     // quad_perm [2,3,0,1]
constexpr int DPP_HALF_MIRROR = 0x141;  // lane i <-> 7-i within each 8 lanes
constexpr int DPP_MIRROR = 0x140;       // lane i <-> 15-i within each 16 lanes

// Every pattern used reads a valid lane, so the destination's previous value
// is never kept and needs no initialisation.
template <int CTRL> PSB_DEV int dpp_mov(int v) {
  return __builtin_amdgcn_mov_dpp(opq(v), CTRL, 0xF, 0xF, false);
}

PSB_DEV i128 make_i128(uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
  const uint64_t lo = ((uint64_t)b << 32) | a, hi = ((uint64_t)d << 32) | c;
  return (i128)(((unsigned __int128)hi << 64) | lo);
}

// One step: the pair (key, arg) of the partner lane replaces this lane's if
// it is smaller (key first, then arg).  The order is evaluated on the two
// 64-bit halves without branches.
template <int CTRL> PSB_DEV void argmin_step(i128& key, int& arg) {
  const unsigned __int128 u = (unsigned __int128)key;
  const uint64_t lo = (uint64_t)u;
  const int64_t hi = (int64_t)(uint64_t)(u >> 64);
  const uint64_t lo2 = ((uint64_t)(uint32_t)dpp_mov<CTRL>((int)(uint32_t)(lo >> 32)) << 32) |
                       (uint32_t)dpp_mov<CTRL>((int)(uint32_t)lo);
  const int64_t hi2 = (int64_t)(((uint64_t)(uint32_t)dpp_mov<CTRL>((int)(uint32_t)((uint64_t)hi >> 32)) << 32) |
                                (uint32_t)dpp_mov<CTRL>((int)(uint32_t)(uint64_t)hi));
  const int a2 = dpp_mov<CTRL>(arg);
  const bool take = (hi2 < hi) | ((hi2 == hi) & ((lo2 < lo) | ((lo2 == lo) & (a2 < arg))));
  const uint64_t nlo = take ? lo2 : lo;
  const int64_t nhi = take ? hi2 : hi;
  arg = take ? a2 : arg;
  key = (i128)(((unsigned __int128)(uint64_t)nhi << 64) | nlo);
}

// Minimum over aligned groups of g lanes (g a power of two <= 16); ties to the
// smaller arg.  Every lane of the group receives its group's result.  All
// lanes of the wavefront must call this.
PSB_DEV void group_argmin(i128& key, int& arg, int g) {
  if (g >= 2) argmin_step<DPP_QUAD_XOR1>(key, arg);
  if (g >= 4) argmin_step<DPP_QUAD_XOR2>(key, arg);
  if (g >= 8) argmin_step<DPP_HALF_MIRROR>(key, arg);
  if (g >= 16) argmin_step<DPP_MIRROR>(key, arg);
}

// Wave-wide (key, arg) minimum; ties broken by the smaller arg.  The four
// row minima are combined as scalars: the result is uniform.
PSB_DEV void wave_argmin(i128& key, int& arg) {
  group_argmin(key, arg, 16);
  const unsigned __int128 u = (unsigned __int128)key;
  const int w0 = opq((int)(uint32_t)(uint64_t)u), w1 = opq((int)(uint32_t)((uint64_t)u >> 32));
  const int w2 = opq((int)(uint32_t)(uint64_t)(u >> 64)), w3 = opq((int)(uint32_t)((uint64_t)(u >> 64) >> 32));
  const int av = opq(arg);
  i128 bk = T_INF_W; int ba = 0x7fffffff;
#pragma unroll
  for (int row = 0; row < 4; ++row) {
    const i128 k2 = make_i128((uint32_t)__builtin_amdgcn_readlane(w0, 16 * row), (uint32_t)__builtin_amdgcn_readlane(w1, 16 * row),
                              (uint32_t)__builtin_amdgcn_readlane(w2, 16 * row), (uint32_t)__builtin_amdgcn_readlane(w3, 16 * row));
    const int a2 = __builtin_amdgcn_readlane(av, 16 * row);
    if (row == 0 || k2 < bk || (k2 == bk && a2 < ba)) { bk = k2; ba = a2; }
  }
  key = bk; arg = ba;
}

PSB_DEV int wave_sum(int v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += shfl_xor_i32(v, m);
  return uni(v);
}

PSB_DEV int wave_max(int v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) { int o = shfl_xor_i32(v, m); v = o > v ? o : v; }
  return uni(v);
}

PSB_DEV int wave_or(int v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v |= shfl_xor_i32(v, m);
  return uni(v);
}

// Exclusive prefix sum across the wave.
PSB_DEV int wave_prefix(int v) {
  int x = v;
#pragma unroll
  for (int d = 1; d < PSB_WAVE; d <<= 1) {
    int y = __shfl_up(opq(x), d, PSB_WAVE);
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

PSB_DEV uint64_t ballot(int pred) { return __ballot(opq(pred)); }
PSB_DEV uint64_t lanemask_lt() { return (lane() == 0) ? 0ull : (~0ull >> (64 - lane())); }
PSB_DEV uint64_t dev_clock() { return wall_clock64(); }
