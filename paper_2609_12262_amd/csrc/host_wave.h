// Single-lane primitives for a host (CPU) build of the decoding engine: the
// same interface as lane_wave.h, with plain host functions.  Used to run the
// engine one shot at a time on the CPU under address and undefined-behaviour
// sanitizers and with the invariant checks compiled in; never linked into
// the library.
#pragma once
#include <stdint.h>

#define PSB_DEV inline
#define PSB_WAVE 1

typedef __int128 i128;

PSB_DEV int lane() { return 0; }
PSB_DEV void wave_sync() {}
PSB_DEV int uni(int v) { return v; }
PSB_DEV int64_t uni64(int64_t v) { return v; }
PSB_DEV i128 uni128(i128 v) { return v; }
PSB_DEV int shfl_xor_i32(int v, int) { return v; }
PSB_DEV int shfl_i32(int v, int) { return v; }
PSB_DEV i128 shfl_xor_i128(i128 v, int) { return v; }
PSB_DEV void wave_argmin(i128&, int&) {}
PSB_DEV void group_argmin(i128&, int&, int) {}
PSB_DEV int wave_sum(int v) { return v; }
PSB_DEV int wave_max(int v) { return v; }
PSB_DEV int wave_or(int v) { return v; }
PSB_DEV int wave_prefix(int) { return 0; }
PSB_DEV int atom_add(int* p, int v) { const int o = *p; *p = o + v; return o; }
PSB_DEV int atom_or(int* p, int v) { const int o = *p; *p = o | v; return o; }
PSB_DEV unsigned atom_xor(unsigned* p, unsigned v) { const unsigned o = *p; *p = o ^ v; return o; }
PSB_DEV int atom_cas(int* p, int cmp, int v) { const int o = *p; if (o == cmp) *p = v; return o; }
PSB_DEV int atom_min(int* p, int v) { const int o = *p; if (v < o) *p = v; return o; }
PSB_DEV unsigned atom_xchg(unsigned* p, unsigned v) { const unsigned o = *p; *p = v; return o; }
PSB_DEV int atom_load(int* p) { return *p; }
PSB_DEV uint64_t ballot(int pred) { return pred ? 1ull : 0ull; }
PSB_DEV uint64_t lanemask_lt() { return 0ull; }
PSB_DEV uint64_t dev_clock() { return 0; }
