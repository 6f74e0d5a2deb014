/* Seeded, counter-based sampler of independent edge flips on a detector graph.
 *
 * Input generator only: it draws the hidden error set N (each edge flips
 * independently with its own probability) and reports what a decoder sees
 * (the detection events = detectors with odd flipped degree) plus the hidden
 * error's observable flips and weight.  It contains none of the decoding
 * method's arithmetic and is shared by the oracle and the GPU path.
 *
 * Random numbers: SplitMix64 (Steele, Lea & Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014).  The k-th output (k >= 1) of
 * a stream seeded with s is mix(s + k * 0x9E3779B97F4A7C15).  Edge e of shot i
 * uses counter k = i * |E| + e + 1 and flips iff (output >> 32) < thr[e],
 * with thr[e] = floor(p_e * 2^32).
 *
 * Syndrome layout: one row of ceil(num_detectors / 8) bytes per shot,
 * detector j is bit (j & 7) of byte (j >> 3) (LSB first).
 */
#include <stdint.h>
#include <string.h>

static inline uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static inline uint64_t sm64_output(uint64_t seed, uint64_t k) {
  return sm64_mix(seed + k * 0x9E3779B97F4A7C15ULL);
}

/* Returns 0 on success, -1 on bad arguments. */
int synth_sample(int64_t num_edges, const int32_t* eu, const int32_t* ev,
                 const uint32_t* thr, const uint64_t* obs_mask, const int32_t* w,
                 int32_t num_detectors, uint64_t seed, int64_t shot0, int64_t n_shots,
                 uint8_t* synd, uint64_t* obs, int64_t* weight) {
  if (num_edges < 0 || num_detectors < 0 || n_shots < 0) return -1;
  const int64_t nbytes = ((int64_t)num_detectors + 7) / 8;
  memset(synd, 0, (size_t)(nbytes * n_shots));
  for (int64_t s = 0; s < n_shots; ++s) {
    const uint64_t i = (uint64_t)(shot0 + s);
    uint8_t* row = synd + s * nbytes;
    uint64_t o = 0;
    int64_t wsum = 0;
    for (int64_t e = 0; e < num_edges; ++e) {
      const uint64_t k = i * (uint64_t)num_edges + (uint64_t)e + 1ULL;
      const uint32_t r = (uint32_t)(sm64_output(seed, k) >> 32);
      if (r < thr[e]) {
        const int32_t a = eu[e], b = ev[e];
        if (a >= 0) row[a >> 3] ^= (uint8_t)(1u << (a & 7));
        if (b >= 0) row[b >> 3] ^= (uint8_t)(1u << (b & 7));
        o ^= obs_mask[e];
        wsum += w[e];
      }
    }
    obs[s] = o;
    weight[s] = wsum;
  }
  return 0;
}
