// Seeded instances generated inside the library (host only): quenched
// disorder, initial configurations and the external values that load every
// Parisi-Rapuano wheel (sec. 3.3 loads the wheels with externally generated
// random values; sec. 2.1 defines the couplings), so that a job can be
// created from a seed alone.
//
// Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable
// pseudorandom number generators", OOPSLA 2014) used as a counter-based
// stream: output u (u = 0, 1, ...) of the stream with key K is
// mix64(K + (u + 1) * GOLDEN), mix64 being the SplitMix64 finaliser; the key
// of stream (seed, tag, a, b) is
//   k = mix64(seed + tag * GOLDEN); k = mix64(k ^ (a + 1) * M1);
//   k = mix64(k ^ (b + 1) * M2).
// Encodings (canonical host formats of include/sg.h):
//   +-1 arrays: bit b of output u gives element 64 u + b, bit 1 <-> -1;
//   Potts spins: bits 2n, 2n + 1 give state bit0 | bit1 << 1 of site n;
//   permutation couplings: element n is permutation number (output n mod 24)
//     in lexicographic order, as the byte pi(0) | pi(1) << 2 | ...;
//   dilution x = 1 - bit, field sign f = 1 - 2 bit (tags 'X', 'F');
//   wheel words: the high 32 bits of outputs 0..60, oldest first, bit 0 of
//     the last forced to 1 (the low-bit lagged-Fibonacci sequence is then
//     never identically zero).
// Tags: 'J' couplings, 'S' spins, 'W' sweep wheels (a = copy, b = wheel),
// 'P' parallel-tempering wheels (a = chain), 'Q' permutation couplings
// (b = 4 for the 4D model), 'X' dilution, 'F' field signs.  Samples, copies
// and chains are numbered globally from sample0, so one campaign split over
// several jobs gets the same inputs.
#include <cstring>
#include <vector>

#include "sg.h"

namespace sg {

static const uint64_t GOLDEN = 0x9E3779B97F4A7C15ull;
static const uint64_t M1 = 0xBF58476D1CE4E5B9ull;
static const uint64_t M2 = 0x94D049BB133111EBull;

static uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * M1;
  z = (z ^ (z >> 27)) * M2;
  return z ^ (z >> 31);
}

static uint64_t stream_key(uint64_t seed, uint64_t tag, uint64_t a, uint64_t b) {
  uint64_t k = mix64(seed + tag * GOLDEN);
  k = mix64(k ^ (a + 1) * M1);
  return mix64(k ^ (b + 1) * M2);
}

static uint64_t out_of(uint64_t key, uint64_t u) { return mix64(key + (u + 1) * GOLDEN); }

// n +-1 values (int8) from the bits of one stream
static void pm1(uint64_t key, uint64_t n, int8_t *dst) {
  for (uint64_t u = 0; u * 64 < n; u++) {
    const uint64_t w = out_of(key, u);
    for (uint64_t b = 0; b < 64 && u * 64 + b < n; b++) dst[u * 64 + b] = ((w >> b) & 1) ? -1 : 1;
  }
}

static void bits01(uint64_t key, uint64_t n, int8_t *dst) {  // 1 - bit
  for (uint64_t u = 0; u * 64 < n; u++) {
    const uint64_t w = out_of(key, u);
    for (uint64_t b = 0; b < 64 && u * 64 + b < n; b++) dst[u * 64 + b] = ((w >> b) & 1) ? 0 : 1;
  }
}

static void potts_states(uint64_t key, uint64_t n, uint8_t *dst) {
  for (uint64_t u = 0; u * 32 < n; u++) {
    const uint64_t w = out_of(key, u);
    for (uint64_t t = 0; t < 32 && u * 32 + t < n; t++) dst[u * 32 + t] = (uint8_t)((w >> (2 * t)) & 3);
  }
}

static void permutation_bytes(uint8_t out[24]) {
  int n = 0;
  for (int a = 0; a < 4; a++)
    for (int b = 0; b < 4; b++)
      for (int c = 0; c < 4; c++)
        for (int d = 0; d < 4; d++)
          if (a != b && a != c && a != d && b != c && b != d && c != d)
            out[n++] = (uint8_t)(a | b << 2 | c << 4 | d << 6);
}

static void wheel_words(uint64_t key, uint32_t *dst) {
  for (int u = 0; u < 61; u++) dst[u] = (uint32_t)(out_of(key, (uint64_t)u) >> 32);
  dst[60] |= 1u;
}

}  // namespace sg

extern "C" int sg_generate(const sg_job_spec *spec, int8_t *J, void *spins, uint32_t *wheels,
                           uint32_t *ptwheels) {
  using namespace sg;
  uint64_t bytes = 0;
  const int rc = sg_job_bytes(spec, &bytes);  // validates the specification
  if (rc) return rc;
  const int32_t NW = sg_model_wheels_per_copy(spec->model, spec->L);
  const uint64_t L = (uint64_t)spec->L, S = spec->n_samples, R = spec->n_replicas,
                 K = spec->n_temps;
  const uint64_t N = spec->model == SG_GPOTTS4 ? L * L * L * L : L * L * L;
  const uint64_t seed = spec->seed, s0 = spec->sample0;
  if (J) {
    uint8_t perm[24];
    permutation_bytes(perm);
    for (uint64_t s = 0; s < S; s++) {
      const uint64_t smp = s0 + s;
      switch (spec->model) {
        case SG_ISING:
        case SG_POTTS:
          pm1(stream_key(seed, 'J', smp, 0), 3 * N, J + s * 3 * N);
          break;
        case SG_GPOTTS:
        case SG_GPOTTS4: {
          const uint64_t dims = spec->model == SG_GPOTTS4 ? 4 : 3;
          const uint64_t key = stream_key(seed, 'Q', smp, spec->model == SG_GPOTTS4 ? 4 : 0);
          uint8_t *P = (uint8_t *)J + s * dims * N;
          for (uint64_t e = 0; e < dims * N; e++) P[e] = perm[out_of(key, e) % 24];
          break;
        }
        default: {  // SG_ISING_GEN: couplings, dilution and field signs all random
          int8_t *D = J + s * 5 * N;
          pm1(stream_key(seed, 'J', smp, 0), 3 * N, D);
          bits01(stream_key(seed, 'X', smp, 0), N, D + 3 * N);
          pm1(stream_key(seed, 'F', smp, 0), N, D + 4 * N);
        }
      }
    }
  }
  const uint64_t C = S * R * K, c0 = s0 * R * K;
  const bool ising = spec->model == SG_ISING || spec->model == SG_ISING_GEN;
  if (spins)
    for (uint64_t c = 0; c < C; c++) {
      const uint64_t key = stream_key(seed, 'S', c0 + c, 0);
      if (ising)
        pm1(key, N, (int8_t *)spins + c * N);
      else
        potts_states(key, N, (uint8_t *)spins + c * N);
    }
  if (wheels)
    for (uint64_t c = 0; c < C; c++)
      for (uint64_t w = 0; w < (uint64_t)NW; w++)
        wheel_words(stream_key(seed, 'W', c0 + c, w), wheels + (c * NW + w) * 61);
  if (ptwheels)
    for (uint64_t h = 0; h < S * R; h++)
      wheel_words(stream_key(seed, 'P', s0 * R + h, 0), ptwheels + h * 61);
  return SG_OK;
}
