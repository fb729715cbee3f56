/*
 * synth.c -- fast host generation of the seeded integer signals defined in
 * synth/__init__.py (SplitMix64, Steele, Lea & Flood, OOPSLA 2014).  It
 * performs no Walsh-Hadamard arithmetic; it exists only because building a
 * 2^30-entry signal with numpy takes minutes.  The test-suite checks it
 * against the numpy definition element by element.
 */
#include <stdint.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* out[i] = output number (start+i) of SplitMix64 begun from `state`. */
void synth_splitmix64(uint64_t state, uint64_t start, uint64_t count, uint64_t *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)count; i++)
        out[i] = mix(state + (start + (uint64_t)i + 1) * GOLDEN);
}

/* Uniform signs, x_i = 1 - 2 (h_i >> 63); elem = 4 (int32) or 8 (int64). */
void synth_signs(uint64_t state, uint64_t start, uint64_t count, void *out, int elem)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)count; i++) {
        uint64_t h = mix(state + (start + (uint64_t)i + 1) * GOLDEN);
        int64_t v = 1 - 2 * (int64_t)(h >> 63);
        if (elem == 4) ((int32_t *)out)[i] = (int32_t)v;
        else           ((int64_t *)out)[i] = v;
    }
}

/* Planted signal x_i = (-1)^(popcount(s & i) xor e_i), e_i = [(h_i >> 32) < thr].
 * Returns the number of e_i = 1 in the slice. */
uint64_t synth_planted(uint64_t state, uint64_t s, uint64_t thr, uint64_t start,
                       uint64_t count, void *out, int elem)
{
    uint64_t errors = 0;
#pragma omp parallel for schedule(static) reduction(+ : errors)
    for (int64_t i = 0; i < (int64_t)count; i++) {
        uint64_t idx = start + (uint64_t)i;
        uint64_t h = mix(state + (idx + 1) * GOLDEN);
        int e = (h >> 32) < thr;
        int par = __builtin_popcountll(s & idx) & 1;
        errors += (uint64_t)e;
        int64_t v = (par ^ e) ? -1 : 1;
        if (elem == 4) ((int32_t *)out)[i] = (int32_t)v;
        else           ((int64_t *)out)[i] = v;
    }
    return errors;
}
