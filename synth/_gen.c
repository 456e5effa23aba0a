/* Candidate-edge draws for the synthetic graph generators (input generation only).
 *
 * Every draw is a pure function of (seed, candidate index, level) through the SplitMix64
 * finaliser (Steele, Lea, Flood, OOPSLA'14), so the arrays are identical for any thread
 * count.  Nothing here belongs to the influence-maximisation method itself.
 */
#include <stdint.h>

static inline uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static inline uint64_t draw64(uint64_t seed, uint64_t idx, uint64_t lane) {
    return mix64(mix64(seed) ^ mix64((idx << 6) | lane));
}

/* R-MAT: for candidate i (first <= i < first+count), at each of `scale` levels pick a
 * quadrant from a 32-bit uniform u: u < ta -> (0,0), ta <= u < tab -> (0,1),
 * tab <= u < tabc -> (1,0), else (1,1).  Candidates with an endpoint >= n are returned
 * as self-loops (the caller drops loops). */
void synth_rmat_draw(int32_t scale, int64_t n, uint64_t seed, int64_t first, int64_t count,
                     uint32_t ta, uint32_t tab, uint32_t tabc, int32_t* src, int32_t* dst) {
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < count; ++j) {
        uint64_t i = (uint64_t)(first + j);
        int64_t s = 0, d = 0;
        for (int32_t level = 0; level < scale; level += 2) {
            uint64_t w = draw64(seed, i, (uint64_t)(level >> 1));
            for (int h = 0; h < 2 && level + h < scale; ++h) {
                uint32_t u = (uint32_t)(w >> (32 * h));
                int64_t bit = (int64_t)1 << (scale - 1 - (level + h));
                if (u >= tab) s += bit;
                if ((u >= ta && u < tab) || u >= tabc) d += bit;
            }
        }
        if (s >= n || d >= n) { s = 0; d = 0; }
        src[j] = (int32_t)s;
        dst[j] = (int32_t)d;
    }
}

/* Uniform ordered pairs for G(n, m). */
void synth_er_draw(int64_t n, uint64_t seed, int64_t first, int64_t count,
                   int32_t* src, int32_t* dst) {
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < count; ++j) {
        uint64_t w = draw64(seed, (uint64_t)(first + j), 0);
        src[j] = (int32_t)(((w & 0xFFFFFFFFull) * (uint64_t)n) >> 32);
        dst[j] = (int32_t)(((w >> 32) * (uint64_t)n) >> 32);
    }
}

/* A seeded 64-bit hash of each key (used to pick a uniform subset of distinct edges). */
void synth_hash_keys(const int64_t* keys, int64_t count, uint64_t seed, uint64_t* out) {
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < count; ++j) out[j] = draw64(seed, (uint64_t)keys[j], 63);
}

/* Barabasi-Albert preferential attachment (the density sweep of gIM Sec. IV-F): a clique
 * of r0 = r + 1 vertices, then vertices r0 .. n-1 one at a time, each joined to r distinct
 * earlier vertices chosen with probability proportional to their current degree (a
 * uniform entry of the list of all edge endpoints so far; a repeated choice is drawn
 * again).  Writes the undirected edges (src[i], dst[i]), new vertex first; returns their
 * number, r0 (r0 - 1) / 2 + (n - r0) r.  Sequential by construction. */
int64_t synth_ba(int32_t n, int32_t r, uint64_t seed, int32_t* src, int32_t* dst, int32_t* ends) {
    const int32_t r0 = r + 1;
    int64_t m = 0, ne = 0;
    for (int32_t a = 0; a < r0 && a < n; ++a)
        for (int32_t b = 0; b < a; ++b) {
            src[m] = a;
            dst[m] = b;
            ++m;
            ends[ne++] = a;
            ends[ne++] = b;
        }
    for (int32_t v = r0; v < n; ++v) {
        const int64_t base = ne;          /* targets of v are chosen among [0, base) */
        uint64_t attempt = 0;
        for (int32_t j = 0; j < r; ++j) {
            int32_t t;
            for (;;) {
                uint64_t w = draw64(seed, (uint64_t)v, attempt++ & 63);
                if (attempt > 64) w = mix64(w ^ attempt);
                t = ends[(int64_t)(((w & 0xFFFFFFFFull) * (uint64_t)base) >> 32)];
                int dup = 0;
                for (int32_t q = 0; q < j; ++q)
                    if (dst[m - j + q] == t) { dup = 1; break; }
                if (!dup) break;
            }
            src[m] = v;
            dst[m] = t;
            ++m;
            ends[ne++] = v;
            ends[ne++] = t;
        }
    }
    return m;
}
