/*
 * Seeded synthetic inputs for the sort workloads.
 *
 * This file draws random keys and sizes and nothing else: it holds none of the
 * sorting arithmetic, and both the CPU oracle's tests and the GPU path take
 * their inputs from it.
 *
 * Every stream is counter based: value i of stream `seed` is the SplitMix64
 * output for state seed + (i + 1) * 0x9E3779B97F4A7C15, using the published
 * SplitMix64 finaliser (Steele, Lea and Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014).  The finaliser is a bijection on 64-bit
 * words, so distinct counters give distinct outputs.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SM64_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t sm64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t sm64_at(uint64_t seed, uint64_t i)
{
    return sm64_mix(seed + (i + 1) * SM64_GAMMA);
}

/* uniform double in [0, 1) from the top 53 bits */
static inline double u01(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

/* uniform integer in [0, m) from the top 32 bits (m <= 2^32) */
static inline uint64_t below(uint64_t x, uint64_t m) { return ((x >> 32) * m) >> 32; }

void wl_u64_stream(uint64_t seed, uint64_t start, uint64_t n, uint64_t *out)
{
    for (uint64_t i = 0; i < n; ++i) out[i] = sm64_at(seed, start + i);
}

/* u32 uniform over [0, 2^32): the high word of each 64-bit output. */
void wl_u32_uniform(uint64_t seed, uint64_t n, uint32_t *out)
{
    for (uint64_t i = 0; i < n; ++i) out[i] = (uint32_t)(sm64_at(seed, i) >> 32);
}

/* Low-entropy u32: bitwise AND of four independent uniform words (outputs
 * 4i .. 4i+3 of the stream), so every bit is 1 with probability 1/16. */
void wl_u32_and4(uint64_t seed, uint64_t n, uint32_t *out)
{
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t a = (uint32_t)(sm64_at(seed, 4 * i + 0) >> 32);
        uint32_t b = (uint32_t)(sm64_at(seed, 4 * i + 1) >> 32);
        uint32_t c = (uint32_t)(sm64_at(seed, 4 * i + 2) >> 32);
        uint32_t d = (uint32_t)(sm64_at(seed, 4 * i + 3) >> 32);
        out[i] = a & b & c & d;
    }
}

/* Pool of `npool` distinct uniform u32 values drawn from stream seed ^ 0x5EED,
 * rejecting repeats. */
static void distinct_u32_pool(uint64_t seed, uint32_t npool, uint32_t *pool)
{
    uint32_t have = 0;
    uint64_t ctr = 0;
    while (have < npool) {
        uint32_t v = (uint32_t)(sm64_at(seed ^ 0x5EEDULL, ctr++) >> 32);
        int dup = 0;
        for (uint32_t j = 0; j < have; ++j)
            if (pool[j] == v) { dup = 1; break; }
        if (!dup) pool[have++] = v;
    }
}

/* Heavy duplicates: key = pool[uniform index], pool of npool distinct values. */
int wl_u32_dup(uint64_t seed, uint64_t n, uint32_t npool, uint32_t *out)
{
    if (npool == 0 || npool > 65536) return -1;
    uint32_t *pool = (uint32_t *)malloc(sizeof(uint32_t) * npool);
    if (!pool) return -3;
    distinct_u32_pool(seed, npool, pool);
    for (uint64_t i = 0; i < n; ++i) out[i] = pool[below(sm64_at(seed, i), npool)];
    free(pool);
    return 0;
}

void wl_u64_uniform(uint64_t seed, uint64_t n, uint64_t *out)
{
    for (uint64_t i = 0; i < n; ++i) out[i] = sm64_at(seed, i);
}

/* Already sorted with a fraction of positions swapped.
 * Sorted by construction: key_i is the running sum of gaps (output >> 27), so
 * it is nondecreasing and never wraps for n <= 2^27.  Each position is then
 * chosen with probability `frac` (stream seed+1); the chosen positions are
 * shuffled by Fisher-Yates (stream seed+2) and swapped in consecutive pairs. */
int wl_u64_nearly_sorted(uint64_t seed, uint64_t n, double frac, uint64_t *out)
{
    uint64_t acc = 0;
    for (uint64_t i = 0; i < n; ++i) {
        acc += sm64_at(seed, i) >> 27;
        out[i] = acc;
    }
    uint64_t thresh = (frac >= 1.0) ? UINT64_MAX : (uint64_t)(frac * 18446744073709551616.0);
    uint64_t m = 0;
    for (uint64_t i = 0; i < n; ++i)
        if (sm64_at(seed + 1, i) < thresh) ++m;
    if (m < 2) return 0;
    uint64_t *pos = (uint64_t *)malloc(sizeof(uint64_t) * m);
    if (!pos) return -3;
    uint64_t k = 0;
    for (uint64_t i = 0; i < n; ++i)
        if (sm64_at(seed + 1, i) < thresh) pos[k++] = i;
    for (uint64_t i = m - 1; i > 0; --i) {
        uint64_t r = sm64_at(seed + 2, i);
        uint64_t j = (uint64_t)(u01(r) * (double)(i + 1));
        if (j > i) j = i;
        uint64_t t = pos[i]; pos[i] = pos[j]; pos[j] = t;
    }
    for (uint64_t i = 0; i + 1 < m; i += 2) {
        uint64_t a = pos[i], b = pos[i + 1];
        uint64_t t = out[a]; out[a] = out[b]; out[b] = t;
    }
    free(pos);
    return 0;
}

/* Zipf(s) over a pool of npool distinct 64-bit values: pool[r] = output r of
 * stream seed ^ 0x2F1F (distinct because the finaliser is a bijection); rank
 * r in [0, npool) has probability proportional to (r + 1)^-s and is drawn by
 * inverse CDF with a binary search over the cumulative weights. */
int wl_u64_zipf(uint64_t seed, uint64_t n, uint32_t npool, double s, uint64_t *out)
{
    if (npool == 0) return -1;
    double *cdf = (double *)malloc(sizeof(double) * npool);
    uint64_t *pool = (uint64_t *)malloc(sizeof(uint64_t) * npool);
    if (!cdf || !pool) { free(cdf); free(pool); return -3; }
    double acc = 0.0;
    for (uint32_t r = 0; r < npool; ++r) {
        acc += pow((double)(r + 1), -s);
        cdf[r] = acc;
    }
    for (uint32_t r = 0; r < npool; ++r) cdf[r] /= acc;
    for (uint32_t r = 0; r < npool; ++r) pool[r] = sm64_at(seed ^ 0x2F1FULL, r);
    for (uint64_t i = 0; i < n; ++i) {
        double u = u01(sm64_at(seed, i));
        uint32_t lo = 0, hi = npool - 1;
        while (lo < hi) {
            uint32_t mid = lo + (hi - lo) / 2;
            if (cdf[mid] > u) hi = mid; else lo = mid + 1;
        }
        out[i] = pool[lo];
    }
    free(cdf);
    free(pool);
    return 0;
}

/* Standard normal from two uniforms (Box-Muller). */
static double std_normal(uint64_t seed, uint64_t i)
{
    double u1 = ((double)(sm64_at(seed, 2 * i) >> 11) + 1.0) * 0x1.0p-53; /* (0, 1] */
    double u2 = u01(sm64_at(seed, 2 * i + 1));
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

/* Lognormal sizes: clip(round(exp(ln(median) + sigma * z)), lo, hi). */
void wl_lognormal_sizes(uint64_t seed, uint64_t count, double median, double sigma,
                        uint64_t lo, uint64_t hi, uint64_t *out)
{
    double mu = log(median);
    for (uint64_t i = 0; i < count; ++i) {
        double v = floor(exp(mu + sigma * std_normal(seed, i)) + 0.5);
        uint64_t x = (v < (double)lo) ? lo : (v > (double)hi ? hi : (uint64_t)v);
        out[i] = x;
    }
}

/* Exponential inter-arrival gaps with the given mean (Poisson arrivals). */
void wl_exponential(uint64_t seed, uint64_t count, double mean, double *out)
{
    for (uint64_t i = 0; i < count; ++i) {
        double u = ((double)(sm64_at(seed, i) >> 11) + 1.0) * 0x1.0p-53;
        out[i] = -mean * log(u);
    }
}

/* Fixed 16-byte lowercase strings sharing a prefix of `prefix_len` bytes
 * (prefix drawn from stream seed ^ 0x9F1C); each remaining byte is uniform in
 * 'a'..'z'.  out holds n * 16 bytes. */
void wl_str16(uint64_t seed, uint64_t n, uint32_t prefix_len, uint8_t *out)
{
    uint8_t prefix[16];
    if (prefix_len > 16) prefix_len = 16;
    for (uint32_t b = 0; b < prefix_len; ++b)
        prefix[b] = (uint8_t)('a' + below(sm64_at(seed ^ 0x9F1CULL, b), 26));
    for (uint64_t i = 0; i < n; ++i) {
        uint8_t *k = out + 16 * i;
        memcpy(k, prefix, prefix_len);
        for (uint32_t b = prefix_len; b < 16; ++b)
            k[b] = (uint8_t)('a' + below(sm64_at(seed, 16 * i + b), 26));
    }
}

/* Uniform integers in [0, m) from stream seed (m <= 2^32). */
void wl_below(uint64_t seed, uint64_t n, uint64_t m, uint64_t *out)
{
    for (uint64_t i = 0; i < n; ++i) out[i] = below(sm64_at(seed, i), m);
}

void wl_iota_u32(uint64_t start, uint64_t n, uint32_t *out)
{
    for (uint64_t i = 0; i < n; ++i) out[i] = (uint32_t)(start + i);
}
