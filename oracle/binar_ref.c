/*
 * CPU oracle for binar sort -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg use
 * this file.  It shares no code with the GPU library and includes none of
 * its headers.  It is deliberately plain and slow: serial, recursive, one
 * bit per partition level, exactly as the paper's method is described,
 * except that each partition is made stable.
 *
 * What it computes (section "Sorting Formalism", Knuth's definition with a
 * stability tie-break): the unique permutation p of 0..n-1 such that the
 * keys K_p(0) <= K_p(1) <= ... in unsigned, MSB-first bit-string order and
 * p(i) < p(i+1) whenever two keys are equal.  keys are rearranged in place;
 * payload (optional) is rearranged with them, so payload = 0,1,2,... yields p.
 *
 * How (section "Operation of Algorithm", its four steps):
 *   1. base case: stop when a sub-array has fewer than two elements or the
 *      key's bits are used up;
 *   2. initialise the working bounds from the passed bounds;
 *   3. partition on bit b (bit 0 = most significant, section "Bit
 *      Extraction"): elements whose bit is 0 form the lower sub-array, those
 *      whose bit is 1 the upper one.  The paper's exchange with the upper
 *      boundary is unstable (section "Conclusion" calls the sort unstable);
 *      here both sub-arrays keep their elements' original order, via a
 *      temporary buffer;
 *   4. recursive call: if the partition left one sub-array only ("pass
 *      through"), continue on the same bounds with the next bit -- by
 *      iteration, the optimisation proposed in section "Optimize the
 *      Algorithm" -- otherwise recurse on both sub-arrays with the next bit.
 *
 * Key views (section "The Other Universal Property": the encoding is the
 * sort property):
 *   key_bytes 4 / 8 : native little-endian unsigned integers, numeric order;
 *   key_bytes 16    : byte strings, memcmp order (byte 0 first, MSB first
 *                     within each byte);
 *   binar_sort_bits_ref: unsigned integers of an arbitrary width 1..64 held
 *                     in uint64 words (the paper's 4-bit nybble example).
 *
 * bit_steps counts element visits, one per element per partition level; the
 * time analysis (section "Recursion Analysis") bounds it by bits * n.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define REF_OK 0
#define REF_EINVAL (-1)
#define REF_ENOMEM (-3)

enum { VIEW_INT = 0, VIEW_STR = 1 };

typedef struct {
    uint8_t *keys;
    uint32_t *payload;
    size_t es;          /* bytes per key */
    int view;           /* VIEW_INT or VIEW_STR */
    uint32_t width;     /* bits per key */
    uint32_t stop_bit;  /* partition bits [0, stop_bit) only */
    uint8_t *tmp_keys;
    uint32_t *tmp_pay;
    uint64_t steps;
} ref_ctx;

/* Bit b (0 = most significant) of element i. */
static int key_bit(const ref_ctx *c, uint64_t i, uint32_t b)
{
    const uint8_t *p = c->keys + i * c->es;
    if (c->view == VIEW_STR) return (p[b >> 3] >> (7 - (b & 7))) & 1;
    uint64_t v = 0;
    if (c->es == 4) {
        uint32_t w;
        memcpy(&w, p, 4);
        v = w;
    } else {
        memcpy(&v, p, 8);
    }
    return (int)((v >> (c->width - 1 - b)) & 1u);
}

static void binar_rec(ref_ctx *c, uint64_t lower, uint64_t upper, uint32_t b)
{
    for (;;) {
        /* step 1: base case */
        if (upper - lower < 2 || b >= c->stop_bit) return;

        /* step 2: working bounds */
        const uint64_t lo = lower, hi = upper, len = upper - lower;

        /* step 3: stable partition on bit b */
        uint64_t zeros = 0;
        for (uint64_t i = lo; i < hi; ++i)
            if (!key_bit(c, i, b)) ++zeros;
        c->steps += len;
        const int pass_through = (zeros == 0 || zeros == len);
        if (!pass_through) {
            uint64_t z = 0, o = zeros;
            for (uint64_t i = lo; i < hi; ++i) {
                uint64_t d = key_bit(c, i, b) ? o++ : z++;
                memcpy(c->tmp_keys + d * c->es, c->keys + i * c->es, c->es);
                if (c->payload) c->tmp_pay[d] = c->payload[i];
            }
            memcpy(c->keys + lo * c->es, c->tmp_keys, len * c->es);
            if (c->payload) memcpy(c->payload + lo, c->tmp_pay, len * sizeof(uint32_t));
        }

        /* step 4: next bit on one sub-array (pass through) or on both */
        if (pass_through) {
            ++b;
            continue;
        }
        binar_rec(c, lo, lo + zeros, b + 1); /* lower sub-array */
        lower = lo + zeros;                  /* upper sub-array, by iteration */
        ++b;
    }
}

static int run(void *keys, size_t es, int view, uint32_t width, uint32_t stop_bit,
               uint64_t n, uint32_t *payload, uint64_t *bit_steps)
{
    if (bit_steps) *bit_steps = 0;
    if (n < 2) return REF_OK;
    if (!keys) return REF_EINVAL;
    ref_ctx c;
    c.keys = (uint8_t *)keys;
    c.payload = payload;
    c.es = es;
    c.view = view;
    c.width = width;
    c.stop_bit = stop_bit < width ? stop_bit : width;
    c.steps = 0;
    c.tmp_keys = (uint8_t *)malloc(n * es);
    c.tmp_pay = payload ? (uint32_t *)malloc(n * sizeof(uint32_t)) : NULL;
    if (!c.tmp_keys || (payload && !c.tmp_pay)) {
        free(c.tmp_keys);
        free(c.tmp_pay);
        return REF_ENOMEM;
    }
    binar_rec(&c, 0, n, 0);
    free(c.tmp_keys);
    free(c.tmp_pay);
    if (bit_steps) *bit_steps = c.steps;
    return REF_OK;
}

static int view_of(uint32_t key_bytes, int *view)
{
    if (key_bytes == 4 || key_bytes == 8) { *view = VIEW_INT; return 1; }
    if (key_bytes == 16) { *view = VIEW_STR; return 1; }
    return 0;
}

/* Full stable binar sort of n keys of key_bytes in {4, 8, 16}. */
int binar_sort_ref(void *keys, uint32_t key_bytes, uint64_t n, uint32_t *payload,
                   uint64_t *bit_steps)
{
    int view;
    if (!view_of(key_bytes, &view)) return REF_EINVAL;
    return run(keys, key_bytes, view, 8u * key_bytes, 8u * key_bytes, n, payload, bit_steps);
}

/* The state after partitioning on the leading nbits bits only: the array is
 * grouped by its top nbits bits, in order, each group in original order. */
int binar_partition_ref(void *keys, uint32_t key_bytes, uint64_t n, uint32_t *payload,
                        uint32_t nbits, uint64_t *bit_steps)
{
    int view;
    if (!view_of(key_bytes, &view)) return REF_EINVAL;
    return run(keys, key_bytes, view, 8u * key_bytes, nbits, n, payload, bit_steps);
}

/* Unsigned keys of width key_bits (1..64) held in uint64 words. */
int binar_sort_bits_ref(uint64_t *keys, uint32_t key_bits, uint64_t n, uint32_t *payload,
                        uint32_t nbits, uint64_t *bit_steps)
{
    if (key_bits == 0 || key_bits > 64) return REF_EINVAL;
    for (uint64_t i = 0; i < n; ++i)
        if (key_bits < 64 && (keys[i] >> key_bits) != 0) return REF_EINVAL;
    return run(keys, 8, VIEW_INT, key_bits, nbits, n, payload, bit_steps);
}

/* Each segment [seg_offsets[s], seg_offsets[s+1]) sorted on its own. */
int binar_sort_segmented_ref(void *keys, uint32_t key_bytes, const uint64_t *seg_offsets,
                             uint64_t num_segments, uint32_t *payload)
{
    int view;
    if (!view_of(key_bytes, &view)) return REF_EINVAL;
    for (uint64_t s = 0; s < num_segments; ++s)
        if (seg_offsets[s + 1] < seg_offsets[s]) return REF_EINVAL;
    for (uint64_t s = 0; s < num_segments; ++s) {
        uint64_t a = seg_offsets[s], len = seg_offsets[s + 1] - a;
        int rc = run((uint8_t *)keys + a * key_bytes, key_bytes, view, 8u * key_bytes,
                     8u * key_bytes, len, payload ? payload + a : NULL, NULL);
        if (rc != REF_OK) return rc;
    }
    return REF_OK;
}
