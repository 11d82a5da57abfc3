/*
 * binar.h -- C ABI of the MI355X (gfx950) binar sort library, libbinar.so.
 *
 * The operation (Gilreath, "Binar Sort", section "Sorting Formalism", with
 * the stability tie-break): rearrange n keys in place into nondecreasing
 * order of their bit strings, most significant bit first, and rearrange an
 * optional uint32 payload with them.  Equal keys keep their input order, so
 * the result is unique; a payload of 0,1,...,n-1 comes back as the sorting
 * permutation p (0-based): payload_out[i] = payload_in[p(i)].
 *
 * The method (sections "Algorithm Synopsis", "Operation of Algorithm",
 * "Algorithm Variants"): partition on the most significant bit(s) first and
 * continue on every sub-array with the next bits, stopping when a sub-array
 * has one element or the bits are used up.  Here every partition is stable,
 * k bits are taken per pass (a stable 2^k-way partition is k stable binary
 * partitions in a row; a one-bit step ranks with wavefront ballots), all
 * live sub-arrays are partitioned in one breadth-first pass, and sub-arrays
 * small enough for on-chip memory (LDS) are finished there: by a
 * workgroup, by one wavefront (up to 1024 keys), or packed many to a
 * wavefront (up to 64 keys).
 *
 * Key views (section "The Other Universal Property": the encoding is what
 * is sorted):
 *   key_bytes == 4  : uint32 values (native little-endian), numeric order;
 *   key_bytes == 8  : uint64 values (native little-endian), numeric order;
 *   key_bytes == 16 : 16-byte strings, memcmp order.
 * 4- and 8-byte keys may instead be read as two's-complement integers or as
 * IEEE-754 values (binar_params.key_kind).
 *
 * Memory and ownership:
 *   keys, payload, seg_offsets are DEVICE pointers owned by the caller; keys
 *   and payload are sorted in place.  The library never frees caller memory.
 *   Scratch memory is either the caller's `workspace` (device, at least
 *   binar_workspace_bytes() bytes, 256-byte aligned) or, when workspace is
 *   NULL, a per-device pool the library grows on demand and keeps until the
 *   process ends.  Two calls that share a workspace (or the pool) must not
 *   overlap in time.
 *   `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *
 * Limits: n (or the sum of segment lengths) < 2^30, because the decoupled
 * look-back packs a prefix count and a 2-bit flag into one 32-bit word.
 *
 * Errors: every call returns a status code.  Arguments are checked before
 * any device work is enqueued, so on an error the caller's buffers are not
 * touched.  Segment offsets live on the device and are checked on the
 * device: an invalid table makes every kernel of that call exit without
 * writing caller memory and is reported by the synchronous calls (and by
 * binar_stats_read) as BINAR_EINVAL.  The _async calls report enqueue
 * errors only; device faults surface at the caller's synchronisation.
 * No C++ exception crosses this interface.
 */
#ifndef BINAR_H
#define BINAR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BINAR_OK 0
#define BINAR_EINVAL (-1)  /* bad key_bytes, NULL pointer with n > 0, bad segment table */
#define BINAR_ERANGE (-2)  /* n or total segment length >= 2^30 */
#define BINAR_ENOMEM (-3)  /* workspace too small, or the pool could not grow */
#define BINAR_EDEVICE (-4) /* a HIP call failed */

#define BINAR_MAX_KEYS ((1u << 30) - 1u)

/* Tuning knobs; a zero field means "library default".
 *   digit_bits : bits taken per global pass: 1, 4, 5, 6, 7 or 8 (1 = the
 *                paper's binary partition step, made stable).
 *   tile_keys  : keys per scatter tile: 4096 for every digit_bits; 2048 for
 *                digit_bits 1, 4 and 8; 8192 for 4-byte keys with digit_bits 8;
 *                6144 for 8-byte keys with digit_bits 8.  Other pairs return
 *                BINAR_EINVAL.
 *   finish_max : largest sub-array finished in on-chip memory (LDS) by one
 *                workgroup; capped by the key width's largest LDS class.
 *   offsets    : how a scatter tile finds where its keys go:
 *                1 = per-chunk counts from the digit-count pass, scanned
 *                    once per segment; each block then walks its chunk of
 *                    tiles in order (no waits between blocks);
 *                2 = decoupled look-back over the segment's earlier tiles
 *                    (tiles taken in ticket order).
 *                0 = default (1).
 *   key_bits   : sort by the leading key_bits bits of each key only (1 ..
 *                8 * key_bytes; 0 = all): keys equal in those bits keep
 *                their input order.  This is the state the method reaches
 *                after partitioning on the first key_bits bits.
 *   key_kind   : how the bits of a 4- or 8-byte key are ordered (the paper
 *                claims the method for any data type whose encoding orders
 *                it; section "The Other Universal Property"):
 *                BINAR_KEY_UNSIGNED (0) unsigned integers;
 *                BINAR_KEY_SIGNED   (1) two's-complement integers;
 *                BINAR_KEY_FLOAT    (2) IEEE-754 binary32 / binary64 in the
 *                  standard's total order: -NaN < -inf < negative values <
 *                  -0 < +0 < positive values < +inf < +NaN (NaNs of one
 *                  sign ordered by payload bits; -0 before +0).
 *                The sort reads each key through an order-preserving
 *                unsigned view (flip the sign bit of signed and non-negative
 *                float keys, every bit of negative float keys) and writes the
 *                caller's bits back unchanged.  16-byte keys take 0 only; a
 *                call's key_kind is never taken from the defaults. */
typedef struct binar_params {
    uint32_t digit_bits;
    uint32_t tile_keys;
    uint32_t finish_max;
    uint32_t offsets;
    uint32_t key_bits;
    uint32_t key_kind;
    uint32_t reserved[2];
} binar_params;

#define BINAR_KEY_UNSIGNED 0u
#define BINAR_KEY_SIGNED 1u
#define BINAR_KEY_FLOAT 2u

/* Counters of the last call that used a workspace (exact integers).
 *   moved[j]       keys scattered by global pass j (pass-through and
 *                  finished sub-arrays move nothing);
 *   hist_keys[j]   keys read by the digit count of pass j;
 *   finish_keys    keys of sub-arrays finished on chip (LDS classes and the
 *                  small path); finish_segments their sub-arrays;
 *   passes         global passes that had work. */
typedef struct binar_stats {
    uint64_t moved[16];
    uint64_t hist_keys[16];
    uint64_t finish_keys;
    uint64_t finish_segments;
    uint32_t passes;
    int32_t status;
    uint64_t finish_class_keys[4];     /* finish_keys split by LDS size class */
    uint64_t finish_class_segments[4];
    uint64_t copyback_keys;            /* finished keys copied from scratch to the caller's buffer */
    uint64_t sorted_keys;              /* keys of sub-arrays found already in order by a digit count
                                          and retired without partitioning (section "Optimize the
                                          Algorithm") */
    uint64_t finish_small_keys;        /* finish_keys of sub-arrays of 2..64 keys, each ranked inside one
                                          64-lane wavefront (in no LDS class) */
    uint64_t finish_small_segments;
} binar_stats;

/* One timed kernel launch (see binar_profile_enable). */
typedef struct binar_launch_time {
    char name[32];   /* "k_hist", "k_plan", "k_scatter", "k_finish_small", "k_finish0".."k_finish3", ... */
    int32_t pass;    /* global pass index, -1 for launches outside the pass loop */
    float ms;        /* elapsed time between the events around the launch */
} binar_launch_time;

/* Sort n keys (and payload, may be NULL) on the null stream with the pool;
 * blocks until the sort has finished. */
int binar_sort(void *keys, uint32_t key_bytes, uint64_t n, uint32_t *payload);

/* Enqueue the same sort on `stream`; returns once enqueued.  workspace may be
 * NULL (pool). */
int binar_sort_async(void *keys, uint32_t key_bytes, uint64_t n, uint32_t *payload,
                     void *stream, void *workspace, size_t workspace_bytes);

/* Sort each segment [seg_offsets[s], seg_offsets[s+1]) of keys independently
 * (payload permuted within its segment), all in one enqueue sequence.
 * seg_offsets: device uint32[num_segments + 1], nondecreasing, in keys;
 * n_total: an upper bound on seg_offsets[num_segments] used to size the
 * scratch (the device checks the table against it).  Empty segments are
 * allowed.  Enqueue only. */
int binar_sort_segmented(void *keys, uint32_t key_bytes, const uint32_t *seg_offsets,
                         uint32_t num_segments, uint64_t n_total, uint32_t *payload,
                         void *stream, void *workspace, size_t workspace_bytes);

/* Same calls with explicit tuning knobs (params may be NULL). */
int binar_sort_ex(void *keys, uint32_t key_bytes, uint64_t n, uint32_t *payload,
                  const uint32_t *seg_offsets, uint32_t num_segments,
                  const binar_params *params, void *stream, void *workspace,
                  size_t workspace_bytes);

/* Scratch bytes a call needs (0 on invalid arguments).  params may be NULL. */
size_t binar_workspace_bytes(uint32_t key_bytes, uint64_t n, int has_payload,
                             uint32_t num_segments, const binar_params *params);

/* Read the counters of the last call that used `workspace` (NULL = the
 * calling device's pool), after synchronising `stream`. */
int binar_stats_read(const void *workspace, void *stream, binar_stats *out);

/* The defaults a call uses for the zero fields of its params (all fields
 * filled in, key_bits = 8 * key_bytes); key_bytes 4, 8, 16.  set replaces
 * them (zero fields: built-in choice; key_bits is ignored) and returns
 * BINAR_EINVAL, changing nothing, for a combination that is not built.  The
 * autotuner installs its choices here. */
int binar_get_default_params(uint32_t key_bytes, int has_payload, binar_params *out);
int binar_set_default_params(uint32_t key_bytes, int has_payload, const binar_params *p);

/* The parameters a call with `params` (may be NULL) would run with, every
 * field filled in (finish_max clamped to the key width's largest LDS class);
 * BINAR_EINVAL for a combination that is not built. */
int binar_resolve_params(uint32_t key_bytes, int has_payload, const binar_params *params, binar_params *out);

/* Launch timing for measurement.  While enabled (on = 1), every kernel the
 * library enqueues is bracketed by two HIP events recorded on the same
 * stream as the kernel.  binar_profile_read waits for the recorded events,
 * copies up to `cap` records (oldest first) to `out`, sets *count to the
 * number copied and clears the log.  Disabling drops unread records. */
int binar_profile_enable(int on);
int binar_profile_read(binar_launch_time *out, uint32_t cap, uint32_t *count);

/* A reusable plan for repeated sorts on resident buffers (batched or served
 * work).  The plan owns a workspace for up to max_keys keys in up to
 * max_segments segments.  The first binar_plan_sort with a given
 * (keys, payload, seg_offsets, num_segments, n_total) captures the call's
 * whole launch sequence into a HIP graph on a stream of the plan's own;
 * later calls with the same values replay that graph on `stream`, whatever
 * the buffers then hold (segment offsets are read on the device, so the
 * segment layout may change between replays within the capacity).  Up to 16
 * graphs are kept per plan.  With seg_offsets, keys and payload must hold
 * max_keys entries and n_total is their length: a call with n_total below
 * max_keys returns BINAR_EINVAL before any device work (the offsets are
 * checked on the device against max_keys), so one graph serves every batch
 * placed in the same buffers.  seg_offsets may be NULL: one array of n_total keys (then
 * n_total is part of the graph's identity).  Calls on one plan must not
 * overlap in time.  binar_plan_stats reads
 * the counters of the plan's last sort; binar_plan_graphs returns how many
 * graphs the plan holds. */
typedef struct binar_plan binar_plan;
int binar_plan_create(binar_plan **out, uint32_t key_bytes, uint64_t max_keys, uint32_t max_segments,
                      int has_payload, const binar_params *params);
int binar_plan_sort(binar_plan *plan, void *keys, uint32_t *payload, const uint32_t *seg_offsets,
                    uint32_t num_segments, uint64_t n_total, void *stream);
int binar_plan_stats(binar_plan *plan, void *stream, binar_stats *out);
/* Enqueue on `stream` a copy of the plan's two device status words (the
 * error flags and the list-overflow flag of its last sort; both zero after
 * a good sort) into host_words[0..1], which should be pinned host memory
 * for the copy to be asynchronous.  The words are valid once the stream
 * has reached the copy; a nonzero error word with bit 0 set means a bad
 * segment table (BINAR_EINVAL), anything else nonzero a broken invariant
 * (BINAR_EDEVICE).  For servers that check every batch without a
 * synchronous read. */
int binar_plan_status_async(const binar_plan *plan, void *stream, uint32_t *host_words);
int binar_plan_graphs(const binar_plan *plan);
size_t binar_plan_workspace_bytes(const binar_plan *plan);
void binar_plan_destroy(binar_plan *plan);

/* Variable-length byte strings (the sort's "strings of average length",
 * section "Performance Analysis"; memcmp order, a proper prefix before its
 * extensions, equal strings in input order).  String i is
 * bytes[offsets[i], offsets[i+1]); bytes and offsets (n + 1 entries,
 * nondecreasing, at most nbytes) are DEVICE memory and are not modified.
 * payload (device, n entries) is permuted into the sorted order:
 * payload_out[i] = payload_in[p(i)]; pass 0..n-1 to receive p.
 * The strings are partitioned MSD-first 15 bytes at a time, each round
 * with the fixed-width 16-byte sort on (next 15 bytes, remaining-length
 * code) keys; only groups still tied go on to the next round.  Blocks
 * until done (one small device-to-host read per round).  An offsets table
 * out of order or past nbytes returns BINAR_EINVAL after reading nothing
 * out of bounds.  workspace may be NULL (pool). */
int binar_sort_strings(const uint8_t *bytes, uint64_t nbytes, const uint32_t *offsets, uint64_t n,
                       uint32_t *payload, void *stream, void *workspace, size_t workspace_bytes);
size_t binar_strings_workspace_bytes(uint64_t n);

/* In-place sort (sections "Space Analysis" and "Algorithm": the partition
 * works inside the caller's array, with extra space that does not grow with
 * the keys' size).  Same result as binar_sort_ex on one array: stable, keys
 * (device, n * key_bytes) and payload (device, n, or NULL) are permuted in
 * their own buffers.  No scratch copy of the keys exists: each pass sorts
 * every tile of a segment by its digit in on-chip memory, writes it back
 * over itself, and then moves every key to its place by following the
 * cycles of the pass's permutation.  The workspace holds only per-segment
 * and per-tile tables, 1 bit per key and a segment map (see
 * binar_inplace_workspace_bytes: about 5% of the data for 4-byte keys with
 * payload and 4-bit digits, against twice the data for binar_sort_ex).
 * params: digit_bits must be 0, 4 or 8 (default 4: twice the passes of 8,
 * but runs of one digit 16 times longer move together, which is faster),
 * tile_keys 0 or 4096, offsets 0 or 1
 * (else BINAR_EINVAL); finish_max is raised to at least 256; key_bits and
 * key_kind as for binar_sort_ex.  Asynchronous on stream; binar_stats_read
 * reads its counters.  workspace may be NULL (pool). */
int binar_sort_inplace(void *keys, uint32_t key_bytes, uint64_t n, uint32_t *payload, const binar_params *params,
                       void *stream, void *workspace, size_t workspace_bytes);
size_t binar_inplace_workspace_bytes(uint32_t key_bytes, uint64_t n, int has_payload, const binar_params *params);

/* Allocation-free sort, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The same operation and result as binar_sort_async on one
 * array (keys and payload are caller-owned device buffers, payload may be
 * NULL), enqueued on `stream`, but the scratch is a fixed array of
 * BINAR_STATIC_SCRATCH_BYTES inside the library, one per device, set up on
 * the first call on that device and held until the process ends.  The call
 * allocates nothing: no hipMalloc, no hipFree, no pool growth, no timing
 * events.  n is bounded by what fits: a call with
 * binar_workspace_bytes(key_bytes, n, payload != NULL, 1, NULL) above
 * BINAR_STATIC_SCRATCH_BYTES returns BINAR_ENOMEM before any device work
 * (about 3.9M 4-byte keys with payload, 3.1M 8-byte keys with payload,
 * 2.2M 16-byte keys with payload).  Every call on one device shares that
 * device's array, which keeps the last call's contents (each call clears
 * what it needs itself): calls that overlap in time on one device race,
 * whatever their streams.  binar_stats_read(NULL, stream, ...) reads the
 * counters of the last such call.  Errors as for binar_sort_async. */
#define BINAR_STATIC_SCRATCH_BYTES (64u << 20)
int binar_sort_static(void *keys, uint32_t key_bytes, uint64_t n, uint32_t *payload, void *stream);

/* Measurement helpers: the rate a plain streaming pass over device memory
 * reaches, to set the sort's passes against (a pass reads and writes its
 * bytes once, a digit count reads them once).  binar_stream_copy copies
 * `bytes` from src to dst (device, 16-byte aligned, bytes a multiple of 16,
 * not overlapping) with streaming stores; binar_stream_read reads src and
 * stores one XOR of its words per block to out (device, at least
 * blocks_per_cu x compute units words).  Both run a persistent grid of
 * blocks_per_cu (1..32) 256-thread blocks per compute unit with `unroll`
 * (2, 4 or 8) 16-byte vectors in flight per thread; BINAR_EINVAL for other
 * arguments.  Asynchronous on stream. */
int binar_stream_copy(void *dst, const void *src, size_t bytes, uint32_t blocks_per_cu, uint32_t unroll,
                      void *stream);
int binar_stream_read(const void *src, size_t bytes, uint32_t *out, uint32_t blocks_per_cu, uint32_t unroll,
                      void *stream);

/* Static description of a status code. */
const char *binar_strerror(int status);

/* The HIP call behind the last BINAR_EDEVICE returned on this thread and
 * HIP's message for it ("" if none); valid until the thread's next call. */
const char *binar_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BINAR_H */
