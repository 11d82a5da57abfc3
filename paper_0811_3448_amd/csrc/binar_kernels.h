// gfx950 kernels of the breadth-first stable binar sort.
//
// One call sorts a set of sub-arrays ("segments") of the keys.  Each global
// pass takes every live segment larger than the LDS-finish threshold T and
// partitions it stably on its next k bits (section "Partition Array into
// Sub-arrays", with the exchange replaced by a stable scatter, k bits at a
// time instead of one; k stable binary partitions in a row are one stable
// 2^k-way partition):
//
//   k_hist    digit counts of every live segment, per "piece" (the tiles of
//             one segment inside one block's chunk), + AND/OR of its keys
//   k_pscan   per segment and digit: exclusive prefix of the piece counts
//             over the segment's pieces, and the segment's digit totals
//   k_plan    per segment: pass-through test (one non-empty digit bin: the
//             iteration of section "Optimize the Algorithm"), bucket bases
//             (exclusive scan over digits), classification of the children:
//             done (one key or no varying bits left: the base cases of
//             section "Evaluate for Recursive Base Case"), LDS finish, or the
//             next pass
//   k_scatter per tile: stable rank by wave64 ballots, LDS staging in digit
//             order, coalesced write of keys and payload.  Bucket offsets
//             come either from the piece prefixes (each block walks its chunk
//             in order, carrying running offsets: no inter-block waits), or,
//             in the look-back variant, from a decoupled look-back over the
//             segment's earlier tiles (Merrill & Garland, 2016).
//
// after which k_finish sorts each small segment inside one workgroup (LDS
// least-significant-digit passes over its remaining varying bits) and
// writes it to the caller's buffer.
//
// Data live in two ping-pong buffer pairs: A (the caller's keys/payload) and
// B (scratch).  A segment's `parity` says which one holds it; a pass always
// writes the other buffer, because other tiles of the same segment may still
// be reading the source range.  Children that are finished (one key, or no
// varying bits left) therefore land in A only when their parent sat in B;
// finished children of a parent in A land in B and are copied back by
// k_copyback (runs of adjacent finished children merged into one range).
// Segments never overlap, so a finished segment is never touched again by
// later passes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "binar_keys.h"

namespace binar {

constexpr int WAVE = 64;
constexpr int THREADS = 256;
constexpr int WAVES = THREADS / WAVE;
constexpr int NCLASS = 4;        // LDS-finish size classes
constexpr uint32_t SMALL_MAX = 64;  // sub-arrays this short are ranked by one wave (k_finish_small)
constexpr int CAT_SMALL = NCLASS + 1;  // block_append category of such a sub-array
constexpr int S_BASE_WORDS = NCLASS + 4;  // block_append's shared bases (+ k_plan's copy-back base)
constexpr int MAX_PASSES = 16;   // statistics slots (128 bits / 8 bits)

constexpr uint32_t SEG_SKIP = 1u;  // segment does not scatter this pass
constexpr uint32_t ST_FLAGS = 3u << 30;
constexpr uint32_t ST_AGG = 1u << 30;  // look-back word: tile aggregate only
constexpr uint32_t ST_INC = 2u << 30;  // look-back word: inclusive prefix
constexpr uint32_t ST_VAL = (1u << 30) - 1u;
// Bound on every look-back wait (s_sleep rounds).  A predecessor tile always
// publishes within microseconds; the bound only guarantees that no wave can
// wait forever if an invariant were ever broken.
constexpr uint32_t SPIN_LIMIT = 1u << 24;
constexpr unsigned ERR_SEGMENTS = 1u;  // bad segment table
constexpr unsigned ERR_INTERNAL = 2u;  // broken invariant (bounds, wait limit)

// A live segment of a global pass.  info = bitpos | parity << 8 | flags << 16
// | (in a pass whose counts came with pass 0's) its digit in pass 0 << 24
struct SegEntry {
    uint32_t begin, len, info, tile_start;
};

// A segment to finish in LDS.  info = len | bitpos << 16 | parity << 24
struct FinEntry {
    uint32_t begin, info;
};

struct Ctl {
    unsigned long long list_ctr[2];  // (entries << 32) | tiles of each pass list
    unsigned int ticket;             // look-back scatter: tile tickets
    unsigned int error;              // ERR_SEGMENTS / ERR_INTERNAL
    unsigned int overflow;           // a list ran out of room (never expected)
    unsigned int passes;
    unsigned int fin_ctr[NCLASS];
    unsigned long long moved[MAX_PASSES];
    unsigned long long hist_keys[MAX_PASSES];
    unsigned long long fin_keys[NCLASS];
    unsigned long long fin_segs[NCLASS];
    unsigned int cpy_ctr;            // copy-back ranges
    unsigned int pad;
    unsigned long long cpy_keys;
    unsigned long long sorted_keys;  // keys of segments found already in order
    unsigned long long small_keys;   // keys and sub-arrays of k_finish_small
    unsigned long long small_segs;
    unsigned int small_ctr;          // entries of the small list
    unsigned int fused_pass;         // pass whose digit counts came with pass 0's (0: none)
    unsigned int fuse_bad;           // pass 0's digit-pair counts overflowed a 16-bit bin
    unsigned int pad3;
};

// A range [begin, begin + len) to copy from B to A after the passes.
struct CopyEntry {
    uint32_t begin, len;
};

struct Work {
    Ctl *ctl;
    SegEntry *list[2];
    uint32_t *counts[2];           // [entry][radix]: digit totals of the segment
    uint32_t *bases[2];            // [entry][radix]: bucket start (global index)
    unsigned long long *andor[2];  // [entry][4]: and.hi, and.lo, or.hi, or.lo
    uint32_t *desc[2];             // [entry]: nonzero once two adjacent keys are found out of order
    uint32_t *pcnt;                // [tile][radix]: piece counts -> piece prefixes (row = piece's first tile)
    uint32_t *status;              // [tile][radix]: look-back words (look-back variant only)
    FinEntry *fin[NCLASS];
    FinEntry *fin_small;           // sub-arrays of 2 .. SMALL_MAX keys
    uint32_t max_small;            // entries the small list can hold
    CopyEntry *cpy;
    uint32_t max_cpy;
    uint32_t fin_cap[NCLASS];      // largest segment of each class
    uint32_t max_fin[NCLASS];      // entries each class can hold
    uint32_t max_big, max_tiles;
    uint32_t finish_max;           // T
    uint32_t tile_keys;
    uint32_t n_total;              // keys in A and B: every index written is below it
    uint32_t chunk_grid;           // blocks of k_hist / k_scatter: fixes the pieces
    uint32_t nbits;                // leading key bits to sort by (the key width unless limited)
    uint32_t kind;                 // KIND_*: how key bits are ordered; loads apply enc, stores dec
    uint32_t inplace;              // passes permute inside A (no B); small children are not listed
    uint32_t pair_rows;            // pass 0 also counts digit pairs (blocks of k_hist that may write a row)
    uint32_t *pair_part;           // [block][R * R / 2]: each k_hist block's pair counts, two 16-bit bins a word
    uint32_t *pair_sum;            // [R][R]: pair counts of the whole array (digit of pass 0, digit of pass 1)
    void *keys[2];                 // A, B
    uint32_t *pay[2];              // A, B (NULL without payload)
};

// ------------------------------------------------------------ small helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Values every lane of a wave holds alike, made visibly uniform so the
// compiler keeps them (and addresses built from them) in scalar registers.
__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ SegEntry uni(const SegEntry &e) {
    return SegEntry{uni(e.begin), uni(e.len), uni(e.info), uni(e.tile_start)};
}

__device__ __forceinline__ FinEntry uni(const FinEntry &e) { return FinEntry{uni(e.begin), uni(e.info)}; }

__device__ __forceinline__ uint32_t ld_agent(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_agent(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive scan of one value per thread over a block of BT threads;
// returns the exclusive prefix and writes the block total to *total.
// tmp: BT / 64 words.
template <int BT = THREADS>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *tmp, uint32_t *total) {
    constexpr int WAVES = BT / WAVE;
    const int lane = lane_id();
    const int wv = threadIdx.x / WAVE;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        uint32_t y = __shfl_up(x, o, WAVE);
        if (lane >= o) x += y;
    }
    if (lane == WAVE - 1) tmp[wv] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
        const uint32_t t = tmp[w];
        if (w < wv) before += t;
        all += t;
    }
    __syncthreads();
    *total = all;
    return before + x - v;
}

// Stable rank of every key of a wave's ITEMS steps (64 consecutive keys per
// step) among the keys with the same digit: keys of earlier steps of this
// wave + earlier lanes of this step.
//   tbl  : this wave's table of R lane masks in LDS, each two 32-bit words
//          (lanes 0-31, lanes 32-63), 8-byte aligned (zero on entry and exit)
//   whist: this wave's R counters in LDS (zero on entry; the wave's digit
//          counts on exit)
// For each step every lane ORs its lane bit into its half of tbl[digit] and
// reads the whole 64-bit mask back -- the lanes holding its digit -- then
// clears its half (32-bit atomics spread a wave's 64 lanes over the LDS banks
// better than 64-bit ones).
// The highest lane of each mask adds the group size to whist[digit] with an
// LDS atomic and the others take the old value from it.  A wave's LDS
// operations execute in issue order, so one table serves every step and the
// counters advance step by step: the ranks follow the input order.  Steps go
// in groups of G whose operations are issued back to back (masks of all G
// steps, then all G counter updates, then all G broadcasts), so a group
// waits for the LDS three times instead of three times per step.  UNI: up
// to two digits of a step bypass the table (below; the check costs
// registers, so only the scatter uses it).  FULL: every key of the tile is
// valid.
constexpr int RANK_GROUP = 2;  // steps per group of wave_rank
constexpr int PEEL_MISSES = 4;  // unproductive steps after which a wave stops peeling digits
constexpr int PEEL_RETRY = 32;  // steps after which a wave that stopped peeling tries again
constexpr int PEEL_GAIN = 32;   // lanes a step's peeling must take out to count as worth it

template <int R, int G, int ITEMS, bool FULL, bool UNI = false>
__device__ __forceinline__ void wave_rank(const uint32_t (&dg)[ITEMS], uint32_t ebase, uint32_t len,
                                          uint32_t *tbl, uint32_t *whist, uint32_t (&rnk)[ITEMS],
                                          int *peel_misses = nullptr) {
    if constexpr (R == 2) {
        // the paper's one-bit step: a ballot of the bit gives each lane the
        // lanes below it with the same bit (mbcnt), its popcount the wave's
        // total; running totals carry the order across steps
        uint32_t c0 = 0u, c1 = 0u;
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const bool valid = FULL || ebase + (uint32_t)j * WAVE < len;
            const uint64_t m1 = __ballot(valid && dg[j] != 0u), m0 = __ballot(valid && dg[j] == 0u);
            rnk[j] = dg[j] ? c1 + lanes_below(m1) : c0 + lanes_below(m0);
            c0 += (uint32_t)__popcll(m0);
            c1 += (uint32_t)__popcll(m1);
        }
        if (lane_id() == 0) {
            whist[0] += c0;
            whist[1] += c1;
        }
        (void)tbl;
        return;
    }
    // the 64-bit view of a mask may alias the 32-bit words it is built from
    typedef unsigned long long __attribute__((may_alias)) mask_t;
    const uint32_t half = (uint32_t)lane_id() >> 5, me = 1u << (lane_id() & 31);
#pragma unroll
    for (int j0 = 0; j0 < ITEMS; j0 += G) {
        bool valid[G];
        unsigned long long m[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int j = j0 + g;
            valid[g] = (j < ITEMS) && (FULL || ebase + (uint32_t)j * WAVE < len);
            m[g] = 0ull;
            // skewed data puts many lanes of a step on one digit (and 64
            // lanes on one LDS word are served one after another).  A step
            // whose valid lanes all hold one digit takes the ballot of its
            // valid lanes as the mask.  In other steps up to two digits are
            // taken out whole (the first remaining lane's digit each time,
            // their masks the ballot of their lanes) and the other lanes go
            // through the table; a wave stops that after PEEL_MISSES mixed
            // steps in a row in which it took out fewer than PEEL_GAIN lanes,
            // and tries again every PEEL_RETRY mixed steps (*peel_misses,
            // kept by the caller across tiles).
            bool peeled = false;
            if constexpr (UNI) {
                const uint32_t dj = dg[j < ITEMS ? j : 0];
                const unsigned long long vm = __ballot(valid[g]);
                const uint32_t d0 = __builtin_amdgcn_readlane(dj, vm ? __builtin_ctzll(vm) : 0);
                const unsigned long long p0 = __ballot(valid[g] && dj == d0);
                if (p0 == vm) {
                    m[g] = valid[g] ? vm : 0ull;
                    peeled = true;
                } else {
                    if (*peel_misses >= PEEL_MISSES && ++*peel_misses >= PEEL_MISSES + PEEL_RETRY)
                        *peel_misses = PEEL_MISSES - 1;
                    if (*peel_misses < PEEL_MISSES) {
                        const unsigned long long rest = vm & ~p0;
                        const uint32_t d1 = __builtin_amdgcn_readlane(dj, __builtin_ctzll(rest));
                        const unsigned long long p1 = __ballot(valid[g] && dj == d1) & rest;
                        peeled = valid[g] && (dj == d0 || dj == d1);
                        if (peeled) m[g] = (dj == d0) ? p0 : p1;
                        *peel_misses = (__popcll(p0) + __popcll(p1) < PEEL_GAIN) ? *peel_misses + 1 : 0;
                    }
                }
            }
            if (!peeled && valid[g]) {
                atomicOr(&tbl[2u * dg[j] + half], me);
                m[g] = *reinterpret_cast<const mask_t *>(&tbl[2u * dg[j]]);
                tbl[2u * dg[j] + half] = 0u;
            }
        }
        uint32_t lead[G], got[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int j = j0 + g;
            got[g] = 0u;
            lead[g] = 0u;
            if (j < ITEMS) {
                const uint32_t r = lanes_below(m[g]);
                const uint32_t c = (uint32_t)__popcll(m[g]);
                lead[g] = 63u - (uint32_t)__clzll(m[g] | 1ull);
                rnk[j] = r;
                if (valid[g] && r + 1u == c) got[g] = atomicAdd(&whist[dg[j]], c);
            }
        }
#pragma unroll
        for (int g = 0; g < G; ++g)
            if (j0 + g < ITEMS) rnk[j0 + g] += (uint32_t)__shfl((int)got[g], (int)lead[g], WAVE);
    }
}

// ------------------------------------------------------------------ k_reset
static __global__ void k_reset(Ctl *ctl) {
    uint32_t *p = reinterpret_cast<uint32_t *>(ctl);
    for (uint32_t i = threadIdx.x; i < sizeof(Ctl) / 4; i += blockDim.x) p[i] = 0u;
}

// Block-aggregated appends of the children a block found: category q of
// thread's child: 0..NCLASS-1 = LDS-finish class, NCLASS = next pass list,
// CAT_SMALL = small list, -1 = none.  Each category reserves one contiguous
// range with one atomic; next-pass entries reserve their list slots and
// tiles together, so the list stays ordered by tile_start.  s_base holds
// S_BASE_WORDS words; word NCLASS + 2 is left to the caller.  slot_out, if
// given, receives the thread's slot in the next list (~0u if it appended
// none there).
template <int R>
__device__ void block_append(const Work &w, int Lnext, int cat, uint32_t begin, uint32_t len, uint32_t bitpos,
                             uint32_t parity, uint32_t *s_tmp, uint32_t *s_base, uint32_t *slot_out = nullptr) {
    if (slot_out) *slot_out = ~0u;
    uint32_t idx[NCLASS + 2];
    uint32_t tot[NCLASS + 2];
#pragma unroll
    for (int q = 0; q <= CAT_SMALL; ++q) idx[q] = block_excl_scan(cat == q ? 1u : 0u, s_tmp, &tot[q]);
    const uint32_t ntiles = (cat == NCLASS) ? (len + w.tile_keys - 1) / w.tile_keys : 0u;
    uint32_t tot_tiles;
    const uint32_t tidx = block_excl_scan(ntiles, s_tmp, &tot_tiles);
    // the finish counters (keys and sub-arrays per class, and of the small
    // path) are kept here, once per block: thousands of finishing waves or
    // blocks adding to one address each would serialise
    __shared__ uint32_t s_fk[NCLASS + 1][THREADS / WAVE];
    uint32_t fkeys[NCLASS + 1];
    {
        const int wv = threadIdx.x / WAVE;
#pragma unroll
        for (int q = 0; q <= NCLASS; ++q) {
            uint32_t x = (cat == (q < NCLASS ? q : CAT_SMALL)) ? len : 0u;
#pragma unroll
            for (int o = 1; o < WAVE; o <<= 1) x += __shfl_xor(x, o, WAVE);
            if (lane_id() == 0) s_fk[q][wv] = x;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q <= NCLASS; ++q) {
            fkeys[q] = 0u;
#pragma unroll
            for (int v = 0; v < THREADS / WAVE; ++v) fkeys[q] += s_fk[q][v];
        }
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NCLASS; ++q) {
            s_base[q] = tot[q] ? atomicAdd(&w.ctl->fin_ctr[q], tot[q]) : 0u;
            if (tot[q]) {
                atomicAdd(&w.ctl->fin_keys[q], (unsigned long long)fkeys[q]);
                atomicAdd(&w.ctl->fin_segs[q], (unsigned long long)tot[q]);
            }
        }
        s_base[NCLASS + 3] = tot[CAT_SMALL] ? atomicAdd(&w.ctl->small_ctr, tot[CAT_SMALL]) : 0u;
        if (tot[CAT_SMALL]) {
            atomicAdd(&w.ctl->small_keys, (unsigned long long)fkeys[NCLASS]);
            atomicAdd(&w.ctl->small_segs, (unsigned long long)tot[CAT_SMALL]);
        }
        if (tot[NCLASS]) {
            const unsigned long long old = atomicAdd(&w.ctl->list_ctr[Lnext],
                                                     ((unsigned long long)tot[NCLASS] << 32) | tot_tiles);
            s_base[NCLASS] = (uint32_t)(old >> 32);
            s_base[NCLASS + 1] = (uint32_t)old;
        }
    }
    __syncthreads();
    if (cat >= 0 && cat < NCLASS) {
        const uint32_t slot = s_base[cat] + idx[cat];
        if (slot < w.max_fin[cat])
            w.fin[cat][slot] = FinEntry{begin, len | (bitpos << 16) | (parity << 24)};
        else
            atomicOr(&w.ctl->overflow, 1u);
    } else if (cat == CAT_SMALL) {
        const uint32_t slot = s_base[NCLASS + 3] + idx[CAT_SMALL];
        if (slot < w.max_small)
            w.fin_small[slot] = FinEntry{begin, len | (bitpos << 16) | (parity << 24)};
        else
            atomicOr(&w.ctl->overflow, 1u);
    } else if (cat == NCLASS) {
        const uint32_t slot = s_base[NCLASS] + idx[NCLASS];
        const uint32_t ts = s_base[NCLASS + 1] + tidx;
        if (slot < w.max_big && ts + ntiles <= w.max_tiles) {
            if (slot_out) *slot_out = slot;
            w.list[Lnext][slot] = SegEntry{begin, len, bitpos | (parity << 8), ts};
            unsigned long long *ao = w.andor[Lnext] + (size_t)slot * 4;
            w.desc[Lnext][slot] = 0u;
            ao[0] = ~0ull;
            ao[1] = ~0ull;
            ao[2] = 0ull;
            ao[3] = 0ull;
        } else {
            atomicOr(&w.ctl->overflow, 1u);
        }
    }
    __syncthreads();
}

// Where a sub-array of 2 .. T keys is finished: the small list, or the
// smallest LDS class that holds it.
__device__ __forceinline__ int fin_class(const Work &w, uint32_t len) {
    if (len <= SMALL_MAX) return CAT_SMALL;
    int c = 0;
    while (c < NCLASS - 1 && len > w.fin_cap[c]) ++c;
    return c;
}

// ------------------------------------------------------------------- k_init
// Classify the caller's segments: <= 1 key: nothing to do (base case);
// <= T keys: finished by one wave (small list) or in LDS; larger: first
// global pass.
template <int R>
__global__ __launch_bounds__(THREADS) void k_init(Work w, const uint32_t *seg_off, uint32_t nseg,
                                                  uint32_t n_single, uint32_t n_limit) {
    __shared__ uint32_t s_tmp[WAVES];
    __shared__ uint32_t s_base[S_BASE_WORDS];
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t s0 = blockIdx.x * blockDim.x; s0 < nseg; s0 += stride) {
        const uint32_t s = s0 + threadIdx.x;
        int cat = -1;
        uint32_t b = 0, len = 0;
        if (s < nseg) {
            uint32_t e = n_single;
            if (seg_off) {
                b = seg_off[s];
                e = seg_off[s + 1];
            }
            if (e < b || e > n_limit) {
                atomicOr(&w.ctl->error, ERR_SEGMENTS);
            } else {
                len = e - b;
                if (len > 1) cat = (len <= w.finish_max) ? fin_class(w, len) : NCLASS;
            }
        }
        block_append<R>(w, 0, cat, b, len, 0u, 0u, s_tmp, s_base);
    }
}

// Segment holding tile t: the last list entry whose tile_start <= t.
__device__ __forceinline__ uint32_t find_slot(const SegEntry *list, uint32_t nslots, uint32_t t) {
    uint32_t lo = 0, hi = nslots - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (list[mid].tile_start <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ uint32_t seg_tile_end(const SegEntry *list, uint32_t slot, uint32_t nslots,
                                                 uint32_t ntiles) {
    return (slot + 1 < nslots) ? list[slot + 1].tile_start : ntiles;
}

// 16-byte vector of keys: 4 (u32), 2 (u64) or 1 (16-byte string).
template <int KB>
struct Vec {
    static constexpr int N = 16 / KB;
};

template <int KB>
__device__ __forceinline__ void load_vec(const void *p, size_t i, typename KeyT<KB>::V (&v)[Vec<KB>::N]) {
    if constexpr (KB == 4) {
        const uint4 x = *reinterpret_cast<const uint4 *>(reinterpret_cast<const uint32_t *>(p) + i);
        v[0] = x.x;
        v[1] = x.y;
        v[2] = x.z;
        v[3] = x.w;
    } else if constexpr (KB == 8) {
        const ulonglong2 x = *reinterpret_cast<const ulonglong2 *>(reinterpret_cast<const uint64_t *>(p) + i);
        v[0] = x.x;
        v[1] = x.y;
    } else {
        v[0] = KeyT<16>::load(p, i);
    }
}

// The key held by the lane below (lane 0: unspecified).  4- and 8-byte keys
// move with a DPP wave shift (a VALU op); 16-byte keys through the LDS
// crossbar.
template <int KB>
__device__ __forceinline__ typename KeyT<KB>::V shfl_up_key(typename KeyT<KB>::V v) {
    constexpr int WAVE_SHR1 = 0x138;
    if constexpr (KB == 4) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, WAVE_SHR1, 0xF, 0xF, false);
    } else if constexpr (KB == 8) {
        const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, WAVE_SHR1, 0xF, 0xF, false);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), WAVE_SHR1, 0xF, 0xF,
                                                                  false);
        return ((uint64_t)hi << 32) | lo;
    } else {
        return U128{(uint64_t)__shfl_up((long long)v.hi, 1u, WAVE), (uint64_t)__shfl_up((long long)v.lo, 1u, WAVE)};
    }
}

// a comes after b in the sort order of the leading bits selected by m (all
// bits when `full`: then a plain integer compare for 4- and 8-byte keys).
template <int KB>
__device__ __forceinline__ bool key_after(typename KeyT<KB>::V a, typename KeyT<KB>::V b, Canon m, bool full) {
    if constexpr (KB != 16) {
        if (full) return a > b;
    }
    return canon_after(KeyT<KB>::canon(a), KeyT<KB>::canon(b), m);
}

// Key i of a buffer in the sorting view (enc), and back.
template <int KB>
__device__ __forceinline__ typename KeyT<KB>::V ld_key(const void *p, size_t i, uint32_t kind) {
    const typename KeyT<KB>::V v = KeyT<KB>::load(p, i);
    return kind ? KeyT<KB>::enc(v, kind) : v;
}

template <int KB>
__device__ __forceinline__ typename KeyT<KB>::V raw_key(typename KeyT<KB>::V v, uint32_t kind) {
    return kind ? KeyT<KB>::dec(v, kind) : v;
}

// ------------------------------------------------------------------- k_hist
// Digit counts (bits [bitpos, bitpos + w) of each key) and AND/OR of every
// live segment of list L.  The tiles of the list are cut into gridDim.x
// contiguous chunks, one per block; the tiles of one segment inside one
// chunk form a piece, whose counts go to row pcnt[first tile of the piece].
// Also resets the next list and the scatter ticket (nothing else touches
// them during this kernel) and, for the look-back scatter, clears the
// look-back words of every tile.
//
// PAIRS (first pass of one array): the digit of the next K bits is counted
// too, per pair (this digit, next digit), in 16-bit LDS bins packed two to a
// word; each block leaves its pair counts in its row of w.pair_part (and
// k_pair_sum adds the rows).  A block that holds more than 65535 keys of
// one digit (so that one of its pair bins could pass 65535) sets
// ctl->fuse_bad: the pair counts are then not used (the piece counts come
// from the exact per-wave counts either way).
// A pass whose counts came with pass 0's (ctl->fused_pass) reads no key.
template <int KB, int K, bool LOOKBACK, int BT, bool PAIRS>
__global__ __launch_bounds__(BT) void k_hist(Work w, int L, int pass) {
    using KT = KeyT<KB>;
    using V = typename KT::V;
    constexpr int R = 1 << K;
    constexpr int VN = Vec<KB>::N;
    constexpr int U = 4;  // vectors in flight per thread
    constexpr int NW = BT / WAVE;
    __shared__ uint32_t s_h[NW][R];
    __shared__ uint32_t s_p[PAIRS ? R * R / 2 : 1];
    __shared__ unsigned long long s_ao[NW][4];

    Ctl *ctl = w.ctl;
    if (ctl->error | ctl->overflow) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->list_ctr[L ^ 1] = 0ull;
        ctl->ticket = 0u;
    }
    if (pass != 0 && (uint32_t)pass == ctl->fused_pass) return;
    const unsigned long long lc = ctl->list_ctr[L];
    const uint32_t nslots = (uint32_t)(lc >> 32), ntiles = (uint32_t)lc;
    if (ntiles == 0) return;
    const uint32_t per = (ntiles + gridDim.x - 1) / gridDim.x;
    const uint32_t t0 = blockIdx.x * per;
    const uint32_t t1 = min(ntiles, t0 + per);
    if (t0 >= t1) return;

    const int wv = threadIdx.x / WAVE, lane = lane_id();
    if (PAIRS)
        for (int i = threadIdx.x; i < R * R / 2; i += BT) s_p[i] = 0u;
    for (int i = threadIdx.x; i < NW * R; i += BT) (&s_h[0][0])[i] = 0u;
    if (LOOKBACK)
        for (size_t i = (size_t)t0 * R + threadIdx.x; i < (size_t)t1 * R; i += BT) w.status[i] = 0u;
    __syncthreads();
    // a pair bin can pass 65535 (and spill into its neighbour) only if its
    // digit has more than 65535 keys in the block: checked on the block's
    // digit totals when they are flushed, so the pair adds need no result
    bool pair_full = false;

    uint32_t slot = find_slot(w.list[L], nslots, t0);
    for (uint32_t t = t0; t < t1;) {
        const SegEntry seg = uni(w.list[L][slot]);
        const uint32_t te = min(t1, seg_tile_end(w.list[L], slot, nslots, ntiles));
        const uint32_t bitpos = seg.info & 0xFFu, parity = (seg.info >> 8) & 1u;
        const int wbits = min(K, (int)w.nbits - (int)bitpos);
        const uint32_t kind = w.kind;
        const void *src = w.keys[parity];
        // already in order?  every key after the segment's first against its
        // predecessor, in the leading bits being sorted
        const Canon km = canon_lead_mask((int)w.nbits);
        const bool full = w.nbits == 8u * KB;
        bool desc = false;
        const size_t g0 = (size_t)seg.begin + (size_t)(t - seg.tile_start) * w.tile_keys;
        const size_t g1 = (size_t)seg.begin + min((size_t)seg.len, (size_t)(te - seg.tile_start) * w.tile_keys);
        V a = KT::ones(), o = KT::zero();
        // one-bit steps count with ballots: per wave step, the popcounts of
        // the active lanes and of those whose bit is 1, added to the wave's
        // counters by its first active lane (the loops below are divergent);
        // wider digits with a per-wave LDS histogram
        // the next digit of the pairs: the K bits after this pass's (the
        // pairs are used only if the next pass starts there)
        const int nbits2 = min(K, (int)w.nbits - (int)bitpos - wbits);
        auto count = [&](const V &v) {
            const uint32_t d = KT::digit(v, bitpos, wbits);
            if constexpr (PAIRS) {
                const uint32_t b = d * R + (nbits2 > 0 ? KT::digit(v, bitpos + wbits, nbits2) : 0u);
                const uint32_t sh = (b & 1u) * 16u;
                atomicAdd(&s_p[b >> 1], 1u << sh);
            }
            if constexpr (K == 1) {
                const uint64_t act = __ballot(true), ones = __ballot(d != 0u);
                if (lane == __builtin_ctzll(act)) {
                    s_h[wv][1] += (uint32_t)__popcll(ones);
                    s_h[wv][0] += (uint32_t)__popcll(act & ~ones);
                }
            } else {
                atomicAdd(&s_h[wv][d], 1u);
            }
        };
        // Skewed or sorted data (duplicates, low-entropy bits, runs) puts
        // many lanes of a wave step on one digit, and 64 lanes adding to one
        // LDS word are served one after another.  So up to PEELS bins of a
        // step are taken out whole: the first remaining lane's bin (its digit,
        // or its digit pair with PAIRS), counted with a ballot and added once;
        // the lanes left after that add one each.  Random keys gain nothing
        // from it and would pay for the ballots at every step, so a wave
        // stops peeling in this piece after MISSES steps in a row in which
        // peeling took out fewer than 16 lanes.
        constexpr int PEELS = 2;
        constexpr int MISSES = 4;
        int misses = (K == 1) ? MISSES : 0;
        auto count_peeled = [&](const V &v) {
            const uint32_t d = KT::digit(v, bitpos, wbits);
            const uint32_t bin = PAIRS ? d * R + (nbits2 > 0 ? KT::digit(v, bitpos + wbits, nbits2) : 0u) : d;
            const uint64_t all = __ballot(true);
            uint64_t rest = all;
#pragma unroll
            for (int it = 0; it < PEELS; ++it) {
                if (rest == 0ull) break;
                const int l0 = __builtin_ctzll(rest);
                const uint32_t b0 = __builtin_amdgcn_readlane(bin, l0);
                const uint64_t m = __ballot(bin == b0) & rest;
                if (lane == l0) {
                    const uint32_t c = (uint32_t)__popcll(m);
                    if constexpr (PAIRS) {
                        const uint32_t sh = (b0 & 1u) * 16u;
                        atomicAdd(&s_p[b0 >> 1], c << sh);
                        atomicAdd(&s_h[wv][b0 / R], c);
                    } else {
                        atomicAdd(&s_h[wv][b0], c);
                    }
                }
                rest &= ~m;
            }
            if ((rest >> lane) & 1ull) count(v);
            misses = (__popcll(all) - __popcll(rest) < 16) ? misses + 1 : 0;
        };
        // head and tail one key at a time, the 16-byte aligned body 16 bytes at
        // a time (keys are at least key-size aligned, so `mis` is whole keys)
        const size_t mis = ((16u - (reinterpret_cast<uintptr_t>(src) & 15u)) & 15u) / KB;
        const size_t b0 = min(g1, g0 + ((mis + VN - (g0 % VN)) % VN));
        const size_t b1 = b0 + (g1 - b0) / VN * VN;
        for (size_t i = g0 + threadIdx.x; i < b0; i += BT) {
            const V v = ld_key<KB>(src, i, kind);
            if (i > seg.begin) desc |= key_after<KB>(ld_key<KB>(src, i - 1, kind), v, km, full);
            count(v);
            a = KT::vand(a, v);
            o = KT::vor(o, v);
        }
        for (size_t i = b1 + threadIdx.x; i < g1; i += BT) {
            const V v = ld_key<KB>(src, i, kind);
            if (i > seg.begin) desc |= key_after<KB>(ld_key<KB>(src, i - 1, kind), v, km, full);
            count(v);
            a = KT::vand(a, v);
            o = KT::vor(o, v);
        }
        for (size_t i = b0 + (size_t)threadIdx.x * VN; i < b1; i += (size_t)BT * VN * U) {
            V v[U][VN];
            V pv[U];  // the key before the vector, where no lane below holds it
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const size_t x = i + (size_t)u * BT * VN;
                if (x < b1) load_vec<KB>(src, x, v[u]);
                if (x < b1 && (lane == 0 || x == b0) && x > seg.begin) pv[u] = KT::load(src, x - 1);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const size_t x = i + (size_t)u * BT * VN;
                // the key before this vector: the last of the lane below's vector
                // (same step), loaded directly for lane 0 and for the body's first
                // vector
                const V pl = shfl_up_key<KB>(v[u][VN - 1]);
                if (x < b1) {
                    if (kind) {
#pragma unroll
                        for (int q = 0; q < VN; ++q) v[u][q] = KT::enc(v[u][q], kind);
                    }
                    V prev = (lane == 0 || x == b0) ? pv[u] : pl;
                    if (kind) prev = KT::enc(prev, kind);
                    if (x > seg.begin) desc |= key_after<KB>(prev, v[u][0], km, full);
#pragma unroll
                    for (int q = 1; q < VN; ++q) desc |= key_after<KB>(v[u][q - 1], v[u][q], km, full);
                    if (misses < MISSES) {
#pragma unroll
                        for (int q = 0; q < VN; ++q) count_peeled(v[u][q]);
                    } else {
#pragma unroll
                        for (int q = 0; q < VN; ++q) count(v[u][q]);
                    }
#pragma unroll
                    for (int q = 0; q < VN; ++q) {
                        a = KT::vand(a, v[u][q]);
                        o = KT::vor(o, v[u][q]);
                    }
                }
            }
        }
        // flush the piece: counts to its row, AND/OR to the segment
        Canon ca = KT::canon(a), co = KT::canon(o);
#pragma unroll
        for (int off = 1; off < WAVE; off <<= 1) {
            ca.hi &= __shfl_xor(ca.hi, off, WAVE);
            ca.lo &= __shfl_xor(ca.lo, off, WAVE);
            co.hi |= __shfl_xor(co.hi, off, WAVE);
            co.lo |= __shfl_xor(co.lo, off, WAVE);
        }
        if (lane == 0) {
            s_ao[wv][0] = ca.hi;
            s_ao[wv][1] = ca.lo;
            s_ao[wv][2] = co.hi;
            s_ao[wv][3] = co.lo;
        }
        if (__syncthreads_or(desc ? 1 : 0) && threadIdx.x == 0) atomicOr(&w.desc[L][slot], 1u);
        uint32_t *row = w.pcnt + (size_t)t * R;
        for (int d = threadIdx.x; d < R; d += BT) {
            uint32_t c = 0;
#pragma unroll
            for (int q = 0; q < NW; ++q) {
                c += s_h[q][d];
                s_h[q][d] = 0u;
            }
            row[d] = c;
            if (PAIRS) pair_full |= c > 0xFFFFu;
        }
        if constexpr (PAIRS) {
            // one piece per block (one array): the pairs go to the block's
            // row, cleared after
            uint32_t *prow = w.pair_part + (size_t)blockIdx.x * (R * R / 2);
            for (int i = threadIdx.x; i < R * R / 2; i += BT) {
                prow[i] = s_p[i];
                s_p[i] = 0u;
            }
            if (__syncthreads_or(pair_full ? 1 : 0) && threadIdx.x == 0) atomicOr(&ctl->fuse_bad, 1u);
        }
        if (threadIdx.x < 4) {
            unsigned long long v = s_ao[0][threadIdx.x];
            for (int q = 1; q < NW; ++q)
                v = (threadIdx.x < 2) ? (v & s_ao[q][threadIdx.x]) : (v | s_ao[q][threadIdx.x]);
            unsigned long long *dst = w.andor[L] + (size_t)slot * 4 + threadIdx.x;
            if (threadIdx.x < 2)
                atomicAnd(dst, v);
            else
                atomicOr(dst, v);
        }
        __syncthreads();
        t = te;
        ++slot;
    }
}

// -------------------------------------------------------------- k_pair_sum
// Pair counts of the whole array: the sum of the rows that k_hist's blocks
// with work left in w.pair_part (block b has work iff b * per < tiles),
// unpacked to 32 bits, into w.pair_sum[d0 * R + d1].
template <int K>
__global__ __launch_bounds__(THREADS) void k_pair_sum(Work w) {
    constexpr int R = 1 << K;
    constexpr uint32_t NPW = R * R / 2;  // words per row
    Ctl *ctl = w.ctl;
    if (ctl->error | ctl->overflow | ctl->fuse_bad) return;
    const unsigned long long lc = ctl->list_ctr[0];
    const uint32_t ntiles = (uint32_t)lc;
    if (ntiles == 0 || (uint32_t)(lc >> 32) != 1u) return;
    const uint32_t per = (ntiles + w.chunk_grid - 1) / w.chunk_grid;
    const uint32_t rows = min(w.pair_rows, (ntiles + per - 1) / per);
    for (uint32_t i = blockIdx.x * THREADS + threadIdx.x; i < NPW; i += gridDim.x * THREADS) {
        uint32_t lo = 0u, hi = 0u;
        uint32_t b = 0;
        for (; b + 8 <= rows; b += 8) {
            uint32_t x[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) x[q] = w.pair_part[(size_t)(b + q) * NPW + i];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                lo += x[q] & 0xFFFFu;
                hi += x[q] >> 16;
            }
        }
        for (; b < rows; ++b) {
            const uint32_t x = w.pair_part[(size_t)b * NPW + i];
            lo += x & 0xFFFFu;
            hi += x >> 16;
        }
        w.pair_sum[2 * i] = lo;
        w.pair_sum[2 * i + 1] = hi;
    }
}

// ------------------------------------------------------------------ k_pscan
// For every live segment and digit: the exclusive prefix of its piece counts
// over the segment's pieces (in tile order, written back in place) and the
// segment's digit total.  One block per (segment, group of up to 32
// digits); THREADS / group lanes split the pieces into contiguous runs.
template <int K>
__global__ __launch_bounds__(THREADS) void k_pscan(Work w, int L, int pass) {
    constexpr int R = 1 << K;
    constexpr int DG = R < 32 ? R : 32;          // digits per block
    constexpr int NG = R / DG;                   // digit groups per segment
    constexpr int Q = THREADS / DG;              // lanes per digit
    constexpr int B = 8;                         // loads in flight per lane
    __shared__ uint32_t s_part[Q][DG];

    Ctl *ctl = w.ctl;
    if (ctl->error | ctl->overflow) return;
    if (pass != 0 && (uint32_t)pass == ctl->fused_pass) return;  // totals set by pass 0's plan, one piece per segment
    const unsigned long long lc = ctl->list_ctr[L];
    const uint32_t nslots = (uint32_t)(lc >> 32), ntiles = (uint32_t)lc;
    if (nslots == 0) return;
    const uint32_t per = (ntiles + w.chunk_grid - 1) / w.chunk_grid;
    const int dl = threadIdx.x % DG, q = threadIdx.x / DG;

    for (uint32_t item = blockIdx.x; item < nslots * NG; item += gridDim.x) {
        const uint32_t slot = item / NG;
        const int d = (int)(item % NG) * DG + dl;
        const SegEntry seg = w.list[L][slot];
        const uint32_t ts = seg.tile_start;
        const uint32_t te = seg_tile_end(w.list[L], slot, nslots, ntiles);
        // pieces: ts, then every chunk start inside (ts, te)
        const uint32_t c0 = ts / per;
        const uint32_t np = (te - 1) / per - c0 + 1;
        const uint32_t p0 = (uint32_t)(((unsigned long long)np * q) / Q);
        const uint32_t p1 = (uint32_t)(((unsigned long long)np * (q + 1)) / Q);
        auto row = [&](uint32_t p) -> uint32_t * {
            const uint32_t t = (p == 0) ? ts : (c0 + p) * per;
            return w.pcnt + (size_t)t * R + d;
        };
        uint32_t part = 0;
        for (uint32_t p = p0; p < p1; p += B) {
            uint32_t v[B];
#pragma unroll
            for (int i = 0; i < B; ++i) v[i] = (p + i < p1) ? *row(p + i) : 0u;
#pragma unroll
            for (int i = 0; i < B; ++i) part += v[i];
        }
        s_part[q][dl] = part;
        __syncthreads();
        uint32_t run = 0, total = 0;
        for (int k = 0; k < Q; ++k) {
            const uint32_t x = s_part[k][dl];
            if (k < q) run += x;
            total += x;
        }
        __syncthreads();
        if (q == 0) w.counts[L][(size_t)slot * R + d] = total;
        for (uint32_t p = p0; p < p1; p += B) {
            uint32_t v[B];
#pragma unroll
            for (int i = 0; i < B; ++i) v[i] = (p + i < p1) ? *row(p + i) : 0u;
#pragma unroll
            for (int i = 0; i < B; ++i) {
                if (p + i < p1) *row(p + i) = run;
                run += v[i];
            }
        }
    }
}

// ------------------------------------------------------------------- k_plan
template <int KB, int K>
__global__ __launch_bounds__(THREADS) void k_plan(Work w, int L, int pass) {
    constexpr int R = 1 << K;
    const int NB = (int)w.nbits;
    __shared__ uint32_t s_tmp[WAVES];
    __shared__ uint32_t s_base[S_BASE_WORDS];
    __shared__ uint32_t s_state[THREADS];
    __shared__ uint32_t s_max;
    Ctl *ctl = w.ctl;
    if (ctl->error | ctl->overflow) return;
    const unsigned long long lc = ctl->list_ctr[L];
    const uint32_t nslots = (uint32_t)(lc >> 32);
    if (nslots == 0) return;
    const bool fused_here = pass != 0 && (uint32_t)pass == ctl->fused_pass;  // no key was read for this pass
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicMax(&ctl->passes, (unsigned)(pass + 1));
    const int ps = pass < MAX_PASSES ? pass : MAX_PASSES - 1;
    const int d = threadIdx.x;
    // statistics: summed per block, one atomic each at the end (per-segment
    // atomics on one address serialise the whole grid)
    unsigned long long st_hist = 0ull, st_moved = 0ull, st_sorted = 0ull;
    unsigned long long st_small_keys = 0ull, st_small_segs = 0ull;  // in place: children ranked from the table

    for (uint32_t s = blockIdx.x; s < nslots; s += gridDim.x) {
        const SegEntry seg = w.list[L][s];
        const uint32_t bitpos = seg.info & 0xFFu, parity = (seg.info >> 8) & 1u;
        const int wbits = min(K, NB - (int)bitpos);
        const uint32_t nbins = 1u << wbits;
        // counts of this segment's digits: from the digit count, or, in the
        // pass whose counts came with pass 0's, row (parent digit) of the
        // pair sums
        const uint32_t *segc = fused_here ? w.pair_sum + (size_t)(seg.info >> 24) * R : w.counts[L] + (size_t)s * R;
        const uint32_t c = (d < (int)nbins) ? segc[d] : 0u;
        const int nz = __syncthreads_count(c != 0u);
        const unsigned long long *ao = w.andor[L] + (size_t)s * 4;
        const Canon diff{ao[0] ^ ao[2], ao[1] ^ ao[3]};
        if (!fused_here) st_hist += seg.len;

        if (w.desc[L][s] == 0u) {
            // already in order (section "Optimize the Algorithm": a sorted
            // sub-array needs no partitioning): in A it is done; in B a stable
            // partition of sorted keys is the identity, so the scatter copies
            // it to A and no child goes on
            uint32_t total;
            const uint32_t excl = block_excl_scan(c, s_tmp, &total);
            if (parity == 1u) {
                if (c != 0u) w.bases[L][(size_t)s * R + d] = seg.begin + excl;
                st_moved += seg.len;
            } else if (d == 0) {
                w.list[L][s].info = seg.info | (SEG_SKIP << 16);
            }
            st_sorted += seg.len;
            block_append<R>(w, L ^ 1, -1, 0u, 0u, 0u, 0u, s_tmp, s_base);
            continue;
        }

        if (nz == 1) {
            // pass-through: every key has the same digit here
            const int nb = first_set_from(diff, bitpos, NB);
            int cat = -1;
            if (nb >= NB) {
                // all keys equal: done; if they sit in B the scatter copies them to A
                if (parity == 1u) {
                    if (c != 0u) w.bases[L][(size_t)s * R + d] = seg.begin;
                    st_moved += seg.len;
                } else if (d == 0) {
                    w.list[L][s].info = seg.info | (SEG_SKIP << 16);
                }
            } else {
                if (d == 0) {
                    w.list[L][s].info = seg.info | (SEG_SKIP << 16);
                    cat = NCLASS;
                }
            }
            block_append<R>(w, L ^ 1, cat, seg.begin, seg.len, nb < NB ? (uint32_t)nb : 0u, parity, s_tmp,
                            s_base);
            continue;
        }

        uint32_t total;
        const uint32_t excl = block_excl_scan(c, s_tmp, &total);
        if (w.inplace) {
            const bool small = c >= 2u && c <= SMALL_MAX;
            uint32_t sk, sc;
            (void)block_excl_scan(small ? c : 0u, s_tmp, &sk);
            (void)block_excl_scan(small ? 1u : 0u, s_tmp, &sc);
            st_small_keys += sk;
            st_small_segs += sc;
        }
        int cat = -1;
        uint32_t cb = 0;
        bool done = false;
        const uint32_t child_parity = w.inplace ? 0u : parity ^ 1u;
        if (c != 0u) {
            cb = (uint32_t)first_set_from(diff, bitpos + wbits, NB);
            done = (c == 1u) || (cb >= (uint32_t)NB);
            w.bases[L][(size_t)s * R + d] = seg.begin + excl;
            if (!done) cat = (c <= w.finish_max) ? fin_class(w, c) : NCLASS;
            // in place, small children are ranked straight from this table
            if (w.inplace && cat == CAT_SMALL) cat = -1;
        }
        st_moved += seg.len;
        if (parity == 0u && !w.inplace) {
            // finished children land in B: one copy-back range per run of
            // adjacent finished children (empty digits do not break a run)
            s_state[d] = (c == 0u) ? 0u : (done ? 1u : 2u);
            __syncthreads();
            bool head = false;
            uint32_t run = 0;
            if (d < R && s_state[d] == 1u) {
                int e = d - 1;
                while (e >= 0 && s_state[e] == 0u) --e;
                head = (e < 0) || (s_state[e] == 2u);
                if (head) {
                    for (int f = d; f < R && s_state[f] != 2u; ++f) run += segc[f];
                }
            }
            uint32_t nh;
            const uint32_t hi = block_excl_scan(head ? 1u : 0u, s_tmp, &nh);
            if (d == 0 && nh) s_base[NCLASS + 2] = atomicAdd(&ctl->cpy_ctr, nh);
            __syncthreads();
            if (head) {
                const uint32_t slot = s_base[NCLASS + 2] + hi;
                if (slot < w.max_cpy)
                    w.cpy[slot] = CopyEntry{seg.begin + excl, run};
                else
                    atomicOr(&ctl->overflow, 1u);
            }
        }
        uint32_t slot = ~0u;
        block_append<R>(w, L ^ 1, cat, seg.begin + excl, c, cb, child_parity, s_tmp, s_base, &slot);
        if (pass == 0 && w.pair_rows != 0u && nslots == 1u && !w.inplace) {
            // the next pass takes its digit counts from pass 0's pair counts
            // if they hold (no bin overflowed, every child's next digit
            // starts right after this one) and one whole child per scatter
            // block balances the work: as many children as blocks at most,
            // the largest within 1/8 of an even share of the tiles
            const uint32_t nt = (cat == NCLASS) ? (c + w.tile_keys - 1) / w.tile_keys : 0u;
            uint32_t tt, nn;
            (void)block_excl_scan(nt, s_tmp, &tt);
            (void)block_excl_scan(cat == NCLASS ? 1u : 0u, s_tmp, &nn);
            if (d == 0) s_max = 0u;
            __syncthreads();
            if (nt) atomicMax(&s_max, nt);
            __syncthreads();
            const uint32_t even = (tt + w.chunk_grid - 1) / w.chunk_grid;
            const bool fuse = nn != 0u && nn <= w.chunk_grid && s_max <= even + even / 8u &&
                              first_set_from(diff, bitpos + wbits, NB) == (int)bitpos + wbits &&
                              ctl->fuse_bad == 0u;
            if (fuse) {
                if (d == 0) ctl->fused_pass = (uint32_t)pass + 1u;
                if (slot != ~0u) {
                    // the child's digit here tags it (its counts are row d of
                    // the pair sums); sortedness unknown; the constant bits of
                    // the parent are constant in the child
                    w.list[L ^ 1][slot].info |= (uint32_t)d << 24;
                    w.desc[L ^ 1][slot] = 1u;
                    unsigned long long *cao = w.andor[L ^ 1] + (size_t)slot * 4;
                    for (int q = 0; q < 4; ++q) cao[q] = ao[q];
                }
            }
        }
    }
    if (d == 0) {
        if (st_hist) atomicAdd(&ctl->hist_keys[ps], st_hist);
        if (st_moved) atomicAdd(&ctl->moved[ps], st_moved);
        if (st_sorted) atomicAdd(&ctl->sorted_keys, st_sorted);
        if (st_small_segs) {
            atomicAdd(&ctl->small_keys, st_small_keys);
            atomicAdd(&ctl->small_segs, st_small_segs);
        }
    }
}

// -------------------------------------------------------------- k_copyback
// Copy the finished ranges that the passes left in B to A.
template <int KB, bool PAY>
__global__ __launch_bounds__(THREADS) void k_copyback(Work w) {
    using KT = KeyT<KB>;
    Ctl *ctl = w.ctl;
    if (ctl->error | ctl->overflow) return;
    const uint32_t n = min(ctl->cpy_ctr, w.max_cpy);
    unsigned long long st_keys = 0ull;
    for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
        const CopyEntry e = w.cpy[i];
        if ((size_t)e.begin + e.len > w.n_total) {
            if (threadIdx.x == 0) atomicOr(&ctl->error, ERR_INTERNAL);
            continue;
        }
        st_keys += e.len;
        for (uint32_t k = threadIdx.x; k < e.len; k += THREADS) {
            const size_t g = (size_t)e.begin + k;
            KT::store(w.keys[0], g, KT::load(w.keys[1], g));
            if (PAY) w.pay[0][g] = w.pay[1][g];
        }
    }
    if (threadIdx.x == 0 && st_keys) atomicAdd(&ctl->cpy_keys, st_keys);
}

// ---------------------------------------------------------------- k_scatter
// One tile = BT * ITEMS keys of one segment.  Wave q owns keys
// [q * ITEMS * 64, (q + 1) * ITEMS * 64) of the tile, 64 consecutive keys per
// step, so the (wave, step, lane) order is the input order and a stable rank
// is: keys of the digit in earlier waves + the rank inside the wave.
//
// Bucket offsets of a tile (gw[d].x = global index of staged position 0
// of digit d):
//   LOOKBACK = false: the block owns the same chunk of tiles as in k_hist and
//     walks it in order, starting each piece from bases + piece prefix and
//     advancing by each tile's counts;
//   LOOKBACK = true: tiles are taken in ticket order and each looks back over
//     the earlier tiles of its segment (decoupled look-back).
// Chunked scatter writes whole aligned bursts of BURST_BYTES of keys: the
// part of each digit's run that does not yet fill a burst is carried in LDS
// to the block's next tile (a partial burst costs the memory a
// read-modify-write).  Only the first and last burst of a digit's run in a
// piece can be partial.
constexpr int BURST_BYTES = 64;

template <int KB, int K, int BT, int ITEMS, bool PAY, bool LOOKBACK>
struct ScatterLds {
    using V = typename KeyT<KB>::V;
    static constexpr int R = 1 << K;
    static constexpr int TILE = BT * ITEMS;
    static constexpr int NW = BT / WAVE;
    static constexpr int P = 1;                      // lane-mask tables per wave
    static constexpr int CB = BURST_BYTES / KB;      // keys per burst
    static constexpr int CR = LOOKBACK ? 1 : R;      // digits that carry
    V keys[TILE];
    uint32_t pay[PAY ? TILE : 1];
    alignas(8) uint32_t tbl[NW][2 * R];  // lane masks of the wave ranking
    uint32_t wh[NW][R];             // per-wave digit counts -> staged offset of (wave, digit)
    // per digit d: .x = global index of staged position 0, .y = staged keys
    // below this global index are written now (chunked scatter only): one
    // 8-byte read gives the write-out both
    uint2 gw[R];
    uint32_t run[R];                // chunked offsets: next global index of digit d in this piece
    uint32_t cc[CR];                // carried keys of digit d (global [run - cc, run))
    uint32_t ccw[CR];               // carried keys written this tile, from global index clo
    uint32_t clo[CR];
    V ckeys[CR][CB];
    uint32_t cpay[PAY ? CR : 1][CB];
    uint32_t tmp[NW];
    uint32_t tile, slot;
};

// Keys (and payloads) of tile t of `seg` into registers, wave-striped, as
// stored (the sorting view is taken when the tile is processed, so that the
// loads of a prefetched tile stay in flight).
template <int KB, int BT, int ITEMS, bool PAY>
__device__ __forceinline__ void load_tile(const Work &w, const SegEntry &seg, uint32_t t,
                                          typename KeyT<KB>::V (&key)[ITEMS], uint32_t (&pay)[ITEMS]) {
    using KT = KeyT<KB>;
    constexpr uint32_t TILE = BT * ITEMS;
    const uint32_t parity = (seg.info >> 8) & 1u;
    const uint32_t off = (t - seg.tile_start) * TILE;
    const uint32_t tlen = min(TILE, seg.len - off);
    const size_t gbase = (size_t)seg.begin + off;
    // tile base pointers are uniform: loads use a scalar base + lane offset
    const char *tsrc = static_cast<const char *>(w.keys[parity]) + gbase * KB;
    const uint32_t *tpsrc = PAY ? w.pay[parity] + gbase : nullptr;
    const uint32_t ebase = (uint32_t)(threadIdx.x / WAVE) * ITEMS * WAVE + (uint32_t)lane_id();
    if (tlen == TILE) {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            key[j] = KT::load(tsrc, ebase + j * WAVE);
            if (PAY) pay[j] = tpsrc[ebase + j * WAVE];
        }
    } else {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t e = ebase + j * WAVE;
            key[j] = (e < tlen) ? KT::load(tsrc, e) : KT::zero();
            if (PAY) pay[j] = (e < tlen) ? tpsrc[e] : 0u;
        }
    }
}

// Rank, offsets, stage and write one tile whose keys are in registers.
template <int KB, int K, int BT, int ITEMS, bool PAY, bool LOOKBACK, bool FULL>
__device__ __forceinline__ void scatter_tile(const Work &w, int L, ScatterLds<KB, K, BT, ITEMS, PAY, LOOKBACK> &S,
                                             const SegEntry &seg, uint32_t t, uint32_t slot,
                                             typename KeyT<KB>::V (&key)[ITEMS], const uint32_t (&pay)[ITEMS],
                                             int &peel_misses) {
    using KT = KeyT<KB>;
    using V = typename KT::V;
    constexpr int R = 1 << K;
    constexpr int TILE = BT * ITEMS;
    constexpr int NW = BT / WAVE;
    Ctl *ctl = w.ctl;
    const int wv = threadIdx.x / WAVE, lane = lane_id();
    const uint32_t bitpos = seg.info & 0xFFu, parity = (seg.info >> 8) & 1u;
    const int wbits = min(K, (int)w.nbits - (int)bitpos);
    const uint32_t lt = t - seg.tile_start;
    const uint32_t off = lt * (uint32_t)TILE;
    const uint32_t tlen = FULL ? (uint32_t)TILE : min((uint32_t)TILE, seg.len - off);
    void *dst = w.keys[parity ^ 1u];
    uint32_t *pdst = w.pay[parity ^ 1u];

    uint32_t dg[ITEMS];
    uint32_t rnk[ITEMS];
    const uint32_t ebase = (uint32_t)wv * ITEMS * WAVE + (uint32_t)lane;
    // the tile's keys, loaded as stored, into the sorting view (in place)
    if (w.kind) {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) key[j] = KT::enc(key[j], w.kind);
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) dg[j] = KT::digit(key[j], bitpos, wbits);
    wave_rank<R, RANK_GROUP, ITEMS, FULL, true>(dg, ebase, tlen, &S.tbl[wv][0], &S.wh[wv][0], rnk, &peel_misses);
    __syncthreads();
    // per digit: staged offset of each wave's keys, tile count, global offset
    uint32_t tcnt = 0;
    if (threadIdx.x < R) {
#pragma unroll
        for (int q = 0; q < NW; ++q) tcnt += S.wh[q][threadIdx.x];
    }
    uint32_t tot;
    const uint32_t dstart = block_excl_scan<BT>(tcnt, S.tmp, &tot);  // every thread: it holds barriers
    if (threadIdx.x < R) {
        uint32_t acc = dstart;
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            const uint32_t x = S.wh[q][threadIdx.x];
            S.wh[q][threadIdx.x] = acc;
            acc += x;
        }
        if (LOOKBACK) {
            uint32_t *st = w.status + (size_t)t * R + threadIdx.x;
            uint32_t excl = 0;
            if (lt == 0) {
                st_agent(st, ST_INC | tcnt);
            } else {
                st_agent(st, ST_AGG | tcnt);
                uint32_t tt = t - 1;
                uint32_t spins = 0;
                for (;;) {
                    uint32_t v;
                    while (((v = ld_agent(w.status + (size_t)tt * R + threadIdx.x)) & ST_FLAGS) == 0u &&
                           spins < SPIN_LIMIT) {
                        __builtin_amdgcn_s_sleep(1);
                        ++spins;
                    }
                    if (spins >= SPIN_LIMIT || tt == seg.tile_start) {
                        if (!(v & ST_INC)) atomicOr(&ctl->error, ERR_INTERNAL);
                        excl += v & ST_VAL;
                        break;
                    }
                    excl += v & ST_VAL;
                    if (v & ST_INC) break;
                    --tt;
                }
                st_agent(st, ST_INC | (excl + tcnt));
            }
            if (tcnt) S.gw[threadIdx.x].x = w.bases[L][(size_t)slot * R + threadIdx.x] + excl - dstart;
        } else {
            // the run of digit d so far: carried [gpos - cc, gpos) + this tile's
            // [gpos, gpos + tcnt); write everything below the last burst
            // boundary, carry the rest
            constexpr uint32_t CB = ScatterLds<KB, K, BT, ITEMS, PAY, LOOKBACK>::CB;
            const uint32_t gpos = S.run[threadIdx.x];
            const uint32_t cc = S.cc[threadIdx.x];
            const uint32_t lo = gpos - cc, hi = gpos + tcnt;
            const uint32_t cut = hi & ~(CB - 1u);
            const uint32_t wlim = cut > lo ? cut : lo;
            S.gw[threadIdx.x] = make_uint2(gpos - dstart, wlim);
            S.ccw[threadIdx.x] = cut > lo ? cc : 0u;
            S.clo[threadIdx.x] = lo;
            S.cc[threadIdx.x] = hi - wlim;
            S.run[threadIdx.x] = hi;
        }
    }
    __syncthreads();
    // stage in digit order; the wave ranking left its counters at zero
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const uint32_t e = ebase + j * WAVE;
        if (FULL || e < tlen) {
            const uint32_t pos = S.wh[wv][dg[j]] + rnk[j];
            S.keys[pos] = key[j];
            if (PAY) S.pay[pos] = pay[j];
        }
    }
    if (!LOOKBACK) {
        // carried keys whose burst this tile completes
        constexpr int CB = ScatterLds<KB, K, BT, ITEMS, PAY, LOOKBACK>::CB;
        for (int i = threadIdx.x; i < R * CB; i += BT) {
            const int d = i / CB, k = i % CB;
            if ((uint32_t)k < S.ccw[d]) {
                const uint32_t g = S.clo[d] + k;
                if (g < w.n_total) {
                    KT::store(dst, g, raw_key<KB>(S.ckeys[d][k], w.kind));
                    if (PAY) pdst[g] = S.cpay[d][k];
                } else {
                    atomicOr(&ctl->error, ERR_INTERNAL);
                }
            }
        }
    }
    __syncthreads();
    // coalesced write: consecutive staged keys of one digit go to consecutive
    // global positions; each wave clears its own counters for the next tile
    for (int i = lane; i < R; i += WAVE) S.wh[wv][i] = 0u;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const uint32_t p = j * BT + threadIdx.x;
        if (FULL || p < tlen) {
            const V k = S.keys[p];
            const uint32_t d = KT::digit(k, bitpos, wbits);
            const uint2 gw = S.gw[d];
            const uint32_t g = gw.x + p;
            if (!LOOKBACK && g >= gw.y) {
                // does not fill a burst yet: carry it to the next tile
                S.ckeys[d][g - gw.y] = k;
                if (PAY) S.cpay[d][g - gw.y] = S.pay[p];
            } else if (g < w.n_total) {
                // whole bursts from this tile: streaming stores (the partial
                // bursts completed from the carry above stay ordinary, so the
                // cache merges their two halves)
                KT::store_nt(dst, g, raw_key<KB>(k, w.kind));
                if (PAY) __builtin_nontemporal_store(S.pay[p], pdst + g);
            } else {
                atomicOr(&ctl->error, ERR_INTERNAL);
            }
        }
    }
    __syncthreads();
}

// End of a piece in the chunked scatter: write the carried keys of every
// digit (the partial last burst of each run).
template <int KB, int K, int BT, int ITEMS, bool PAY>
__device__ __forceinline__ void flush_carry(const Work &w, ScatterLds<KB, K, BT, ITEMS, PAY, false> &S,
                                            uint32_t parity) {
    using KT = KeyT<KB>;
    constexpr int R = 1 << K;
    constexpr int CB = ScatterLds<KB, K, BT, ITEMS, PAY, false>::CB;
    void *dst = w.keys[parity ^ 1u];
    uint32_t *pdst = w.pay[parity ^ 1u];
    for (int i = threadIdx.x; i < R * CB; i += BT) {
        const int d = i / CB, k = i % CB;
        if ((uint32_t)k < S.cc[d]) {
            const uint32_t g = S.run[d] - S.cc[d] + k;
            if (g < w.n_total) {
                KT::store(dst, g, raw_key<KB>(S.ckeys[d][k], w.kind));
                if (PAY) pdst[g] = S.cpay[d][k];
            } else {
                atomicOr(&w.ctl->error, ERR_INTERNAL);
            }
        }
    }
    __syncthreads();
}

// A pass whose digit counts came with pass 0's (ctl->fused_pass) has no
// piece counts: block b takes the whole segment in slot b of the list (the
// plan chose this only for at most as many, evenly sized, segments as
// blocks), starting at the segment's bucket bases.
template <int KB, int K, int BT, int ITEMS, bool PAY, bool LOOKBACK>
__global__ __launch_bounds__(BT) void k_scatter(Work w, int L, int pass) {
    using V = typename KeyT<KB>::V;
    constexpr int R = 1 << K;
    constexpr uint32_t TILE = BT * ITEMS;
    constexpr int NW = BT / WAVE;
    __shared__ ScatterLds<KB, K, BT, ITEMS, PAY, LOOKBACK> S;

    Ctl *ctl = w.ctl;
    if (ctl->error | ctl->overflow) return;
    const unsigned long long lc = ctl->list_ctr[L];
    const uint32_t nslots = (uint32_t)(lc >> 32), ntiles = (uint32_t)lc;
    if (ntiles == 0) return;
    const bool whole = !LOOKBACK && pass != 0 && (uint32_t)pass == ctl->fused_pass;
    uint32_t t0 = 0, t1 = 0;
    if (!LOOKBACK) {
        if (whole) {
            if (blockIdx.x >= nslots) return;
            t0 = w.list[L][blockIdx.x].tile_start;
            t1 = seg_tile_end(w.list[L], blockIdx.x, nslots, ntiles);
        } else {
            const uint32_t per = (ntiles + gridDim.x - 1) / gridDim.x;
            t0 = blockIdx.x * per;
            t1 = min(ntiles, t0 + per);
        }
        if (t0 >= t1) return;
    }
    for (int i = threadIdx.x; i < NW * R; i += BT) (&S.wh[0][0])[i] = 0u;
    for (int i = threadIdx.x; i < NW * 2 * R; i += BT) (&S.tbl[0][0])[i] = 0u;
    __syncthreads();

    V key[ITEMS];
    uint32_t pay[ITEMS];
    int peel_misses = 0;  // the ranking's digit peeling (see wave_rank)
    if constexpr (LOOKBACK) {
        // tiles in ticket order; each looks back over its segment's earlier tiles
        for (;;) {
            if (threadIdx.x == 0) {
                const uint32_t tk = atomicAdd(&ctl->ticket, 1u);
                S.tile = tk;
                S.slot = (tk < ntiles) ? find_slot(w.list[L], nslots, tk) : 0u;
            }
            __syncthreads();
            const uint32_t t = uni(S.tile);
            if (t >= ntiles) break;
            const uint32_t slot = uni(S.slot);
            const SegEntry seg = uni(w.list[L][slot]);
            __syncthreads();
            if ((seg.info >> 16) & SEG_SKIP) continue;
            load_tile<KB, BT, ITEMS, PAY>(w, seg, t, key, pay);
            if (seg.len - (t - seg.tile_start) * TILE >= TILE)
                scatter_tile<KB, K, BT, ITEMS, PAY, true, true>(w, L, S, seg, t, slot, key, pay, peel_misses);
            else
                scatter_tile<KB, K, BT, ITEMS, PAY, true, false>(w, L, S, seg, t, slot, key, pay, peel_misses);
        }
    } else {
    // chunked: walk tiles t0 .. t1 in order; the next tile of the same segment
    // is loaded into a second register set while the current one is processed
    V keyn[ITEMS];
    uint32_t payn[ITEMS];
    uint32_t t = t0;
    uint32_t slot = whole ? blockIdx.x : uni(find_slot(w.list[L], nslots, t));
    SegEntry seg = uni(w.list[L][slot]);
    uint32_t seg_end = uni(seg_tile_end(w.list[L], slot, nslots, ntiles));
    bool loaded = false;
    while (t < t1) {
        if (!loaded) {
            // entering a segment: skip it if it does not move, else start its piece
            if ((seg.info >> 16) & SEG_SKIP) {
                t = seg_end;
                if (t >= t1) break;
                ++slot;
                seg = uni(w.list[L][slot]);
                seg_end = uni(seg_tile_end(w.list[L], slot, nslots, ntiles));
                continue;
            }
            if (threadIdx.x < R) {
                S.run[threadIdx.x] =
                    w.bases[L][(size_t)slot * R + threadIdx.x] + (whole ? 0u : w.pcnt[(size_t)t * R + threadIdx.x]);
                S.cc[threadIdx.x] = 0u;
            }
            load_tile<KB, BT, ITEMS, PAY>(w, seg, t, key, pay);
            loaded = true;
        }
        const uint32_t tn = t + 1;
        const bool pref = tn < t1 && tn < seg_end;
        if (pref) load_tile<KB, BT, ITEMS, PAY>(w, seg, tn, keyn, payn);
        if (seg.len - (t - seg.tile_start) * TILE >= TILE)
            scatter_tile<KB, K, BT, ITEMS, PAY, false, true>(w, L, S, seg, t, slot, key, pay, peel_misses);
        else
            scatter_tile<KB, K, BT, ITEMS, PAY, false, false>(w, L, S, seg, t, slot, key, pay, peel_misses);
        t = tn;
        if (pref) {
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                key[j] = keyn[j];
                if (PAY) pay[j] = payn[j];
            }
        } else {
            // the piece ends here
            flush_carry<KB, K, BT, ITEMS, PAY>(w, S, (seg.info >> 8) & 1u);
        }
        if (!pref && t < t1) {
            ++slot;
            seg = uni(w.list[L][slot]);
            seg_end = uni(seg_tile_end(w.list[L], slot, nslots, ntiles));
            loaded = false;
        }
    }
    }
}

// ----------------------------------------------------------------- k_finish
// One workgroup per small segment (at most BT * ITEMS keys): find the bits
// that vary inside it (AND/OR), sort stably by them with
// least-significant-first LDS passes of up to 8 bits, write to A.
// Copies between a segment's range [g0, g1) of a global buffer and LDS
// (element g of the range at lds[g - g0]): the 16-byte aligned body as whole
// vectors, the unaligned head and tail one element at a time.  Loads issue
// every vector of the thread before the first LDS write, so the whole range
// is in flight at once; NV bounds the vectors per thread.
template <int VN, int ES>
__device__ __forceinline__ void aligned_body(const void *base, size_t g0, size_t g1, size_t &b0, size_t &b1) {
    const size_t mis = ((16u - (reinterpret_cast<uintptr_t>(base) & 15u)) & 15u) / ES;
    b0 = min(g1, g0 + ((mis + VN - (g0 % VN)) % VN));
    b1 = b0 + (g1 - b0) / VN * VN;
}

// Loading a sub-array into LDS in two halves, so that a block can issue the
// next sub-array's loads before it sorts the current one: issue = the 16-byte
// vector loads of the aligned body into registers; commit = the few keys
// before and after the body, and everything into LDS (AND/OR on the way).
template <int KB, int NV, int BT>
__device__ __forceinline__ void fin_issue_keys(const void *src, size_t g0, size_t g1,
                                               typename KeyT<KB>::V (&v)[NV][Vec<KB>::N]) {
    constexpr int VN = Vec<KB>::N;
    size_t b0, b1;
    aligned_body<VN, KB>(src, g0, g1, b0, b1);
#pragma unroll
    for (int u = 0; u < NV; ++u) {
        const size_t x = b0 + ((size_t)u * BT + threadIdx.x) * VN;
        if (x < b1) load_vec<KB>(src, x, v[u]);
    }
}

template <int KB, int NV, int BT>
__device__ __forceinline__ void fin_commit_keys(const void *src, size_t g0, size_t g1,
                                                typename KeyT<KB>::V (&v)[NV][Vec<KB>::N],
                                                typename KeyT<KB>::V *lds, typename KeyT<KB>::V &a,
                                                typename KeyT<KB>::V &o, uint32_t kind) {
    using KT = KeyT<KB>;
    using V = typename KT::V;
    constexpr int VN = Vec<KB>::N;
    size_t b0, b1;
    aligned_body<VN, KB>(src, g0, g1, b0, b1);
    for (size_t i = g0 + threadIdx.x; i < b0; i += BT) {
        const V k = ld_key<KB>(src, i, kind);
        lds[i - g0] = k;
        a = KT::vand(a, k);
        o = KT::vor(o, k);
    }
    for (size_t i = b1 + threadIdx.x; i < g1; i += BT) {
        const V k = ld_key<KB>(src, i, kind);
        lds[i - g0] = k;
        a = KT::vand(a, k);
        o = KT::vor(o, k);
    }
#pragma unroll
    for (int u = 0; u < NV; ++u) {
        const size_t x = b0 + ((size_t)u * BT + threadIdx.x) * VN;
        if (x < b1) {
#pragma unroll
            for (int q = 0; q < VN; ++q) {
                if (kind) v[u][q] = KT::enc(v[u][q], kind);
                lds[x - g0 + q] = v[u][q];
                a = KT::vand(a, v[u][q]);
                o = KT::vor(o, v[u][q]);
            }
        }
    }
}

template <int KB, int NV, int BT>
__device__ __forceinline__ void fin_load_keys(const void *src, size_t g0, size_t g1, typename KeyT<KB>::V *lds,
                                              typename KeyT<KB>::V &a, typename KeyT<KB>::V &o, uint32_t kind) {
    typename KeyT<KB>::V v[NV][Vec<KB>::N];
    fin_issue_keys<KB, NV, BT>(src, g0, g1, v);
    fin_commit_keys<KB, NV, BT>(src, g0, g1, v, lds, a, o, kind);
}

template <int NV, int BT>
__device__ __forceinline__ void fin_issue_pay(const uint32_t *src, size_t g0, size_t g1, uint4 (&v)[NV]) {
    size_t b0, b1;
    aligned_body<4, 4>(src, g0, g1, b0, b1);
#pragma unroll
    for (int u = 0; u < NV; ++u) {
        const size_t x = b0 + ((size_t)u * BT + threadIdx.x) * 4;
        if (x < b1) v[u] = *reinterpret_cast<const uint4 *>(src + x);
    }
}

template <int NV, int BT>
__device__ __forceinline__ void fin_commit_pay(const uint32_t *src, size_t g0, size_t g1, uint4 (&v)[NV],
                                               uint32_t *lds) {
    size_t b0, b1;
    aligned_body<4, 4>(src, g0, g1, b0, b1);
    for (size_t i = g0 + threadIdx.x; i < b0; i += BT) lds[i - g0] = src[i];
    for (size_t i = b1 + threadIdx.x; i < g1; i += BT) lds[i - g0] = src[i];
#pragma unroll
    for (int u = 0; u < NV; ++u) {
        const size_t x = b0 + ((size_t)u * BT + threadIdx.x) * 4;
        if (x < b1) {
            uint32_t *d = lds + (x - g0);
            d[0] = v[u].x;
            d[1] = v[u].y;
            d[2] = v[u].z;
            d[3] = v[u].w;
        }
    }
}

template <int NV, int BT>
__device__ __forceinline__ void fin_load_pay(const uint32_t *src, size_t g0, size_t g1, uint32_t *lds) {
    uint4 v[NV];
    fin_issue_pay<NV, BT>(src, g0, g1, v);
    fin_commit_pay<NV, BT>(src, g0, g1, v, lds);
}

template <int KB, int BT>
__device__ __forceinline__ void fin_store_keys(void *dst, size_t g0, size_t g1, const typename KeyT<KB>::V *lds,
                                               uint32_t kind) {
    using KT = KeyT<KB>;
    constexpr int VN = Vec<KB>::N;
    size_t b0, b1;
    aligned_body<VN, KB>(dst, g0, g1, b0, b1);
    for (size_t i = g0 + threadIdx.x; i < b0; i += BT) KT::store(dst, i, raw_key<KB>(lds[i - g0], kind));
    for (size_t i = b1 + threadIdx.x; i < g1; i += BT) KT::store(dst, i, raw_key<KB>(lds[i - g0], kind));
    for (size_t x = b0 + (size_t)threadIdx.x * VN; x < b1; x += (size_t)BT * VN) {
        const typename KT::V *s = lds + (x - g0);
        if constexpr (KB == 4) {
            *reinterpret_cast<uint4 *>(reinterpret_cast<uint32_t *>(dst) + x) =
                make_uint4(raw_key<KB>(s[0], kind), raw_key<KB>(s[1], kind), raw_key<KB>(s[2], kind),
                           raw_key<KB>(s[3], kind));
        } else if constexpr (KB == 8) {
            ulonglong2 r;
            r.x = raw_key<KB>(s[0], kind);
            r.y = raw_key<KB>(s[1], kind);
            *reinterpret_cast<ulonglong2 *>(reinterpret_cast<uint64_t *>(dst) + x) = r;
        } else {
            KT::store(dst, x, raw_key<KB>(s[0], kind));
        }
    }
}

template <int BT>
__device__ __forceinline__ void fin_store_pay(uint32_t *dst, size_t g0, size_t g1, const uint32_t *lds) {
    size_t b0, b1;
    aligned_body<4, 4>(dst, g0, g1, b0, b1);
    for (size_t i = g0 + threadIdx.x; i < b0; i += BT) dst[i] = lds[i - g0];
    for (size_t i = b1 + threadIdx.x; i < g1; i += BT) dst[i] = lds[i - g0];
    for (size_t x = b0 + (size_t)threadIdx.x * 4; x < b1; x += (size_t)BT * 4) {
        const uint32_t *s = lds + (x - g0);
        *reinterpret_cast<uint4 *>(dst + x) = make_uint4(s[0], s[1], s[2], s[3]);
    }
}

template <int KB, int BT, int ITEMS, bool PAY>
struct FinishLds {
    using V = typename KeyT<KB>::V;
    static constexpr int R = 256;
    static constexpr int CAP = BT * ITEMS;
    static constexpr int NW = BT / WAVE;
    V keys[CAP];
    uint32_t pay[PAY ? CAP : 1];
    alignas(8) uint32_t tbl[NW][2 * R];  // lane masks; between passes also the list of runs to fix
    uint32_t wh[NW][R];
    uint32_t tmp[NW];
    unsigned long long ao[NW][4];
    uint32_t long_run;
};

// Keys [wb, we) of a sub-array of len keys held by wave wv of a BT-thread
// block: the keys are spread evenly over the waves (it = ceil(len / (waves
// * 64)) steps of 64 consecutive keys each, at most ITEMS), so (wave, step,
// lane) order is the input order.  Lanes past we hold nothing in any step.
template <int BT, int ITEMS>
__device__ __forceinline__ void wave_share(uint32_t len, int wv, uint32_t &wb, uint32_t &we) {
    constexpr uint32_t NW = BT / WAVE;
    uint32_t it = (len + NW * WAVE - 1) / (NW * WAVE);
    it = it < (uint32_t)ITEMS ? it : (uint32_t)ITEMS;
    wb = uni((uint32_t)wv * it * WAVE);
    we = uni(min(len, wb + it * WAVE));
}

// Per digit: the staged offset of each wave's keys (exclusive scan over the
// digits of the block's counts, then over the waves), left in S.wh in place
// of the wave counts.  Every thread calls it (it holds barriers).
template <int BT, class L>
__device__ __forceinline__ void fin_offsets(L &S) {
    constexpr int R = 256;
    constexpr int NW = BT / WAVE;
    __syncthreads();
    uint32_t tcnt = 0;
    if (threadIdx.x < R) {
#pragma unroll
        for (int q = 0; q < NW; ++q) tcnt += S.wh[q][threadIdx.x];
    }
    uint32_t tot;
    uint32_t acc = block_excl_scan<BT>(tcnt, S.tmp, &tot);  // every thread: it holds barriers
    if (threadIdx.x < R) {
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            const uint32_t x = S.wh[q][threadIdx.x];
            S.wh[q][threadIdx.x] = acc;
            acc += x;
        }
    }
    __syncthreads();
}

// Stable LDS passes over the varying bits of the segment in S with bit
// index in [bitpos, end] (MSB-first indices), least significant window of up
// to 8 bits first; constant windows are skipped.  The order lives in S
// between passes.  Each wave ranks its share [ebase - lane, we)
// (wave_share).  REGFIRST: the first window takes key e = ebase + 64 j from
// key_at(j) (registers) instead of the keys in LDS in input order.
template <int KB, int BT, int ITEMS, bool PAY, bool REGFIRST, class F>
__device__ __forceinline__ void lds_passes(FinishLds<KB, BT, ITEMS, PAY> &S, Canon diff, int bitpos, int end,
                                           uint32_t ebase, uint32_t we, F &&key_at) {
    using KT = KeyT<KB>;
    using V = typename KT::V;
    constexpr int KL = 8;
    constexpr int R = 1 << KL;
    const int wv = threadIdx.x / WAVE, lane = lane_id();
    // one window [lo, lo + wbits) over keys key_of(j)
    auto window = [&](int lo, int wbits, auto &&key_of) {
        V key[ITEMS];
        uint32_t dg[ITEMS], rnk[ITEMS];
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t e = ebase + j * WAVE;
            key[j] = (e < we) ? key_of(j) : KT::zero();
            dg[j] = KT::digit(key[j], lo, wbits);
        }
        wave_rank<R, RANK_GROUP, ITEMS, false>(dg, ebase, we, &S.tbl[wv][0], &S.wh[wv][0], rnk);
        uint32_t pay[ITEMS];
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t e = ebase + j * WAVE;
            if (PAY) pay[j] = (e < we) ? S.pay[e] : 0u;
        }
        fin_offsets<BT>(S);
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t e = ebase + j * WAVE;
            if (e < we) {
                const uint32_t pos = S.wh[wv][dg[j]] + rnk[j];
                S.keys[pos] = key[j];
                if (PAY) S.pay[pos] = pay[j];
            }
        }
        __syncthreads();
        // each wave clears its own counters: only it touches them before
        // the next barrier
        for (int i = lane; i < R; i += WAVE) S.wh[wv][i] = 0u;
    };
    int hib = last_set_below(diff, bitpos, end + 1);
    if constexpr (REGFIRST) {
        if (hib < bitpos) return;
        const int lo = max(bitpos, hib - KL + 1);
        window(lo, hib - lo + 1, key_at);
        hib = last_set_below(diff, bitpos, lo);
    }
    auto in_lds = [&](int j) -> V { return S.keys[ebase + j * WAVE]; };
    while (hib >= bitpos) {
        const int lo = max(bitpos, hib - KL + 1);
        window(lo, hib - lo + 1, in_lds);
        hib = last_set_below(diff, bitpos, lo);
    }
}

// The 16 bits [s, s + 16) (MSB-first) of a 4- or 8-byte key, and a key
// rebuilt from them over the bits `base` has outside that field.
template <int KB>
__device__ __forceinline__ uint32_t field16(typename KeyT<KB>::V v, int s) {
    return (uint32_t)(v >> (8 * KB - 16 - s)) & 0xFFFFu;
}

template <int KB>
__device__ __forceinline__ typename KeyT<KB>::V unfield16(typename KeyT<KB>::V base, uint32_t f, int s) {
    using V = typename KeyT<KB>::V;
    const int sh = 8 * KB - 16 - s;
    return (base & ~((V)0xFFFFu << sh)) | ((V)f << sh);
}

// The same passes for a sub-array whose varying bits all lie in the 16 bits
// [s, s + 16) (MSB-first): each key travels as one 32-bit word, (those 16
// bits << 16) | its index in the sub-array, so that a pass moves 4 bytes per
// key whatever the key width, and the payload stays where it was loaded.
// Windows of up to 8 bits from lb down to fb.  The caller passes the
// words of its keys (key e of the sub-array at (wave, step, lane) = e); on
// return the words in sorted order are in S.keys, read as 32-bit words
// (word i = the i-th key).
template <int KB, int BT, int ITEMS, bool PAY, class F>
__device__ __forceinline__ void packed_passes(FinishLds<KB, BT, ITEMS, PAY> &S, Canon diff, int fb, int lb, int s,
                                              uint32_t ebase, uint32_t we, F &&key_at) {
    typedef uint32_t __attribute__((may_alias)) word_t;
    word_t *pk = reinterpret_cast<word_t *>(&S.keys[0]);
    constexpr int R = 256;
    const int wv = threadIdx.x / WAVE, lane = lane_id();
    uint32_t pw[ITEMS];
    // the words (key_at(j) = key e = ebase + 64 j, from registers or from the
    // keys in LDS in input order: every read comes before the barriers of
    // the first window, every write after them)
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const uint32_t e = ebase + j * WAVE;
        pw[j] = (e < we) ? (field16<KB>(key_at(j), s) << 16) | e : 0u;
    }
    int hib = lb;
    bool first = true;
    while (hib >= fb) {
        const int lo = max(fb, hib - 7);
        const uint32_t mask = (1u << (hib - lo + 1)) - 1u;
        const int sh = 31 - (hib - s);  // the window's least significant bit in a word
        uint32_t dg[ITEMS], rnk[ITEMS];
        if (!first) {
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                const uint32_t e = ebase + j * WAVE;
                pw[j] = (e < we) ? pk[e] : 0u;
            }
        }
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) dg[j] = (pw[j] >> sh) & mask;
        wave_rank<R, RANK_GROUP, ITEMS, false>(dg, ebase, we, &S.tbl[wv][0], &S.wh[wv][0], rnk);
        fin_offsets<BT>(S);
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t e = ebase + j * WAVE;
            if (e < we) pk[S.wh[wv][dg[j]] + rnk[j]] = pw[j];
        }
        __syncthreads();
        for (int i = lane; i < R; i += WAVE) S.wh[wv][i] = 0u;
        hib = last_set_below(diff, fb, lo);
        first = false;
    }
}

// The packed sort's result from LDS to [g0, g1) of A: word i of pk is the
// i-th key's 16-bit field and its index in the sub-array, whose payload is
// pay[index]; keys are rebuilt over `base` (the bits every key shares).
// Whole 16-byte vectors for the aligned body of each buffer.
template <int KB, int BT, bool PAY>
__device__ __forceinline__ void fin_store_packed(const Work &w, size_t g0, size_t g1, const uint32_t *pk,
                                                 const uint32_t *pay, typename KeyT<KB>::V base, int s) {
    using KT = KeyT<KB>;
    constexpr int VN = Vec<KB>::N;
    void *dst = w.keys[0];
    size_t b0, b1;
    aligned_body<VN, KB>(dst, g0, g1, b0, b1);
    for (size_t i = g0 + threadIdx.x; i < b0; i += BT)
        KT::store(dst, i, raw_key<KB>(unfield16<KB>(base, pk[i - g0] >> 16, s), w.kind));
    for (size_t i = b1 + threadIdx.x; i < g1; i += BT)
        KT::store(dst, i, raw_key<KB>(unfield16<KB>(base, pk[i - g0] >> 16, s), w.kind));
    for (size_t x = b0 + (size_t)threadIdx.x * VN; x < b1; x += (size_t)BT * VN) {
        const uint32_t *q = pk + (x - g0);
        if constexpr (KB == 4) {
            *reinterpret_cast<uint4 *>(reinterpret_cast<uint32_t *>(dst) + x) =
                make_uint4(raw_key<KB>(unfield16<KB>(base, q[0] >> 16, s), w.kind),
                           raw_key<KB>(unfield16<KB>(base, q[1] >> 16, s), w.kind),
                           raw_key<KB>(unfield16<KB>(base, q[2] >> 16, s), w.kind),
                           raw_key<KB>(unfield16<KB>(base, q[3] >> 16, s), w.kind));
        } else {
            ulonglong2 r;
            r.x = raw_key<KB>(unfield16<KB>(base, q[0] >> 16, s), w.kind);
            r.y = raw_key<KB>(unfield16<KB>(base, q[1] >> 16, s), w.kind);
            *reinterpret_cast<ulonglong2 *>(reinterpret_cast<uint64_t *>(dst) + x) = r;
        }
    }
    if constexpr (PAY) {
        uint32_t *pdst = w.pay[0];
        aligned_body<4, 4>(pdst, g0, g1, b0, b1);
        for (size_t i = g0 + threadIdx.x; i < b0; i += BT) pdst[i] = pay[pk[i - g0] & 0xFFFFu];
        for (size_t i = b1 + threadIdx.x; i < g1; i += BT) pdst[i] = pay[pk[i - g0] & 0xFFFFu];
        for (size_t x = b0 + (size_t)threadIdx.x * 4; x < b1; x += (size_t)BT * 4) {
            const uint32_t *q = pk + (x - g0);
            *reinterpret_cast<uint4 *>(pdst + x) = make_uint4(pay[q[0] & 0xFFFFu], pay[q[1] & 0xFFFFu],
                                                              pay[q[2] & 0xFFFFu], pay[q[3] & 0xFFFFu]);
        }
    }
}

// Packs sub-arrays of at most 64 elements into the lanes of one wave.  Lane
// l describes sub-array l by its length len (0: none).  For each group of
// whole sub-arrays that fits into 64 lanes, in order, every lane calls
// fn(l, i, head, act, el, ml): the sub-array l of the element it carries,
// the element's index i there, the lane holding element 0 (head), whether
// it carries an element at all (act), the sub-array's length el and the
// longest length of the group (ml, the same in every lane).
template <class F>
__device__ __forceinline__ void wave_pack(uint32_t len, F &&fn) {
    const int lane = lane_id();
    uint32_t incl = len;  // sub-array l owns elements [incl - len, incl)
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, WAVE);
        if (lane >= o) incl += y;
    }
    const uint32_t total = __builtin_amdgcn_readlane(incl, WAVE - 1);
    for (uint32_t done = 0u; done < total;) {
        // the sub-arrays that end within the next 64 elements (a leading
        // run of lanes, as incl never decreases); the one holding element
        // `done` is always among them, since none exceeds 64 elements
        const uint64_t fits = __ballot(incl <= done + WAVE);
        const int last = 63 - __builtin_clzll(fits);
        const uint32_t end = __builtin_amdgcn_readlane(incl, last);
        const uint32_t q = done + (uint32_t)lane;
        // sub-array of element q: the number of sub-arrays that end at or before q
        int l = 0;
#pragma unroll
        for (int step = WAVE / 2; step > 0; step >>= 1)
            if ((uint32_t)__shfl(incl, l + step - 1, WAVE) <= q) l += step;
        const uint32_t el = __shfl(len, l, WAVE);
        const uint32_t i = q - ((uint32_t)__shfl(incl, l, WAVE) - el);
        const bool act = q < end;
        uint32_t ml = act ? el : 0u;
#pragma unroll
        for (int o = 1; o < WAVE; o <<= 1) ml = max(ml, (uint32_t)__shfl_xor(ml, o, WAVE));
        fn(l, i, (lane - (int)i) & (WAVE - 1), act, el, ml);
        done = end;
    }
}

// Place of element i among the el elements of its sub-array (held by lanes
// head .. head + el - 1, keys ck): the number of elements that come before
// it in the stable order, smaller or equal and earlier.  Every lane of the
// wave takes part (ml: the longest sub-array of the wave's group).
template <int KB>
__device__ __forceinline__ uint32_t pack_rank(Canon ck, uint32_t i, uint32_t el, int head, uint32_t ml) {
    uint32_t r = 0u;
    for (uint32_t j = 0; j < ml; ++j) {
        const int src = (head + (int)j) & (WAVE - 1);
        Canon cj;
        if constexpr (KB == 4) {
            cj.hi = (uint64_t)(uint32_t)__shfl((uint32_t)(ck.hi >> 32), src, WAVE) << 32;
            cj.lo = 0ull;
        } else {
            cj.hi = __shfl(ck.hi, src, WAVE);
            cj.lo = (KB == 16) ? __shfl(ck.lo, src, WAVE) : 0ull;
        }
        const bool before = canon_less(cj, ck) || (cj.hi == ck.hi && cj.lo == ck.lo && j < i);
        if (j < el && before) ++r;
    }
    return r;
}

// The segment in S is sorted stably by its bits [0, pe]: keys equal on them
// form runs, each in input order, still to be ordered by the bits after pe
// (the recursion on sub-arrays, done in LDS).  Runs of up to 64 keys are
// ranked inside one wave, as many packed into its lanes at once as fit: a
// key's new place is the number of run members that are smaller on the
// leading nb bits, or equal there and earlier.  Returns true, with nothing
// of a longer run moved, if some run is longer than 64 keys.
template <int KB, int BT, int ITEMS, bool PAY>
__device__ bool fix_runs(FinishLds<KB, BT, ITEMS, PAY> &S, int pe, uint32_t len, int nb) {
    using KT = KeyT<KB>;
    using V = typename KT::V;
    constexpr int NW = BT / WAVE;
    constexpr int CAP = BT * ITEMS;
    // run starts as 16-bit positions in the (zero) lane-mask table
    typedef uint16_t __attribute__((may_alias)) pos16_t;
    constexpr uint32_t LIST = NW * 2 * (1u << 8) * 2;
    static_assert(LIST >= CAP / 2 && CAP <= 65536, "run list must hold every possible run start");
    pos16_t *list = reinterpret_cast<pos16_t *>(&S.tbl[0][0]);
    const int wv = threadIdx.x / WAVE, lane = lane_id();
    Canon pm;
    pm.hi = pe >= 63 ? ~0ull : ~(~0ull >> (pe + 1));
    pm.lo = pe >= 127 ? ~0ull : (pe < 64 ? 0ull : ~(~0ull >> (pe - 63)));
    if (threadIdx.x == 0) S.long_run = 0u;
    // run starts: first key of a run of two or more
    auto is_start = [&](uint32_t p) -> bool {
        if (p + 1 >= len) return false;
        const Canon k = KT::canon(S.keys[p]);
        if (!canon_eq_under(KT::canon(S.keys[p + 1]), k, pm)) return false;
        return p == 0 || !canon_eq_under(KT::canon(S.keys[p - 1]), k, pm);
    };
    // each thread tests its keys once and keeps the answers as bits (at most
    // ITEMS keys a thread)
    static_assert(ITEMS <= 32, "run-start bits must fit one word");
    uint32_t cnt = 0, starts = 0;
    for (uint32_t p = threadIdx.x, i = 0; p < len; p += BT, ++i)
        if (is_start(p)) {
            ++cnt;
            starts |= 1u << i;
        }
    uint32_t nruns;
    uint32_t at = block_excl_scan<BT>(cnt, S.tmp, &nruns);  // every thread: it holds barriers
    if (nruns == 0u) return false;                         // no tied run: nothing to order
    for (uint32_t p = threadIdx.x, i = 0; p < len; p += BT, ++i)
        if ((starts >> i) & 1u) list[at++] = (uint16_t)p;
    __syncthreads();
    const Canon km = canon_lead_mask(nb);
    for (uint32_t r0 = (uint32_t)wv * WAVE; r0 < nruns; r0 += NW * WAVE) {
        // lane l: run r0 + l, its start and its length (a walk over the keys
        // equal to the first; a key past the run differs from it however
        // another wave may be permuting that key's own run)
        uint32_t s0 = 0u, L = 0u;
        if (r0 + (uint32_t)lane < nruns) {
            s0 = list[r0 + lane];
            const Canon ks = KT::canon(S.keys[s0]);
            L = 2u;  // a run start has an equal successor
            while (L <= (uint32_t)WAVE && s0 + L < len && canon_eq_under(KT::canon(S.keys[s0 + L]), ks, pm)) ++L;
            if (L > (uint32_t)WAVE) {
                S.long_run = 1u;  // left in place for the passes over every varying bit
                L = 0u;
            }
        }
        wave_pack(L, [&](int l, uint32_t i, int head, bool act, uint32_t el, uint32_t ml) {
            const uint32_t s = __shfl(s0, l, WAVE);
            V k = KT::zero();
            uint32_t pv = 0u;
            if (act) {
                k = S.keys[s + i];
                if (PAY) pv = S.pay[s + i];
            }
            Canon ck = KT::canon(k);
            ck.hi &= km.hi;
            ck.lo &= km.lo;
            const uint32_t r = pack_rank<KB>(ck, i, el, head, ml);
            if (act) {
                S.keys[s + r] = k;
                if (PAY) S.pay[s + r] = pv;
            }
        });
    }
    __syncthreads();
    const bool lng = S.long_run != 0u;
    // the ranking tables start at zero
    for (uint32_t i = threadIdx.x; i < (nruns + 1u) / 2u; i += BT) (&S.tbl[0][0])[i] = 0u;
    __syncthreads();
    return lng;
}

// Waves per SIMD that the register budget must allow for a finish class:
// as many blocks as fit a CU by LDS (160 KiB), capped below.
template <int KB, int BT, int ITEMS, bool PAY>
struct FinOcc {
    static constexpr int blocks = (160 * 1024) / (int)sizeof(FinishLds<KB, BT, ITEMS, PAY>);
    static constexpr int lds_waves = (blocks * (BT / WAVE) + 3) / 4;
    // at most 4 (5 for a class of 8 keys a thread with a payload, whose
    // LDS fits five blocks): a higher floor makes the keys-only classes spill
    static constexpr int cap = (ITEMS <= 8 && PAY) ? 5 : 4;
    static constexpr int waves = lds_waves < cap ? lds_waves : cap;
};

template <int KB, int BT, int ITEMS, bool PAY>
__global__ __launch_bounds__(BT) __attribute__((amdgpu_waves_per_eu(FinOcc<KB, BT, ITEMS, PAY>::waves)))
void k_finish(Work w, int cls) {
    using KT = KeyT<KB>;
    using V = typename KT::V;
    constexpr int KL = 8;
    constexpr int R = 1 << KL;
    constexpr int CAP = BT * ITEMS;
    constexpr int NW = BT / WAVE;
    const int NB = (int)w.nbits;
    __shared__ FinishLds<KB, BT, ITEMS, PAY> S;

    Ctl *ctl = w.ctl;
    if (ctl->error | ctl->overflow) return;
    const uint32_t nfin = min(ctl->fin_ctr[cls], w.max_fin[cls]);
    const int wv = threadIdx.x / WAVE, lane = lane_id();
    for (int i = threadIdx.x; i < NW * R; i += BT) (&S.wh[0][0])[i] = 0u;
    for (int i = threadIdx.x; i < NW * 2 * R; i += BT) (&S.tbl[0][0])[i] = 0u;
    __syncthreads();

    constexpr int NVK = (CAP + Vec<KB>::N * BT - 1) / (Vec<KB>::N * BT);
    constexpr int NVP = (CAP + 4 * BT - 1) / (4 * BT);
    for (uint32_t f = blockIdx.x; f < nfin; f += gridDim.x) {
        const FinEntry fe = uni(w.fin[cls][f]);
        const uint32_t len = fe.info & 0xFFFFu;
        const int bitpos = (int)((fe.info >> 16) & 0xFFu);
        const uint32_t parity = (fe.info >> 24) & 1u;
        if (len > (uint32_t)CAP || (size_t)fe.begin + len > w.n_total) {
            if (threadIdx.x == 0) atomicOr(&ctl->error, ERR_INTERNAL);
            continue;
        }
        // each wave's share of the keys (wave_share): 4-byte keys with a
        // payload are loaded in that order into registers, one per lane and
        // step, so that the first LDS pass can rank them from there; other
        // keys go to LDS in input order with 16-byte vectors (keys-only
        // classes run more waves per SIMD and have no registers to spare).
        // AND/OR on the way.
        constexpr bool REGK = KB == 4 && PAY;
        uint32_t wb = 0u, we = 0u;
        if constexpr (REGK) wave_share<BT, ITEMS>(len, wv, wb, we);
        V a = KT::ones(), o = KT::zero();
        V kr[REGK ? ITEMS : 1];
        if constexpr (REGK) {
            const uint32_t ebase = wb + (uint32_t)lane;
            // every load is valid (indices clamped into the sub-array), the
            // lanes past the wave's share drop theirs
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                const uint32_t e = ebase + j * WAVE;
                kr[j] = ld_key<KB>(w.keys[parity], (size_t)fe.begin + min(e, len - 1u), w.kind);
            }
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                if (ebase + j * WAVE < we) {
                    a = KT::vand(a, kr[j]);
                    o = KT::vor(o, kr[j]);
                }
            }
        } else {
            fin_load_keys<KB, NVK, BT>(w.keys[parity], fe.begin, (size_t)fe.begin + len, S.keys, a, o, w.kind);
        }
        if constexpr (PAY) fin_load_pay<NVP, BT>(w.pay[parity], fe.begin, (size_t)fe.begin + len, S.pay);
        Canon ca = KT::canon(a), co = KT::canon(o);
#pragma unroll
        for (int off = 1; off < WAVE; off <<= 1) {
            ca.hi &= __shfl_xor(ca.hi, off, WAVE);
            ca.lo &= __shfl_xor(ca.lo, off, WAVE);
            co.hi |= __shfl_xor(co.hi, off, WAVE);
            co.lo |= __shfl_xor(co.lo, off, WAVE);
        }
        if (lane == 0) {
            S.ao[wv][0] = ca.hi;
            S.ao[wv][1] = ca.lo;
            S.ao[wv][2] = co.hi;
            S.ao[wv][3] = co.lo;
        }
        __syncthreads();
        Canon diff{0ull, 0ull};
        unsigned long long ah = ~0ull;  // bits every key has (the high word)
        {
            unsigned long long al = ~0ull, oh = 0ull, ol = 0ull;
#pragma unroll
            for (int q = 0; q < NW; ++q) {
                ah &= S.ao[q][0];
                al &= S.ao[q][1];
                oh |= S.ao[q][2];
                ol |= S.ao[q][3];
            }
            diff.hi = ah ^ oh;
            diff.lo = al ^ ol;
        }
        const int lb = last_set_below(diff, bitpos, NB);  // least significant varying bit
        if (lb < bitpos && parity == 0u) {
            // nothing varies and the keys already sit in A: nothing to write
            __syncthreads();
            continue;
        }
        if constexpr (!REGK) wave_share<BT, ITEMS>(len, wv, wb, we);
        const uint32_t ebase = wb + (uint32_t)lane;
        const int fb = first_set_from(diff, bitpos, NB);
        if constexpr (KB != 16) {
            // every varying bit of the keys (those after the sorted ones
            // included) inside one 16-bit field: sort one word per key
            const int s = min(fb, 8 * KB - 16);
            const uint64_t fmask = (0xFFFFull << 48) >> s;  // the field in the left-aligned word
            if (lb >= bitpos && lb - s <= 15 && ((diff.hi & ~fmask) | diff.lo) == 0ull) {
                // the keys in registers (REGK) or in LDS in input order
                packed_passes<KB, BT, ITEMS, PAY>(S, diff, fb, lb, s, ebase, we, [&](int j) -> V {
                    if constexpr (REGK) return kr[j];
                    else return S.keys[ebase + j * WAVE];
                });
                typedef uint32_t __attribute__((may_alias)) word_t;
                const V base = (KB == 4) ? (V)(ah >> 32) : (V)ah;
                fin_store_packed<KB, BT, PAY>(w, fe.begin, (size_t)fe.begin + len,
                                              reinterpret_cast<const word_t *>(&S.keys[0]), S.pay, base, s);
                __syncthreads();
                continue;
            }
        }
        // the first window ranks the keys in registers where the class has
        // registers to spare for it (at most 12 keys a thread); otherwise
        // they go to LDS in input order first
        constexpr bool REGW = REGK && ITEMS <= 12;
        if constexpr (REGK && !REGW) {
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                const uint32_t e = ebase + j * WAVE;
                if (e < we) S.keys[e] = kr[j];
            }
            __syncthreads();
        }
        auto in_lds = [&](int j) -> V { return S.keys[ebase + j * WAVE]; };
        if (lb >= bitpos) {
            // sort by the two leading 8-bit windows that start at varying bits;
            // keys still tied on them are ordered by fix_runs, or, if a tied
            // run is long, by passes over every varying bit
            const int f2 = first_set_from(diff, min(fb + 8, NB), NB);
            const int pe = (f2 >= NB) ? lb : min(lb, f2 + 7);
            lds_passes<KB, BT, ITEMS, PAY, REGW>(S, diff, bitpos, pe, ebase, we, [&](int j) -> V {
                if constexpr (REGW) return kr[j];
                else return in_lds(j);
            });
            if (pe < lb && fix_runs<KB, BT, ITEMS, PAY>(S, pe, len, NB))
                lds_passes<KB, BT, ITEMS, PAY, false>(S, diff, bitpos, lb, ebase, we, in_lds);
        } else if constexpr (REGW) {
            // nothing varies (the keys sit in B): written out as they are
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                const uint32_t e = ebase + j * WAVE;
                if (e < we) S.keys[e] = kr[j];
            }
            __syncthreads();
        }
        fin_store_keys<KB, BT>(w.keys[0], fe.begin, (size_t)fe.begin + len, S.keys, w.kind);
        if constexpr (PAY) fin_store_pay<BT>(w.pay[0], fe.begin, (size_t)fe.begin + len, S.pay);
        __syncthreads();
    }
}

// ----------------------------------------------------------- k_finish_wave
// Sub-arrays of up to FW_CAP keys (the smallest LDS class), one per wave:
// the same steps as k_finish -- AND/OR, the two leading varying windows as
// LSD passes in LDS, tied runs ranked in the wave, passes over every varying
// bit if a run is longer than 64 -- in a slice of LDS of the wave's own,
// with wave-level scans instead of block barriers.  A workgroup per short
// sub-array spends most of its time in barriers; here the waves of a block
// never wait for each other.
constexpr int FW_CAP = 1024;
constexpr int FW_ITEMS = FW_CAP / WAVE;

template <int KB, bool PAY>
struct WaveFinLds {
    using V = typename KeyT<KB>::V;
    V keys[FW_CAP];
    uint32_t pay[PAY ? FW_CAP : 1];
    alignas(8) uint32_t tbl[2 * 256];  // lane masks; between passes the list of tied runs
    uint32_t wh[256];
    uint32_t long_run;
};

// Stable passes over the varying bits in [bitpos, end] of the wave's slice,
// least significant window of up to 8 bits first.
template <int KB, bool PAY, int IT>
__device__ __forceinline__ void wave_passes(WaveFinLds<KB, PAY> &S, Canon diff, int bitpos, int end, uint32_t len) {
    using KT = KeyT<KB>;
    using V = typename KT::V;
    constexpr int R = 256;
    const int lane = lane_id();
    int hib = last_set_below(diff, bitpos, end + 1);
    while (hib >= bitpos) {
        const int lo = max(bitpos, hib - 7);
        const int wbits = hib - lo + 1;
        V key[IT];
        uint32_t dg[IT], rnk[IT], pv[IT];
#pragma unroll
        for (int j = 0; j < IT; ++j) {
            const uint32_t e = (uint32_t)lane + j * WAVE;
            key[j] = (e < len) ? S.keys[e] : KT::zero();
            dg[j] = KT::digit(key[j], lo, wbits);
        }
        wave_rank<R, RANK_GROUP, IT, false>(dg, (uint32_t)lane, len, S.tbl, S.wh, rnk);
#pragma unroll
        for (int j = 0; j < IT; ++j) {
            const uint32_t e = (uint32_t)lane + j * WAVE;
            pv[j] = (PAY && e < len) ? S.pay[e] : 0u;
        }
        // exclusive scan of the digit counts: lane l holds digits 4l .. 4l+3
        {
            const uint32_t c0 = S.wh[4 * lane], c1 = S.wh[4 * lane + 1], c2 = S.wh[4 * lane + 2],
                           c3 = S.wh[4 * lane + 3];
            const uint32_t sum = c0 + c1 + c2 + c3;
            uint32_t x = sum;
#pragma unroll
            for (int o = 1; o < WAVE; o <<= 1) {
                const uint32_t y = __shfl_up(x, o, WAVE);
                if (lane >= o) x += y;
            }
            const uint32_t b = x - sum;
            S.wh[4 * lane] = b;
            S.wh[4 * lane + 1] = b + c0;
            S.wh[4 * lane + 2] = b + c0 + c1;
            S.wh[4 * lane + 3] = b + c0 + c1 + c2;
        }
#pragma unroll
        for (int j = 0; j < IT; ++j) {
            const uint32_t e = (uint32_t)lane + j * WAVE;
            if (e < len) {
                const uint32_t pos = S.wh[dg[j]] + rnk[j];
                S.keys[pos] = key[j];
                if (PAY) S.pay[pos] = pv[j];
            }
        }
        for (int i = lane; i < R; i += WAVE) S.wh[i] = 0u;
        hib = last_set_below(diff, bitpos, lo);
    }
}

// Tied runs of the wave's slice after sorting by bits [0, pe]: runs of up to
// 64 keys ranked in the wave on the leading nb bits (packed, as in
// fix_runs); true, with nothing of a longer run moved, if a run is longer.
template <int KB, bool PAY, int IT>
__device__ bool wave_fix_runs(WaveFinLds<KB, PAY> &S, int pe, uint32_t len, int nb) {
    using KT = KeyT<KB>;
    using V = typename KT::V;
    typedef uint16_t __attribute__((may_alias)) pos16_t;
    static_assert(2 * 256 * 2 >= FW_CAP / 2, "run list must hold every possible run start");
    pos16_t *list = reinterpret_cast<pos16_t *>(&S.tbl[0]);
    const int lane = lane_id();
    Canon pm;
    pm.hi = pe >= 63 ? ~0ull : ~(~0ull >> (pe + 1));
    pm.lo = pe >= 127 ? ~0ull : (pe < 64 ? 0ull : ~(~0ull >> (pe - 63)));
    const Canon km = canon_lead_mask(nb);
    bool lng = false;
    // run starts in position order (position = lane + 64 j)
    uint32_t nruns = 0;
#pragma unroll
    for (int j = 0; j < IT; ++j) {
        const uint32_t p = (uint32_t)lane + j * WAVE;
        bool st = false;
        if (p + 1 < len) {
            const Canon k = KT::canon(S.keys[p]);
            st = canon_eq_under(KT::canon(S.keys[p + 1]), k, pm) &&
                 (p == 0 || !canon_eq_under(KT::canon(S.keys[p - 1]), k, pm));
        }
        const uint64_t b = __ballot(st);
        if (st) list[nruns + lanes_below(b)] = (uint16_t)p;
        nruns += (uint32_t)__popcll(b);
    }
    for (uint32_t r0 = 0; r0 < nruns; r0 += WAVE) {
        uint32_t s0 = 0u, L = 0u;
        if (r0 + (uint32_t)lane < nruns) {
            s0 = list[r0 + lane];
            const Canon ks = KT::canon(S.keys[s0]);
            L = 2u;
            while (L <= (uint32_t)WAVE && s0 + L < len && canon_eq_under(KT::canon(S.keys[s0 + L]), ks, pm)) ++L;
            if (L > (uint32_t)WAVE) {
                lng = true;
                L = 0u;
            }
        }
        wave_pack(L, [&](int l, uint32_t i, int head, bool act, uint32_t el, uint32_t ml) {
            const uint32_t s = __shfl(s0, l, WAVE);
            V k = KT::zero();
            uint32_t pv = 0u;
            if (act) {
                k = S.keys[s + i];
                if (PAY) pv = S.pay[s + i];
            }
            Canon ck = KT::canon(k);
            ck.hi &= km.hi;
            ck.lo &= km.lo;
            const uint32_t r = pack_rank<KB>(ck, i, el, head, ml);
            if (act) {
                S.keys[s + r] = k;
                if (PAY) S.pay[s + r] = pv;
            }
        });
    }
    // the ranking tables start at zero
    for (uint32_t i = lane; i < (nruns + 1u) / 2u; i += WAVE) S.tbl[i] = 0u;
    return __ballot(lng) != 0ull;
}

template <int KB>
struct FinWaves {
    static constexpr int n = (KB == 16) ? 2 : 4;  // waves per block: LDS per wave grows with the key
};

template <int KB, bool PAY>
__global__ __launch_bounds__(FinWaves<KB>::n * WAVE) void k_finish_wave(Work w, int cls) {
    using KT = KeyT<KB>;
    using V = typename KT::V;
    constexpr int NWB = FinWaves<KB>::n;
    const int NB = (int)w.nbits;
    __shared__ WaveFinLds<KB, PAY> SS[NWB];
    Ctl *ctl = w.ctl;
    if (ctl->error | ctl->overflow) return;
    const uint32_t nfin = min(ctl->fin_ctr[cls], w.max_fin[cls]);
    const int wv = threadIdx.x / WAVE, lane = lane_id();
    WaveFinLds<KB, PAY> &S = SS[wv];
    for (int i = lane; i < 2 * 256; i += WAVE) S.tbl[i] = 0u;
    for (int i = lane; i < 256; i += WAVE) S.wh[i] = 0u;
    const uint32_t gw = blockIdx.x * NWB + wv, nw = gridDim.x * NWB;
    for (uint32_t f = gw; f < nfin; f += nw) {
        const FinEntry fe = uni(w.fin[cls][f]);
        const uint32_t len = fe.info & 0xFFFFu;
        const int bitpos = (int)((fe.info >> 16) & 0xFFu);
        const uint32_t parity = (fe.info >> 24) & 1u;
        if (len > (uint32_t)FW_CAP || (size_t)fe.begin + len > w.n_total) {
            if (lane == 0) atomicOr(&ctl->error, ERR_INTERNAL);
            continue;
        }
        V a = KT::ones(), o = KT::zero();
        for (uint32_t p = lane; p < len; p += WAVE) {
            const V k = ld_key<KB>(w.keys[parity], (size_t)fe.begin + p, w.kind);
            S.keys[p] = k;
            a = KT::vand(a, k);
            o = KT::vor(o, k);
            if (PAY) S.pay[p] = w.pay[parity][fe.begin + p];
        }
        Canon ca = KT::canon(a), co = KT::canon(o);
#pragma unroll
        for (int off = 1; off < WAVE; off <<= 1) {
            ca.hi &= __shfl_xor(ca.hi, off, WAVE);
            ca.lo &= __shfl_xor(ca.lo, off, WAVE);
            co.hi |= __shfl_xor(co.hi, off, WAVE);
            co.lo |= __shfl_xor(co.lo, off, WAVE);
        }
        const Canon diff{ca.hi ^ co.hi, ca.lo ^ co.lo};
        const int lb = last_set_below(diff, bitpos, NB);
        if (lb < bitpos && parity == 0u) continue;  // nothing varies and the keys sit in A
        if (lb >= bitpos) {
            const int fb = first_set_from(diff, bitpos, NB);
            const int f2 = first_set_from(diff, min(fb + 8, NB), NB);
            const int pe = (f2 >= NB) ? lb : min(lb, f2 + 7);
            // loops sized to the sub-array: 2, 4, 8 or 16 keys per lane
            auto sort_it = [&](auto it) {
                constexpr int IT = decltype(it)::value;
                wave_passes<KB, PAY, IT>(S, diff, bitpos, pe, len);
                if (pe < lb && wave_fix_runs<KB, PAY, IT>(S, pe, len, NB))
                    wave_passes<KB, PAY, IT>(S, diff, bitpos, lb, len);
            };
            if (len <= 2u * WAVE)
                sort_it(std::integral_constant<int, 2>());
            else if (len <= 4u * WAVE)
                sort_it(std::integral_constant<int, 4>());
            else if (len <= 8u * WAVE)
                sort_it(std::integral_constant<int, 8>());
            else
                sort_it(std::integral_constant<int, FW_ITEMS>());
        }
        for (uint32_t p = lane; p < len; p += WAVE) {
            KT::store(w.keys[0], (size_t)fe.begin + p, raw_key<KB>(S.keys[p], w.kind));
            if (PAY) w.pay[0][fe.begin + p] = S.pay[p];
        }
    }
}

// ---------------------------------------------------------- k_finish_small
// Sub-arrays of 2 .. SMALL_MAX keys.  A block per sub-array would spend its
// time on barriers; instead each wave takes 64 list entries at a time and
// packs as many whole sub-arrays as fit into its 64 lanes, one key per lane.
// A key's place in its sub-array is the number of keys there that come
// before it in the stable order (smaller on the leading nbits bits, or equal
// and earlier in the input), so the result is the stable sort.  Every lane
// loads its key before any lane of the wave stores, and distinct sub-arrays
// never overlap, so reading and writing the same buffer is safe.
template <int KB, bool PAY>
__global__ __launch_bounds__(THREADS) void k_finish_small(Work w) {
    using KT = KeyT<KB>;
    using V = typename KT::V;
    Ctl *ctl = w.ctl;
    if (ctl->error | ctl->overflow) return;
    const uint32_t nent = min(ctl->small_ctr, w.max_small);
    const int lane = lane_id();
    const uint32_t wave_id = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const uint32_t nwaves = gridDim.x * (blockDim.x / WAVE);
    const Canon km = canon_lead_mask((int)w.nbits);
    // entries per wave: about 256 keys' worth (four packed rounds), from the
    // bound n_total / entries on their mean length -- pairs fill a window
    // of 64, sub-arrays of 60 keys get one entry per wave instead of 64
    // serial rounds on a few waves
    const unsigned long long wfit = (256ull * nent) / (w.n_total ? w.n_total : 1u);
    const uint32_t win = wfit >= (unsigned long long)WAVE ? (uint32_t)WAVE : (wfit ? (uint32_t)wfit : 1u);
    for (uint32_t e0 = wave_id * win; e0 < nent; e0 += nwaves * win) {
        // lane l < win holds entry e0 + l
        uint32_t b = 0u, len = 0u, par = 0u;
        if ((uint32_t)lane < win && e0 + lane < nent) {
            const FinEntry fe = w.fin_small[e0 + lane];
            b = fe.begin;
            len = fe.info & 0xFFFFu;
            par = (fe.info >> 24) & 1u;
            if (len > SMALL_MAX || (size_t)b + len > w.n_total) {
                atomicOr(&ctl->error, ERR_INTERNAL);
                len = 0u;
            }
        }
        wave_pack(len, [&](int l, uint32_t i, int head, bool act, uint32_t el, uint32_t ml) {
            const uint32_t eb = __shfl(b, l, WAVE), ep = __shfl(par, l, WAVE);
            V k = KT::zero();
            uint32_t pv = 0u;
            if (act) {
                k = ld_key<KB>(w.keys[ep], (size_t)eb + i, w.kind);
                if constexpr (PAY) pv = w.pay[ep][eb + i];
            }
            Canon ck = KT::canon(k);
            ck.hi &= km.hi;
            ck.lo &= km.lo;
            const uint32_t r = pack_rank<KB>(ck, i, el, head, ml);
            if (act) {
                KT::store(w.keys[0], (size_t)eb + r, raw_key<KB>(k, w.kind));
                if constexpr (PAY) w.pay[0][eb + r] = pv;
            }
        });
    }
}

}  // namespace binar
