// gfx950 kernels of the breadth-first stable binar sort.
//
// One call sorts a set of sub-arrays ("segments") of the keys.  Each global
// pass takes every live segment larger than the LDS-finish threshold T and
// partitions it stably on its next k bits (section "Partition Array into
// Sub-arrays", with the exchange replaced by a stable scatter, k bits at a
// time instead of one):
//
//   k_hist    digit counts of every live segment + AND/OR of its keys
//   k_plan    per segment: pass-through test (one non-empty digit bin, the
//             iteration of section "Optimize the Algorithm"), bucket bases
//             (exclusive scan), classification of the children: done (one
//             key or no varying bits left: the base cases of section
//             "Evaluate for Recursive Base Case"), LDS finish, or next pass
//   k_scatter per tile: stable rank by wave64 ballots, decoupled look-back
//             prefix across the segment's tiles, LDS staging in digit order,
//             coalesced write of keys and payload
//
// after which k_finish sorts each small segment inside one workgroup (LDS
// least-significant-digit passes over its remaining varying bits) and
// writes it to the caller's buffer.
//
// Data live in two ping-pong buffer pairs: A (the caller's keys/payload) and
// B (scratch).  A segment's `parity` says which one holds it; every pass
// writes the other one, except that finished children are written straight
// to A.  Segments never overlap, so a finished segment is never touched
// again by later passes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "binar_keys.h"

namespace binar {

constexpr int WAVE = 64;
constexpr int THREADS = 256;
constexpr int WAVES = THREADS / WAVE;
constexpr int MAX_RADIX = 256;
constexpr int NCLASS = 4;        // LDS-finish size classes
constexpr int MAX_PASSES = 16;   // 128 bits / 8 bits

constexpr uint32_t SEG_SKIP = 1u;  // segment does not scatter this pass
constexpr uint32_t ST_FLAGS = 3u << 30;
constexpr uint32_t ST_AGG = 1u << 30;  // status word: tile aggregate only
constexpr uint32_t ST_INC = 2u << 30;  // status word: inclusive prefix
constexpr uint32_t ST_VAL = (1u << 30) - 1u;
// Bound on every look-back wait (s_sleep rounds).  A predecessor tile always
// publishes within microseconds; the bound only guarantees that no wave can
// wait forever if an invariant were ever broken.
constexpr uint32_t SPIN_LIMIT = 1u << 24;
constexpr unsigned ERR_SEGMENTS = 1u;  // bad segment table
constexpr unsigned ERR_INTERNAL = 2u;  // broken invariant (bounds, wait limit)

// A live segment of a global pass.  info = bitpos | parity << 8 | flags << 16
struct SegEntry {
    uint32_t begin, len, info, tile_start;
};

// A segment to finish in LDS.  info = len | bitpos << 16 | parity << 24
struct FinEntry {
    uint32_t begin, info;
};

struct Ctl {
    unsigned long long list_ctr[2];  // (entries << 32) | tiles of each pass list
    unsigned int ticket;             // scatter tile tickets
    unsigned int error;              // ERR_SEGMENTS / ERR_INTERNAL
    unsigned int overflow;           // a list ran out of room (never expected)
    unsigned int passes;
    unsigned int fin_ctr[NCLASS];
    unsigned long long moved[MAX_PASSES];
    unsigned long long hist_keys[MAX_PASSES];
    unsigned long long fin_keys;
    unsigned long long fin_segs;
};

struct Work {
    Ctl *ctl;
    SegEntry *list[2];
    uint32_t *counts[2];        // [entry][radix]
    uint32_t *bases[2];         // [entry][radix]: bucket start
    uint8_t *to_a[2];           // [entry][radix]: 1 = write this bucket to A
    unsigned long long *andor[2];  // [entry][4]: and.hi, and.lo, or.hi, or.lo
    uint32_t *status;           // [tile][radix]
    FinEntry *fin[NCLASS];
    uint32_t fin_cap[NCLASS];   // largest segment of each class
    uint32_t max_fin[NCLASS];   // entries each class can hold
    uint32_t max_big, max_tiles;
    uint32_t finish_max;        // T
    uint32_t tile_keys;
    uint32_t n_total;           // keys in A and B: every index written is below it
    void *keys[2];              // A, B
    uint32_t *pay[2];           // A, B (NULL without payload)
};

// ------------------------------------------------------------ small helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t ld_acquire_agent(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_agent(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long ld_u64(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive scan of one value per thread over the block; returns the
// exclusive prefix and writes the block total to *total.  tmp: WAVES words.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *tmp, uint32_t *total) {
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

// Stable multisplit rank inside a wave: lanes holding the same digit d are
// ranked by lane order.  Returns this lane's rank among them and the number
// of lanes holding d (valid lanes only).
template <int K>
__device__ __forceinline__ void wave_match(uint32_t d, bool valid, uint32_t &rank, uint32_t &cnt) {
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < K; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bal = __ballot(bit);
        m &= bit ? bal : ~bal;
    }
    rank = lanes_below(m);
    cnt = (uint32_t)__popcll(m);
}

// Append a live segment to pass list L; its counts / AND-OR slot is cleared.
template <int R>
__device__ void append_big(const Work &w, int L, uint32_t begin, uint32_t len, uint32_t bitpos,
                           uint32_t parity) {
    const uint32_t ntiles = (len + w.tile_keys - 1) / w.tile_keys;
    const unsigned long long old = atomicAdd(&w.ctl->list_ctr[L], (1ull << 32) | (unsigned long long)ntiles);
    const uint32_t slot = (uint32_t)(old >> 32);
    if (slot >= w.max_big || (uint32_t)old + ntiles > w.max_tiles) {
        atomicOr(&w.ctl->overflow, 1u);
        return;
    }
    w.list[L][slot] = SegEntry{begin, len, bitpos | (parity << 8), (uint32_t)old};
    uint32_t *c = w.counts[L] + (size_t)slot * R;
    for (int d = 0; d < R; ++d) c[d] = 0u;
    unsigned long long *ao = w.andor[L] + (size_t)slot * 4;
    ao[0] = ~0ull;
    ao[1] = ~0ull;
    ao[2] = 0ull;
    ao[3] = 0ull;
}

__device__ __forceinline__ void append_fin(const Work &w, uint32_t begin, uint32_t len, uint32_t bitpos,
                                           uint32_t parity) {
    int c = 0;
    while (c < NCLASS - 1 && len > w.fin_cap[c]) ++c;
    const uint32_t slot = atomicAdd(&w.ctl->fin_ctr[c], 1u);
    if (slot >= w.max_fin[c]) {
        atomicOr(&w.ctl->overflow, 1u);
        return;
    }
    w.fin[c][slot] = FinEntry{begin, len | (bitpos << 16) | (parity << 24)};
}

// ------------------------------------------------------------------ k_reset
__global__ void k_reset(Ctl *ctl) {
    uint32_t *p = reinterpret_cast<uint32_t *>(ctl);
    for (uint32_t i = threadIdx.x; i < sizeof(Ctl) / 4; i += blockDim.x) p[i] = 0u;
}

// ------------------------------------------------------------------- k_init
// Classify the caller's segments: <= 1 key: nothing to do (base case);
// <= T keys: LDS finish; larger: first global pass.
template <int R>
__global__ __launch_bounds__(THREADS) void k_init(Work w, const uint32_t *seg_off, uint32_t nseg,
                                                  uint32_t n_single, uint32_t n_limit) {
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < nseg; s += gridDim.x * blockDim.x) {
        uint32_t b = 0, e = n_single;
        if (seg_off) {
            b = seg_off[s];
            e = seg_off[s + 1];
            if (e < b || e > n_limit) {
                atomicOr(&w.ctl->error, ERR_SEGMENTS);
                continue;
            }
        }
        const uint32_t len = e - b;
        if (len <= 1) continue;
        if (len <= w.finish_max)
            append_fin(w, b, len, 0u, 0u);
        else
            append_big<R>(w, 0, b, len, 0u, 0u);
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

// ------------------------------------------------------------------- k_hist
// Digit counts (bits [bitpos, bitpos + w) of each key) and AND/OR of every
// live segment of list L.  Each block takes a contiguous run of tiles and
// flushes its LDS counts whenever the segment changes.  Also clears the
// look-back status words of its tiles and resets the next list and the
// scatter ticket (nothing else touches them during this kernel).
template <int KB, int K>
__global__ __launch_bounds__(THREADS) void k_hist(Work w, int L) {
    using KT = KeyT<KB>;
    using V = typename KT::V;
    constexpr int R = 1 << K;
    constexpr int U = 4;  // keys in flight per thread
    __shared__ uint32_t s_h[WAVES][R];
    __shared__ unsigned long long s_ao[WAVES][4];

    Ctl *ctl = w.ctl;
    if (ctl->error | ctl->overflow) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->list_ctr[L ^ 1] = 0ull;
        ctl->ticket = 0u;
    }
    const unsigned long long lc = ctl->list_ctr[L];
    const uint32_t nslots = (uint32_t)(lc >> 32), ntiles = (uint32_t)lc;
    if (ntiles == 0) return;
    const uint32_t per = (ntiles + gridDim.x - 1) / gridDim.x;
    const uint32_t t0 = blockIdx.x * per;
    const uint32_t t1 = min(ntiles, t0 + per);
    if (t0 >= t1) return;

    const int wv = threadIdx.x / WAVE, lane = lane_id();
    for (int i = threadIdx.x; i < WAVES * R; i += THREADS) (&s_h[0][0])[i] = 0u;
    __syncthreads();

    uint32_t slot = find_slot(w.list[L], nslots, t0);
    SegEntry seg = w.list[L][slot];
    uint32_t next_start = (slot + 1 < nslots) ? w.list[L][slot + 1].tile_start : 0xFFFFFFFFu;
    V a = KT::ones(), o = KT::zero();

    auto flush = [&](uint32_t fslot) {
        __syncthreads();
        uint32_t *cnt = w.counts[L] + (size_t)fslot * R;
        for (int d = threadIdx.x; d < R; d += THREADS) {
            uint32_t c = 0;
#pragma unroll
            for (int q = 0; q < WAVES; ++q) {
                c += s_h[q][d];
                s_h[q][d] = 0u;
            }
            if (c) atomicAdd(&cnt[d], c);
        }
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
        __syncthreads();
        if (threadIdx.x < 4) {
            unsigned long long v = s_ao[0][threadIdx.x];
            for (int q = 1; q < WAVES; ++q) v = (threadIdx.x < 2) ? (v & s_ao[q][threadIdx.x]) : (v | s_ao[q][threadIdx.x]);
            unsigned long long *dst = w.andor[L] + (size_t)fslot * 4 + threadIdx.x;
            if (threadIdx.x < 2)
                atomicAnd(dst, v);
            else
                atomicOr(dst, v);
        }
        a = KT::ones();
        o = KT::zero();
        __syncthreads();
    };

    for (uint32_t t = t0; t < t1; ++t) {
        if (t >= next_start) {
            flush(slot);
            while (slot + 1 < nslots && w.list[L][slot + 1].tile_start <= t) ++slot;
            seg = w.list[L][slot];
            next_start = (slot + 1 < nslots) ? w.list[L][slot + 1].tile_start : 0xFFFFFFFFu;
        }
        // clear this tile's look-back status words
        for (int d = threadIdx.x; d < R; d += THREADS) w.status[(size_t)t * R + d] = 0u;

        const uint32_t bitpos = seg.info & 0xFFu, parity = (seg.info >> 8) & 1u;
        const int wbits = min(K, KT::NBITS - (int)bitpos);
        const void *src = w.keys[parity];
        const uint32_t lt = t - seg.tile_start;
        const uint32_t e0 = lt * w.tile_keys;
        const uint32_t e1 = min(seg.len, e0 + w.tile_keys);
        for (uint32_t e = e0 + threadIdx.x; e < e1; e += THREADS * U) {
            V v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t x = e + u * THREADS;
                v[u] = (x < e1) ? KT::load(src, (size_t)seg.begin + x) : KT::zero();
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t x = e + u * THREADS;
                if (x < e1) {
                    atomicAdd(&s_h[wv][KT::digit(v[u], bitpos, wbits)], 1u);
                    a = KT::vand(a, v[u]);
                    o = KT::vor(o, v[u]);
                }
            }
        }
    }
    flush(slot);
}

// ------------------------------------------------------------------- k_plan
template <int KB, int K>
__global__ __launch_bounds__(THREADS) void k_plan(Work w, int L, int pass) {
    using KT = KeyT<KB>;
    constexpr int R = 1 << K;
    constexpr int NB = KT::NBITS;
    __shared__ uint32_t s_tmp[WAVES];
    Ctl *ctl = w.ctl;
    if (ctl->error | ctl->overflow) return;
    const unsigned long long lc = ctl->list_ctr[L];
    const uint32_t nslots = (uint32_t)(lc >> 32);
    if (nslots == 0) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicMax(&ctl->passes, (unsigned)(pass + 1));
    const int d = threadIdx.x;

    for (uint32_t s = blockIdx.x; s < nslots; s += gridDim.x) {
        const SegEntry seg = w.list[L][s];
        const uint32_t bitpos = seg.info & 0xFFu, parity = (seg.info >> 8) & 1u;
        const int wbits = min(K, NB - (int)bitpos);
        const uint32_t nbins = 1u << wbits;
        const uint32_t c = (d < (int)nbins) ? w.counts[L][(size_t)s * R + d] : 0u;
        const int nz = __syncthreads_count(c != 0u);
        const unsigned long long *ao = w.andor[L] + (size_t)s * 4;
        const Canon diff{ao[0] ^ ao[2], ao[1] ^ ao[3]};
        const int ps = pass < MAX_PASSES ? pass : MAX_PASSES - 1;
        if (d == 0) atomicAdd(&ctl->hist_keys[ps], (unsigned long long)seg.len);

        if (nz == 1) {
            // pass-through: every key has the same digit here
            const int nb = first_set_from(diff, bitpos, NB);
            if (nb >= NB) {
                // all keys equal: done; if they sit in B the scatter copies them to A
                if (parity == 1u) {
                    if (c != 0u) {
                        w.bases[L][(size_t)s * R + d] = seg.begin;
                        w.to_a[L][(size_t)s * R + d] = 1;
                    }
                    if (d == 0) atomicAdd(&ctl->moved[ps], (unsigned long long)seg.len);
                } else if (d == 0) {
                    w.list[L][s].info = seg.info | (SEG_SKIP << 16);
                }
            } else if (d == 0) {
                w.list[L][s].info = seg.info | (SEG_SKIP << 16);
                append_big<R>(w, L ^ 1, seg.begin, seg.len, (uint32_t)nb, parity);
            }
            __syncthreads();
            continue;
        }

        uint32_t total;
        const uint32_t excl = block_excl_scan(c, s_tmp, &total);
        if (c != 0u) {
            const uint32_t cb = (uint32_t)first_set_from(diff, bitpos + wbits, NB);
            const uint32_t child_parity = parity ^ 1u;
            const bool done = (c == 1u) || (cb >= (uint32_t)NB);
            w.bases[L][(size_t)s * R + d] = seg.begin + excl;
            w.to_a[L][(size_t)s * R + d] = (done || child_parity == 0u) ? 1 : 0;
            if (!done) {
                if (c <= w.finish_max)
                    append_fin(w, seg.begin + excl, c, cb, child_parity);
                else
                    append_big<R>(w, L ^ 1, seg.begin + excl, c, cb, child_parity);
            }
        }
        if (d == 0) atomicAdd(&ctl->moved[ps], (unsigned long long)seg.len);
        __syncthreads();
    }
}

// ---------------------------------------------------------------- k_scatter
// One tile = THREADS * ITEMS keys of one segment.  Wave q owns keys
// [q * ITEMS * 64, (q + 1) * ITEMS * 64) of the tile, 64 consecutive keys per
// step, so the (wave, step, lane) order is the input order and a stable rank
// is: keys of the digit in earlier waves + earlier steps of this wave +
// earlier lanes of this step.
template <int KB, int K, int ITEMS, bool PAY>
__global__ __launch_bounds__(THREADS) void k_scatter(Work w, int L) {
    using KT = KeyT<KB>;
    using V = typename KT::V;
    constexpr int R = 1 << K;
    constexpr int TILE = THREADS * ITEMS;
    __shared__ V s_keys[TILE];
    __shared__ uint32_t s_pay[PAY ? TILE : 1];
    __shared__ uint32_t s_wh[WAVES][R];   // per-wave digit counts -> wave offsets
    __shared__ uint32_t s_dstart[R];      // digit start inside the staged tile
    __shared__ uint32_t s_gofs[R];        // global index of staged position 0 of digit d
    __shared__ uint8_t s_toa[R];
    __shared__ uint32_t s_tmp[WAVES];
    __shared__ uint32_t s_tile, s_slot;

    Ctl *ctl = w.ctl;
    if (ctl->error | ctl->overflow) return;
    const unsigned long long lc = ctl->list_ctr[L];
    const uint32_t nslots = (uint32_t)(lc >> 32), ntiles = (uint32_t)lc;
    if (ntiles == 0) return;
    const int wv = threadIdx.x / WAVE, lane = lane_id();

    for (;;) {
        if (threadIdx.x == 0) {
            const uint32_t t = atomicAdd(&ctl->ticket, 1u);
            s_tile = t;
            s_slot = (t < ntiles) ? find_slot(w.list[L], nslots, t) : 0u;
        }
        for (int i = threadIdx.x; i < WAVES * R; i += THREADS) (&s_wh[0][0])[i] = 0u;
        __syncthreads();
        const uint32_t t = s_tile;
        if (t >= ntiles) break;
        const uint32_t slot = s_slot;
        const SegEntry seg = w.list[L][slot];
        if ((seg.info >> 16) & SEG_SKIP) {
            __syncthreads();
            continue;
        }
        const uint32_t bitpos = seg.info & 0xFFu, parity = (seg.info >> 8) & 1u;
        const int wbits = min(K, KT::NBITS - (int)bitpos);
        const uint32_t lt = t - seg.tile_start;
        const uint32_t off = lt * (uint32_t)TILE;
        const uint32_t tlen = min((uint32_t)TILE, seg.len - off);
        const void *src = w.keys[parity];
        const uint32_t *psrc = w.pay[parity];
        const size_t gbase = (size_t)seg.begin + off;

        V key[ITEMS];
        uint32_t pay[ITEMS];
        uint32_t rnk[ITEMS];
        const uint32_t ebase = (uint32_t)wv * ITEMS * WAVE + (uint32_t)lane;
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t e = ebase + j * WAVE;
            key[j] = (e < tlen) ? KT::load(src, gbase + e) : KT::zero();
            if (PAY) pay[j] = (e < tlen) ? psrc[gbase + e] : 0u;
        }
        // stable rank inside the wave, step by step
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t e = ebase + j * WAVE;
            const bool valid = e < tlen;
            const uint32_t dg = valid ? KT::digit(key[j], bitpos, wbits) : 0u;
            uint32_t r, c;
            wave_match<K>(dg, valid, r, c);
            uint32_t before = 0;
            if (valid) before = s_wh[wv][dg];
            rnk[j] = before + r;
            if (valid && r + 1 == c) s_wh[wv][dg] = before + c;
        }
        __syncthreads();
        // per digit: wave offsets and tile count
        uint32_t tcnt = 0;
        if (threadIdx.x < R) {
#pragma unroll
            for (int q = 0; q < WAVES; ++q) {
                const uint32_t x = s_wh[q][threadIdx.x];
                s_wh[q][threadIdx.x] = tcnt;
                tcnt += x;
            }
        }
        uint32_t tot;
        const uint32_t dstart = block_excl_scan(tcnt, s_tmp, &tot);
        // decoupled look-back over the earlier tiles of this segment
        if (threadIdx.x < R) {
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
                    while (((v = ld_acquire_agent(w.status + (size_t)tt * R + threadIdx.x)) & ST_FLAGS) == 0u &&
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
            const size_t bi = (size_t)slot * R + threadIdx.x;
            s_dstart[threadIdx.x] = dstart;
            if (tcnt) {
                s_gofs[threadIdx.x] = w.bases[L][bi] + excl - dstart;
                s_toa[threadIdx.x] = w.to_a[L][bi];
            }
        }
        __syncthreads();
        // stage in digit order
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t e = ebase + j * WAVE;
            if (e < tlen) {
                const uint32_t dg = KT::digit(key[j], bitpos, wbits);
                const uint32_t pos = s_dstart[dg] + s_wh[wv][dg] + rnk[j];
                s_keys[pos] = key[j];
                if (PAY) s_pay[pos] = pay[j];
            }
        }
        __syncthreads();
        // coalesced write: consecutive staged keys of one digit go to
        // consecutive global positions
#pragma unroll 4
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t p = j * THREADS + threadIdx.x;
            if (p < tlen) {
                const V k = s_keys[p];
                const uint32_t dg = KT::digit(k, bitpos, wbits);
                const uint32_t a = s_toa[dg];
                const uint32_t g = s_gofs[dg] + p;
                if (g < w.n_total) {
                    KT::store(w.keys[a ? 0 : 1], g, k);
                    if (PAY) w.pay[a ? 0 : 1][g] = s_pay[p];
                } else {
                    atomicOr(&ctl->error, ERR_INTERNAL);
                }
            }
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------- k_finish
// One workgroup per small segment (at most THREADS * ITEMS keys): find the
// bits that vary inside it (AND/OR), sort stably by them with
// least-significant-first LDS passes of up to 8 bits, write to A.
template <int KB, int ITEMS, bool PAY>
__global__ __launch_bounds__(THREADS) void k_finish(Work w, int cls) {
    using KT = KeyT<KB>;
    using V = typename KT::V;
    constexpr int KL = 8;
    constexpr int R = 1 << KL;
    constexpr int CAP = THREADS * ITEMS;
    constexpr int NB = KT::NBITS;
    __shared__ V s_keys[CAP];
    __shared__ uint32_t s_pay[PAY ? CAP : 1];
    __shared__ uint32_t s_wh[WAVES][R];
    __shared__ uint32_t s_dstart[R];
    __shared__ uint32_t s_tmp[WAVES];
    __shared__ unsigned long long s_ao[WAVES][4];

    Ctl *ctl = w.ctl;
    if (ctl->error | ctl->overflow) return;
    const uint32_t nfin = min(ctl->fin_ctr[cls], w.max_fin[cls]);
    const int wv = threadIdx.x / WAVE, lane = lane_id();
    const uint32_t ebase = (uint32_t)wv * ITEMS * WAVE + (uint32_t)lane;

    for (uint32_t f = blockIdx.x; f < nfin; f += gridDim.x) {
        const FinEntry fe = w.fin[cls][f];
        const uint32_t len = fe.info & 0xFFFFu;
        const int bitpos = (int)((fe.info >> 16) & 0xFFu);
        const uint32_t parity = (fe.info >> 24) & 1u;
        const void *src = w.keys[parity];
        const uint32_t *psrc = w.pay[parity];
        const size_t gbase = fe.begin;
        if (len > (uint32_t)CAP || (size_t)fe.begin + len > w.n_total) {
            if (threadIdx.x == 0) atomicOr(&ctl->error, ERR_INTERNAL);
            continue;
        }
        if (threadIdx.x == 0) {
            atomicAdd(&ctl->fin_keys, (unsigned long long)len);
            atomicAdd(&ctl->fin_segs, 1ull);
        }

        V key[ITEMS];
        uint32_t pay[ITEMS];
        V a = KT::ones(), o = KT::zero();
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t e = ebase + j * WAVE;
            key[j] = (e < len) ? KT::load(src, gbase + e) : KT::zero();
            if (PAY) pay[j] = (e < len) ? psrc[gbase + e] : 0u;
            if (e < len) {
                a = KT::vand(a, key[j]);
                o = KT::vor(o, key[j]);
            }
        }
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
        __syncthreads();
        Canon diff{0ull, 0ull};
        {
            unsigned long long ah = ~0ull, al = ~0ull, oh = 0ull, ol = 0ull;
#pragma unroll
            for (int q = 0; q < WAVES; ++q) {
                ah &= s_ao[q][0];
                al &= s_ao[q][1];
                oh |= s_ao[q][2];
                ol |= s_ao[q][3];
            }
            diff.hi = ah ^ oh;
            diff.lo = al ^ ol;
        }
        __syncthreads();

        int hib = last_set_below(diff, bitpos, NB);
        bool staged = false;  // true when the sorted order sits in LDS
        while (hib >= bitpos) {
            const int lo = max(bitpos, hib - KL + 1);
            const int wbits = hib - lo + 1;
            if (staged) {
                // reload the previous pass's order into registers
#pragma unroll
                for (int j = 0; j < ITEMS; ++j) {
                    const uint32_t e = ebase + j * WAVE;
                    if (e < len) {
                        key[j] = s_keys[e];
                        if (PAY) pay[j] = s_pay[e];
                    }
                }
            }
            for (int i = threadIdx.x; i < WAVES * R; i += THREADS) (&s_wh[0][0])[i] = 0u;
            __syncthreads();
            uint32_t rnk[ITEMS];
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                const uint32_t e = ebase + j * WAVE;
                const bool valid = e < len;
                const uint32_t dg = valid ? KT::digit(key[j], lo, wbits) : 0u;
                uint32_t r, c;
                wave_match<KL>(dg, valid, r, c);
                uint32_t before = 0;
                if (valid) before = s_wh[wv][dg];
                rnk[j] = before + r;
                if (valid && r + 1 == c) s_wh[wv][dg] = before + c;
            }
            __syncthreads();
            uint32_t tcnt = 0;
            if (threadIdx.x < R) {
#pragma unroll
                for (int q = 0; q < WAVES; ++q) {
                    const uint32_t x = s_wh[q][threadIdx.x];
                    s_wh[q][threadIdx.x] = tcnt;
                    tcnt += x;
                }
            }
            uint32_t tot;
            const uint32_t ds = block_excl_scan(tcnt, s_tmp, &tot);
            if (threadIdx.x < R) s_dstart[threadIdx.x] = ds;
            __syncthreads();
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                const uint32_t e = ebase + j * WAVE;
                if (e < len) {
                    const uint32_t dg = KT::digit(key[j], lo, wbits);
                    const uint32_t pos = s_dstart[dg] + s_wh[wv][dg] + rnk[j];
                    s_keys[pos] = key[j];
                    if (PAY) s_pay[pos] = pay[j];
                }
            }
            __syncthreads();
            staged = true;
            hib = last_set_below(diff, bitpos, lo);
        }
        if (staged) {
            for (uint32_t p = threadIdx.x; p < len; p += THREADS) {
                KT::store(w.keys[0], gbase + p, s_keys[p]);
                if (PAY) w.pay[0][gbase + p] = s_pay[p];
            }
        } else if (parity == 1u) {
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                const uint32_t e = ebase + j * WAVE;
                if (e < len) {
                    KT::store(w.keys[0], gbase + e, key[j]);
                    if (PAY) w.pay[0][gbase + e] = pay[j];
                }
            }
        }
        __syncthreads();
    }
}

}  // namespace binar
