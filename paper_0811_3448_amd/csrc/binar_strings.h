// Variable-length byte strings (memcmp order, a proper prefix first).
//
// The method is the same MSD partition, taken 15 bytes at a time: every
// round builds a 16-byte key per active string -- the next 15 bytes from the
// round's depth (zero past the string's end) and, in the last byte, how many
// of its bytes remain, capped at 16 -- and sorts the round's groups with the
// fixed-width 16-byte sort (stable, memcmp order of keys).  Keys that tie
// with the last byte 16 belong to strings that still go on: each such run is
// a group of the next round, 15 bytes deeper.  Everything else is final.
//
// Strings are never moved: the sort permutes string ids (0 .. n-1), and the
// caller's payload is gathered through them at the end.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "binar_kernels.h"

namespace binar {

constexpr uint32_t STR_WIN = 15;   // string bytes per round
constexpr int STR_BT = 1024;       // threads per block of the round kernels

struct StrCtl {
    uint32_t n_next;     // active strings of the next round
    uint32_t seg_next;   // groups of the next round
    uint32_t error;      // an offset table entry out of order or past the byte buffer
    uint32_t pad;
};

// Key of compact entry c: the string's next STR_WIN bytes from `depth` and a
// remaining-length code.  Offsets are checked; a bad entry reads nothing and
// sets the error flag.
__global__ __launch_bounds__(256) void k_str_keys(const uint8_t *bytes, uint64_t nbytes, const uint32_t *offs,
                                                  uint32_t n_strings, const uint32_t *ids, uint32_t n_active,
                                                  uint32_t depth, uint8_t *keys, StrCtl *ctl) {
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n_active; c += gridDim.x * blockDim.x) {
        const uint32_t id = ids[c];
        uint32_t s = 0, e = 0;
        if (id < n_strings) {
            s = offs[id];
            e = offs[id + 1];
        }
        if (id >= n_strings || e < s || (uint64_t)e > nbytes) {
            atomicOr(&ctl->error, 1u);
            s = e = 0;
        }
        const uint32_t len = e - s;
        const uint32_t rem = len > depth ? len - depth : 0u;
        const uint32_t take = rem < STR_WIN ? rem : STR_WIN;
        // the window's bytes, little-endian in four words: up to five aligned
        // 4-byte loads, shifted into place; a word reaching outside the
        // caller's buffer is read byte by byte, and only the window's bytes
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (take) {
            const uintptr_t pa = reinterpret_cast<uintptr_t>(bytes) + s + depth;
            const uintptr_t lo = reinterpret_cast<uintptr_t>(bytes), hi = lo + nbytes;
            const uintptr_t d0 = pa & ~(uintptr_t)3;
            const uint32_t off = (uint32_t)(pa - d0);
            uint32_t wd[5];
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                const uintptr_t da = d0 + 4u * q;
                wd[q] = 0u;
                if (da < pa + take) {
                    if (da >= lo && da + 4u <= hi) {
                        wd[q] = *reinterpret_cast<const uint32_t *>(da);
                    } else {
#pragma unroll
                        for (uint32_t b = 0; b < 4; ++b)
                            if (da + b >= pa && da + b < pa + take)
                                wd[q] |= (uint32_t)*reinterpret_cast<const uint8_t *>(da + b) << (8u * b);
                    }
                }
            }
            v.x = __builtin_amdgcn_alignbyte(wd[1], wd[0], off);
            v.y = __builtin_amdgcn_alignbyte(wd[2], wd[1], off);
            v.z = __builtin_amdgcn_alignbyte(wd[3], wd[2], off);
            v.w = __builtin_amdgcn_alignbyte(wd[4], wd[3], off);
            // bytes past the string's end (or past the window) are zero
            auto keep = [&](uint32_t word) -> uint32_t {
                const int n = (int)take - 4 * (int)word;
                return n >= 4 ? 0xFFFFFFFFu : (n <= 0 ? 0u : ((1u << (8 * n)) - 1u));
            };
            v.x &= keep(0);
            v.y &= keep(1);
            v.z &= keep(2);
            v.w &= keep(3);
        }
        v.w = (v.w & 0x00FFFFFFu) | ((rem < 16u ? rem : 16u) << 24);
        reinterpret_cast<uint4 *>(keys)[c] = v;
    }
}

// Mark the first entry of every group of this round (tag = round number, so
// the marks never need clearing).
__global__ __launch_bounds__(256) void k_str_mark(const uint32_t *seg_off, uint32_t nseg, uint32_t *mark,
                                                  uint32_t tag) {
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < nseg; s += gridDim.x * blockDim.x)
        mark[seg_off[s]] = tag;
}

// After the round's sort: put every id where it belongs in the full order.
__global__ __launch_bounds__(256) void k_str_place(const uint32_t *ids_c, const uint32_t *pos_c, uint32_t n_active,
                                                   uint32_t *ids) {
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n_active; c += gridDim.x * blockDim.x)
        ids[pos_c[c]] = ids_c[c];
}

// Entry c continues into the next round: its key ties with a neighbour of
// the same group and the string has bytes beyond this window.
__device__ __forceinline__ void str_flags(const uint4 *keys, const uint32_t *mark, uint32_t tag, uint32_t n_active,
                                          uint32_t c, bool &cont, bool &head) {
    cont = head = false;
    if (c >= n_active) return;
    const uint4 k = keys[c];
    if ((k.w >> 24) != 16u) return;
    const bool first = mark[c] == tag;
    const bool eq_prev = !first && [&] {
        const uint4 p = keys[c - 1];
        return p.x == k.x && p.y == k.y && p.z == k.z && p.w == k.w;
    }();
    const bool eq_next = (c + 1 < n_active) && mark[c + 1] != tag && [&] {
        const uint4 q = keys[c + 1];
        return q.x == k.x && q.y == k.y && q.z == k.z && q.w == k.w;
    }();
    cont = eq_prev || eq_next;
    head = cont && !eq_prev;
}

// Pass 1 of the compaction: entries and run heads that continue, per block.
__global__ __launch_bounds__(STR_BT) void k_str_count(const uint4 *keys, const uint32_t *mark, uint32_t tag,
                                                      uint32_t n_active, uint32_t *blk) {
    __shared__ uint32_t s_tmp[STR_BT / WAVE];
    const uint32_t c = blockIdx.x * STR_BT + threadIdx.x;
    bool cont, head;
    str_flags(keys, mark, tag, n_active, c, cont, head);
    uint32_t tot_c, tot_h;
    (void)block_excl_scan<STR_BT>(cont ? 1u : 0u, s_tmp, &tot_c);
    (void)block_excl_scan<STR_BT>(head ? 1u : 0u, s_tmp, &tot_h);
    if (threadIdx.x == 0) {
        blk[2 * blockIdx.x] = tot_c;
        blk[2 * blockIdx.x + 1] = tot_h;
    }
}

// Pass 2: exclusive scan of the per-block totals (one block), totals to ctl.
__global__ __launch_bounds__(STR_BT) void k_str_scan(uint32_t *blk, uint32_t nblk, StrCtl *ctl) {
    __shared__ uint32_t s_tmp[STR_BT / WAVE];
    __shared__ uint32_t s_carry[2];
    if (threadIdx.x == 0) s_carry[0] = s_carry[1] = 0u;
    __syncthreads();
    for (uint32_t b0 = 0; b0 < nblk; b0 += STR_BT) {
        const uint32_t b = b0 + threadIdx.x;
        const uint32_t vc = b < nblk ? blk[2 * b] : 0u, vh = b < nblk ? blk[2 * b + 1] : 0u;
        uint32_t tc, th;
        const uint32_t ec = block_excl_scan<STR_BT>(vc, s_tmp, &tc);
        const uint32_t eh = block_excl_scan<STR_BT>(vh, s_tmp, &th);
        if (b < nblk) {
            blk[2 * b] = s_carry[0] + ec;
            blk[2 * b + 1] = s_carry[1] + eh;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            s_carry[0] += tc;
            s_carry[1] += th;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        ctl->n_next = s_carry[0];
        ctl->seg_next = s_carry[1];
    }
}

// Pass 3: write the continuing entries (id and place in the full order) and
// the next round's group offsets (closed by the total).
__global__ __launch_bounds__(STR_BT) void k_str_compact(const uint4 *keys, const uint32_t *mark, uint32_t tag,
                                                        uint32_t n_active, const uint32_t *blk, const uint32_t *ids_c,
                                                        const uint32_t *pos_c, uint32_t *ids_n, uint32_t *pos_n,
                                                        uint32_t *seg_n, const StrCtl *ctl) {
    __shared__ uint32_t s_tmp[STR_BT / WAVE];
    const uint32_t c = blockIdx.x * STR_BT + threadIdx.x;
    bool cont, head;
    str_flags(keys, mark, tag, n_active, c, cont, head);
    uint32_t tot;
    const uint32_t oc = blk[2 * blockIdx.x] + block_excl_scan<STR_BT>(cont ? 1u : 0u, s_tmp, &tot);
    const uint32_t oh = blk[2 * blockIdx.x + 1] + block_excl_scan<STR_BT>(head ? 1u : 0u, s_tmp, &tot);
    if (cont) {
        ids_n[oc] = ids_c[c];
        pos_n[oc] = pos_c[c];
    }
    if (head) seg_n[oh] = oc;
    if (blockIdx.x == 0 && threadIdx.x == 0) seg_n[ctl->seg_next] = ctl->n_next;
}

// Start: every string active, in input order, one group (marked for round
// 1); the control word cleared.
__global__ __launch_bounds__(256) void k_str_iota(uint32_t *ids_c, uint32_t *pos_c, uint32_t *mark, uint32_t *seg_c,
                                                  uint32_t n, StrCtl *ctl) {
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
        ids_c[c] = c;
        pos_c[c] = c;
        mark[c] = c == 0 ? 1u : 0u;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        seg_c[0] = 0u;
        seg_c[1] = n;
        ctl->n_next = ctl->seg_next = ctl->error = ctl->pad = 0u;
    }
}

// End: the caller's payload in the sorted order, through the ids.
__global__ __launch_bounds__(256) void k_str_gather(const uint32_t *ids, const uint32_t *pay_in, uint32_t n,
                                                    uint32_t *pay_out) {
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x)
        pay_out[c] = pay_in[ids[c]];
}

__global__ __launch_bounds__(256) void k_str_copy(const uint32_t *src, uint32_t n, uint32_t *dst) {
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) dst[c] = src[c];
}

}  // namespace binar
