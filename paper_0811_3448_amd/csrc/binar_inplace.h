// In-place passes: no scratch copy of the keys.
//
// The paper's partition works inside the array it is given, and the space it
// needs beyond the array does not grow with the data (section "Space
// Analysis").  Its exchange of two keys is not stable; the passes here keep
// the stable order of the scatter passes and still move the keys only within
// the caller's buffer.  One pass over the live segments of list L:
//
//   k_local   every tile of a segment that is partitioned sorts itself
//             stably by the pass digit in LDS and is written back over
//             itself.  Keys of one digit in one tile then sit in one run
//             whose place after the pass is known (bucket base + the
//             digit's count in the segment's earlier tiles), so every key
//             of the run moves by the same distance: one int32 per (tile,
//             digit), in a table that takes the place of the piece prefixes
//             it was computed from.
//   k_cycle   applies the permutation  i -> i + dist[tile(i)][digit(key i)]
//             by following its cycles: a walk carries one key to its place,
//             picks up the key found there and carries that one on (a lane
//             runs several walks side by side).  One claim bit per position
//             makes every key picked up exactly once and every place
//             written exactly once.  With 4-bit digits a tile's runs are
//             long, so neighbouring walks stay together and their accesses
//             coalesce.
//   k_small_pairs  children of 2..SMALL_MAX keys, read straight from the
//             pass's count table and ranked inside a wave (no list).
//
// The extra memory is the per-segment and per-tile tables, 1 bit per key and
// 16 bytes per IP_GRANULE positions: a small fraction of the data.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "binar_kernels.h"

namespace binar {

constexpr uint32_t IP_GRANULE = 256;     // positions per entry of the segment map
constexpr uint32_t IP_NONE = 0xFFFFFFFFu;
// digit bits of the in-place passes: 4 or 8 (template parameter K)
constexpr int IP_BT = 512, IP_ITEMS = 8;  // one tile = 4096 keys
constexpr uint32_t IP_TILE = IP_BT * IP_ITEMS;

// Where position i lies: the segment map holds, for every granule of
// IP_GRANULE positions, the live segment holding its first position and the
// one holding its last, each as (begin, first tile | bit position << 24).  A
// live segment is longer than a granule (T >= IP_GRANULE), so it holds the
// first or the last position of every granule it touches, and a position at
// or after the begin of the second lies in the second.
struct IpMaps {
    int32_t *dist;      // [tile][R]: aliases the piece-prefix table
    uint4 *segmap;      // [granule]: (first-position segment, last-position segment)
    uint32_t *state;    // 1 bit per position: claimed (its first claimer took the key it held)
};

// Clear the state bits and the segment map before a pass.
static __global__ __launch_bounds__(THREADS) void k_ip_clear(IpMaps m, uint32_t nstate, uint32_t nmap) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nstate; i += stride) m.state[i] = 0u;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nmap; i += stride)
        m.segmap[i] = make_uint4(IP_NONE, 0u, IP_NONE, 0u);
}

template <int KB, bool PAY, int K>
struct LocalLds {
    using V = typename KeyT<KB>::V;
    static constexpr int R = 1 << K;
    static constexpr int NW = IP_BT / WAVE;
    V keys[IP_TILE];
    uint32_t pay[PAY ? IP_TILE : 1];
    alignas(8) uint32_t tbl[NW][2 * R];
    uint32_t wh[NW][R];
    uint32_t run[R];   // place after the pass of the next key of digit d in this piece
    uint32_t tmp[NW];
};

// The tiles of list L are cut into gridDim.x chunks exactly as in k_hist, so
// the piece prefixes line up; the grid must be the one k_hist ran with.
template <int KB, bool PAY, int K>
__global__ __launch_bounds__(IP_BT) void k_local(Work w, int L, IpMaps m) {
    using KT = KeyT<KB>;
    using V = typename KT::V;
    constexpr int R = 1 << K;
    constexpr int NW = IP_BT / WAVE;
    __shared__ LocalLds<KB, PAY, K> S;
    Ctl *ctl = w.ctl;
    if (ctl->error | ctl->overflow) return;
    const unsigned long long lc = ctl->list_ctr[L];
    const uint32_t nslots = (uint32_t)(lc >> 32), ntiles = (uint32_t)lc;
    if (ntiles == 0) return;
    const uint32_t per = (ntiles + gridDim.x - 1) / gridDim.x;
    const uint32_t t0 = blockIdx.x * per, t1 = min(ntiles, t0 + per);
    if (t0 >= t1) return;
    const int wv = threadIdx.x / WAVE, lane = lane_id();
    for (int i = threadIdx.x; i < NW * R; i += IP_BT) (&S.wh[0][0])[i] = 0u;
    for (int i = threadIdx.x; i < NW * 2 * R; i += IP_BT) (&S.tbl[0][0])[i] = 0u;
    __syncthreads();

    uint32_t t = t0;
    uint32_t slot = uni(find_slot(w.list[L], nslots, t));
    SegEntry seg = uni(w.list[L][slot]);
    uint32_t seg_end = uni(seg_tile_end(w.list[L], slot, nslots, ntiles));
    bool entered = false;
    const uint32_t ebase = (uint32_t)wv * IP_ITEMS * WAVE + (uint32_t)lane;
    // the next tile of the same segment is loaded (as stored) while the
    // current one is sorted; tiles are disjoint, so its loads may still be
    // in flight while the current tile is written back
    V kn[IP_ITEMS];
    uint32_t pn[IP_ITEMS];
    bool have_next = false;
    auto load_raw = [&](uint32_t tt, V (&kk)[IP_ITEMS], uint32_t (&pp)[IP_ITEMS]) {
        const uint32_t o = (tt - seg.tile_start) * IP_TILE;
        const uint32_t ln = min(IP_TILE, seg.len - o);
        const uint32_t b0 = seg.begin + o;
#pragma unroll
        for (int j = 0; j < IP_ITEMS; ++j) {
            const uint32_t e = ebase + j * WAVE;
            kk[j] = (e < ln) ? KT::load(w.keys[0], (size_t)b0 + e) : KT::zero();
            pp[j] = (PAY && e < ln) ? w.pay[0][b0 + e] : 0u;
        }
    };
    while (t < t1) {
        if (!entered) {
            if (((seg.info >> 16) & SEG_SKIP) || ((seg.info >> 8) & 1u)) {
                // not partitioned this pass (an odd parity never occurs in place)
                if ((seg.info >> 8) & 1u) {
                    if (threadIdx.x == 0) atomicOr(&ctl->error, ERR_INTERNAL);
                }
                t = seg_end;
                if (t >= t1) break;
                ++slot;
                seg = uni(w.list[L][slot]);
                seg_end = uni(seg_tile_end(w.list[L], slot, nslots, ntiles));
                continue;
            }
            if (threadIdx.x < R)
                S.run[threadIdx.x] = w.bases[L][(size_t)slot * R + threadIdx.x] + w.pcnt[(size_t)t * R + threadIdx.x];
            entered = true;
            __syncthreads();
        }
        const uint32_t bitpos = seg.info & 0xFFu;
        const int wbits = min(K, (int)w.nbits - (int)bitpos);
        const uint32_t off = (t - seg.tile_start) * IP_TILE;
        const uint32_t tlen = min(IP_TILE, seg.len - off);
        const uint32_t tb = seg.begin + off;
        if ((size_t)tb + tlen > w.n_total) {
            if (threadIdx.x == 0) atomicOr(&ctl->error, ERR_INTERNAL);
            break;
        }
        V key[IP_ITEMS];
        uint32_t pay[IP_ITEMS], dg[IP_ITEMS], rnk[IP_ITEMS];
        if (have_next) {
#pragma unroll
            for (int j = 0; j < IP_ITEMS; ++j) {
                key[j] = kn[j];
                pay[j] = pn[j];
            }
        } else {
            load_raw(t, key, pay);
        }
        have_next = t + 1 < t1 && t + 1 < seg_end && (size_t)seg.begin + seg.len <= w.n_total;
        if (have_next) load_raw(t + 1, kn, pn);
#pragma unroll
        for (int j = 0; j < IP_ITEMS; ++j) {
            if (w.kind) key[j] = KT::enc(key[j], w.kind);
            dg[j] = KT::digit(key[j], bitpos, wbits);
        }
        wave_rank<R, RANK_GROUP, IP_ITEMS, false>(dg, ebase, tlen, &S.tbl[wv][0], &S.wh[wv][0], rnk);
        __syncthreads();
        uint32_t tcnt = 0;
        if (threadIdx.x < R) {
#pragma unroll
            for (int q = 0; q < NW; ++q) tcnt += S.wh[q][threadIdx.x];
        }
        uint32_t tot;
        const uint32_t dstart = block_excl_scan<IP_BT>(tcnt, S.tmp, &tot);  // every thread: it holds barriers
        if (threadIdx.x < R) {
            uint32_t acc = dstart;
#pragma unroll
            for (int q = 0; q < NW; ++q) {
                const uint32_t x = S.wh[q][threadIdx.x];
                S.wh[q][threadIdx.x] = acc;
                acc += x;
            }
            // a key of digit d at tile position dstart + r goes to run + r;
            // this row was read (as the piece prefix) only by this block
            const uint32_t run = S.run[threadIdx.x];
            m.dist[(size_t)t * R + threadIdx.x] = (int32_t)(run - (tb + dstart));
            S.run[threadIdx.x] = run + tcnt;
        }
        // the segment map for the granules this tile touches
        {
            const uint32_t g0 = tb / IP_GRANULE, g1 = (tb + tlen - 1) / IP_GRANULE;
            const uint32_t sb = seg.begin, se = seg.begin + seg.len;
            const uint32_t inf = seg.tile_start | (bitpos << 24);
            for (uint32_t g = g0 + threadIdx.x; g <= g1; g += IP_BT) {
                const uint32_t first = g * IP_GRANULE, last = first + IP_GRANULE - 1;
                if (first >= sb && first < se) {
                    m.segmap[g].x = sb;
                    m.segmap[g].y = inf;
                }
                if (last >= sb && last < se) {
                    m.segmap[g].z = sb;
                    m.segmap[g].w = inf;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < IP_ITEMS; ++j) {
            const uint32_t e = ebase + j * WAVE;
            if (e < tlen) {
                const uint32_t pos = S.wh[wv][dg[j]] + rnk[j];
                S.keys[pos] = key[j];
                if (PAY) S.pay[pos] = pay[j];
            }
        }
        __syncthreads();
        for (int i = lane; i < R; i += WAVE) S.wh[wv][i] = 0u;
        // every key of the tile is in LDS: write it back over the tile
#pragma unroll
        for (int j = 0; j < IP_ITEMS; ++j) {
            const uint32_t p = j * IP_BT + threadIdx.x;
            if (p < tlen) {
                KT::store(w.keys[0], (size_t)tb + p, raw_key<KB>(S.keys[p], w.kind));
                if (PAY) w.pay[0][tb + p] = S.pay[p];
            }
        }
        __syncthreads();
        ++t;
        if (t == seg_end && t < t1) {
            ++slot;
            seg = uni(w.list[L][slot]);
            seg_end = uni(seg_tile_end(w.list[L], slot, nslots, ntiles));
            entered = false;
        }
    }
}

// Position i's claim bit: the word and the bit.
__device__ __forceinline__ uint32_t *ip_word(uint32_t *state, uint32_t i) { return state + (i >> 5); }
__device__ __forceinline__ uint32_t ip_bit(uint32_t i) { return 1u << (i & 31u); }

// A hardware wait for every memory operation the wave has issued (the
// compiler keeps memory operations on their side of the signal fences).
__device__ __forceinline__ void ip_wait_all() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Claim bit `tgt` for every lane that wants it; the lane that claims it
// first wins.  Neighbouring lanes whose bits share a state word (runs of one
// digit move together, so they mostly do) are served by one atomic, the OR of
// their bits, issued by the last lane of the run; inside the run, lanes count
// as claiming in lane order.  Split in two so that the atomics of several
// walks per lane are in flight together: ip_claim_issue leaves the word's
// old value in the issuing lane, ip_claim_won tells every lane its outcome.
struct IpClaim {
    uint32_t old, earlier;
    int last;
};

__device__ __forceinline__ IpClaim ip_claim_issue(uint32_t *state, uint32_t tgt, bool want) {
    const int lane = lane_id();
    const uint32_t wd = want ? (tgt >> 5) : IP_NONE;
    const uint32_t prev = __shfl_up(wd, 1, WAVE);
    const bool head = want && (lane == 0 || prev != wd);
    const uint64_t heads = __ballot(head) | __ballot(!want);  // a lane that wants nothing is its own run
    const int hd = 63 - __builtin_clzll(heads & (~0ull >> (63 - lane)));
    uint32_t acc = want ? ip_bit(tgt) : 0u;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        const uint32_t y = __shfl_up(acc, o, WAVE);
        if (lane - o >= hd) acc |= y;
    }
    const uint64_t after = (lane == 63) ? 0ull : (heads & (~0ull << (lane + 1)));
    IpClaim c;
    c.last = after ? __builtin_ctzll(after) - 1 : 63;
    // two lanes of a run may want one bit (a start and a carried key's
    // place): the earlier lane is its first claimer
    const uint32_t before = __shfl_up(acc, 1, WAVE);
    c.earlier = (lane > hd) ? before : 0u;
    c.old = 0u;
    if (want && lane == c.last)
        c.old = __hip_atomic_fetch_or(state + (tgt >> 5), acc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return c;
}

__device__ __forceinline__ bool ip_claim_won(const IpClaim &c, uint32_t tgt, bool want) {
    const uint32_t old = __shfl(c.old, c.last, WAVE);
    return want && ((old | c.earlier) & ip_bit(tgt)) == 0u;
}

// Where position i lies, from the segment map entry gm of its granule: the
// tile and the bit position of its segment (t = IP_NONE if the map has no
// segment for it, never expected for a position of a partitioned segment).
struct IpLoc {
    uint32_t t, bitpos;
};

__device__ __forceinline__ IpLoc ip_loc(uint4 gm, uint32_t i) {
    uint32_t b, inf;
    if (gm.z != IP_NONE && i >= gm.z) {
        b = gm.z;
        inf = gm.w;
    } else if (gm.x != IP_NONE) {
        b = gm.x;
        inf = gm.y;
    } else {
        return IpLoc{IP_NONE, 0u};
    }
    return IpLoc{(inf & 0xFFFFFFu) + (i - b) / IP_TILE, inf >> 24};
}

// Every position of every partitioned segment of list L starts a walk once
// (unless a walk has claimed it already).  Per step, every walk has a
// target: a new start, or the place of the key it carries.  It reads the key
// at the target, waits for the read, then claims the target; after the claim
// has returned it puts its carried key (if any) down there.  The first
// claimer of a place goes on with the key it read; any other claimer's walk
// ends.  Why that is exact: every place is claimed first exactly once, and
// the key its first claimer read is the one that was there at the start -- a
// place is only written after its writer's claim has returned, and every
// claim of a place but the first comes after the first claim, which was
// issued after the first claimer's read had returned.  Each place receives
// its key once (from the unique carrier of that key), and no lane ever waits
// for another.
//
// Each lane runs NS walks side by side (their reads, claims and writes in
// flight together), and the distance of a picked-up key is loaded right
// after its claim, so a step waits for three memory round trips: distance,
// read, claim.
template <int KB, bool PAY, int NS, int K>
__global__ __launch_bounds__(THREADS) void k_cycle(Work w, int L, IpMaps m) {
    using KT = KeyT<KB>;
    using V = typename KT::V;
    constexpr uint32_t R = 1u << K;
    Ctl *ctl = w.ctl;
    if (ctl->error | ctl->overflow) return;
    const unsigned long long lc = ctl->list_ctr[L];
    const uint32_t nslots = (uint32_t)(lc >> 32), ntiles = (uint32_t)lc;
    if (ntiles == 0) return;
    const uint32_t wave_id = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const uint32_t nwaves = gridDim.x * (blockDim.x / WAVE);

    bool carry[NS];
    V x[NS];                 // carried key (as stored)
    uint32_t px[NS], src[NS];
    int32_t dist[NS];        // carried key's distance to its place
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        carry[q] = false;
        x[q] = KT::zero();
        px[q] = src[q] = 0u;
        dist[q] = 0;
    }
    uint32_t t = wave_id;    // this wave's next tile of start positions
    uint32_t cur = 0u, tb = 0u, tlen = 0u;
    bool tiles_left = true;
    for (;;) {
        // the next tile with start positions left
        while (tiles_left && cur >= tlen) {
            if (t >= ntiles) {
                tiles_left = false;
                break;
            }
            const uint32_t slot = uni(find_slot(w.list[L], nslots, t));
            const SegEntry seg = uni(w.list[L][slot]);
            if (((seg.info >> 16) & SEG_SKIP) || ((seg.info >> 8) & 1u)) {
                t += nwaves;
                continue;
            }
            const uint32_t off = (t - seg.tile_start) * IP_TILE;
            tb = seg.begin + off;
            tlen = min(IP_TILE, seg.len - off);
            cur = 0u;
            t += nwaves;
        }
        bool any = false;
#pragma unroll
        for (int q = 0; q < NS; ++q) any = any || carry[q];
        if (!tiles_left && __ballot(any) == 0ull) break;  // no start left, nothing carried
        // targets: idle walks take consecutive start positions
        uint32_t tgt[NS];
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            tgt[q] = IP_NONE;
            const bool idle = !carry[q];
            const uint64_t idle_m = __ballot(idle);
            if (idle) {
                const uint32_t r = cur + lanes_below(idle_m);
                if (tiles_left && r < tlen) tgt[q] = tb + r;
            } else {
                tgt[q] = (uint32_t)((int32_t)src[q] + dist[q]);
                if (tgt[q] >= w.n_total) {
                    atomicOr(&ctl->error, ERR_INTERNAL);
                    carry[q] = false;
                    tgt[q] = IP_NONE;
                }
            }
            if (tiles_left) cur += (uint32_t)__builtin_popcountll(idle_m);
        }
        // read every target, its segment map entry and, for a start, whether
        // a walk has claimed it already
        V y[NS];
        uint32_t py[NS], claimed[NS];
        uint4 gm[NS];
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            y[q] = KT::zero();
            py[q] = claimed[q] = 0u;
            gm[q] = make_uint4(IP_NONE, 0u, IP_NONE, 0u);
            if (tgt[q] != IP_NONE) {
                y[q] = KT::load(w.keys[0], tgt[q]);
                if (PAY) py[q] = w.pay[0][tgt[q]];
                gm[q] = m.segmap[tgt[q] / IP_GRANULE];
                if (!carry[q])
                    claimed[q] = __hip_atomic_load(ip_word(m.state, tgt[q]), __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        ip_wait_all();
        IpClaim c[NS];
        bool want[NS];
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            want[q] = tgt[q] != IP_NONE && !(claimed[q] & ip_bit(tgt[q]));
            c[q] = ip_claim_issue(m.state, tgt[q], want[q]);
        }
        bool won[NS];
#pragma unroll
        for (int q = 0; q < NS; ++q) won[q] = ip_claim_won(c[q], tgt[q], want[q]);
        ip_wait_all();
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            if (carry[q]) {
                KT::store(w.keys[0], tgt[q], x[q]);
                if (PAY) w.pay[0][tgt[q]] = px[q];
            }
            carry[q] = won[q];
            if (won[q]) {
                x[q] = y[q];
                px[q] = py[q];
                src[q] = tgt[q];
                const IpLoc loc = ip_loc(gm[q], tgt[q]);
                if (loc.t == IP_NONE) {
                    atomicOr(&ctl->error, ERR_INTERNAL);
                    carry[q] = false;
                } else {
                    const int wbits = min(K, (int)w.nbits - (int)loc.bitpos);
                    const uint32_t d = KT::digit(w.kind ? KT::enc(y[q], w.kind) : y[q], (int)loc.bitpos, wbits);
                    dist[q] = m.dist[(size_t)loc.t * R + d];
                }
            }
        }
    }
}

// Children of 2..SMALL_MAX keys of the segments partitioned with list L,
// taken from its count and base tables: each wave takes 64 (segment, digit)
// pairs at a time and ranks the small ones, packed into its lanes, in place.
template <int KB, bool PAY, int K>
__global__ __launch_bounds__(THREADS) void k_small_pairs(Work w, int L) {
    using KT = KeyT<KB>;
    using V = typename KT::V;
    constexpr uint32_t R = 1u << K;
    Ctl *ctl = w.ctl;
    if (ctl->error | ctl->overflow) return;
    const unsigned long long lc = ctl->list_ctr[L];
    const uint32_t nslots = (uint32_t)(lc >> 32);
    if (nslots == 0) return;
    const uint32_t npairs = nslots * R;
    const int lane = lane_id();
    const uint32_t wave_id = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const uint32_t nwaves = gridDim.x * (blockDim.x / WAVE);
    const Canon km = canon_lead_mask((int)w.nbits);
    // (k_plan counts these children: per-wave counter atomics serialise)
    for (uint32_t e0 = wave_id * WAVE; e0 < npairs; e0 += nwaves * WAVE) {
        const uint32_t e = e0 + lane;
        uint32_t b = 0u, len = 0u;
        if (e < npairs) {
            const SegEntry seg = w.list[L][e / R];
            const bool moved = !((seg.info >> 16) & SEG_SKIP) && !((seg.info >> 8) & 1u);
            const uint32_t c = moved ? w.counts[L][e] : 0u;
            if (c >= 2u && c <= SMALL_MAX) {
                b = w.bases[L][e];
                len = c;
                if (b < seg.begin || b - seg.begin + c > seg.len) {
                    atomicOr(&ctl->error, ERR_INTERNAL);
                    len = 0u;
                }
            }
        }
        wave_pack(len, [&](int l, uint32_t i, int head, bool act, uint32_t el, uint32_t ml) {
            const uint32_t eb = __shfl(b, l, WAVE);
            V k = KT::zero();
            uint32_t pv = 0u;
            if (act) {
                k = ld_key<KB>(w.keys[0], (size_t)eb + i, w.kind);
                if constexpr (PAY) pv = w.pay[0][eb + i];
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
