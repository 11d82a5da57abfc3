// Host side of libbinar.so: argument checks, scratch layout, kernel
// sequence, the C ABI declared in include/binar.h.
//
// Enqueue sequence of one call (all on the caller's stream, no host sync):
//   k_reset, k_init, then for every possible global pass j < ceil(bits / k):
//   k_hist, k_plan, k_scatter (each exits at once when its list is empty),
//   then k_finish for each LDS size class.  The sequence is fixed for a
//   given (key width, k, n, segment count), so it can be captured in a HIP
//   graph; the number of passes that do work depends on the data.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "binar.h"
#include "binar_host.h"
#include "binar_strings.h"

namespace binar {

// Text of the last HIP failure seen on this thread (binar_last_error).
thread_local char t_err[192];

int hip_fail(const char *what, hipError_t e) {
    std::snprintf(t_err, sizeof(t_err), "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
    return BINAR_EDEVICE;
}

OccCache g_occ;
Prof g_prof;
thread_local bool t_capturing = false;

int cu_count() {
    static int cus = 0;
    if (!cus) {
        int dev = 0, c = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && c > 0)
            cus = c;
        else
            cus = 256;
    }
    return cus;
}

namespace {

binar_params g_defaults[3][2];  // [kb index][has payload]
std::mutex g_mu;

int kb_index(uint32_t kb) { return kb == 4 ? 0 : (kb == 8 ? 1 : 2); }

bool valid_kb(uint32_t kb) { return kb == 4 || kb == 8 || kb == 16; }

bool supported_k(uint32_t k) { return k == 1 || (k >= 4 && k <= 8); }

bool supported_tile(uint32_t t) { return t == 2048 || t == 4096 || t == 6144 || t == 8192; }

// Effective parameters: the nonzero fields of p over the defaults d, then
// the built-in choices for what is still zero.
int resolve_over(uint32_t kb, bool pay, binar_params d, const binar_params *p, Resolved *r) {
    if (p) {
        if (p->digit_bits) d.digit_bits = p->digit_bits;
        if (p->tile_keys) d.tile_keys = p->tile_keys;
        if (p->finish_max) d.finish_max = p->finish_max;
        if (p->offsets) d.offsets = p->offsets;
    }
    if (!d.digit_bits) d.digit_bits = 8;
    if (!d.tile_keys) d.tile_keys = (d.digit_bits != 8) ? 4096 : (kb == 4) ? 8192 : (kb == 8) ? 6144 : 4096;
    if (!d.offsets) d.offsets = 1;
    const uint32_t tmax = fin_cap(kb, NCLASS - 1);
    if (!d.finish_max) d.finish_max = tmax;
    if (!supported_k(d.digit_bits) || !supported_tile(d.tile_keys) || d.offsets > 2) return BINAR_EINVAL;
    if (d.tile_keys == 8192 && (kb != 4 || d.digit_bits != 8)) return BINAR_EINVAL;
    if (d.tile_keys == 6144 && (kb != 8 || d.digit_bits != 8)) return BINAR_EINVAL;
    if (d.tile_keys == 2048 && d.digit_bits > 4 && d.digit_bits < 8) return BINAR_EINVAL;
    const uint32_t nbits = (p && p->key_bits) ? p->key_bits : 8u * kb;
    if (nbits > 8u * kb) return BINAR_EINVAL;
    // the key kind belongs to the call, never to the defaults
    const uint32_t kind = p ? p->key_kind : 0u;
    if (kind > KIND_FLOAT || (kind != KIND_UNSIGNED && kb == 16)) return BINAR_EINVAL;
    r->nbits = nbits;
    r->kind = kind;
    r->kb = kb;
    r->k = d.digit_bits;
    r->tile = d.tile_keys;
    r->T = std::min(std::max(d.finish_max, 1u), tmax);
    r->pay = pay;
    r->lookback = d.offsets == 2;
    return BINAR_OK;
}

int resolve(uint32_t kb, bool pay, const binar_params *p, Resolved *r) {
    binar_params d;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        d = g_defaults[kb_index(kb)][pay ? 1 : 0];
    }
    return resolve_over(kb, pay, d, p, r);
}

Layout make_layout(const Resolved &r, uint64_t n, bool single = true) {
    Layout L{};
    const uint32_t R = 1u << r.k;
    L.max_big = (uint32_t)(n / (r.T + 1ull) + 1ull);
    L.max_tiles = (uint32_t)(n / r.tile + L.max_big + 1ull);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    L.ctl = take(sizeof(Ctl));
    for (int i = 0; i < 2; ++i) {
        L.list[i] = take((size_t)L.max_big * sizeof(SegEntry));
        L.counts[i] = take((size_t)L.max_big * R * 4);
        L.bases[i] = take((size_t)L.max_big * R * 4);
        L.andor[i] = take((size_t)L.max_big * 32);
        L.desc[i] = take((size_t)L.max_big * 4);
    }
    L.pcnt = take((size_t)L.max_tiles * R * 4);
    L.status = take(r.lookback ? (size_t)L.max_tiles * R * 4 : 0);
    // sub-arrays of 2 .. SMALL_MAX keys go to the small list, longer ones up
    // to T to the smallest LDS class that holds them; in place, only the
    // caller's array can be listed there (small children of a pass are
    // ranked from its count table)
    L.max_small = (r.T >= 2u) ? (r.inplace ? 1u : (uint32_t)(n / 2ull + 1ull)) : 0u;
    L.fin_small = take((size_t)L.max_small * sizeof(FinEntry));
    uint32_t prev = SMALL_MAX;
    for (int c = 0; c < NCLASS; ++c) {
        L.fin_cap[c] = fin_cap(r.kb, c);
        L.max_fin[c] = (prev >= r.T) ? 0u : (uint32_t)(n / (prev + 1ull) + 1ull);
        L.fin[c] = take((size_t)L.max_fin[c] * sizeof(FinEntry));
        prev = L.fin_cap[c];
    }
    // copy-back runs: each is bounded by a child that is not finished (two
    // or more keys) or by its parent's end
    L.max_cpy = r.inplace ? 1u : (uint32_t)(n / 2 + L.max_big + 2);
    L.cpy = take((size_t)L.max_cpy * sizeof(CopyEntry));
    L.keys_b = take(r.inplace ? 0 : (size_t)n * r.kb);
    L.pay_b = take((r.pay && !r.inplace) ? (size_t)n * 4 : 0);
    L.nmap = r.inplace ? (uint32_t)(n / IP_GRANULE + 2) : 0u;
    L.nstate = r.inplace ? (uint32_t)(n / 32 + 2) : 0u;
    L.segmap = take((size_t)L.nmap * sizeof(uint4));
    L.state = take((size_t)L.nstate * 4);
    // pass 0's digit-pair counts (one array of at least PAIR_MIN_KEYS keys):
    // a row per digit-count block (at most two per compute unit) and the sum
    L.pair_rows = (single && !r.inplace && !r.lookback && r.k >= 4 && n >= PAIR_MIN_KEYS)
                      ? (uint32_t)(2 * cu_count())
                      : 0u;
    const size_t pair_words = ((size_t)R * R) / 2;
    L.pair_part = take((size_t)L.pair_rows * pair_words * 4);
    L.pair_sum = take(L.pair_rows ? (size_t)R * R * 4 : 0);
    L.total = off;
    return L;
}

// ------------------------------------------------------------- device pool
struct Pool {
    void *ptr = nullptr;
    size_t bytes = 0;
};
std::mutex g_pool_mu;
std::vector<Pool> g_pools;
constexpr int MAX_WS_DEVICES = 64;
const void *g_last_ws[MAX_WS_DEVICES];  // per device: workspace of the last call

int pool_get(int dev, size_t bytes, void **out) {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    if ((int)g_pools.size() <= dev) g_pools.resize(dev + 1);
    Pool &p = g_pools[dev];
    if (p.bytes < bytes) {
        if (p.ptr) {
            BINAR_HIP_TRY(hipDeviceSynchronize());
            BINAR_HIP_TRY(hipFree(p.ptr));
            p.ptr = nullptr;
            p.bytes = 0;
        }
        void *q = nullptr;
        if (hipMalloc(&q, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return BINAR_ENOMEM;
        }
        p.ptr = q;
        p.bytes = bytes;
    }
    *out = p.ptr;
    return BINAR_OK;
}

void note_ws(int dev, const void *ws) {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    if (dev >= 0 && dev < MAX_WS_DEVICES) g_last_ws[dev] = ws;
}

Work make_work(const Layout &L, const Resolved &r, char *ws, void *keys, uint32_t *pay, uint32_t n_total) {
    Work w{};
    w.ctl = reinterpret_cast<Ctl *>(ws + L.ctl);
    for (int i = 0; i < 2; ++i) {
        w.list[i] = reinterpret_cast<SegEntry *>(ws + L.list[i]);
        w.counts[i] = reinterpret_cast<uint32_t *>(ws + L.counts[i]);
        w.bases[i] = reinterpret_cast<uint32_t *>(ws + L.bases[i]);
        w.andor[i] = reinterpret_cast<unsigned long long *>(ws + L.andor[i]);
        w.desc[i] = reinterpret_cast<uint32_t *>(ws + L.desc[i]);
    }
    w.pcnt = reinterpret_cast<uint32_t *>(ws + L.pcnt);
    w.status = reinterpret_cast<uint32_t *>(ws + L.status);
    for (int c = 0; c < NCLASS; ++c) {
        w.fin[c] = reinterpret_cast<FinEntry *>(ws + L.fin[c]);
        w.fin_cap[c] = L.fin_cap[c];
        w.max_fin[c] = L.max_fin[c];
    }
    w.fin_small = reinterpret_cast<FinEntry *>(ws + L.fin_small);
    w.max_small = L.max_small;
    w.cpy = reinterpret_cast<CopyEntry *>(ws + L.cpy);
    w.max_cpy = L.max_cpy;
    w.max_big = L.max_big;
    w.max_tiles = L.max_tiles;
    w.finish_max = r.T;
    w.tile_keys = r.tile;
    w.nbits = r.nbits;
    w.kind = r.kind;
    w.inplace = r.inplace ? 1u : 0u;
    w.n_total = n_total;
    w.pair_rows = L.pair_rows;
    w.pair_part = reinterpret_cast<uint32_t *>(ws + L.pair_part);
    w.pair_sum = reinterpret_cast<uint32_t *>(ws + L.pair_sum);
    w.keys[0] = keys;
    w.keys[1] = r.inplace ? nullptr : ws + L.keys_b;
    w.pay[0] = pay;
    w.pay[1] = (r.pay && !r.inplace) ? reinterpret_cast<uint32_t *>(ws + L.pay_b) : nullptr;
    return w;
}

int dispatch(const Resolved &r, const Work &w, const Layout &L, const uint32_t *so, uint32_t ns, uint32_t n,
             hipStream_t st) {
    switch (r.kb) {
        case 4: return r.pay ? launch_sort<4, true>(r, w, L, so, ns, n, st) : launch_sort<4, false>(r, w, L, so, ns, n, st);
        case 8: return r.pay ? launch_sort<8, true>(r, w, L, so, ns, n, st) : launch_sort<8, false>(r, w, L, so, ns, n, st);
        case 16:
            return r.pay ? launch_sort<16, true>(r, w, L, so, ns, n, st) : launch_sort<16, false>(r, w, L, so, ns, n, st);
    }
    return BINAR_EINVAL;
}

int check_buffers(void *keys, uint32_t kb, uint32_t *payload) {
    if (keys == nullptr) return BINAR_EINVAL;
    if (kb == 16 && (reinterpret_cast<uintptr_t>(keys) & 15u)) return BINAR_EINVAL;
    if ((reinterpret_cast<uintptr_t>(keys) & 3u) || (reinterpret_cast<uintptr_t>(payload) & 3u))
        return BINAR_EINVAL;
    if (kb == 8 && (reinterpret_cast<uintptr_t>(keys) & 7u)) return BINAR_EINVAL;
    return BINAR_OK;
}

int run(void *keys, uint32_t kb, uint64_t n, uint32_t *payload, const uint32_t *seg_off, uint32_t nseg,
        const binar_params *params, hipStream_t st, void *ws, size_t ws_bytes) {
    if (!valid_kb(kb)) return BINAR_EINVAL;
    if (n > BINAR_MAX_KEYS) return BINAR_ERANGE;
    if (seg_off == nullptr && n < 2) return BINAR_OK;  // base case: nothing to order
    if (seg_off != nullptr && nseg == 0) return BINAR_OK;
    if (int rc = check_buffers(keys, kb, payload)) return rc;
    Resolved r;
    int rc = resolve(kb, payload != nullptr, params, &r);
    if (rc) return rc;
    const Layout L = make_layout(r, n, seg_off == nullptr);
    int dev = 0;
    BINAR_HIP_TRY(hipGetDevice(&dev));
    if (ws) {
        if (ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) & (ALIGN - 1))) return BINAR_ENOMEM;
    } else {
        rc = pool_get(dev, L.total, &ws);
        if (rc) return rc;
    }
    note_ws(dev, ws);
    (void)hipGetLastError();  // a stale error of earlier, unrelated HIP calls is not ours
    const Work w = make_work(L, r, static_cast<char *>(ws), keys, payload, (uint32_t)n);
    return dispatch(r, w, L, seg_off, seg_off ? nseg : 1u, (uint32_t)n, st);
}

// ------------------------------------------------------------ in place
// Parameters of the in-place passes: 4- or 8-bit digits (default IP_K_DEFAULT),
// 4096-key tiles, chunked piece prefixes, and T at least a segment-map
// granule.
constexpr uint32_t IP_K_DEFAULT = 4;

int resolve_inplace(uint32_t kb, bool pay, const binar_params *p, Resolved *r) {
    if (p && ((p->digit_bits && p->digit_bits != 4u && p->digit_bits != 8u) ||
              (p->tile_keys && p->tile_keys != IP_TILE) || p->offsets == 2))
        return BINAR_EINVAL;
    const uint32_t k = (p && p->digit_bits) ? p->digit_bits : IP_K_DEFAULT;
    binar_params d;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        d = g_defaults[kb_index(kb)][pay ? 1 : 0];
    }
    d.digit_bits = k;
    d.tile_keys = IP_TILE;
    d.offsets = 1;
    binar_params q = p ? *p : binar_params{};
    q.digit_bits = 0;
    q.tile_keys = 0;
    q.offsets = 0;
    if (int rc = resolve_over(kb, pay, d, p ? &q : nullptr, r)) return rc;
    r->T = std::max(r->T, IP_GRANULE);
    r->inplace = true;
    return BINAR_OK;
}

int run_inplace(void *keys, uint32_t kb, uint64_t n, uint32_t *payload, const binar_params *params, hipStream_t st,
                void *ws, size_t ws_bytes) {
    if (!valid_kb(kb)) return BINAR_EINVAL;
    if (n > BINAR_MAX_KEYS) return BINAR_ERANGE;
    if (n < 2) return BINAR_OK;  // base case: nothing to order
    if (int rc = check_buffers(keys, kb, payload)) return rc;
    Resolved r;
    int rc = resolve_inplace(kb, payload != nullptr, params, &r);
    if (rc) return rc;
    const Layout L = make_layout(r, n);
    if (L.max_tiles >= (1u << 24)) return BINAR_ERANGE;  // tile numbers share a word with the bit position
    int dev = 0;
    BINAR_HIP_TRY(hipGetDevice(&dev));
    if (ws) {
        if (ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) & (ALIGN - 1))) return BINAR_ENOMEM;
    } else {
        rc = pool_get(dev, L.total, &ws);
        if (rc) return rc;
    }
    note_ws(dev, ws);
    (void)hipGetLastError();
    char *b = static_cast<char *>(ws);
    const Work w = make_work(L, r, b, keys, payload, (uint32_t)n);
    switch (kb) {
        case 4: return r.pay ? launch_inplace<4, true>(r, w, L, b, (uint32_t)n, st)
                             : launch_inplace<4, false>(r, w, L, b, (uint32_t)n, st);
        case 8: return r.pay ? launch_inplace<8, true>(r, w, L, b, (uint32_t)n, st)
                             : launch_inplace<8, false>(r, w, L, b, (uint32_t)n, st);
        default: return r.pay ? launch_inplace<16, true>(r, w, L, b, (uint32_t)n, st)
                              : launch_inplace<16, false>(r, w, L, b, (uint32_t)n, st);
    }
}

// ------------------------------------------------------------ strings
struct StrLayout {
    size_t ctl, ids, ids_c, pos_c, ids_n, pos_n, seg_c, seg_n, mark, blk, keys, inner, inner_bytes, total;
};

StrLayout str_layout(uint64_t n) {
    StrLayout S{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    const size_t nblk = (n + STR_BT - 1) / STR_BT + 1;
    S.ctl = take(sizeof(StrCtl));
    S.ids = take(4 * n);
    S.ids_c = take(4 * n);
    S.pos_c = take(4 * n);
    S.ids_n = take(4 * n);
    S.pos_n = take(4 * n);
    S.seg_c = take(4 * (n + 2));
    S.seg_n = take(4 * (n + 2));
    S.mark = take(4 * n);
    S.blk = take(8 * nblk);
    S.keys = take(16 * n);
    Resolved r;
    (void)resolve(16, true, nullptr, &r);
    S.inner_bytes = make_layout(r, n < 2 ? 2 : n, false).total;  // the inner sorts are segmented
    S.inner = take(S.inner_bytes);
    S.total = off;
    return S;
}

uint32_t grid1d(uint64_t n) { return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, 4096)); }

int sort_strings(const uint8_t *bytes, uint64_t nbytes, const uint32_t *offs, uint64_t n, uint32_t *payload,
                 hipStream_t st, void *ws, size_t ws_bytes) {
    if (n > BINAR_MAX_KEYS) return BINAR_ERANGE;
    if (n < 2) return BINAR_OK;  // base case
    if (!offs || !payload || (!bytes && nbytes)) return BINAR_EINVAL;
    const StrLayout L = str_layout(n);
    int dev = 0;
    BINAR_HIP_TRY(hipGetDevice(&dev));
    if (ws) {
        if (ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) & (ALIGN - 1))) return BINAR_ENOMEM;
    } else if (int rc = pool_get(dev, L.total, &ws)) {
        return rc;
    }
    (void)hipGetLastError();
    char *b = static_cast<char *>(ws);
    StrCtl *ctl = reinterpret_cast<StrCtl *>(b + L.ctl);
    uint32_t *ids = reinterpret_cast<uint32_t *>(b + L.ids);
    uint32_t *ids_c = reinterpret_cast<uint32_t *>(b + L.ids_c), *ids_n = reinterpret_cast<uint32_t *>(b + L.ids_n);
    uint32_t *pos_c = reinterpret_cast<uint32_t *>(b + L.pos_c), *pos_n = reinterpret_cast<uint32_t *>(b + L.pos_n);
    uint32_t *seg_c = reinterpret_cast<uint32_t *>(b + L.seg_c), *seg_n = reinterpret_cast<uint32_t *>(b + L.seg_n);
    uint32_t *mark = reinterpret_cast<uint32_t *>(b + L.mark);
    uint32_t *blk = reinterpret_cast<uint32_t *>(b + L.blk);
    uint8_t *keys = reinterpret_cast<uint8_t *>(b + L.keys);
    void *inner = b + L.inner;
    const uint32_t nn = (uint32_t)n;
    hipLaunchKernelGGL(k_str_iota, dim3(grid1d(n)), dim3(256), 0, st, ids_c, pos_c, mark, seg_c, nn, ctl);
    uint32_t n_active = nn, nseg = 1, depth = 0, round = 1;
    for (;;) {
        hipLaunchKernelGGL(k_str_keys, dim3(grid1d(n_active)), dim3(256), 0, st, bytes, nbytes, offs, nn, ids_c,
                           n_active, depth, keys, ctl);
        BINAR_HIP_TRY(hipGetLastError());
        if (int rc = run(keys, 16, n_active, ids_c, seg_c, nseg, nullptr, st, inner, L.inner_bytes)) return rc;
        hipLaunchKernelGGL(k_str_place, dim3(grid1d(n_active)), dim3(256), 0, st, ids_c, pos_c, n_active, ids);
        if (round > 1)
            hipLaunchKernelGGL(k_str_mark, dim3(grid1d(nseg)), dim3(256), 0, st, seg_c, nseg, mark, round);
        const uint32_t nblk = (n_active + STR_BT - 1) / STR_BT;
        hipLaunchKernelGGL(k_str_count, dim3(nblk), dim3(STR_BT), 0, st, reinterpret_cast<const uint4 *>(keys), mark,
                           round, n_active, blk);
        hipLaunchKernelGGL(k_str_scan, dim3(1), dim3(STR_BT), 0, st, blk, nblk, ctl);
        BINAR_HIP_TRY(hipGetLastError());
        // the totals decide whether a next round exists: the compaction runs
        // only if it does
        StrCtl h{};
        BINAR_HIP_TRY(hipMemcpyAsync(&h, ctl, sizeof(h), hipMemcpyDeviceToHost, st));
        BINAR_HIP_TRY(hipStreamSynchronize(st));
        if (h.error) return BINAR_EINVAL;
        if (h.n_next == 0) break;
        hipLaunchKernelGGL(k_str_compact, dim3(nblk), dim3(STR_BT), 0, st, reinterpret_cast<const uint4 *>(keys),
                           mark, round, n_active, blk, ids_c, pos_c, ids_n, pos_n, seg_n, ctl);
        BINAR_HIP_TRY(hipGetLastError());
        std::swap(ids_c, ids_n);
        std::swap(pos_c, pos_n);
        std::swap(seg_c, seg_n);
        n_active = h.n_next;
        nseg = h.seg_next;
        depth += STR_WIN;
        ++round;
    }
    // the payload follows the ids: copy it aside, then gather
    hipLaunchKernelGGL(k_str_copy, dim3(grid1d(n)), dim3(256), 0, st, payload, nn, ids_n);
    hipLaunchKernelGGL(k_str_gather, dim3(grid1d(n)), dim3(256), 0, st, ids, ids_n, nn, payload);
    BINAR_HIP_TRY(hipGetLastError());
    BINAR_HIP_TRY(hipStreamSynchronize(st));
    return BINAR_OK;
}

const void *last_ws(int dev) {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    return (dev >= 0 && dev < MAX_WS_DEVICES) ? g_last_ws[dev] : nullptr;
}

}  // namespace
}  // namespace binar

// ------------------------------------------------------------------- plans
struct binar_plan {
    int dev = 0;
    binar::Resolved r{};
    binar::Layout L{};
    uint64_t max_keys = 0;
    uint32_t max_segments = 0;
    void *ws = nullptr;
    hipStream_t cap = nullptr;  // capture stream (never runs work)
    struct Graph {
        void *keys;
        uint32_t *pay;
        const uint32_t *off;
        uint32_t nseg;
        uint64_t n;
        hipGraph_t g;
        hipGraphExec_t ge;
    };
    std::vector<Graph> graphs;
};

namespace {
void plan_free(binar_plan *p) {
    for (auto &g : p->graphs) {
        (void)hipGraphExecDestroy(g.ge);
        (void)hipGraphDestroy(g.g);
    }
    p->graphs.clear();
    if (p->cap) (void)hipStreamDestroy(p->cap);
    if (p->ws) (void)hipFree(p->ws);
    delete p;
}
}  // namespace

extern "C" {

int binar_plan_create(binar_plan **out, uint32_t key_bytes, uint64_t max_keys, uint32_t max_segments,
                      int has_payload, const binar_params *params) {
    using namespace binar;
    if (!out) return BINAR_EINVAL;
    *out = nullptr;
    if (!valid_kb(key_bytes) || max_segments == 0) return BINAR_EINVAL;
    if (max_keys > BINAR_MAX_KEYS) return BINAR_ERANGE;
    binar_plan *p = new (std::nothrow) binar_plan();
    if (!p) return BINAR_ENOMEM;
    int rc = resolve(key_bytes, has_payload != 0, params, &p->r);
    if (rc) {
        delete p;
        return rc;
    }
    p->max_keys = max_keys < 2 ? 2 : max_keys;
    p->max_segments = max_segments;
    p->L = make_layout(p->r, p->max_keys, max_segments == 1u);
    if (const hipError_t e = hipGetDevice(&p->dev)) {
        delete p;
        return hip_fail("hipGetDevice", e);
    }
    if (hipMalloc(&p->ws, p->L.total) != hipSuccess) {
        (void)hipGetLastError();
        p->ws = nullptr;
        plan_free(p);
        return BINAR_ENOMEM;
    }
    if (const hipError_t e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking)) {
        plan_free(p);
        return hip_fail("hipStreamCreateWithFlags", e);
    }
    *out = p;
    return BINAR_OK;
}

int binar_plan_sort(binar_plan *p, void *keys, uint32_t *payload, const uint32_t *seg_offsets,
                    uint32_t num_segments, uint64_t n_total, void *stream) {
    using namespace binar;
    if (!p) return BINAR_EINVAL;
    if (n_total > p->max_keys) return BINAR_ERANGE;
    if (seg_offsets ? (num_segments == 0 || num_segments > p->max_segments) : false) return BINAR_EINVAL;
    if ((payload != nullptr) != p->r.pay) return BINAR_EINVAL;
    if (!seg_offsets && n_total < 2) return BINAR_OK;
    if (int rc = check_buffers(keys, p->r.kb, payload)) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const uint32_t nseg = seg_offsets ? num_segments : 1u;
    // segmented: the buffers hold the plan's capacity and the device checks
    // the offsets against it, so one graph serves every batch on them; a
    // caller whose buffers are shorter than that capacity is refused, since
    // a table within the capacity could then reach past them
    if (seg_offsets) {
        if (n_total < p->max_keys) return BINAR_EINVAL;
        n_total = p->max_keys;
    }
    (void)hipGetLastError();  // a stale error of earlier, unrelated HIP calls is not ours
    for (auto &g : p->graphs)
        if (g.keys == keys && g.pay == payload && g.off == seg_offsets && g.nseg == nseg && g.n == n_total) {
            note_ws(p->dev, p->ws);
            BINAR_HIP_TRY(hipGraphLaunch(g.ge, st));
            return BINAR_OK;
        }
    // capture the launch sequence once for these buffers
    Work w = make_work(p->L, p->r, static_cast<char *>(p->ws), keys, payload, (uint32_t)n_total);
    BINAR_HIP_TRY(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
    t_capturing = true;
    int rc = dispatch(p->r, w, p->L, seg_offsets, nseg, (uint32_t)n_total, p->cap);
    t_capturing = false;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(p->cap, &g);
    if (rc || e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return rc ? rc : hip_fail("hipStreamEndCapture", e != hipSuccess ? e : hipErrorUnknown);
    }
    hipGraphExec_t ge = nullptr;
    if (const hipError_t ei = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0)) {
        (void)hipGraphDestroy(g);
        return hip_fail("hipGraphInstantiate", ei);
    }
    if (p->graphs.size() >= 16) {
        (void)hipGraphExecDestroy(p->graphs.front().ge);
        (void)hipGraphDestroy(p->graphs.front().g);
        p->graphs.erase(p->graphs.begin());
    }
    p->graphs.push_back(binar_plan::Graph{keys, payload, seg_offsets, nseg, n_total, g, ge});
    note_ws(p->dev, p->ws);
    BINAR_HIP_TRY(hipGraphLaunch(ge, st));
    return BINAR_OK;
}

int binar_plan_stats(binar_plan *p, void *stream, binar_stats *out) {
    if (!p) return BINAR_EINVAL;
    return binar_stats_read(p->ws, stream, out);
}

int binar_plan_status_async(const binar_plan *p, void *stream, uint32_t *host_words) {
    using namespace binar;
    if (!p || !host_words) return BINAR_EINVAL;
    // error and overflow are adjacent words of the control block
    static_assert(offsetof(Ctl, overflow) == offsetof(Ctl, error) + 4, "status words must be adjacent");
    const char *src = static_cast<const char *>(p->ws) + p->L.ctl + offsetof(Ctl, error);
    BINAR_HIP_TRY(hipMemcpyAsync(host_words, src, 8, hipMemcpyDeviceToHost, static_cast<hipStream_t>(stream)));
    return BINAR_OK;
}

int binar_plan_graphs(const binar_plan *p) { return p ? (int)p->graphs.size() : 0; }

size_t binar_plan_workspace_bytes(const binar_plan *p) { return p ? p->L.total : 0; }

void binar_plan_destroy(binar_plan *p) {
    if (p) plan_free(p);
}

}  // extern "C"

using namespace binar;

extern "C" {

int binar_sort_ex(void *keys, uint32_t key_bytes, uint64_t n, uint32_t *payload, const uint32_t *seg_offsets,
                  uint32_t num_segments, const binar_params *params, void *stream, void *workspace,
                  size_t workspace_bytes) {
    return run(keys, key_bytes, n, payload, seg_offsets, num_segments, params,
               static_cast<hipStream_t>(stream), workspace, workspace_bytes);
}

int binar_sort_async(void *keys, uint32_t key_bytes, uint64_t n, uint32_t *payload, void *stream,
                     void *workspace, size_t workspace_bytes) {
    return run(keys, key_bytes, n, payload, nullptr, 0, nullptr, static_cast<hipStream_t>(stream), workspace,
               workspace_bytes);
}

int binar_sort_segmented(void *keys, uint32_t key_bytes, const uint32_t *seg_offsets, uint32_t num_segments,
                         uint64_t n_total, uint32_t *payload, void *stream, void *workspace,
                         size_t workspace_bytes) {
    if (seg_offsets == nullptr && num_segments > 0) return BINAR_EINVAL;
    return run(keys, key_bytes, n_total, payload, seg_offsets, num_segments, nullptr,
               static_cast<hipStream_t>(stream), workspace, workspace_bytes);
}

int binar_sort(void *keys, uint32_t key_bytes, uint64_t n, uint32_t *payload) {
    int rc = run(keys, key_bytes, n, payload, nullptr, 0, nullptr, nullptr, nullptr, 0);
    if (rc) return rc;
    if (n < 2) return BINAR_OK;
    binar_stats st;
    rc = binar_stats_read(nullptr, nullptr, &st);
    return rc ? rc : st.status;
}

size_t binar_workspace_bytes(uint32_t key_bytes, uint64_t n, int has_payload, uint32_t num_segments,
                             const binar_params *params) {
    if (!valid_kb(key_bytes) || n > BINAR_MAX_KEYS) return 0;
    Resolved r;
    if (resolve(key_bytes, has_payload != 0, params, &r)) return 0;
    return make_layout(r, n, num_segments <= 1u).total;
}

int binar_stats_read(const void *workspace, void *stream, binar_stats *out) {
    if (!out) return BINAR_EINVAL;
    std::memset(out, 0, sizeof(*out));
    int dev = 0;
    BINAR_HIP_TRY(hipGetDevice(&dev));
    const void *ws = workspace ? workspace : last_ws(dev);
    if (!ws) return BINAR_EINVAL;
    BINAR_HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    Ctl c;
    BINAR_HIP_TRY(hipMemcpy(&c, ws, sizeof(Ctl), hipMemcpyDeviceToHost));
    for (int j = 0; j < MAX_PASSES; ++j) {
        out->moved[j] = c.moved[j];
        out->hist_keys[j] = c.hist_keys[j];
    }
    for (int k = 0; k < NCLASS; ++k) {
        out->finish_class_keys[k] = c.fin_keys[k];
        out->finish_class_segments[k] = c.fin_segs[k];
        out->finish_keys += c.fin_keys[k];
        out->finish_segments += c.fin_segs[k];
    }
    out->finish_small_keys = c.small_keys;
    out->finish_small_segments = c.small_segs;
    out->finish_keys += c.small_keys;
    out->finish_segments += c.small_segs;
    out->passes = c.passes;
    out->copyback_keys = c.cpy_keys;
    out->sorted_keys = c.sorted_keys;
    out->status = (c.error & ERR_SEGMENTS) ? BINAR_EINVAL
                  : ((c.error & ERR_INTERNAL) || c.overflow) ? BINAR_EDEVICE : BINAR_OK;
    return BINAR_OK;
}

int binar_resolve_params(uint32_t key_bytes, int has_payload, const binar_params *params, binar_params *out) {
    if (!valid_kb(key_bytes) || !out) return BINAR_EINVAL;
    Resolved r;
    int rc = resolve(key_bytes, has_payload != 0, params, &r);
    if (rc) return rc;
    std::memset(out, 0, sizeof(*out));
    out->digit_bits = r.k;
    out->tile_keys = r.tile;
    out->finish_max = r.T;
    out->offsets = r.lookback ? 2u : 1u;
    out->key_bits = r.nbits;
    out->key_kind = r.kind;
    return BINAR_OK;
}

int binar_get_default_params(uint32_t key_bytes, int has_payload, binar_params *out) {
    return binar_resolve_params(key_bytes, has_payload, nullptr, out);
}

int binar_set_default_params(uint32_t key_bytes, int has_payload, const binar_params *p) {
    if (!valid_kb(key_bytes) || !p) return BINAR_EINVAL;
    binar_params d = *p;
    d.key_bits = 0;  // the defaults always sort whole keys
    d.key_kind = 0;  // and say nothing about how keys are read
    Resolved r;
    if (int rc = resolve_over(key_bytes, has_payload != 0, d, nullptr, &r)) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    g_defaults[kb_index(key_bytes)][has_payload ? 1 : 0] = d;
    return BINAR_OK;
}

int binar_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.on = on != 0;
    if (!g_prof.on) {
        for (auto &r : g_prof.recs) {
            g_prof.spare.push_back(r.a);
            g_prof.spare.push_back(r.b);
        }
        g_prof.recs.clear();
    }
    return BINAR_OK;
}

int binar_profile_read(binar_launch_time *out, uint32_t cap, uint32_t *count) {
    if (!count || (!out && cap)) return BINAR_EINVAL;
    std::lock_guard<std::mutex> lk(g_prof.mu);
    uint32_t k = 0;
    int rc = BINAR_OK;
    for (auto &r : g_prof.recs) {
        if (k < cap) {
            float ms = 0.f;
            hipError_t e = hipEventSynchronize(r.b);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
            if (e != hipSuccess) rc = hip_fail("binar_profile_read", e);
            std::memcpy(out[k].name, r.name, sizeof(out[k].name));
            out[k].pass = r.pass;
            out[k].ms = ms;
            ++k;
        }
        g_prof.spare.push_back(r.a);
        g_prof.spare.push_back(r.b);
    }
    g_prof.recs.clear();
    *count = k;
    return rc;
}

const char *binar_last_error(void) { return binar::t_err; }

int binar_sort_inplace(void *keys, uint32_t key_bytes, uint64_t n, uint32_t *payload, const binar_params *params,
                       void *stream, void *workspace, size_t workspace_bytes) {
    return binar::run_inplace(keys, key_bytes, n, payload, params, static_cast<hipStream_t>(stream), workspace,
                              workspace_bytes);
}

size_t binar_inplace_workspace_bytes(uint32_t key_bytes, uint64_t n, int has_payload, const binar_params *params) {
    using namespace binar;
    if (!valid_kb(key_bytes) || n > BINAR_MAX_KEYS) return 0;
    Resolved r;
    if (resolve_inplace(key_bytes, has_payload != 0, params, &r)) return 0;
    return make_layout(r, n).total;
}

size_t binar_strings_workspace_bytes(uint64_t n) {
    if (n > BINAR_MAX_KEYS) return 0;
    return binar::str_layout(n).total;
}

int binar_sort_strings(const uint8_t *bytes, uint64_t nbytes, const uint32_t *offsets, uint64_t n, uint32_t *payload,
                       void *stream, void *workspace, size_t workspace_bytes) {
    return binar::sort_strings(bytes, nbytes, offsets, n, payload, static_cast<hipStream_t>(stream), workspace,
                               workspace_bytes);
}

const char *binar_strerror(int status) {
    switch (status) {
        case BINAR_OK:
            return "ok";
        case BINAR_EINVAL:
            return "invalid argument (key width, pointer, alignment, tuning knob or segment table)";
        case BINAR_ERANGE:
            return "too many keys: the limit is 2^30 - 1";
        case BINAR_ENOMEM:
            return "workspace too small or device memory exhausted";
        case BINAR_EDEVICE:
            return "HIP runtime error";
    }
    return "unknown status";
}

}  // extern "C"
