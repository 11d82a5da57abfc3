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
#include "binar_inplace.h"
#include "binar_kernels.h"
#include "binar_strings.h"

namespace binar {
namespace {

constexpr size_t ALIGN = 256;

// Text of the last HIP failure seen on this thread (binar_last_error).
thread_local char t_err[192];

int hip_fail(const char *what, hipError_t e) {
    std::snprintf(t_err, sizeof(t_err), "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
    return BINAR_EDEVICE;
}

#define BINAR_HIP_TRY(call)                                   \
    do {                                                      \
        const hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return hip_fail(#call, e_);     \
    } while (0)

size_t align_up(size_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

// The digit count streams keys at full bandwidth: big blocks, so that even one
// block per CU (the 8192-key tile grid) keeps enough loads in flight.
constexpr int HIST_BT = 1024;

// LDS-finish classes per key width: (threads per block, keys per thread);
// capacities 1024, 3072, 5120, 8192 keys (16-byte keys: 1024, 2048, 3072,
// 5120).  The finish is bound by LDS work: 256-thread blocks let several
// independent blocks share a CU, so one block's loads and stores overlap
// another's LDS passes.  Where even a 256-thread block is alone on its CU
// (the largest class of 8- and 16-byte keys), 512 threads keep more waves.
template <int KB>
struct FinShape;
template <>
struct FinShape<4> {
    static constexpr int bt[NCLASS] = {256, 256, 256, 256};
    static constexpr int items[NCLASS] = {4, 12, 20, 32};
};
template <>
struct FinShape<8> {
    static constexpr int bt[NCLASS] = {256, 256, 256, 512};
    static constexpr int items[NCLASS] = {4, 12, 20, 16};
};
template <>
struct FinShape<16> {
    static constexpr int bt[NCLASS] = {256, 256, 256, 512};
    static constexpr int items[NCLASS] = {4, 8, 12, 10};
};

uint32_t fin_cap(uint32_t kb, int c) {
    switch (kb) {
        case 4: return (uint32_t)(FinShape<4>::bt[c] * FinShape<4>::items[c]);
        case 8: return (uint32_t)(FinShape<8>::bt[c] * FinShape<8>::items[c]);
        default: return (uint32_t)(FinShape<16>::bt[c] * FinShape<16>::items[c]);
    }
}

// Scatter tiles: (threads per block, keys per thread) per tile size.
template <int TILE>
struct ScatterShape;
template <>
struct ScatterShape<2048> {
    static constexpr int BT = 256, ITEMS = 8;
};
template <>
struct ScatterShape<4096> {
    static constexpr int BT = 512, ITEMS = 8;
};
template <>
struct ScatterShape<8192> {
    static constexpr int BT = 1024, ITEMS = 8;
};

struct Resolved {
    uint32_t kb, k, tile, T, nbits, kind;
    bool pay;
    bool lookback;
    bool inplace = false;
};

struct Layout {
    size_t ctl, list[2], counts[2], bases[2], andor[2], desc[2], pcnt, status, fin[NCLASS], fin_small, cpy, keys_b,
        pay_b, segmap, state, total;
    uint32_t nmap, nstate;  // in place: segment-map entries and state words
    uint32_t max_big, max_tiles, max_fin[NCLASS], fin_cap[NCLASS], max_small, max_cpy;
};

binar_params g_defaults[3][2];  // [kb index][has payload]
std::mutex g_mu;

int kb_index(uint32_t kb) { return kb == 4 ? 0 : (kb == 8 ? 1 : 2); }

bool valid_kb(uint32_t kb) { return kb == 4 || kb == 8 || kb == 16; }

bool supported_k(uint32_t k) { return k == 1 || (k >= 4 && k <= 8); }

bool supported_tile(uint32_t t) { return t == 2048 || t == 4096 || t == 8192; }

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
    if (!d.tile_keys) d.tile_keys = (kb == 4 && d.digit_bits == 8) ? 8192 : 4096;
    if (!d.offsets) d.offsets = 1;
    const uint32_t tmax = fin_cap(kb, NCLASS - 1);
    if (!d.finish_max) d.finish_max = tmax;
    if (!supported_k(d.digit_bits) || !supported_tile(d.tile_keys) || d.offsets > 2) return BINAR_EINVAL;
    if (d.tile_keys == 8192 && (kb != 4 || d.digit_bits != 8)) return BINAR_EINVAL;
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

Layout make_layout(const Resolved &r, uint64_t n) {
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
std::vector<const void *> g_last_ws;  // per device: workspace of the last call

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
    if ((int)g_last_ws.size() <= dev) g_last_ws.resize(dev + 1, nullptr);
    g_last_ws[dev] = ws;
}

// Blocks each kernel keeps resident per CU (cached per kernel).
struct OccCache {
    std::mutex mu;
    std::vector<std::pair<const void *, int>> v;
    int get(const void *fn, int block) {
        std::lock_guard<std::mutex> lk(mu);
        for (auto &e : v)
            if (e.first == fn) return e.second;
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, fn, block, 0) != hipSuccess || b < 1) {
            (void)hipGetLastError();
            b = 1;
        }
        v.emplace_back(fn, b);
        return b;
    }
} g_occ;

int g_cus = 0;
int cu_count() {
    if (!g_cus) {
        int dev = 0, c = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && c > 0)
            g_cus = c;
        else
            g_cus = 256;
    }
    return g_cus;
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
    w.keys[0] = keys;
    w.keys[1] = r.inplace ? nullptr : ws + L.keys_b;
    w.pay[0] = pay;
    w.pay[1] = (r.pay && !r.inplace) ? reinterpret_cast<uint32_t *>(ws + L.pay_b) : nullptr;
    return w;
}

// ---------------------------------------------------------------- profiler
// Optional launch timing: an event pair on the launch stream around every
// kernel, read back by binar_profile_read.
struct Prof {
    std::mutex mu;
    bool on = false;
    struct Rec {
        hipEvent_t a, b;
        char name[32];
        int pass;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> spare;

    hipEvent_t ev() {
        if (!spare.empty()) {
            hipEvent_t e = spare.back();
            spare.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
} g_prof;

// Set while this thread captures a launch sequence into a graph: no timing
// events are recorded into graphs.
thread_local bool t_capturing = false;

struct Timed {
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    const char *name;
    int pass;
    Timed(hipStream_t s, const char *n, int p) : st(s), name(n), pass(p) {
        if (t_capturing) return;
        std::lock_guard<std::mutex> lk(g_prof.mu);
        if (!g_prof.on) return;
        a = g_prof.ev();
        b = g_prof.ev();
        if (a && b) (void)hipEventRecord(a, st);
    }
    ~Timed() {
        std::lock_guard<std::mutex> lk(g_prof.mu);
        if (!a || !b) return;
        (void)hipEventRecord(b, st);
        Prof::Rec r;
        r.a = a;
        r.b = b;
        std::snprintf(r.name, sizeof(r.name), "%s", name);
        r.pass = pass;
        g_prof.recs.push_back(r);
    }
};

template <typename F>
uint32_t grid_for(F fn, uint32_t work_items, int block = THREADS) {
    const uint32_t per_cu = (uint32_t)g_occ.get(reinterpret_cast<const void *>(fn), block);
    const uint32_t g = (uint32_t)cu_count() * per_cu;
    return std::max(1u, std::min(g, work_items));
}

template <int KB, bool PAY, int C>
void launch_finish(const Work &w, const Layout &L, hipStream_t st) {
    constexpr int BT = FinShape<KB>::bt[C], IT = FinShape<KB>::items[C];
    if (!L.max_fin[C]) return;
    static const char *names[NCLASS] = {"k_finish0", "k_finish1", "k_finish2", "k_finish3"};
    Timed tm(st, names[C], -1);
    hipLaunchKernelGGL((k_finish<KB, BT, IT, PAY>), dim3(grid_for(k_finish<KB, BT, IT, PAY>, L.max_fin[C], BT)),
                       dim3(BT), 0, st, w, C);
}

// The smallest class (up to FW_CAP keys) is finished one sub-array per wave
// for 4- and 8-byte keys.  16-byte keys keep a workgroup per sub-array: a
// wave's 16 keys per lane take 64 registers and the occupancy halves (the
// 2^24-string sort measured 2.43 ms against 2.29).
template <int KB, bool PAY>
void launch_finish_wave(const Work &w, const Layout &L, hipStream_t st) {
    if constexpr (KB == 16) {
        launch_finish<KB, PAY, 0>(w, L, st);
    } else {
        static_assert(FinShape<KB>::bt[0] * FinShape<KB>::items[0] == FW_CAP, "class 0 is the wave finish");
        if (!L.max_fin[0]) return;
        constexpr int NWB = FinWaves<KB>::n;
        Timed tm(st, "k_finish0", -1);
        const uint32_t blocks = (L.max_fin[0] + NWB - 1) / NWB;
        hipLaunchKernelGGL((k_finish_wave<KB, PAY>), dim3(grid_for(k_finish_wave<KB, PAY>, blocks, NWB * WAVE)),
                           dim3(NWB * WAVE), 0, st, w, 0);
    }
}

template <int KB, int K, int TILE, bool PAY, bool LB>
int enqueue(Work w, const Layout &L, const uint32_t *seg_off, uint32_t nseg, uint32_t n, hipStream_t st) {
    constexpr int SBT = ScatterShape<TILE>::BT, SIT = ScatterShape<TILE>::ITEMS;
    constexpr int R = 1 << K;
    const int passes = ((int)w.nbits + K - 1) / K;
    {
        Timed tm(st, "k_reset", -1);
        hipLaunchKernelGGL(k_reset, dim3(1), dim3(THREADS), 0, st, w.ctl);
    }
    const uint32_t ig = std::max(1u, std::min(1024u, (nseg + THREADS - 1) / THREADS));
    {
        Timed tm(st, "k_init", -1);
        hipLaunchKernelGGL(k_init<R>, dim3(ig), dim3(THREADS), 0, st, w, seg_off, nseg, n, n);
    }
    // the chunked scatter and the digit count share one grid: it fixes the
    // pieces whose prefixes k_pscan computes
    const uint32_t sg = grid_for(k_scatter<KB, K, SBT, SIT, PAY, LB>, L.max_tiles, SBT);
    w.chunk_grid = sg;
    const uint32_t hg = sg;
    const uint32_t pg = std::max(1u, std::min(L.max_big, 1024u));
    constexpr uint32_t NG = (R < 32) ? 1u : (uint32_t)R / 32u;
    const uint32_t qg = std::max(1u, std::min(L.max_big * NG, 2048u));
    for (int j = 0; j < passes; ++j) {
        const int Lc = j & 1;
        {
            Timed tm(st, "k_hist", j);
            hipLaunchKernelGGL((k_hist<KB, K, LB, HIST_BT>), dim3(hg), dim3(HIST_BT), 0, st, w, Lc);
        }
        {
            Timed tm(st, "k_pscan", j);
            hipLaunchKernelGGL((k_pscan<K>), dim3(qg), dim3(THREADS), 0, st, w, Lc);
        }
        {
            Timed tm(st, "k_plan", j);
            hipLaunchKernelGGL((k_plan<KB, K>), dim3(pg), dim3(THREADS), 0, st, w, Lc, j);
        }
        {
            Timed tm(st, "k_scatter", j);
            hipLaunchKernelGGL((k_scatter<KB, K, SBT, SIT, PAY, LB>), dim3(sg), dim3(SBT), 0, st, w, Lc);
        }
    }
    {
        Timed tm(st, "k_copyback", -1);
        hipLaunchKernelGGL((k_copyback<KB, PAY>), dim3(grid_for(k_copyback<KB, PAY>, L.max_cpy)), dim3(THREADS), 0,
                           st, w);
    }
    if (L.max_small) {
        Timed tm(st, "k_finish_small", -1);
        // one wave per 64 list entries, at most what fits the device at once
        const uint32_t waves = (L.max_small + WAVE - 1) / WAVE;
        hipLaunchKernelGGL((k_finish_small<KB, PAY>),
                           dim3(grid_for(k_finish_small<KB, PAY>, (waves + WAVES - 1) / WAVES)), dim3(THREADS), 0,
                           st, w);
    }
    launch_finish_wave<KB, PAY>(w, L, st);
    launch_finish<KB, PAY, 1>(w, L, st);
    launch_finish<KB, PAY, 2>(w, L, st);
    launch_finish<KB, PAY, 3>(w, L, st);
    BINAR_HIP_TRY(hipGetLastError());
    return BINAR_OK;
}

template <int KB, bool PAY>
int dispatch_k(const Resolved &r, const Work &w, const Layout &L, const uint32_t *so, uint32_t ns,
               uint32_t n, hipStream_t st) {
#define BINAR_CASE(KK, TT)                                                  \
    if (r.k == KK && r.tile == TT)                                          \
        return r.lookback ? enqueue<KB, KK, TT, PAY, true>(w, L, so, ns, n, st) \
                          : enqueue<KB, KK, TT, PAY, false>(w, L, so, ns, n, st);
    if constexpr (KB == 4) {
        BINAR_CASE(8, 8192)  // wider keys: 8192 of them do not fit in LDS
    }
    BINAR_CASE(8, 4096)
    BINAR_CASE(8, 2048)
    BINAR_CASE(7, 4096)
    BINAR_CASE(6, 4096)
    BINAR_CASE(5, 4096)
    BINAR_CASE(4, 4096)
    BINAR_CASE(4, 2048)
    BINAR_CASE(1, 4096)
    BINAR_CASE(1, 2048)
#undef BINAR_CASE
    return BINAR_EINVAL;
}

int dispatch(const Resolved &r, const Work &w, const Layout &L, const uint32_t *so, uint32_t ns, uint32_t n,
             hipStream_t st) {
    switch (r.kb) {
        case 4:
            return r.pay ? dispatch_k<4, true>(r, w, L, so, ns, n, st) : dispatch_k<4, false>(r, w, L, so, ns, n, st);
        case 8:
            return r.pay ? dispatch_k<8, true>(r, w, L, so, ns, n, st) : dispatch_k<8, false>(r, w, L, so, ns, n, st);
        case 16:
            return r.pay ? dispatch_k<16, true>(r, w, L, so, ns, n, st)
                         : dispatch_k<16, false>(r, w, L, so, ns, n, st);
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
    const Layout L = make_layout(r, n);
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
constexpr int IP_WALKS = 4;  // walks per lane in the cycle walk

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

template <int KB, bool PAY, int K>
int enqueue_inplace(Work w, const Layout &L, char *ws, uint32_t n, hipStream_t st) {
    constexpr int R = 1 << K;
    const int passes = ((int)w.nbits + K - 1) / K;
    IpMaps m;
    m.dist = reinterpret_cast<int32_t *>(w.pcnt);  // each row replaces the piece prefix it came from
    m.segmap = reinterpret_cast<uint4 *>(ws + L.segmap);
    m.state = reinterpret_cast<uint32_t *>(ws + L.state);
    {
        Timed tm(st, "k_reset", -1);
        hipLaunchKernelGGL(k_reset, dim3(1), dim3(THREADS), 0, st, w.ctl);
    }
    {
        Timed tm(st, "k_init", -1);
        hipLaunchKernelGGL(k_init<R>, dim3(1), dim3(THREADS), 0, st, w, nullptr, 1u, n, n);
    }
    // the local sort and the digit count share one grid: it fixes the pieces
    const uint32_t lg = grid_for(k_local<KB, PAY, K>, L.max_tiles, IP_BT);
    w.chunk_grid = lg;
    const uint32_t pg = std::max(1u, std::min(L.max_big, 1024u));
    constexpr uint32_t NG = (R < 32) ? 1u : (uint32_t)R / 32u;
    const uint32_t qg = std::max(1u, std::min(L.max_big * NG, 2048u));
    const uint32_t cg = grid_for(k_cycle<KB, PAY, IP_WALKS, K>, L.max_tiles);
    const uint32_t clr = grid_for(k_ip_clear, (L.nstate + THREADS - 1) / THREADS);
    const uint32_t spg = grid_for(k_small_pairs<KB, PAY, K>, (L.max_big * (uint32_t)R + THREADS - 1) / THREADS);
    for (int j = 0; j < passes; ++j) {
        const int Lc = j & 1;
        {
            Timed tm(st, "k_hist", j);
            hipLaunchKernelGGL((k_hist<KB, K, false, HIST_BT>), dim3(lg), dim3(HIST_BT), 0, st, w, Lc);
        }
        {
            Timed tm(st, "k_pscan", j);
            hipLaunchKernelGGL((k_pscan<K>), dim3(qg), dim3(THREADS), 0, st, w, Lc);
        }
        {
            Timed tm(st, "k_plan", j);
            hipLaunchKernelGGL((k_plan<KB, K>), dim3(pg), dim3(THREADS), 0, st, w, Lc, j);
        }
        {
            Timed tm(st, "k_ip_clear", j);
            hipLaunchKernelGGL(k_ip_clear, dim3(clr), dim3(THREADS), 0, st, m, L.nstate, L.nmap);
        }
        {
            Timed tm(st, "k_local", j);
            hipLaunchKernelGGL((k_local<KB, PAY, K>), dim3(lg), dim3(IP_BT), 0, st, w, Lc, m);
        }
        {
            Timed tm(st, "k_cycle", j);
            hipLaunchKernelGGL((k_cycle<KB, PAY, IP_WALKS, K>), dim3(cg), dim3(THREADS), 0, st, w, Lc, m);
        }
        {
            Timed tm(st, "k_small_pairs", j);
            hipLaunchKernelGGL((k_small_pairs<KB, PAY, K>), dim3(spg), dim3(THREADS), 0, st, w, Lc);
        }
    }
    {
        Timed tm(st, "k_finish_small", -1);
        hipLaunchKernelGGL((k_finish_small<KB, PAY>), dim3(1), dim3(THREADS), 0, st, w);
    }
    launch_finish_wave<KB, PAY>(w, L, st);
    launch_finish<KB, PAY, 1>(w, L, st);
    launch_finish<KB, PAY, 2>(w, L, st);
    launch_finish<KB, PAY, 3>(w, L, st);
    BINAR_HIP_TRY(hipGetLastError());
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
#define BINAR_IP(KK)                                                                                   \
    switch (kb) {                                                                                      \
        case 4:                                                                                        \
            return payload ? enqueue_inplace<4, true, KK>(w, L, b, (uint32_t)n, st)                  \
                           : enqueue_inplace<4, false, KK>(w, L, b, (uint32_t)n, st);                \
        case 8:                                                                                        \
            return payload ? enqueue_inplace<8, true, KK>(w, L, b, (uint32_t)n, st)                  \
                           : enqueue_inplace<8, false, KK>(w, L, b, (uint32_t)n, st);                \
        default:                                                                                       \
            return payload ? enqueue_inplace<16, true, KK>(w, L, b, (uint32_t)n, st)                 \
                           : enqueue_inplace<16, false, KK>(w, L, b, (uint32_t)n, st);               \
    }
    if (r.k == 4) {
        BINAR_IP(4)
    }
    BINAR_IP(8)
#undef BINAR_IP
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
    S.inner_bytes = make_layout(r, n < 2 ? 2 : n).total;
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
    return (dev < (int)g_last_ws.size()) ? g_last_ws[dev] : nullptr;
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
    p->L = make_layout(p->r, p->max_keys);
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
    // the offsets against it, so one graph serves every batch on them
    if (seg_offsets) n_total = p->max_keys;
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
    (void)num_segments;
    if (!valid_kb(key_bytes) || n > BINAR_MAX_KEYS) return 0;
    Resolved r;
    if (resolve(key_bytes, has_payload != 0, params, &r)) return 0;
    return make_layout(r, n).total;
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
