// Host-side pieces shared by the library's translation units: launch
// shapes, resolved parameters, scratch layout, launch timing and the
// enqueue sequences of the fixed-width and in-place sorts.  The sequences
// are templates over key width, digit width and tile; each key width is
// instantiated per key width and payload in translation units of their own
// (binar_launch_<kb><p|k>.hip) so that they compile in parallel.
#pragma once

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

namespace binar {

constexpr size_t ALIGN = 256;

// Text of the last HIP failure seen on this thread (binar_last_error).
extern thread_local char t_err[192];

int hip_fail(const char *what, hipError_t e);

#define BINAR_HIP_TRY(call)                                   \
    do {                                                      \
        const hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return hip_fail(#call, e_);     \
    } while (0)

inline size_t align_up(size_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

// The digit count streams keys at full bandwidth: big blocks, so that even one
// block per CU (the 8192-key tile grid) keeps enough loads in flight.
constexpr int HIST_BT = 1024;

// LDS-finish classes per key width: (threads per block, keys per thread);
// capacities 1024, 2048, 5120, 8192 keys (8-byte keys: 1024, 2304, 5120,
// 8192; 16-byte keys: 1024, 2048, 3072, 5120).  The finish is bound by LDS
// work: 256-thread blocks let several independent blocks share a CU, so one
// block's loads and stores overlap another's LDS passes.  Where even a
// 256-thread block is alone on its CU (the largest class of 8- and 16-byte
// keys), 512 threads keep more waves.  The second class of 8-byte keys
// holds 2304 (40 KiB of LDS: four blocks a CU), which takes the 2048-key
// sub-arrays that two 8-bit passes leave of 2^27 uniform keys; that of
// 4-byte keys holds 2048 (28 KiB: five blocks a CU).
template <int KB>
struct FinShape;
template <>
struct FinShape<4> {
    static constexpr int bt[NCLASS] = {256, 256, 256, 256};
    static constexpr int items[NCLASS] = {4, 8, 20, 32};
};
template <>
struct FinShape<8> {
    static constexpr int bt[NCLASS] = {256, 256, 256, 512};
    static constexpr int items[NCLASS] = {4, 9, 20, 16};
};
template <>
struct FinShape<16> {
    static constexpr int bt[NCLASS] = {256, 256, 256, 512};
    static constexpr int items[NCLASS] = {4, 8, 12, 10};
};

inline uint32_t fin_cap(uint32_t kb, int c) {
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
struct ScatterShape<6144> {
    static constexpr int BT = 768, ITEMS = 8;
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
        pay_b, segmap, state, pair_part, pair_sum, total;
    uint32_t nmap, nstate;  // in place: segment-map entries and state words
    uint32_t max_big, max_tiles, max_fin[NCLASS], fin_cap[NCLASS], max_small, max_cpy;
    uint32_t pair_rows;     // rows of pass 0's pair counts (0: the next pass counts its own digits)
};

// One array of at least this many keys counts digit pairs in its first
// pass, so that the second reads no key for its counts (below it the pair
// rows cost more than the read they save).
constexpr uint64_t PAIR_MIN_KEYS = 1ull << 26;

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
};
extern OccCache g_occ;

// Compute units of the current device (256 on MI355X).
int cu_count();

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
};
extern Prof g_prof;

// Set while this thread captures a launch sequence into a graph: no timing
// events are recorded into graphs.
extern thread_local bool t_capturing;

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
    // digit pairs in the first pass: one array (no segment table), chunk
    // offsets, a pair row for every digit-count block, two passes or more
    const bool pairs = !LB && K >= 4 && seg_off == nullptr && nseg == 1u && L.pair_rows != 0u && hg <= L.pair_rows &&
                       passes >= 2;
    if (!pairs) w.pair_rows = 0u;
    for (int j = 0; j < passes; ++j) {
        const int Lc = j & 1;
        {
            Timed tm(st, "k_hist", j);
            if (j == 0 && pairs) {
                if constexpr (!LB && K >= 4)
                    hipLaunchKernelGGL((k_hist<KB, K, false, HIST_BT, true>), dim3(hg), dim3(HIST_BT), 0, st, w, Lc,
                                       j);
            } else {
                hipLaunchKernelGGL((k_hist<KB, K, LB, HIST_BT, false>), dim3(hg), dim3(HIST_BT), 0, st, w, Lc, j);
            }
        }
        if (j == 0 && pairs) {
            Timed tm(st, "k_pair_sum", j);
            constexpr uint32_t words = (1u << K) * (1u << K) / 2u;
            hipLaunchKernelGGL(k_pair_sum<K>, dim3(std::max(1u, std::min(1024u, words / THREADS))), dim3(THREADS), 0,
                               st, w);
        }
        {
            Timed tm(st, "k_pscan", j);
            hipLaunchKernelGGL((k_pscan<K>), dim3(qg), dim3(THREADS), 0, st, w, Lc, j);
        }
        {
            Timed tm(st, "k_plan", j);
            hipLaunchKernelGGL((k_plan<KB, K>), dim3(pg), dim3(THREADS), 0, st, w, Lc, j);
        }
        {
            Timed tm(st, "k_scatter", j);
            hipLaunchKernelGGL((k_scatter<KB, K, SBT, SIT, PAY, LB>), dim3(sg), dim3(SBT), 0, st, w, Lc, j);
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
    if constexpr (KB == 8) {
        BINAR_CASE(8, 6144)  // the most 8-byte keys a 1024-thread tile stages in LDS
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

// Walks per lane in the in-place cycle walk.
constexpr int IP_WALKS = 4;

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
            hipLaunchKernelGGL((k_hist<KB, K, false, HIST_BT, false>), dim3(lg), dim3(HIST_BT), 0, st, w, Lc, j);
        }
        {
            Timed tm(st, "k_pscan", j);
            hipLaunchKernelGGL((k_pscan<K>), dim3(qg), dim3(THREADS), 0, st, w, Lc, j);
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

// Enqueue of one fixed-width sort (all global passes, the copy-back and
// the finish) for key width KB, with or without payload, with the digit
// width and tile of r; and of one in-place sort.  Each (KB, PAY) pair is
// instantiated in binar_launch_<KB><p|k>.hip.
template <int KB, bool PAY>
int launch_sort(const Resolved &r, const Work &w, const Layout &L, const uint32_t *so, uint32_t ns, uint32_t n,
                hipStream_t st) {
    return dispatch_k<KB, PAY>(r, w, L, so, ns, n, st);
}

template <int KB, bool PAY>
int launch_inplace(const Resolved &r, const Work &w, const Layout &L, char *ws, uint32_t n, hipStream_t st) {
    return r.k == 4 ? enqueue_inplace<KB, PAY, 4>(w, L, ws, n, st) : enqueue_inplace<KB, PAY, 8>(w, L, ws, n, st);
}

#define BINAR_EXTERN_LAUNCH(KB, PAY)                                                                        \
    extern template int launch_sort<KB, PAY>(const Resolved &, const Work &, const Layout &, const uint32_t *, \
                                             uint32_t, uint32_t, hipStream_t);                              \
    extern template int launch_inplace<KB, PAY>(const Resolved &, const Work &, const Layout &, char *, uint32_t, \
                                                hipStream_t);
BINAR_EXTERN_LAUNCH(4, true)
BINAR_EXTERN_LAUNCH(4, false)
BINAR_EXTERN_LAUNCH(8, true)
BINAR_EXTERN_LAUNCH(8, false)
BINAR_EXTERN_LAUNCH(16, true)
BINAR_EXTERN_LAUNCH(16, false)
#undef BINAR_EXTERN_LAUNCH

}  // namespace binar
