/*
 * CPU baselines for the benchmark -- TEST INFRASTRUCTURE ONLY.
 *
 * Two reference timings beside the oracle, used by the benchmark's
 * CPU-baseline leg and checked against the oracle by the tests.  They share
 * no code with the GPU library.
 *
 *   ref_stable_sort    : std::stable_sort of (key, payload) pairs on one
 *                        thread: a library comparison sort, stable, so its
 *                        result is the oracle's (section "Sorting
 *                        Formalism" with the stability tie-break).
 *   ref_parallel_binar : the paper's parallel variant (section "Algorithm
 *                        Variants": sub-arrays left by a partition are
 *                        independent and can be sorted by separate
 *                        processors): one stable partition on the leading
 *                        8 bits (a counting pass), then the 256 buckets
 *                        sorted by the oracle's binar sort on `threads`
 *                        threads, each taking the next unsorted bucket.
 *
 * Keys: 4- or 8-byte unsigned integers (native little-endian) or 16-byte
 * strings in memcmp order; payload (may be NULL) uint32, moved with its key.
 */
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

extern "C" int binar_sort_ref(void *keys, uint32_t key_bytes, uint64_t n, uint32_t *payload, uint64_t *bit_steps);

namespace {

template <int KB>
struct Rec {
    uint8_t k[KB];
    uint32_t p;
};

template <int KB>
bool key_less(const uint8_t *a, const uint8_t *b) {
    if (KB == 4) {
        uint32_t x, y;
        std::memcpy(&x, a, 4);
        std::memcpy(&y, b, 4);
        return x < y;
    }
    if (KB == 8) {
        uint64_t x, y;
        std::memcpy(&x, a, 8);
        std::memcpy(&y, b, 8);
        return x < y;
    }
    return std::memcmp(a, b, 16) < 0;
}

template <int KB>
int stable_sort_kb(uint8_t *keys, uint64_t n, uint32_t *payload) {
    std::vector<Rec<KB>> v(n);
    for (uint64_t i = 0; i < n; ++i) {
        std::memcpy(v[i].k, keys + i * KB, KB);
        v[i].p = payload ? payload[i] : 0u;
    }
    std::stable_sort(v.begin(), v.end(),
                     [](const Rec<KB> &a, const Rec<KB> &b) { return key_less<KB>(a.k, b.k); });
    for (uint64_t i = 0; i < n; ++i) {
        std::memcpy(keys + i * KB, v[i].k, KB);
        if (payload) payload[i] = v[i].p;
    }
    return 0;
}

// leading byte of a key in the sort order: the most significant byte of an
// integer, byte 0 of a string
template <int KB>
uint32_t lead_byte(const uint8_t *k) {
    return (KB == 16) ? k[0] : k[KB - 1];
}

template <int KB>
int parallel_kb(uint8_t *keys, uint64_t n, uint32_t *payload, int threads) {
    // stable counting partition on the leading byte
    uint64_t cnt[257] = {0};
    for (uint64_t i = 0; i < n; ++i) ++cnt[lead_byte<KB>(keys + i * KB) + 1];
    for (int b = 0; b < 256; ++b) cnt[b + 1] += cnt[b];
    std::vector<uint8_t> tk(n * KB);
    std::vector<uint32_t> tp(payload ? n : 0);
    uint64_t at[256];
    std::memcpy(at, cnt, sizeof(at));
    for (uint64_t i = 0; i < n; ++i) {
        const uint64_t j = at[lead_byte<KB>(keys + i * KB)]++;
        std::memcpy(&tk[j * KB], keys + i * KB, KB);
        if (payload) tp[j] = payload[i];
    }
    std::memcpy(keys, tk.data(), n * KB);
    if (payload) std::memcpy(payload, tp.data(), n * 4);
    // the buckets on the threads
    std::atomic<int> next{0}, err{0};
    auto work = [&]() {
        for (int b; (b = next.fetch_add(1)) < 256;) {
            const uint64_t lo = cnt[b], hi = cnt[b + 1];
            if (hi - lo < 2) continue;
            if (binar_sort_ref(keys + lo * KB, KB, hi - lo, payload ? payload + lo : nullptr, nullptr) != 0) err = 1;
        }
    };
    std::vector<std::thread> pool;
    for (int t = 1; t < threads; ++t) pool.emplace_back(work);
    work();
    for (auto &t : pool) t.join();
    return err.load() ? -1 : 0;
}

}  // namespace

extern "C" int ref_stable_sort(void *keys, uint32_t key_bytes, uint64_t n, uint32_t *payload) {
    if (!keys && n) return -1;
    switch (key_bytes) {
        case 4: return stable_sort_kb<4>(static_cast<uint8_t *>(keys), n, payload);
        case 8: return stable_sort_kb<8>(static_cast<uint8_t *>(keys), n, payload);
        case 16: return stable_sort_kb<16>(static_cast<uint8_t *>(keys), n, payload);
    }
    return -1;
}

extern "C" int ref_parallel_binar(void *keys, uint32_t key_bytes, uint64_t n, uint32_t *payload, int threads) {
    if ((!keys && n) || threads < 1) return -1;
    switch (key_bytes) {
        case 4: return parallel_kb<4>(static_cast<uint8_t *>(keys), n, payload, threads);
        case 8: return parallel_kb<8>(static_cast<uint8_t *>(keys), n, payload, threads);
        case 16: return parallel_kb<16>(static_cast<uint8_t *>(keys), n, payload, threads);
    }
    return -1;
}
