// Key views for the gfx950 binar sort kernels.
//
// A key is a bit string read most significant bit first (bit index 0 is the
// MSB), which is the encoding the paper sorts by (section "The Other
// Universal Property"; bit extraction in section "Bit Extraction").
//   4-byte keys : uint32 values, numeric order;
//   8-byte keys : uint64 values, numeric order;
//   16-byte keys: byte strings in memcmp order.  In registers they are held
//                 as two big-endian 64-bit halves (hi = bytes 0..7), so the
//                 numeric order of (hi, lo) is the memcmp order of the bytes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace binar {

struct U128 {
    uint64_t hi, lo;
};

// The same key as a left-aligned 128-bit word (bit 0 = MSB of hi).  Used for
// the AND/OR reductions that find bits constant over a sub-array.
struct Canon {
    uint64_t hi, lo;
};

__device__ __forceinline__ uint64_t bswap64(uint64_t x) { return __builtin_bswap64(x); }

// How the bits of a key are ordered: as an unsigned integer (the paper's
// bit-string order), as a two's-complement integer, or as an IEEE-754 value
// in the standard's total order (-NaN < -inf < ... < -0 < +0 < ... < +inf <
// +NaN).  The kernels sort the unsigned view enc(v), which flips the sign bit
// of signed and non-negative float keys and every bit of negative float keys.
constexpr uint32_t KIND_UNSIGNED = 0, KIND_SIGNED = 1, KIND_FLOAT = 2;

template <int KB>
struct KeyT;

template <>
struct KeyT<4> {
    using V = uint32_t;
    static constexpr int NBITS = 32;
    __device__ static __forceinline__ V load(const void *p, size_t i) {
        return reinterpret_cast<const uint32_t *>(p)[i];
    }
    __device__ static __forceinline__ void store(void *p, size_t i, V v) {
        reinterpret_cast<uint32_t *>(p)[i] = v;
    }
    // streaming store: the data is not read again soon, keep it out of the caches
    __device__ static __forceinline__ void store_nt(void *p, size_t i, V v) {
        __builtin_nontemporal_store(v, reinterpret_cast<uint32_t *>(p) + i);
    }
    // bits [pos, pos + w) counted from the MSB, 1 <= w <= 8, pos + w <= 32
    __device__ static __forceinline__ uint32_t digit(V v, int pos, int w) {
        return (v >> (32 - pos - w)) & ((1u << w) - 1u);
    }
    __device__ static __forceinline__ V zero() { return 0u; }
    __device__ static __forceinline__ V ones() { return ~0u; }
    __device__ static __forceinline__ V vand(V a, V b) { return a & b; }
    __device__ static __forceinline__ V vor(V a, V b) { return a | b; }
    __device__ static __forceinline__ Canon canon(V v) { return Canon{(uint64_t)v << 32, 0ull}; }
    // the order-preserving unsigned view of a signed (KIND_SIGNED) or IEEE-754
    // (KIND_FLOAT) key, and its inverse
    __device__ static __forceinline__ V enc(V v, uint32_t kind) {
        const V sb = 0x80000000u;
        if (kind == KIND_SIGNED) return v ^ sb;
        return v ^ ((V)((int32_t)v >> 31) | sb);
    }
    __device__ static __forceinline__ V dec(V e, uint32_t kind) {
        const V sb = 0x80000000u;
        if (kind == KIND_SIGNED) return e ^ sb;
        return e ^ ((e & sb) ? sb : ~0u);
    }
};

template <>
struct KeyT<8> {
    using V = uint64_t;
    static constexpr int NBITS = 64;
    __device__ static __forceinline__ V load(const void *p, size_t i) {
        return reinterpret_cast<const uint64_t *>(p)[i];
    }
    __device__ static __forceinline__ void store(void *p, size_t i, V v) {
        reinterpret_cast<uint64_t *>(p)[i] = v;
    }
    __device__ static __forceinline__ void store_nt(void *p, size_t i, V v) {
        __builtin_nontemporal_store(v, reinterpret_cast<uint64_t *>(p) + i);
    }
    __device__ static __forceinline__ uint32_t digit(V v, int pos, int w) {
        return (uint32_t)(v >> (64 - pos - w)) & ((1u << w) - 1u);
    }
    __device__ static __forceinline__ V zero() { return 0ull; }
    __device__ static __forceinline__ V ones() { return ~0ull; }
    __device__ static __forceinline__ V vand(V a, V b) { return a & b; }
    __device__ static __forceinline__ V vor(V a, V b) { return a | b; }
    __device__ static __forceinline__ Canon canon(V v) { return Canon{v, 0ull}; }
    __device__ static __forceinline__ V enc(V v, uint32_t kind) {
        const V sb = 0x8000000000000000ull;
        if (kind == KIND_SIGNED) return v ^ sb;
        return v ^ ((V)((int64_t)v >> 63) | sb);
    }
    __device__ static __forceinline__ V dec(V e, uint32_t kind) {
        const V sb = 0x8000000000000000ull;
        if (kind == KIND_SIGNED) return e ^ sb;
        return e ^ ((e & sb) ? sb : ~0ull);
    }
};

template <>
struct KeyT<16> {
    using V = U128;
    static constexpr int NBITS = 128;
    __device__ static __forceinline__ V load(const void *p, size_t i) {
        const ulonglong2 raw = reinterpret_cast<const ulonglong2 *>(p)[i];
        return U128{bswap64(raw.x), bswap64(raw.y)};
    }
    __device__ static __forceinline__ void store(void *p, size_t i, V v) {
        ulonglong2 raw;
        raw.x = bswap64(v.hi);
        raw.y = bswap64(v.lo);
        reinterpret_cast<ulonglong2 *>(p)[i] = raw;
    }
    __device__ static __forceinline__ void store_nt(void *p, size_t i, V v) {
        typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
        u64x2 raw;
        raw.x = bswap64(v.hi);
        raw.y = bswap64(v.lo);
        __builtin_nontemporal_store(raw, reinterpret_cast<u64x2 *>(p) + i);
    }
    __device__ static __forceinline__ uint32_t digit(V v, int pos, int w) {
        const uint32_t m = (1u << w) - 1u;
        if (pos + w <= 64) return (uint32_t)(v.hi >> (64 - pos - w)) & m;
        if (pos >= 64) return (uint32_t)(v.lo >> (128 - pos - w)) & m;
        const int s = pos + w - 64;  // 1 .. w-1 bits come from lo
        return (uint32_t)((v.hi << s) | (v.lo >> (64 - s))) & m;
    }
    __device__ static __forceinline__ V zero() { return U128{0ull, 0ull}; }
    __device__ static __forceinline__ V ones() { return U128{~0ull, ~0ull}; }
    __device__ static __forceinline__ V vand(V a, V b) { return U128{a.hi & b.hi, a.lo & b.lo}; }
    __device__ static __forceinline__ V vor(V a, V b) { return U128{a.hi | b.hi, a.lo | b.lo}; }
    __device__ static __forceinline__ Canon canon(V v) { return Canon{v.hi, v.lo}; }
    // byte strings have no other view
    __device__ static __forceinline__ V enc(V v, uint32_t) { return v; }
    __device__ static __forceinline__ V dec(V v, uint32_t) { return v; }
};

// First bit index >= pos (MSB-first) set in the left-aligned word d, or
// `limit` if there is none below limit.
__device__ __forceinline__ int first_set_from(Canon d, int pos, int limit) {
    if (pos >= limit) return limit;
    if (pos < 64) {
        const uint64_t h = (pos == 0) ? d.hi : (d.hi & (~0ull >> pos));
        if (h) {
            const int b = __clzll(h);
            return b < limit ? b : limit;
        }
        pos = 64;
    }
    const int p = pos - 64;
    const uint64_t l = (p == 0) ? d.lo : (p >= 64 ? 0ull : (d.lo & (~0ull >> p)));
    if (l) {
        const int b = 64 + __clzll(l);
        return b < limit ? b : limit;
    }
    return limit;
}

// a and b agree on the bits set in m
__device__ __forceinline__ bool canon_eq_under(Canon a, Canon b, Canon m) {
    return (((a.hi ^ b.hi) & m.hi) | ((a.lo ^ b.lo) & m.lo)) == 0ull;
}

__device__ __forceinline__ bool canon_less(Canon a, Canon b) {
    return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo);
}

// The leading `bits` bits (MSB-first) of a left-aligned word.
__device__ __forceinline__ Canon canon_lead_mask(int bits) {
    Canon m;
    m.hi = bits >= 64 ? ~0ull : (bits <= 0 ? 0ull : ~(~0ull >> bits));
    m.lo = bits >= 128 ? ~0ull : (bits <= 64 ? 0ull : ~(~0ull >> (bits - 64)));
    return m;
}

// a comes after b in the order of the leading bits selected by m
__device__ __forceinline__ bool canon_after(Canon a, Canon b, Canon m) {
    return canon_less(Canon{b.hi & m.hi, b.lo & m.lo}, Canon{a.hi & m.hi, a.lo & m.lo});
}

// Last bit index in [pos, end) set in d, or -1 if none.
__device__ __forceinline__ int last_set_below(Canon d, int pos, int end) {
    // mask bits [pos, end) of the 128-bit left-aligned word
    for (int half = 1; half >= 0; --half) {
        const int base = half * 64;
        int a = pos > base ? pos - base : 0;
        int b = end < base + 64 ? end - base : 64;
        if (b <= a) continue;
        uint64_t w = half ? d.lo : d.hi;
        // keep bits with MSB-first index in [a, b): clear the first a bits and
        // the bits from b on
        if (a > 0) w &= (~0ull >> a);
        if (b < 64) w &= ~(~0ull >> b);
        if (w) return base + 63 - __builtin_ctzll(w);
    }
    return -1;
}

}  // namespace binar
