// Streaming copy and read kernels: the rate a plain pass over HBM reaches on
// this device, measured beside the sort's passes (a sort pass reads and
// writes its bytes once, so it cannot beat a copy of the same bytes; a
// digit count reads them once, so it cannot beat a read).
//
// Both kernels run a persistent grid (blocks_per_cu blocks of 256 threads on
// every compute unit) that walks the buffer in grid-strided rounds; in each
// round a thread has U 16-byte vectors in flight, and each wave's loads and
// stores cover 1 KiB of consecutive bytes.  The copy writes with streaming
// (non-temporal) stores, so that written lines do not evict the lines still
// to be read.  Only the 16-byte body is handled: callers pass sizes that are
// multiples of 16 bytes.
#include <hip/hip_runtime.h>

#include "binar.h"
#include "binar_host.h"

namespace binar {
namespace {

constexpr int STREAM_BT = 256;
typedef uint32_t v4u __attribute__((ext_vector_type(4)));  // 16 bytes, a type the streaming-store builtin takes

template <int U>
__global__ __launch_bounds__(STREAM_BT) void k_stream_copy(const v4u *__restrict__ src, v4u *__restrict__ dst,
                                                           size_t nvec) {
    const size_t stride = (size_t)gridDim.x * STREAM_BT * U;
    for (size_t base = (size_t)blockIdx.x * STREAM_BT * U + threadIdx.x; base < nvec; base += stride) {
        v4u v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const size_t i = base + (size_t)u * STREAM_BT;
            if (i < nvec) v[u] = src[i];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const size_t i = base + (size_t)u * STREAM_BT;
            if (i < nvec) __builtin_nontemporal_store(v[u], dst + i);
        }
    }
}

// Read-only: every word is folded into an XOR that each block stores once,
// so the loads cannot be dropped.
template <int U>
__global__ __launch_bounds__(STREAM_BT) void k_stream_read(const v4u *__restrict__ src, size_t nvec,
                                                           uint32_t *__restrict__ out) {
    const size_t stride = (size_t)gridDim.x * STREAM_BT * U;
    uint32_t x = 0u;
    for (size_t base = (size_t)blockIdx.x * STREAM_BT * U + threadIdx.x; base < nvec; base += stride) {
        v4u v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const size_t i = base + (size_t)u * STREAM_BT;
            v[u] = (i < nvec) ? src[i] : v4u{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int u = 0; u < U; ++u) x ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) x ^= (uint32_t)__shfl_xor((int)x, o, WAVE);
    __shared__ uint32_t s_x[STREAM_BT / WAVE];
    if (lane_id() == 0) s_x[threadIdx.x / WAVE] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t y = 0u;
#pragma unroll
        for (int q = 0; q < STREAM_BT / WAVE; ++q) y ^= s_x[q];
        out[blockIdx.x] = y;
    }
}

int stream_args(const void *p, size_t bytes, uint32_t blocks_per_cu, uint32_t unroll) {
    if (!p || (reinterpret_cast<uintptr_t>(p) & 15u) || (bytes & 15u)) return BINAR_EINVAL;
    if (blocks_per_cu == 0 || blocks_per_cu > 32) return BINAR_EINVAL;
    if (unroll != 2 && unroll != 4 && unroll != 8) return BINAR_EINVAL;
    return BINAR_OK;
}

}  // namespace
}  // namespace binar

extern "C" int binar_stream_copy(void *dst, const void *src, size_t bytes, uint32_t blocks_per_cu, uint32_t unroll,
                                 void *stream) {
    using namespace binar;
    if (int rc = stream_args(src, bytes, blocks_per_cu, unroll)) return rc;
    if (int rc = stream_args(dst, bytes, blocks_per_cu, unroll)) return rc;
    if (bytes == 0) return BINAR_OK;
    const size_t nvec = bytes / 16;
    const dim3 grid((uint32_t)cu_count() * blocks_per_cu);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const v4u *s = static_cast<const v4u *>(src);
    v4u *d = static_cast<v4u *>(dst);
    (void)hipGetLastError();
    switch (unroll) {
        case 2: hipLaunchKernelGGL(k_stream_copy<2>, grid, dim3(STREAM_BT), 0, st, s, d, nvec); break;
        case 4: hipLaunchKernelGGL(k_stream_copy<4>, grid, dim3(STREAM_BT), 0, st, s, d, nvec); break;
        default: hipLaunchKernelGGL(k_stream_copy<8>, grid, dim3(STREAM_BT), 0, st, s, d, nvec); break;
    }
    BINAR_HIP_TRY(hipGetLastError());
    return BINAR_OK;
}

extern "C" int binar_stream_read(const void *src, size_t bytes, uint32_t *out, uint32_t blocks_per_cu,
                                 uint32_t unroll, void *stream) {
    using namespace binar;
    if (int rc = stream_args(src, bytes, blocks_per_cu, unroll)) return rc;
    if (!out) return BINAR_EINVAL;
    if (bytes == 0) return BINAR_OK;
    const size_t nvec = bytes / 16;
    const dim3 grid((uint32_t)cu_count() * blocks_per_cu);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const v4u *s = static_cast<const v4u *>(src);
    (void)hipGetLastError();
    switch (unroll) {
        case 2: hipLaunchKernelGGL(k_stream_read<2>, grid, dim3(STREAM_BT), 0, st, s, nvec, out); break;
        case 4: hipLaunchKernelGGL(k_stream_read<4>, grid, dim3(STREAM_BT), 0, st, s, nvec, out); break;
        default: hipLaunchKernelGGL(k_stream_read<8>, grid, dim3(STREAM_BT), 0, st, s, nvec, out); break;
    }
    BINAR_HIP_TRY(hipGetLastError());
    return BINAR_OK;
}
