// Bandwidth reference kernels for the benchmark; not part of the solver.
//
// They measure what trivial access patterns reach on this GPU: a streaming
// read (16-byte loads, non-temporal or plain, and 4-byte loads), a copy, and
// a read with a write stream one eighth its size (the byte mix of a fused
// SpMV pass).  That puts the solver kernels' fraction of the 8 TB/s HBM peak
// beside the fraction an access pattern with no gathers and no arithmetic
// attains on the same device.  The kernels are grid-stride loops over whole
// 16-byte (or 4-byte) units; sizes must be multiples of the unit.
//
// Built into libppa_bwprobe.so, loaded only by the benchmark.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int TPB = 256;
constexpr int UNROLL = 4;

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <bool NT, typename T>
__device__ __forceinline__ T ld(const T* p) {
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

__device__ __forceinline__ uint32_t fold(u32x4 v) { return v.x ^ v.y ^ v.z ^ v.w; }
__device__ __forceinline__ uint32_t fold(uint32_t v) { return v; }

// Reads n units of T; the XOR of everything read is stored only when it
// equals `never`, which the caller chooses so that the store (practically)
// never happens while the loads stay live.
template <typename T, bool NT>
__global__ __launch_bounds__(TPB) void k_read(const T* __restrict__ x, int64_t n, uint32_t never,
                                              uint32_t* __restrict__ sink) {
    const int64_t stride = (int64_t)gridDim.x * TPB;
    int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    uint32_t acc = 0;
    for (; i + (UNROLL - 1) * stride < n; i += UNROLL * stride) {
        T v[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) v[u] = ld<NT>(x + i + u * stride);
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) acc ^= fold(v[u]);
    }
    for (; i < n; i += stride) acc ^= fold(ld<NT>(x + i));
    if (acc == never) sink[blockIdx.x * TPB + threadIdx.x] = acc;
}

// y[i] = x[i] for n 16-byte units.
__global__ __launch_bounds__(TPB) void k_copy(const u32x4* __restrict__ x, u32x4* __restrict__ y,
                                              int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * TPB;
    int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    for (; i + (UNROLL - 1) * stride < n; i += UNROLL * stride) {
        u32x4 v[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) v[u] = x[i + u * stride];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) y[i + u * stride] = v[u];
    }
    for (; i < n; i += stride) y[i] = x[i];
}

// Reads n 16-byte units of x (non-temporal) and writes n / 8 units of y:
// unit i with i % 8 == 0 stores what it read to y[i / 8], so each wave
// writes one contiguous 128-byte piece per 1 KiB it reads.
__global__ __launch_bounds__(TPB) void k_read_write8(const u32x4* __restrict__ x,
                                                     u32x4* __restrict__ y, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * TPB;
    int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    for (; i + (UNROLL - 1) * stride < n; i += UNROLL * stride) {
        u32x4 v[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) v[u] = __builtin_nontemporal_load(x + i + u * stride);
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int64_t k = i + u * stride;
            if ((k & 7) == 0) y[k >> 3] = v[u];
        }
    }
    for (; i < n; i += stride) {
        const u32x4 v = __builtin_nontemporal_load(x + i);
        if ((i & 7) == 0) y[i >> 3] = v;
    }
}

int grid_for(int64_t n, int blocks) {
    if (blocks <= 0) blocks = 4096;
    const int64_t need = (n + TPB - 1) / TPB;
    return (int)(need < blocks ? (need > 0 ? need : 1) : blocks);
}

}  // namespace

extern "C" {

// Streaming read of `bytes` bytes at x (device).  width: 16 (16-byte loads)
// or 4 (4-byte loads); nontemporal: nonzero for non-temporal loads (16-byte
// only).  sink: device buffer of at least blocks * 256 uint32 entries,
// written only when the XOR of the data equals `never`.  blocks <= 0 picks
// 4096.  Returns 0, or -1 for a size or width that does not fit, or the HIP
// error code of the launch.
int ppa_probe_read(const void* x, int64_t bytes, int width, int nontemporal, uint32_t never,
                   uint32_t* sink, int blocks, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    if (bytes < 0 || (width != 16 && width != 4) || bytes % width != 0) return -1;
    const int64_t n = bytes / width;
    if (n == 0) return 0;
    const int g = grid_for(n, blocks);
    if (width == 16) {
        if (nontemporal)
            hipLaunchKernelGGL((k_read<u32x4, true>), dim3(g), dim3(TPB), 0, s,
                               (const u32x4*)x, n, never, sink);
        else
            hipLaunchKernelGGL((k_read<u32x4, false>), dim3(g), dim3(TPB), 0, s,
                               (const u32x4*)x, n, never, sink);
    } else {
        if (nontemporal) return -1;
        hipLaunchKernelGGL((k_read<uint32_t, false>), dim3(g), dim3(TPB), 0, s,
                           (const uint32_t*)x, n, never, sink);
    }
    return (int)hipGetLastError();
}

// y = x for `bytes` bytes (multiple of 16), 16-byte loads and stores.
int ppa_probe_copy(const void* x, void* y, int64_t bytes, int blocks, void* stream) {
    if (bytes < 0 || bytes % 16 != 0) return -1;
    const int64_t n = bytes / 16;
    if (n == 0) return 0;
    hipLaunchKernelGGL(k_copy, dim3(grid_for(n, blocks)), dim3(TPB), 0, (hipStream_t)stream,
                       (const u32x4*)x, (u32x4*)y, n);
    return (int)hipGetLastError();
}

// Reads `bytes` bytes at x (a multiple of 128) and writes bytes / 8 at y.
int ppa_probe_read_write8(const void* x, void* y, int64_t bytes, int blocks, void* stream) {
    if (bytes < 0 || bytes % 128 != 0) return -1;
    const int64_t n = bytes / 16;
    if (n == 0) return 0;
    hipLaunchKernelGGL(k_read_write8, dim3(grid_for(n, blocks)), dim3(TPB), 0, (hipStream_t)stream,
                       (const u32x4*)x, (u32x4*)y, n);
    return (int)hipGetLastError();
}

}  // extern "C"
