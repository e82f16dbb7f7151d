// Bandwidth reference kernels for the benchmark; not part of the solver.
//
// They measure what trivial access patterns reach on this GPU: a streaming
// read (16-byte loads, non-temporal or plain, and 4-byte loads), a copy, and
// a read with a write stream one eighth its size (the byte mix of a fused
// SpMV pass).  That puts the solver kernels' fraction of the 8 TB/s HBM peak
// beside the fraction an access pattern with no gathers and no arithmetic
// attains on the same device.  Each kernel walks whole 16-byte (or 4-byte)
// units, eight loads in flight per thread, either as one grid-stride walk or
// as one contiguous range per workgroup; sizes must be multiples of the unit.
// Workgroups have 256 threads; the read also comes with 1024 (the shape of
// the sliding-window SpMV: one 1024-thread workgroup per CU).
//
// Built into libppa_bwprobe.so, loaded only by the benchmark.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int TPB = 256;
constexpr int UNROLL = 8;

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

// The units a thread visits: i, i + step, ... below end.  CONTIG: workgroup
// b owns units [b * per, (b + 1) * per) and its BS lanes walk them together;
// otherwise the whole grid strides over all n units.
struct Walk {
    int64_t i, end, step;
};
template <bool CONTIG, int BS = TPB>
__device__ __forceinline__ Walk walk(int64_t n, int64_t per) {
    if constexpr (CONTIG) {
        const int64_t s = (int64_t)blockIdx.x * per;
        return {s + threadIdx.x, s + per < n ? s + per : n, BS};
    } else {
        return {(int64_t)blockIdx.x * BS + threadIdx.x, n, (int64_t)gridDim.x * BS};
    }
}

// Reads n units of T with workgroups of BS threads; each thread's XOR of
// what it read is stored to sink[global thread index] only when it equals
// `never`.  The caller picks `never` so that the store (practically) never
// happens while the loads stay live, or, with data that is zero but for one
// unit and never = 0, to see that exactly one thread read that unit, once.
template <typename T, bool NT, bool CONTIG, int BS>
__global__ __launch_bounds__(BS) void k_read(const T* __restrict__ x, int64_t n, int64_t per,
                                             uint32_t never, uint32_t* __restrict__ sink) {
    Walk w = walk<CONTIG, BS>(n, per);
    uint32_t acc = 0;
    for (; w.i + (UNROLL - 1) * w.step < w.end; w.i += UNROLL * w.step) {
        T v[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) v[u] = ld<NT>(x + w.i + u * w.step);
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) acc ^= fold(v[u]);
    }
    for (; w.i < w.end; w.i += w.step) acc ^= fold(ld<NT>(x + w.i));
    if (acc == never) sink[(int64_t)blockIdx.x * BS + threadIdx.x] = acc;
}

// y[i] = x[i] for n 16-byte units.
template <bool CONTIG>
__global__ __launch_bounds__(TPB) void k_copy(const u32x4* __restrict__ x, u32x4* __restrict__ y,
                                              int64_t n, int64_t per) {
    Walk w = walk<CONTIG>(n, per);
    for (; w.i + (UNROLL - 1) * w.step < w.end; w.i += UNROLL * w.step) {
        u32x4 v[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) v[u] = __builtin_nontemporal_load(x + w.i + u * w.step);
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) y[w.i + u * w.step] = v[u];
    }
    for (; w.i < w.end; w.i += w.step) y[w.i] = __builtin_nontemporal_load(x + w.i);
}

// Reads n 16-byte units of x (non-temporal) and writes n / 8 units of y:
// unit k with k % 8 == 0 stores what it read to y[k / 8], so a wave writes
// one contiguous 128-byte piece per 1 KiB it reads.
template <bool CONTIG>
__global__ __launch_bounds__(TPB) void k_read_write8(const u32x4* __restrict__ x,
                                                     u32x4* __restrict__ y, int64_t n, int64_t per) {
    Walk w = walk<CONTIG>(n, per);
    for (; w.i + (UNROLL - 1) * w.step < w.end; w.i += UNROLL * w.step) {
        u32x4 v[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) v[u] = __builtin_nontemporal_load(x + w.i + u * w.step);
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int64_t k = w.i + u * w.step;
            if ((k & 7) == 0) y[k >> 3] = v[u];
        }
    }
    for (; w.i < w.end; w.i += w.step) {
        const u32x4 v = __builtin_nontemporal_load(x + w.i);
        if ((w.i & 7) == 0) y[w.i >> 3] = v;
    }
}

int grid_for(int64_t n, int blocks, int bs = TPB) {
    if (blocks <= 0) blocks = 4096;
    const int64_t need = (n + bs - 1) / bs;
    return (int)(need < blocks ? (need > 0 ? need : 1) : blocks);
}

template <int BS>
void launch_read(const void* x, int64_t n, int width, bool nt, bool contiguous, int g, int64_t per,
                 uint32_t never, uint32_t* sink, hipStream_t s) {
    if (width == 16) {
        const u32x4* p = (const u32x4*)x;
        if (nt && contiguous)
            hipLaunchKernelGGL((k_read<u32x4, true, true, BS>), dim3(g), dim3(BS), 0, s, p, n, per, never, sink);
        else if (nt)
            hipLaunchKernelGGL((k_read<u32x4, true, false, BS>), dim3(g), dim3(BS), 0, s, p, n, per, never, sink);
        else if (contiguous)
            hipLaunchKernelGGL((k_read<u32x4, false, true, BS>), dim3(g), dim3(BS), 0, s, p, n, per, never, sink);
        else
            hipLaunchKernelGGL((k_read<u32x4, false, false, BS>), dim3(g), dim3(BS), 0, s, p, n, per, never, sink);
    } else {
        const uint32_t* p = (const uint32_t*)x;
        if (contiguous)
            hipLaunchKernelGGL((k_read<uint32_t, false, true, BS>), dim3(g), dim3(BS), 0, s, p, n, per, never, sink);
        else
            hipLaunchKernelGGL((k_read<uint32_t, false, false, BS>), dim3(g), dim3(BS), 0, s, p, n, per, never, sink);
    }
}

template <class K, class... A>
int launch(K kern, int64_t n, int blocks, hipStream_t s, A... args) {
    const int g = grid_for(n, blocks);
    const int64_t per = (n + g - 1) / g;
    hipLaunchKernelGGL(kern, dim3(g), dim3(TPB), 0, s, args..., n, per);
    return (int)hipGetLastError();
}

}  // namespace

extern "C" {

// Streaming read of `bytes` bytes at x (device).  width: 16 (16-byte loads)
// or 4 (4-byte loads); nontemporal: nonzero for non-temporal loads (16-byte
// only); contiguous: nonzero for one contiguous range per workgroup, zero for
// a grid-stride walk.  threads: workgroup size, 256 or 1024.  blocks:
// workgroups, <= 0 picks 4096 (never more than the units need).  sink:
// device buffer of at least threads * blocks uint32 entries (threads * 4096
// when blocks <= 0); entry t is written (with the XOR of what thread t read)
// only when that XOR equals `never`.  Returns 0, -1 for a size, width or
// workgroup size that does not fit, or the HIP error code of the launch.
int ppa_probe_read_wg(const void* x, int64_t bytes, int width, int nontemporal, int contiguous,
                      int threads, uint32_t never, uint32_t* sink, int blocks, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    if (bytes < 0 || (width != 16 && width != 4) || bytes % width != 0) return -1;
    if (width == 4 && nontemporal) return -1;
    if (threads != 256 && threads != 1024) return -1;
    const int64_t n = bytes / width;
    if (n == 0) return 0;
    const int g = grid_for(n, blocks, threads);
    const int64_t per = (n + g - 1) / g;
    if (threads == 256)
        launch_read<256>(x, n, width, nontemporal != 0, contiguous != 0, g, per, never, sink, s);
    else
        launch_read<1024>(x, n, width, nontemporal != 0, contiguous != 0, g, per, never, sink, s);
    return (int)hipGetLastError();
}

// ppa_probe_read_wg with 256-thread workgroups.
int ppa_probe_read(const void* x, int64_t bytes, int width, int nontemporal, int contiguous,
                   uint32_t never, uint32_t* sink, int blocks, void* stream) {
    return ppa_probe_read_wg(x, bytes, width, nontemporal, contiguous, 256, never, sink, blocks, stream);
}

// y = x for `bytes` bytes (a multiple of 16): non-temporal 16-byte loads,
// 16-byte stores.  contiguous and blocks as for the read.
int ppa_probe_copy(const void* x, void* y, int64_t bytes, int contiguous, int blocks, void* stream) {
    if (bytes < 0 || bytes % 16 != 0) return -1;
    const int64_t n = bytes / 16;
    if (n == 0) return 0;
    hipStream_t s = (hipStream_t)stream;
    return contiguous ? launch(k_copy<true>, n, blocks, s, (const u32x4*)x, (u32x4*)y)
                      : launch(k_copy<false>, n, blocks, s, (const u32x4*)x, (u32x4*)y);
}

// Reads `bytes` bytes at x (a multiple of 128) and writes bytes / 8 at y.
int ppa_probe_read_write8(const void* x, void* y, int64_t bytes, int contiguous, int blocks,
                          void* stream) {
    if (bytes < 0 || bytes % 128 != 0) return -1;
    const int64_t n = bytes / 16;
    if (n == 0) return 0;
    hipStream_t s = (hipStream_t)stream;
    return contiguous ? launch(k_read_write8<true>, n, blocks, s, (const u32x4*)x, (u32x4*)y)
                      : launch(k_read_write8<false>, n, blocks, s, (const u32x4*)x, (u32x4*)y);
}

}  // extern "C"
