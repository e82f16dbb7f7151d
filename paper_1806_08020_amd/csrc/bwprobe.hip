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
// the sliding-window SpMV: one 1024-thread workgroup per CU), and with one
// to four streams per workgroup.  A last kernel issues the sliding-window
// SpMV's memory streams without its arithmetic: its index, value and
// vector loads per chunk, three chunks ahead, with or without its output
// stores, to see what those streams alone reach.
//
// Built into libppa_bwprobe.so, loaded only by the benchmark.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>

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

// NS equal streams (stream s: units [s L, (s + 1) L)) read by workgroups of
// BS threads; workgroup b reads units [b per, (b + 1) per) of every stream,
// each thread UNROLL / NS units of each stream per step, so that eight loads
// are in flight per thread whatever NS.
template <int NS, int BS>
__global__ __launch_bounds__(BS) void k_read_streams(const u32x4* __restrict__ x, int64_t L, int64_t per,
                                                     uint32_t never, uint32_t* __restrict__ sink) {
    constexpr int UPS = UNROLL / NS;
    const int64_t s0 = (int64_t)blockIdx.x * per;
    const int64_t end = s0 + per < L ? s0 + per : L;
    uint32_t acc = 0;
    int64_t i = s0 + threadIdx.x;
    for (; i + (UPS - 1) * BS < end; i += UPS * BS) {
        u32x4 v[NS][UPS];
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int u = 0; u < UPS; ++u) v[s][u] = __builtin_nontemporal_load(x + s * L + i + u * BS);
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int u = 0; u < UPS; ++u) acc ^= fold(v[s][u]);
    }
    for (; i < end; i += BS)
#pragma unroll
        for (int s = 0; s < NS; ++s) acc ^= fold(__builtin_nontemporal_load(x + s * L + i));
    if (acc == never) sink[(int64_t)blockIdx.x * BS + threadIdx.x] = acc;
}

// The sliding-window SpMV's memory streams without its arithmetic, in its
// shape: workgroups of MIX_BS threads, each walking chunks [b q, (b + 1) q)
// of MIX_CH nonzeros.  Per chunk a thread loads the column indices and
// values of its MIX_CH / MIX_BS nonzeros two per lane (8-byte index loads,
// 16-byte value loads, non-temporal) and one 8-byte vector entry (the new
// ring entry), MIX_D chunks ahead in registers, and folds what it loaded
// into a running XOR.  Chunk c owns output rows [c R, (c + 1) R), R <= MIX_BS;
// thread t < R gives row c R + t its running XOR.  STORE 0: nothing is
// stored (the XOR goes to the sink only when it equals `never`); 1: one
// 8-byte store per row at the end of each chunk, as the kernel does; 2: the
// rows' values kept in LDS and written after the workgroup's last chunk
// (q R <= MIX_DEFER_MAX).  Modes 1 and 2 store the same values.
constexpr int MIX_BS = 1024, MIX_CH = 4096, MIX_D = 3, MIX_DEFER_MAX = 8192;
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

struct MixSlot {
    u32x2 c[MIX_CH / MIX_BS / 2];
    u32x4 v[MIX_CH / MIX_BS / 2];
    u32x2 w;
};

template <class F, int... I>
__device__ __forceinline__ void unroll_impl(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void unroll_n(F&& f) {
    unroll_impl(f, std::make_integer_sequence<int, N>{});
}

template <int STORE>
__global__ __launch_bounds__(MIX_BS) void k_spmv_mix(const u32x2* __restrict__ idx, const u32x4* __restrict__ val,
                                                     const u32x2* __restrict__ vec, u32x2* __restrict__ out,
                                                     int64_t q, int rows, uint32_t never,
                                                     uint32_t* __restrict__ sink) {
    constexpr int NG = MIX_CH / MIX_BS / 2;
    __shared__ u32x2 keep[STORE == 2 ? MIX_DEFER_MAX : 1];
    const int tid = threadIdx.x;
    const int64_t c0 = (int64_t)blockIdx.x * q, c1 = c0 + q;
    uint32_t acc = 0;
    auto load = [&](MixSlot& S, int64_t c) {
        c = c < c1 ? c : c1 - 1;
        S.w = vec[c * rows + (tid < rows ? tid : rows - 1)];
        const int64_t b = c * (MIX_CH / 2);       // in pairs of nonzeros
#pragma unroll
        for (int k = 0; k < NG; ++k) {
            S.c[k] = __builtin_nontemporal_load(idx + b + tid + k * MIX_BS);
            S.v[k] = __builtin_nontemporal_load(val + b + tid + k * MIX_BS);
        }
    };
    auto use = [&](const MixSlot& S, int64_t c) {
#pragma unroll
        for (int k = 0; k < NG; ++k) acc ^= S.c[k].x ^ S.c[k].y ^ fold(S.v[k]);
        acc ^= S.w.x ^ S.w.y;
        if constexpr (STORE != 0) {
            if (tid < rows) {
                const u32x2 o = {acc, ~acc};
                if constexpr (STORE == 1)
                    out[c * rows + tid] = o;
                else
                    keep[(c - c0) * rows + tid] = o;
            }
        }
    };
    MixSlot S[MIX_D];
    unroll_n<MIX_D>([&](auto i) { load(S[decltype(i)::value], c0 + decltype(i)::value); });
    for (int64_t c = c0; c < c1; c += MIX_D) {
        unroll_n<MIX_D>([&](auto i) {
            constexpr int j = decltype(i)::value;
            if (c + j < c1) {
                use(S[j], c + j);
                load(S[j], c + j + MIX_D);
            }
        });
    }
    if constexpr (STORE == 2) {
        // each thread wrote only its own entries of keep: no barrier needed
        for (int64_t c = c0; c < c1; ++c)
            if (tid < rows) out[c * rows + tid] = keep[(c - c0) * rows + tid];
    }
    if (acc == never) sink[(int64_t)blockIdx.x * MIX_BS + tid] = acc;
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

// Reads `bytes` bytes at x as `streams` equal streams (1, 2 or 4; bytes a
// multiple of 16 * streams) with workgroups of `threads` threads (256 or
// 1024), each workgroup one contiguous range of every stream, non-temporal
// 16-byte loads.  blocks, sink and never as for ppa_probe_read_wg.  Returns
// 0, -1 for arguments that do not fit, or the HIP error of the launch.
int ppa_probe_read_streams(const void* x, int64_t bytes, int streams, int threads, uint32_t never,
                           uint32_t* sink, int blocks, void* stream) {
    if (bytes < 0 || (streams != 1 && streams != 2 && streams != 4) || bytes % (16 * streams) != 0)
        return -1;
    if (threads != 256 && threads != 1024) return -1;
    const int64_t L = bytes / 16 / streams;
    if (L == 0) return 0;
    const int g = grid_for(L, blocks, threads);
    const int64_t per = (L + g - 1) / g;
    hipStream_t s = (hipStream_t)stream;
    const u32x4* p = (const u32x4*)x;
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(g), dim3(threads), 0, s, p, L, per, never, sink);
    };
    if (threads == 256)
        streams == 1 ? go(k_read_streams<1, 256>) : streams == 2 ? go(k_read_streams<2, 256>) : go(k_read_streams<4, 256>);
    else
        streams == 1 ? go(k_read_streams<1, 1024>) : streams == 2 ? go(k_read_streams<2, 1024>) : go(k_read_streams<4, 1024>);
    return (int)hipGetLastError();
}

// The sliding-window SpMV's memory streams (k_spmv_mix above): `chunks`
// chunks of 4096 nonzeros, `chunks_per_group` per 1024-thread workgroup
// (chunks a multiple of it), `rows` output rows per chunk (1..1024).  idx:
// 4 * 4096 * chunks bytes (column indices), val: 8 * 4096 * chunks bytes
// (values), vec and out: 8 * rows * chunks bytes each; all device pointers,
// 16-byte aligned.  store: 0 none, 1 per chunk, 2 after each workgroup's
// last chunk (chunks_per_group * rows <= 8192).  sink: 1024 uint32 per
// workgroup, written where a thread's XOR equals `never`.  Returns 0, -1 for
// arguments that do not fit, or the HIP error of the launch.
int ppa_probe_spmv_mix(const void* idx, const void* val, const void* vec, void* out, int64_t chunks,
                       int64_t chunks_per_group, int rows, int store, uint32_t never, uint32_t* sink,
                       void* stream) {
    if (chunks <= 0 || chunks_per_group <= 0 || chunks % chunks_per_group != 0) return -1;
    if (rows < 1 || rows > MIX_BS || store < 0 || store > 2) return -1;
    if (store == 2 && chunks_per_group * rows > MIX_DEFER_MAX) return -1;
    for (const void* ptr : {idx, val, vec, (const void*)out})
        if (reinterpret_cast<uintptr_t>(ptr) % 16 != 0) return -1;
    const int64_t groups = chunks / chunks_per_group;
    if (groups > 65535) return -1;
    hipStream_t s = (hipStream_t)stream;
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3((unsigned)groups), dim3(MIX_BS), 0, s, (const u32x2*)idx,
                           (const u32x4*)val, (const u32x2*)vec, (u32x2*)out, chunks_per_group, rows,
                           never, sink);
    };
    store == 0 ? go(k_spmv_mix<0>) : store == 1 ? go(k_spmv_mix<1>) : go(k_spmv_mix<2>);
    return (int)hipGetLastError();
}

}  // extern "C"
