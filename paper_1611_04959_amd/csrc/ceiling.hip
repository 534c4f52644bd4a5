// ceiling.hip -- read rates the summing scan of the chop is measured against
// (it reads every raw sample once and writes almost nothing).
//
// k_read_stream reads a buffer once with 16-byte non-temporal loads (eight
// in flight per thread, grid-stride), folds the words with XOR so the loads
// cannot be dropped, and leaves one word per wave in a sink.
// k_read_tiles reads calorimeter fills in the scan's own pattern (tiles of
// 4,096 samples x every channel row, 9 rows in flight, the same halo
// overlap) and does nothing else: the rate of that access pattern alone.
// Its two other modes model a single pass that writes the islands from the
// scan: after each tile the threads of a fixed one-in-seven pattern of
// 8-sample groups (islands of 88 samples every 560) read their group of
// every row again (mode 1), and also write those words, packed tile by tile,
// to an output buffer (mode 2).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "daq.h"

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
#define DAQ_GLOBAL __attribute__((address_space(1)))

// layout 0: grid-stride (wave w of the grid reads word w, then w + grid, ...);
// layout 1: each work-group reads one contiguous chunk (a grid's worth of
// streams far apart in memory at any moment).
__global__ void __launch_bounds__(256) k_read_stream(const u32x4 *p, int64_t n16, unsigned int *sink, int layout) {
    constexpr int K = 8;  // loads in flight per thread
    int64_t i, end, stride;
    if (layout == 1) {
        const int64_t chunk = (n16 + gridDim.x - 1) / gridDim.x;
        i = (int64_t)blockIdx.x * chunk + threadIdx.x;
        end = (int64_t)(blockIdx.x + 1) * chunk < n16 ? (int64_t)(blockIdx.x + 1) * chunk : n16;
        stride = blockDim.x;
    } else {
        i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        end = n16;
        stride = (int64_t)gridDim.x * blockDim.x;
    }
    const DAQ_GLOBAL u32x4 *q = (const DAQ_GLOBAL u32x4 *)p;
    u32x4 x = {0, 0, 0, 0};
    for (; i + (K - 1) * stride < end; i += K * stride) {
        u32x4 v[K];
#pragma unroll
        for (int k = 0; k < K; k++) v[k] = __builtin_nontemporal_load(q + i + k * stride);
#pragma unroll
        for (int k = 0; k < K; k++) x ^= v[k];
    }
    for (; i < end; i += stride) x ^= __builtin_nontemporal_load(q + i);
    unsigned int v = x.x ^ x.y ^ x.z ^ x.w;
    for (int d = 32; d > 0; d >>= 1) v ^= __shfl_xor(v, d, 64);
    if ((threadIdx.x & 63) == 0) sink[(blockIdx.x * blockDim.x + threadIdx.x) >> 6] = v;
}

// Tile geometry of the split scan at 512 threads with halos of 4 and 2
// groups of 8 samples (post <= 31, pre <= 15): 512 groups read, 506 owned.
constexpr int kTileThreads = 512;
constexpr int kTileOwned = 4048;
constexpr int kTileLeft = 32;
constexpr int kTileRows = 9;

// Groups of the island pattern of modes 1 and 2: group index (sample / 8)
// of the row modulo 70 below 11.
constexpr int kPatPeriod = 70;
constexpr int kPatGroups = 11;

// Tile t of fill f = t / tiles_per_fill covers samples [lt * 4048 - 32,
// lt * 4048 + 4064) of every channel row; thread i reads the 16-byte group
// at lt * 4048 - 32 + 8 i of each row when it lies inside the row. Each wave
// leaves the wrapping sum of the 32-bit words it read in sink[wave of grid].
// MODE 1 and 2: pattern threads then read their group of every row again
// (9 rows in flight) and add it to the sum; MODE 2 also stores each such
// word to out[(t * C + c) * 512 + k], k the thread's rank among the tile's
// pattern threads.
template <int MODE>
__global__ void __launch_bounds__(kTileThreads) k_read_tiles(const int16_t *raw, int32_t n_fills, int32_t C,
                                                             int64_t n, int64_t tiles_per_fill, unsigned int *sink,
                                                             u32x4 *out) {
    __shared__ int s_cnt[kTileThreads / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t total = (int64_t)n_fills * tiles_per_fill;
    unsigned int acc = 0;
    for (int64_t tile = blockIdx.x; tile < total; tile += gridDim.x) {
        const int64_t f = tile / tiles_per_fill, lt = tile - f * tiles_per_fill;
        const int64_t p = lt * kTileOwned - kTileLeft + (int64_t)threadIdx.x * 8;
        const bool in = p >= 0 && p + 8 <= n;
        const DAQ_GLOBAL int16_t *base = (const DAQ_GLOBAL int16_t *)raw + f * C * n;
        for (int c = 0; c < C; c += kTileRows) {
            u32x4 v[kTileRows];
#pragma unroll
            for (int u = 0; u < kTileRows; u++) {
                if (in && c + u < C)
                    v[u] = __builtin_nontemporal_load((const DAQ_GLOBAL u32x4 *)(base + (int64_t)(c + u) * n + p));
                else
                    v[u] = u32x4{0, 0, 0, 0};
            }
#pragma unroll
            for (int u = 0; u < kTileRows; u++) acc += v[u].x + v[u].y + v[u].z + v[u].w;
        }
        if constexpr (MODE > 0) {
            const bool pat = in && ((p >> 3) % kPatPeriod) < kPatGroups;
            int k = 0;
            if constexpr (MODE == 2) {  // rank among the tile's pattern threads
                const uint64_t b = __ballot(pat);
                if (lane == 0) s_cnt[wid] = __popcll(b);
                __syncthreads();
                for (int w = 0; w < wid; w++) k += s_cnt[w];
                k += __popcll(b & ((1ull << lane) - 1ull));
                __syncthreads();
            } else {
                __syncthreads();
            }
            if (pat) {
                for (int c = 0; c < C; c += kTileRows) {
                    u32x4 v[kTileRows];
#pragma unroll
                    for (int u = 0; u < kTileRows; u++)
                        v[u] = c + u < C ? *(const DAQ_GLOBAL u32x4 *)(base + (int64_t)(c + u) * n + p)
                                         : u32x4{0, 0, 0, 0};
#pragma unroll
                    for (int u = 0; u < kTileRows; u++) {
                        acc += v[u].x + v[u].y + v[u].z + v[u].w;
                        if (MODE == 2 && c + u < C)
                            __builtin_nontemporal_store(
                                v[u], (DAQ_GLOBAL u32x4 *)out + (tile * C + c + u) * kTileThreads + k);
                    }
                }
            }
        }
    }
    for (int d = 32; d > 0; d >>= 1) acc += __shfl_xor(acc, d, 64);
    if ((threadIdx.x & 63) == 0) sink[(blockIdx.x * blockDim.x + threadIdx.x) >> 6] = acc;
}

}  // namespace

extern "C" int daq_read_tiles(const int16_t *d_raw, int32_t n_fills, int32_t channels, int64_t n_samples,
                              unsigned int *d_sink, int32_t blocks, int32_t mode, void *d_out, void *stream) {
    if (!d_raw || !d_sink || n_fills < 1 || channels < 1 || n_samples < 8 || (n_samples & 7) != 0 || blocks < 1 ||
        ((uintptr_t)d_raw & 15u) != 0 || mode < 0 || mode > 2 || (mode == 2 && (!d_out || ((uintptr_t)d_out & 15u))))
        return DAQ_EINVAL;
    const int64_t tiles = (n_samples + kTileOwned - 1) / kTileOwned;
    const hipStream_t s = (hipStream_t)stream;
    u32x4 *out = (u32x4 *)d_out;
    if (mode == 0)
        hipLaunchKernelGGL(k_read_tiles<0>, dim3(blocks), dim3(kTileThreads), 0, s, d_raw, n_fills, channels,
                           n_samples, tiles, d_sink, out);
    else if (mode == 1)
        hipLaunchKernelGGL(k_read_tiles<1>, dim3(blocks), dim3(kTileThreads), 0, s, d_raw, n_fills, channels,
                           n_samples, tiles, d_sink, out);
    else
        hipLaunchKernelGGL(k_read_tiles<2>, dim3(blocks), dim3(kTileThreads), 0, s, d_raw, n_fills, channels,
                           n_samples, tiles, d_sink, out);
    return hipGetLastError() == hipSuccess ? DAQ_OK : DAQ_EHIP;
}

extern "C" int daq_read_stream(const void *d_buf, int64_t bytes, unsigned int *d_sink, int32_t blocks,
                               int32_t layout, void *stream) {
    if (!d_buf || !d_sink || bytes < 16 || blocks < 1 || ((uintptr_t)d_buf & 15u) != 0 || layout < 0 || layout > 1)
        return DAQ_EINVAL;
    hipLaunchKernelGGL(k_read_stream, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (const u32x4 *)d_buf,
                       bytes / 16, d_sink, (int)layout);
    return hipGetLastError() == hipSuccess ? DAQ_OK : DAQ_EHIP;
}
