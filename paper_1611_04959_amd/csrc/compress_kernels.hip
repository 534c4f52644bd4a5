// compress_kernels.hip -- gfx950 kernels of libdaqisland: lossless
// compression of the chopped islands.
//
// Section 3: the frontend compresses the chopped data losslessly before the
// event builder (the algorithm is not named). The format is the one stated in
// include/daq.h: each channel's packed row of L samples in blocks of 64; per
// block a header word (first sample, bit width w) and the zigzag-coded
// differences of consecutive samples as a little-endian bit stream of w bits
// each, the blocks' payloads back to back.
//
// A wave takes a group of 8 consecutive blocks of one row: lane l holds the
// 8 samples 8 l .. 8 l + 7 of the group (one 16-byte load), so block j of the
// group is lanes 8 j .. 8 j + 7. Three kernels, each over up to kZMaxFills
// fills (blockIdx.y): the size pass (block headers, group payload sizes), an
// exclusive scan of the group sizes (one work-group per fill), and the pack
// pass (block offsets; each wave ORs its codes into the group's contiguous
// payload in LDS, then stores it with coalesced writes).
#include "chop_internal.h"

namespace daqk {
namespace {

constexpr int kZBlock = 64;              // samples per block
constexpr int kZGroup = 8;               // blocks per wave
constexpr int kZMaxWords = 34;           // ceil(63 * 17 / 32): the widest block's payload
constexpr int kZGroupWords = kZGroup * kZMaxWords;
constexpr int kZWaves = 4;               // waves per work-group of the size and pack passes
constexpr int kZScanThreads = 1024;
constexpr int kZScanPer = 8;             // consecutive sizes per scan thread and round

struct ZGeom {
    int64_t L;       // samples per row
    int64_t nb;      // blocks per row
    int64_t gpr;     // groups per row
    int64_t groups;  // groups of the fill
};

// Samples each row of fill f compresses: its total_len, clamped to [0, max_len].
__device__ __forceinline__ ZGeom z_geom(const ZFillDev &f) {
    const int64_t tl = *reinterpret_cast<const volatile int64_t *>(&f.counts->total_len);
    ZGeom g;
    g.L = tl < f.max_len ? (tl > 0 ? tl : 0) : f.max_len;
    g.nb = (g.L + kZBlock - 1) / kZBlock;
    g.gpr = (g.nb + kZGroup - 1) / kZGroup;
    g.groups = g.gpr * f.C;
    return g;
}

// What a lane knows of its block after reading group gi.
struct ZLane {
    uint32_t z[kVec];  // zigzag codes of its 8 samples (0 where there is none)
    int16_t first;     // the block's first sample
    int64_t b;         // the block's index in the fill (valid when n > 0)
    int n;             // samples in the block (0: no such block)
    uint32_t w;        // the block's bit width
    int64_t nw;        // the block's payload words
};

__device__ __forceinline__ uint32_t zigzag(int32_t r) { return ((uint32_t)r << 1) ^ (uint32_t)(r >> 31); }

__device__ __forceinline__ void z_read(const ZFillDev &f, const ZGeom &g, int64_t gi, int lane, ZLane &o) {
    const int64_t c = gi / g.gpr;
    const int64_t kb0 = (gi - c * g.gpr) * kZGroup;  // first block of the group in its row
    const int j = lane >> 3, sub = lane & 7;
    const int64_t kb = kb0 + j;
    const int64_t t0 = kb * kZBlock + sub * kVec;     // first sample of the lane
    int32_t s[kVec];
    if (t0 < g.L) {
        const int4 q = *reinterpret_cast<const int4 *>(f.packed + c * f.stride + t0);
        const int16_t *h = reinterpret_cast<const int16_t *>(&q);
#pragma unroll
        for (int e = 0; e < kVec; e++) s[e] = h[e];
    } else {
#pragma unroll
        for (int e = 0; e < kVec; e++) s[e] = 0;
    }
    const int32_t prev = __shfl_up(s[kVec - 1], 1, 64);
    o.n = kb < g.nb ? (int)(g.L - kb * kZBlock < kZBlock ? g.L - kb * kZBlock : kZBlock) : 0;
    o.b = c * g.nb + kb;
    o.first = (int16_t)__shfl(s[0], lane & ~7, 64);
    uint32_t zmax = 0;
#pragma unroll
    for (int e = 0; e < kVec; e++) {
        const int i = sub * kVec + e;  // index in the block
        const int32_t before = e ? s[e - 1] : prev;
        o.z[e] = (i >= 1 && i < o.n) ? zigzag(s[e] - before) : 0u;
        zmax = o.z[e] > zmax ? o.z[e] : zmax;
    }
#pragma unroll
    for (int d = 1; d < 8; d <<= 1) {
        const uint32_t u = __shfl_xor(zmax, d, 64);
        zmax = u > zmax ? u : zmax;
    }
    o.w = zmax ? 32u - (uint32_t)__clz(zmax) : 0u;
    o.nw = o.n > 0 ? ((int64_t)(o.n - 1) * o.w + 31) / 32 : 0;
}

__global__ void __launch_bounds__(kZWaves * 64) k_z_size(ZArgs a) {
    const ZFillDev &f = a.f[blockIdx.y];
    const ZGeom g = z_geom(f);
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * kZWaves;
    for (int64_t gi = (int64_t)blockIdx.x * kZWaves + (threadIdx.x >> 6); gi < g.groups; gi += waves) {
        ZLane o;
        z_read(f, g, gi, lane, o);
        if ((lane & 7) == 0 && o.n > 0) f.hdr[o.b] = (uint32_t)(uint16_t)o.first | (o.w << 16);
        int64_t tot = o.nw;  // the same on the 8 lanes of a block: sum over blocks
#pragma unroll
        for (int d = 8; d < 64; d <<= 1) tot += __shfl_xor(tot, d, 64);
        if (lane == 0) f.gofs[gi] = tot;
    }
}

// Exclusive scan of fill blockIdx.y's group sizes in place, in rounds of
// kZScanThreads * kZScanPer sizes staged through LDS; the total goes to
// *n_words.
__global__ void __launch_bounds__(kZScanThreads) k_z_scan(ZArgs a) {
    constexpr int kRound = kZScanThreads * kZScanPer;
    __shared__ int64_t s_v[kRound];
    __shared__ int64_t s_w[kZScanThreads / 64];
    const ZFillDev &f = a.f[blockIdx.y];
    const ZGeom g = z_geom(f);
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    int64_t carry = 0;
    for (int64_t base = 0; base < g.groups; base += kRound) {
        for (int j = tid; j < kRound; j += kZScanThreads) s_v[j] = base + j < g.groups ? f.gofs[base + j] : 0;
        __syncthreads();
        int64_t v[kZScanPer], mine = 0;
#pragma unroll
        for (int j = 0; j < kZScanPer; j++) {
            v[j] = s_v[tid * kZScanPer + j];
            mine += v[j];
        }
        int64_t inc = mine;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int64_t u = __shfl_up(inc, d, 64);
            if (lane >= d) inc += u;
        }
        if (lane == 63) s_w[wid] = inc;
        __syncthreads();
        int64_t before = carry, all = carry;
        for (int w = 0; w < kZScanThreads / 64; w++) {
            before += w < wid ? s_w[w] : 0;
            all += s_w[w];
        }
        int64_t run = before + inc - mine;
#pragma unroll
        for (int j = 0; j < kZScanPer; j++) {
            s_v[tid * kZScanPer + j] = run;
            run += v[j];
        }
        __syncthreads();
        for (int j = tid; j < kRound; j += kZScanThreads)
            if (base + j < g.groups) f.gofs[base + j] = s_v[j];
        carry = all;
        __syncthreads();
    }
    if (tid == 0) *f.n_words = carry;
}

// The loop bound is uniform over the work-group (kZWaves consecutive
// groups), so every wave reaches the barriers.
__global__ void __launch_bounds__(kZWaves * 64) k_z_pack(ZArgs a) {
    __shared__ uint32_t s_words[kZWaves][kZGroupWords + 2];
    const ZFillDev &f = a.f[blockIdx.y];
    const ZGeom g = z_geom(f);
    const int lane = threadIdx.x & 63;
    const int wl = threadIdx.x >> 6;
    uint32_t *acc = s_words[wl];
    const int64_t step = (int64_t)gridDim.x * kZWaves;
    for (int64_t g0 = (int64_t)blockIdx.x * kZWaves; g0 < g.groups; g0 += step) {
        const int64_t gi = g0 + wl;
        const bool live = gi < g.groups;
        ZLane o;
        if (live) {
            z_read(f, g, gi, lane, o);
        } else {
            o.n = 0;
            o.nw = 0;
            o.w = 0;
        }
        // exclusive prefix of the payload sizes over the group's blocks
        int64_t inc = o.nw;
#pragma unroll
        for (int d = 8; d < 64; d <<= 1) {
            const int64_t u = __shfl_up(inc, d, 64);
            if (lane >= d) inc += u;
        }
        const int64_t base = inc - o.nw;                 // words before this block in the group
        const int64_t total = __shfl(inc, 63, 64);       // the group's payload words
        const int64_t start = live ? f.gofs[gi] : 0;
        if (live && f.offsets && (lane & 7) == 0 && o.n > 0) f.offsets[o.b] = start + base;
        for (int k = lane; k < kZGroupWords + 2; k += 64) acc[k] = 0u;
        __syncthreads();
        if (o.w > 0) {
#pragma unroll
            for (int e = 0; e < kVec; e++) {
                const int i = (lane & 7) * kVec + e;
                if (i >= 1 && i < o.n) {
                    const uint32_t p = (uint32_t)base * 32u + (uint32_t)(i - 1) * o.w;
                    const uint32_t jw = p >> 5, s = p & 31u;
                    atomicOr(&acc[jw], o.z[e] << s);
                    if (s + o.w > 32u) atomicOr(&acc[jw + 1], o.z[e] >> (32u - s));
                }
            }
        }
        __syncthreads();
        for (int k = lane; k < total; k += 64) {
            const int64_t at = start + k;
            if (at < f.cap) f.words[at] = acc[k];
        }
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_z(const ZArgs &a, int grid, hipStream_t s) {
    if (a.n < 1 || a.n > kZMaxFills) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_z_size, dim3(grid, a.n), dim3(kZWaves * 64), 0, s, a);
    hipLaunchKernelGGL(k_z_scan, dim3(1, a.n), dim3(kZScanThreads), 0, s, a);
    hipLaunchKernelGGL(k_z_pack, dim3(grid, a.n), dim3(kZWaves * 64), 0, s, a);
    return hipGetLastError();
}

}  // namespace daqk
