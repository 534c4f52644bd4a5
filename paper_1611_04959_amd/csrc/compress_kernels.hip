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
// A wave takes groups of 8 consecutive blocks of one row: lane l holds the 8
// samples 8 l .. 8 l + 7 of a group (one 16-byte load), so block j of the
// group is lanes 8 j .. 8 j + 7. The groups of a fill are cut into one
// contiguous range per wave of the grid (fill = blockIdx.y). Two kernels:
// the size pass writes the block headers and each wave's payload words; the
// pack pass starts each wave at the sum of the sizes of the waves before it,
// walks its groups in order, ORs each lane's codes into the group's payload
// in LDS (a 64-bit bit writer per lane, one atomic per 32 bits) and stores
// the payload with coalesced writes. Every wave touches only its own LDS, so
// there are no work-group barriers.
#include "chop_internal.h"

namespace daqk {
namespace {

constexpr int kZBlock = 64;     // samples per block
constexpr int kZGroup = 8;      // blocks per wave
constexpr int kZMaxWords = 34;  // ceil(63 * 17 / 32): the widest block's payload
constexpr int kZGroupWords = kZGroup * kZMaxWords;
// Groups a wave loads before it uses them, in the size and the pack pass.
#ifndef DAQ_Z_UNROLL
#define DAQ_Z_UNROLL 4
#endif
#ifndef DAQ_Z_PACK_UNROLL
#define DAQ_Z_PACK_UNROLL 2
#endif
constexpr int kZUnroll = DAQ_Z_UNROLL;
constexpr int kZPackUnroll = DAQ_Z_PACK_UNROLL;

struct ZGeom {
    int64_t L;       // samples per row
    int64_t nb;      // blocks per row
    int64_t gpr;     // groups per row
    int64_t groups;  // groups of the fill
};

// Samples each row of fill f compresses: its total_len, clamped to [0, max_len].
__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// (The length comes from a vector load: taking it through readfirstlane lets
// the compiler keep the whole geometry in scalar registers.)
__device__ __forceinline__ ZGeom z_geom(const ZFillDev &f) {
    const int64_t tl = uniform_i64(*reinterpret_cast<const volatile int64_t *>(&f.counts->total_len));
    ZGeom g;
    g.L = tl < f.max_len ? (tl > 0 ? tl : 0) : f.max_len;
    g.nb = (g.L + kZBlock - 1) / kZBlock;
    g.gpr = (g.nb + kZGroup - 1) / kZGroup;
    g.groups = g.gpr * f.C;
    return g;
}

// The contiguous range of groups of wave v of W.
__device__ __forceinline__ void z_range(const ZGeom &g, int64_t v, int64_t W, int64_t *lo, int64_t *hi) {
    *lo = g.groups * v / W;
    *hi = g.groups * (v + 1) / W;
}

__device__ __forceinline__ uint32_t zigzag(int32_t r) { return ((uint32_t)r << 1) ^ (uint32_t)(r >> 31); }

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Where a group sits: its row and its index in the row (wave-uniform).
struct ZAt {
    int64_t c, gr;
};

// The lane's 8 samples of the group at `at` (zeros past the row's end).
__device__ __forceinline__ int4 z_load(const ZFillDev &f, const ZGeom &g, ZAt at, int lane) {
    const int64_t t0 = at.gr * (kZGroup * kZBlock) + lane * kVec;
    if (t0 >= g.L) return make_int4(0, 0, 0, 0);
    return *reinterpret_cast<const int4 *>(f.packed + at.c * f.stride + t0);
}

__device__ __forceinline__ void z_next(const ZGeom &g, ZAt &at) {
    if (++at.gr == g.gpr) {
        at.gr = 0;
        at.c++;
    }
}

// Lane-to-lane moves within rows of 16 lanes (DPP): the value of lane l - 1
// (lanes 16 k keep their own), and an OR over the 8 lanes of a block. The
// moves keep the lane's own value as the fallback, which stops the compiler
// from folding them into the arithmetic that uses them: a row shift folded
// into a reverse subtract gave wrong differences on gfx950.
__device__ __forceinline__ int32_t dpp_prev(int32_t v) { return __builtin_amdgcn_update_dpp(v, v, 0x111, 0xF, 0xF, false); }
__device__ __forceinline__ uint32_t or8(uint32_t m) {
    m |= (uint32_t)__builtin_amdgcn_update_dpp((int)m, (int)m, 0xB1, 0xF, 0xF, false);   // lanes 1 0 3 2
    m |= (uint32_t)__builtin_amdgcn_update_dpp((int)m, (int)m, 0x4E, 0xF, 0xF, false);   // lanes 2 3 0 1
    m |= (uint32_t)__builtin_amdgcn_update_dpp((int)m, (int)m, 0x141, 0xF, 0xF, false);  // 7 - i within 8
    return m;
}

// Samples in the lane's block (lane >> 3 of the group at `at`): 0 past the row.
__device__ __forceinline__ int z_block_len(const ZGeom &g, ZAt at, int lane) {
    const int64_t left = g.L - (at.gr * kZGroup + (lane >> 3)) * kZBlock;
    return left <= 0 ? 0 : (left < kZBlock ? (int)left : kZBlock);
}

// Zigzag codes of the lane's 8 samples, sample i = 8 sub + e of its block of
// n samples; 0 where there is no code (i = 0 or i >= n). kFull: n = 64.
template <bool kFull>
__device__ __forceinline__ void z_codes(int4 q, int sub, int n, uint32_t z[kVec]) {
    const int16_t *h = reinterpret_cast<const int16_t *>(&q);
    int32_t s[kVec];
#pragma unroll
    for (int e = 0; e < kVec; e++) s[e] = h[e];
    // lanes 16 k have no previous lane in their DPP row: they start a block
    const int32_t prev = dpp_prev(s[kVec - 1]);
#pragma unroll
    for (int e = 0; e < kVec; e++) {
        const uint32_t zz = zigzag(s[e] - (e ? s[e - 1] : prev));
        const int i = sub * kVec + e;
        if (kFull)
            z[e] = (e == 0 && sub == 0) ? 0u : zz;
        else
            z[e] = (i >= 1 && i < n) ? zz : 0u;
    }
}

__device__ __forceinline__ uint32_t z_width(const uint32_t z[kVec]) {
    uint32_t m = 0;
#pragma unroll
    for (int e = 0; e < kVec; e++) m |= z[e];
    m = or8(m);  // the bit length of the OR is that of the largest code
    return m ? 32u - (uint32_t)__clz(m) : 0u;
}

__device__ __forceinline__ uint32_t z_words(int n, uint32_t w) {
    return n > 0 ? ((uint32_t)(n - 1) * w + 31u) >> 5 : 0u;
}

__global__ void __launch_bounds__(kZWaves * 64) k_z_size(ZArgs a) {
    const ZFillDev &f = a.f[blockIdx.y];
    const ZGeom g = z_geom(f);
    const int lane = threadIdx.x & 63, sub = lane & 7;
    const int64_t W = (int64_t)gridDim.x * kZWaves;
    const int64_t v = (int64_t)blockIdx.x * kZWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int64_t lo, hi;
    z_range(g, v, W, &lo, &hi);
    ZAt at;
    at.c = g.gpr ? lo / g.gpr : 0;
    at.gr = lo - at.c * g.gpr;
    int64_t mine = 0;  // payload words of the lane's blocks (on each block's first lane)
    for (int64_t g0 = lo; g0 < hi; g0 += kZUnroll) {
        int4 q[kZUnroll];
        ZAt ats[kZUnroll];
#pragma unroll
        for (int u = 0; u < kZUnroll; u++) {
            ats[u] = at;
            q[u] = g0 + u < hi ? z_load(f, g, at, lane) : make_int4(0, 0, 0, 0);
            z_next(g, at);
        }
#pragma unroll
        for (int u = 0; u < kZUnroll; u++) {
            if (g0 + u >= hi) break;
            const bool full = (ats[u].gr + 1) * (kZGroup * kZBlock) <= g.L;
            const int n = full ? kZBlock : z_block_len(g, ats[u], lane);
            uint32_t z[kVec];
            if (full)
                z_codes<true>(q[u], sub, n, z);
            else
                z_codes<false>(q[u], sub, n, z);
            const uint32_t w = z_width(z);
            if (sub == 0 && n > 0) {
                f.hdr[ats[u].c * g.nb + ats[u].gr * kZGroup + (lane >> 3)] = ((uint32_t)q[u].x & 0xFFFFu) | (w << 16);
                mine += z_words(n, w);
            }
        }
    }
    const int64_t tot = wave_sum_i64(mine);
    if (lane == 0) f.gofs[v] = tot;
}

// Ordering of one wave's own LDS accesses (clear, OR, read back, clear).
__device__ __forceinline__ void wave_lds_order() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__global__ void __launch_bounds__(kZWaves * 64) k_z_pack(ZArgs a) {
    __shared__ uint32_t s_words[kZWaves][kZGroupWords + 2];
    const ZFillDev &f = a.f[blockIdx.y];
    const ZGeom g = z_geom(f);
    const int lane = threadIdx.x & 63;
    const int sub = lane & 7, jb = lane >> 3;
    const int wl = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint32_t *acc = s_words[wl];
    const int64_t W = (int64_t)gridDim.x * kZWaves;
    const int64_t v = (int64_t)blockIdx.x * kZWaves + wl;
    int64_t lo, hi;
    z_range(g, v, W, &lo, &hi);
    // where this wave's payload starts: the sizes of the waves before it
    int64_t before = 0;
#pragma unroll
    for (int r = 0; r < kZMaxGrid * kZWaves / 64; r++) {
        const int64_t k = lane + 64 * r;
        if (k < v) before += f.gofs[k];
    }
    int64_t carry = uniform_i64(wave_sum_i64(before));
    ZAt at;
    at.c = g.gpr ? lo / g.gpr : 0;
    at.gr = lo - at.c * g.gpr;
    for (int64_t g0 = lo; g0 < hi; g0 += kZPackUnroll) {
        int4 q[kZPackUnroll];
        uint32_t hw[kZPackUnroll];
        ZAt ats[kZPackUnroll];
#pragma unroll
        for (int u = 0; u < kZPackUnroll; u++) {
            ats[u] = at;
            const int64_t kb = at.gr * kZGroup + jb;
            q[u] = g0 + u < hi ? z_load(f, g, at, lane) : make_int4(0, 0, 0, 0);
            hw[u] = (g0 + u < hi && kb < g.nb) ? f.hdr[at.c * g.nb + kb] : 0u;
            z_next(g, at);
        }
#pragma unroll
        for (int u = 0; u < kZPackUnroll; u++) {
            if (g0 + u >= hi) break;
            const bool full = (ats[u].gr + 1) * (kZGroup * kZBlock) <= g.L;
            const int n = full ? kZBlock : z_block_len(g, ats[u], lane);
            uint32_t z[kVec];
            if (full)
                z_codes<true>(q[u], sub, n, z);
            else
                z_codes<false>(q[u], sub, n, z);
            const uint32_t w = hw[u] >> 16;
            const uint32_t nw = z_words(n, w);
            // the group's blocks' payload sizes: where the lane's block starts, and the total
            uint32_t base = 0, total = 0;
#pragma unroll
            for (int j = 0; j < kZGroup; j++) {
                const uint32_t t = (uint32_t)__builtin_amdgcn_readlane((int)nw, 8 * j);
                base += j < jb ? t : 0u;
                total += t;
            }
            if (f.offsets && sub == 0 && n > 0)
                f.offsets[ats[u].c * g.nb + ats[u].gr * kZGroup + jb] = carry + base;
            for (uint32_t k = lane; k < total; k += 64) acc[k] = 0u;
            wave_lds_order();
            // code i of the block sits at bit (i - 1) w of its payload; up to
            // 16 bits wide, two neighbouring codes go in with one OR pair
            if (w <= 16) {
#pragma unroll
                for (int m = 0; m < kVec / 2; m++) {
                    // the lane's first pair on a block's first lane is code 1 alone
                    const bool lead = sub == 0 && m == 0;
                    const uint32_t pv = lead ? z[1] : (z[2 * m] | (z[2 * m + 1] << w));
                    if (pv) {
                        const uint32_t pos = base * 32u + (uint32_t)(lead ? 0 : sub * kVec + 2 * m - 1) * w;
                        const uint64_t val = (uint64_t)pv << (pos & 31u);
                        atomicOr(&acc[pos >> 5], (uint32_t)val);
                        if ((uint32_t)(val >> 32)) atomicOr(&acc[(pos >> 5) + 1], (uint32_t)(val >> 32));
                    }
                }
            } else {
#pragma unroll
                for (int e = 0; e < kVec; e++) {
                    if (z[e]) {
                        const uint32_t pos = base * 32u + (uint32_t)(sub * kVec + e - 1) * w;
                        const uint64_t val = (uint64_t)z[e] << (pos & 31u);
                        atomicOr(&acc[pos >> 5], (uint32_t)val);
                        if ((uint32_t)(val >> 32)) atomicOr(&acc[(pos >> 5) + 1], (uint32_t)(val >> 32));
                    }
                }
            }
            wave_lds_order();
            for (uint32_t k = lane; k < total; k += 64) {
                const int64_t at_w = carry + k;
                if (at_w < f.cap) f.words[at_w] = acc[k];
            }
            wave_lds_order();
            carry += total;
        }
    }
    if (v == W - 1 && lane == 0) *f.n_words = carry;
}

// ---- decompression ------------------------------------------------------------
//
// The same 8-block groups: a wave copies the group's payload words (contiguous
// in the stream) into its LDS, then lane l decodes the codes of samples
// 8 l .. 8 l + 7 of the group (each from one or two words), undoes the
// zigzag, and adds the differences up: a prefix within the lane, then across
// the block's 8 lanes, plus the block's first sample. Words past n_words are
// read as zero, so a damaged stream cannot make the kernel read out of bounds.
__global__ void __launch_bounds__(kZWaves * 64) k_unz(ZDecArgs a) {
    __shared__ uint32_t s_words[kZWaves][kZGroupWords + 2];
    const ZStreamDev &f = a.f[blockIdx.y];
    const int lane = threadIdx.x & 63;
    const int sub = lane & 7, jb = lane >> 3;
    const int wl = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint32_t *buf = s_words[wl];
    const int64_t L = f.L;
    const int64_t nb = (L + kZBlock - 1) / kZBlock;
    const int64_t gpr = (nb + kZGroup - 1) / kZGroup;
    const int64_t groups = gpr * f.C;
    const int64_t step = (int64_t)gridDim.x * kZWaves;
    for (int64_t gi = (int64_t)blockIdx.x * kZWaves + wl; gi < groups; gi += step) {
        const int64_t c = gi / gpr;
        const int64_t kb0 = (gi - c * gpr) * kZGroup;
        const int64_t kb = kb0 + jb;
        const int64_t left = L - kb * kZBlock;
        const int n = left <= 0 ? 0 : (left < kZBlock ? (int)left : kZBlock);
        const int64_t b = c * nb + kb;
        uint32_t hw = 0;
        int64_t off = 0;
        if (n > 0) {
            hw = f.hdr[b];
            off = f.offsets[b];
        }
        uint32_t w = hw >> 16;
        w = w > 17u ? 17u : w;
        const uint32_t nw = n > 0 ? ((uint32_t)(n - 1) * w + 31u) >> 5 : 0u;
        // the group's payload: from its first block's offset to the end of its last block
        const int64_t start = __shfl(off, 0, 64);
        const int last = (int)((nb - kb0 < kZGroup ? nb - kb0 : kZGroup) - 1);
        const int64_t end = __shfl(off + (int64_t)nw, 8 * last, 64);
        int64_t span = end - start;
        span = span < 0 ? 0 : (span > kZGroupWords ? kZGroupWords : span);
        for (int k = lane; k < span + 2 && k < kZGroupWords + 2; k += 64) {
            const int64_t at = start + k;
            buf[k] = (at >= 0 && at < f.n_words && k < span) ? f.words[at] : 0u;
        }
        wave_lds_order();
        int32_t v[kVec];
        int32_t run = 0;
        if ((kb0 + kZGroup) * kZBlock <= L) {
            // every block of the group holds 64 samples (wave-uniform): no
            // per-code tests, 32-bit positions, one funnel shift per code;
            // the word index is clamped into the buffer (a damaged offset
            // reads other words of the group, never outside it)
            const int64_t rel64 = off - start;
            const int rel = (int)(rel64 < 0 ? 0 : (rel64 > kZGroupWords ? kZGroupWords : rel64));
            const uint32_t mask = (1u << w) - 1u;  // w <= 17; 0 for a constant block
            int pos = rel * 32 + (sub * kVec - 1) * (int)w;
#pragma unroll
            for (int e = 0; e < kVec; e++) {
                const int p = pos < 0 ? 0 : pos;  // sample 0 of a block has no code
                const int wi = (p >> 5) < kZGroupWords ? (p >> 5) : kZGroupWords;
                const uint32_t z = __builtin_amdgcn_alignbit(buf[wi + 1], buf[wi], (uint32_t)p & 31u) & mask;
                int32_t d = (int32_t)(z >> 1) ^ -(int32_t)(z & 1u);
                if (e == 0 && sub == 0) d = 0;
                run += d;
                v[e] = run;
                pos += (int)w;
            }
        } else {
#pragma unroll
            for (int e = 0; e < kVec; e++) {
                const int i = sub * kVec + e;
                int32_t d = 0;
                if (i >= 1 && i < n && w > 0) {
                    const int64_t pos = (off - start) * 32 + (int64_t)(i - 1) * w;
                    const int64_t wi = pos >> 5;
                    const uint32_t sh = (uint32_t)(pos & 31);
                    uint64_t pair = 0;
                    if (wi >= 0 && wi < kZGroupWords) pair = (uint64_t)buf[wi] | ((uint64_t)buf[wi + 1] << 32);
                    const uint32_t z = (uint32_t)(pair >> sh) & ((1u << w) - 1u);
                    d = (int32_t)(z >> 1) ^ -(int32_t)(z & 1u);
                }
                run += d;
                v[e] = run;
            }
        }
        // exclusive prefix of the lane totals over the block's 8 lanes
        int32_t inc = run;
#pragma unroll
        for (int dd = 1; dd < 8; dd <<= 1) {
            const int32_t t = __shfl_up(inc, dd, 64);
            if (sub >= dd) inc += t;
        }
        const int32_t before = inc - run + (int32_t)(int16_t)(hw & 0xFFFFu);
        wave_lds_order();
        if (n > 0) {
            int16_t *row = f.out + c * f.out_stride + kb * kZBlock + sub * kVec;
            const int valid = n - sub * kVec;
            if (valid >= kVec) {
                uint4 q;
                q.x = (uint32_t)(uint16_t)(before + v[0]) | ((uint32_t)(uint16_t)(before + v[1]) << 16);
                q.y = (uint32_t)(uint16_t)(before + v[2]) | ((uint32_t)(uint16_t)(before + v[3]) << 16);
                q.z = (uint32_t)(uint16_t)(before + v[4]) | ((uint32_t)(uint16_t)(before + v[5]) << 16);
                q.w = (uint32_t)(uint16_t)(before + v[6]) | ((uint32_t)(uint16_t)(before + v[7]) << 16);
                *reinterpret_cast<uint4 *>(row) = q;
            } else {
                for (int e = 0; e < valid; e++) row[e] = (int16_t)(before + v[e]);
            }
        }
    }
}

}  // namespace

hipError_t launch_unz(const ZDecArgs &a, int grid, hipStream_t s) {
    if (a.n < 1 || a.n > kZMaxFills || grid < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_unz, dim3(grid, a.n), dim3(kZWaves * 64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_z(const ZArgs &a, int grid, hipStream_t s) {
    if (a.n < 1 || a.n > kZMaxFills || grid < 1 || grid > kZMaxGrid) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_z_size, dim3(grid, a.n), dim3(kZWaves * 64), 0, s, a);
    hipLaunchKernelGGL(k_z_pack, dim3(grid, a.n), dim3(kZWaves * 64), 0, s, a);
    return hipGetLastError();
}

}  // namespace daqk
