// chop_kernels.hip -- gfx950 kernels of libdaqisland.
//
// T-method island chopping (Section 3, T-method paragraph; Table 2):
// pedestals, calorimeter sum, threshold, pre/post dilation, merge, island
// array and packed island samples, all in integers.
//
// k_prepare  per fill: pedestals (Table 2 pedestal row) and the effective
//            threshold thr + sum(ped); clears the look-back words.
// k_chop     the fused pass. A work-group owns a tile of T = threads x 8
//            consecutive samples of every channel of one fill:
//              1. 16-byte loads of each channel row, int32 sums per sample
//                 (Table 2 waveform-sum row), compare (threshold row) ->
//                 one flag bit per sample, written to an LDS bitmap that also
//                 covers a halo of post + 1 samples on the left and pre + 1 on
//                 the right (flags there are recomputed from the raw data);
//              2. dilation (pre/post row) as "some flag in [t - post, t + pre]"
//                 via popcount prefixes of the bitmap; island edges follow;
//              3. a decoupled look-back over the fill's earlier tiles gives
//                 the number of island samples and islands before the tile;
//              4. island records (island-array row) and, when requested, the
//                 packed raw samples of every channel (the chopped islands).
//            Each record field has exactly one writer: the tile holding an
//            island's first sample writes start and offset, the tile holding
//            its last sample writes stop. No second pass is needed.
// k_gather   packed samples from an existing island table (two-pass path).
//
// Look-back words are 64 bits: flag (2) | samples (31) | islands (31). They
// carry all the data a reader needs, so relaxed agent-scope atomics suffice:
// no other memory is published through them.
#include "chop_internal.h"

namespace daqk {
namespace {

constexpr uint64_t kFlagAgg = 1ull << 62;   // tile total published
constexpr uint64_t kFlagIncl = 2ull << 62;  // inclusive prefix published
constexpr uint64_t kValMask = (1ull << 62) - 1;
constexpr uint64_t kField = 0x7FFFFFFFull;

__device__ __forceinline__ int64_t floor_div(int64_t a, int64_t b) {  // b > 0
    int64_t q = a / b;
    return (a - q * b < 0) ? q - 1 : q;
}

__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v, int lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Descriptor of fill f: from the device table, or the single fill passed in
// the kernel arguments. Returned by value so that no pointer to the kernel
// arguments is formed.
__device__ __forceinline__ FillDev fill_at(const KArgs &a, int f) {
    if (a.table) return a.table[f];
    return a.one;
}

__device__ __forceinline__ int64_t tile_base_at(const KArgs &a, int f) {
    return a.table ? a.table[f].tile_base : a.one.tile_base;
}

// Adds the eight int16 samples of one 16-byte row chunk to eight sums.
__device__ __forceinline__ void add8(int32_t (&s)[kVec], const uint4 v) {
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; i++) {
        s[2 * i] += (int32_t)(int16_t)(w[i] & 0xFFFFu);
        s[2 * i + 1] += ((int32_t)w[i]) >> 16;
    }
}

__device__ __forceinline__ uint32_t flags8(const int32_t (&s)[kVec], int32_t thr_eff, int64_t valid) {
    uint32_t fb = 0;
#pragma unroll
    for (int k = 0; k < kVec; k++) fb |= (s[k] < thr_eff ? 1u : 0u) << k;
    if (valid < kVec) fb &= (1u << valid) - 1u;
    return fb;
}

__device__ __forceinline__ uint4 load16(const int16_t *p) {
    return *reinterpret_cast<const uint4 *>(p);
}

// Flags of 8 samples starting at p (all C rows read, nothing kept).
__device__ uint32_t group_flags(const int16_t *p, int64_t stride, int C, int32_t thr_eff,
                                int64_t valid) {
    int32_t s[kVec] = {0, 0, 0, 0, 0, 0, 0, 0};
    int c = 0;
    for (; c + 6 <= C; c += 6) {
        uint4 v[6];
#pragma unroll
        for (int u = 0; u < 6; u++) v[u] = load16(p + (int64_t)(c + u) * stride);
#pragma unroll
        for (int u = 0; u < 6; u++) add8(s, v[u]);
    }
    for (; c < C; c++) add8(s, load16(p + (int64_t)c * stride));
    return flags8(s, thr_eff, valid);
}

// Number of set bits of the LDS bitmap below bit q.
__device__ __forceinline__ uint32_t prefix_bits(const uint64_t *words, const uint32_t *pc, int q) {
    const int w = q >> 6;
    const int b = q & 63;
    const uint64_t below = b ? (words[w] & ((1ull << b) - 1ull)) : 0ull;
    return pc[w] + (uint32_t)__popcll(below);
}

// Sum of the published values of this fill's tiles [0, lt): the exclusive
// prefix of (island samples, islands). Executed by one whole wave.
__device__ uint64_t look_back(uint64_t *st, int64_t lt, int lane) {
    uint64_t acc = 0;
    int64_t hi = lt - 1;
    for (;;) {
        const int64_t j = hi - lane;
        uint64_t s = kFlagIncl;  // before the fill's first tile: empty prefix
        if (j >= 0) s = __hip_atomic_load(st + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t flag = s & ~kValMask;
        const uint64_t b_incl = __ballot(flag == kFlagIncl);
        const uint64_t b_none = __ballot(flag == 0);
        const uint64_t first = b_incl & (0ull - b_incl);         // lowest lane with a prefix
        const uint64_t need = b_incl ? (first | (first - 1ull)) : ~0ull;
        if (b_none & need) {  // a tile we depend on has not published yet
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        const bool mine = (need >> lane) & 1ull;
        acc += wave_sum_u64(mine ? (s & kValMask) : 0ull);
        if (b_incl) return acc;
        hi -= 64;
    }
}

// Packed-output store of a thread's 8 samples of one channel row.
__device__ __forceinline__ void store_packed(int16_t *orow, int64_t pos0, uint32_t mm,
                                             const uint4 v, int64_t ostride) {
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
    if (mm == 0xFFu && pos0 + kVec <= ostride) {
        int16_t *dst = orow + pos0;
        const uintptr_t addr = reinterpret_cast<uintptr_t>(dst);
        if ((addr & 15u) == 0) {
            *reinterpret_cast<uint4 *>(dst) = v;
            return;
        }
        if ((addr & 3u) == 0) {
#pragma unroll
            for (int i = 0; i < 4; i++) reinterpret_cast<uint32_t *>(dst)[i] = w[i];
            return;
        }
    }
    int64_t pos = pos0;
#pragma unroll
    for (int k = 0; k < kVec; k++) {
        if ((mm >> k) & 1u) {
            if (pos < ostride) {
                const uint32_t word = w[k >> 1];
                orow[pos] = (int16_t)((k & 1) ? (word >> 16) : (word & 0xFFFFu));
            }
            pos++;
        }
    }
}

template <int NT, bool RESIDENT>
__device__ __forceinline__ void chop_tile(const KArgs &a, const FillDev &fd, int f, int64_t tile, uint8_t *s_bits,
                          uint32_t *s_pc, uint32_t *s_wsum, uint64_t *s_excl) {
    constexpr int T = NT * kVec;
    constexpr int NW = NT / 64;
    constexpr int CR = RESIDENT ? kResidentChannels : 1;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;

    const int64_t lt = tile - fd.tile_base;
    const int64_t t0 = lt * T;
    const int64_t N = fd.n;
    const int C = fd.C;
    const int64_t stride = fd.stride;
    const int16_t *raw = fd.raw;
    const int gl = (fd.post + 1 + kVec - 1) / kVec;  // left halo groups
    const int gr = (fd.pre + 1 + kVec - 1) / kVec;   // right halo groups
    const int G = gl + NT + gr;
    const int64_t base = t0 - (int64_t)gl * kVec;    // sample at bitmap bit 0
    int64_t te = a.thr_eff[f];
    te = te > 2147483647LL ? 2147483647LL : (te < -2147483648LL ? -2147483648LL : te);
    const int32_t thr_eff = (int32_t)te;

    // 1a. main group: 8 samples of every channel
    const int64_t p = t0 + (int64_t)tid * kVec;
    uint4 xr[CR];
    uint32_t fb = 0;
    if (p < N) {
        if constexpr (RESIDENT) {
#pragma unroll
            for (int c = 0; c < kResidentChannels; c++) xr[c] = load16(raw + p + (int64_t)c * stride);
            int32_t s[kVec] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
            for (int c = 0; c < kResidentChannels; c++) add8(s, xr[c]);
            fb = flags8(s, thr_eff, N - p);
        } else {
            fb = group_flags(raw + p, stride, C, thr_eff, N - p);
        }
    }
    s_bits[gl + tid] = (uint8_t)fb;
    // 1b. halo groups (flags only)
    for (int h = tid; h < gl + gr; h += NT) {
        const int g = (h < gl) ? h : (NT + h);
        const int64_t q = base + (int64_t)g * kVec;
        uint32_t hb = 0;
        if (q >= 0 && q < N) hb = group_flags(raw + q, stride, C, thr_eff, N - q);
        s_bits[g] = (uint8_t)hb;
    }
    const int Wn = (G + 7) >> 3;  // bitmap words; word Wn stays zero
    for (int g = G + tid; g < (Wn + 1) * 8; g += NT) s_bits[g] = 0;
    __syncthreads();

    // 2a. exclusive popcount prefix over the bitmap words (wave 0)
    const uint64_t *words = reinterpret_cast<const uint64_t *>(s_bits);
    if (wid == 0) {
        uint32_t carry = 0;
        for (int w0 = 0; w0 <= Wn; w0 += 64) {
            const int w = w0 + lane;
            const uint32_t c = (w <= Wn) ? (uint32_t)__popcll(words[w]) : 0u;
            const uint32_t inc = wave_incl_scan_u32(c, lane);
            if (w <= Wn) s_pc[w] = carry + inc - c;
            carry += __shfl(inc, 63, 64);
        }
    }
    __syncthreads();

    // 2b. dilated mask for samples p-1 .. p+8 and island edges of p .. p+7
    uint32_t m10 = 0;
    {
        const int r0 = (gl + tid) * kVec;
#pragma unroll
        for (int k = -1; k <= kVec; k++) {
            const int64_t t = p + k;
            const uint32_t lo = prefix_bits(words, s_pc, r0 + k - fd.post);
            const uint32_t hi = prefix_bits(words, s_pc, r0 + k + fd.pre + 1);
            const bool in = (hi != lo) && t >= 0 && t < N;
            m10 |= (in ? 1u : 0u) << (k + 1);
        }
    }
    const uint32_t mm = (m10 >> 1) & 0xFFu;
    const uint32_t rise = mm & ~(((mm << 1) | (m10 & 1u)) & 0xFFu);
    const uint32_t fall = mm & ~((mm >> 1) | (((m10 >> 9) & 1u) << 7));

    // 2c. work-group exclusive scan of (island samples << 16 | islands)
    const uint32_t mine = ((uint32_t)__popc(mm) << 16) | (uint32_t)__popc(rise);
    const uint32_t inc = wave_incl_scan_u32(mine, lane);
    if (lane == 63) s_wsum[wid] = inc;
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < NW; w++) {
        const uint32_t v = s_wsum[w];
        before += (w < wid) ? v : 0u;
        total += v;
    }
    const uint32_t excl = before + inc - mine;
    const int64_t th_m = excl >> 16, th_i = excl & 0xFFFFu;
    const uint64_t tile_m = total >> 16, tile_i = total & 0xFFFFu;

    // 3. decoupled look-back over the fill's earlier tiles (wave 0)
    if (wid == 0) {
        uint64_t *st = a.tile_state + fd.tile_base;
        const uint64_t agg = (tile_m << 31) | tile_i;
        uint64_t ex = 0;
        if (lt == 0) {
            if (lane == 0) __hip_atomic_store(st, kFlagIncl | agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            if (lane == 0) __hip_atomic_store(st + lt, kFlagAgg | agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ex = look_back(st, lt, lane);
            if (lane == 0)
                __hip_atomic_store(st + lt, kFlagIncl | (ex + agg), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (lane == 0) *s_excl = ex;
    }
    __syncthreads();
    const uint64_t ex = *s_excl;
    const int64_t m_before = (int64_t)((ex >> 31) & kField);
    const int64_t i_before = (int64_t)(ex & kField);
    const int64_t mbase = m_before + th_m;  // packed position of this thread's first island sample
    const int64_t ibase = i_before + th_i;  // islands starting before this thread's samples

    // 4a. island records
    if (rise | fall) {
        daq_island *isl = fd.isl;
        const int64_t cap = fd.cap;
#pragma unroll
        for (int k = 0; k < kVec; k++) {
            if ((rise >> k) & 1u) {
                const int64_t idx = ibase + __popc(rise & ((1u << k) - 1u));
                if (idx < cap) {
                    isl[idx].start = p + k;
                    isl[idx].offset = mbase + __popc(mm & ((1u << k) - 1u));
                }
            }
            if ((fall >> k) & 1u) {
                const int64_t idx = ibase + __popc(rise & ((2u << k) - 1u)) - 1;
                if (idx >= 0 && idx < cap) isl[idx].stop = p + k + 1;
            }
        }
    }

    // 4b. packed raw samples of every channel (chopped islands)
    if (fd.out != nullptr && mm != 0) {
        const int64_t ostride = fd.out_stride;
        if constexpr (RESIDENT) {
#pragma unroll
            for (int c = 0; c < kResidentChannels; c++)
                store_packed(fd.out + (int64_t)c * ostride, mbase, mm, xr[c], ostride);
        } else {
            for (int c = 0; c < C; c++)
                store_packed(fd.out + (int64_t)c * ostride, mbase, mm, load16(raw + p + (int64_t)c * stride),
                             ostride);
        }
    }

    // 5. totals, written by the fill's last tile
    if (tid == 0 && lt == fd.n_tiles - 1 && fd.counts != nullptr) {
        const int64_t n_isl = i_before + (int64_t)tile_i;
        const int64_t tl = m_before + (int64_t)tile_m;
        int32_t status = (n_isl > fd.cap) ? DAQ_STATUS_CAPACITY : 0;
        if (fd.out != nullptr && tl > fd.out_stride) status |= DAQ_STATUS_OUT_STRIDE;
        fd.counts->n_islands = n_isl;
        fd.counts->total_len = tl;
        fd.counts->status = status;
        fd.counts->reserved = 0;
    }
}

template <int NT>
struct ChopLds {
    static constexpr int kGroups = 2 * kMaxHaloGroups + NT;
    static constexpr int kWords = (kGroups + 7) / 8 + 1;
};

template <int NT, bool RESIDENT>
__global__ void __launch_bounds__(NT) k_chop(KArgs a) {
    __shared__ __align__(16) uint8_t s_bits[ChopLds<NT>::kWords * 8];
    __shared__ uint32_t s_pc[ChopLds<NT>::kWords + 1];
    __shared__ uint32_t s_wsum[NT / 64];
    __shared__ uint64_t s_excl;
    __shared__ int64_t s_tile;

    const int nf = a.hdr ? a.hdr->n_fills : a.n_fills;
    const int64_t total = a.hdr ? a.hdr->total_tiles : a.total_tiles;
    for (;;) {
        if (threadIdx.x == 0) s_tile = (int64_t)atomicAdd(a.ticket, 1u);
        __syncthreads();
        const int64_t tile = s_tile;
        if (tile >= total) break;
        // the fill owning this tile: the last one whose first tile is <= tile
        int lo = 0, hi = nf - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tile_base_at(a, mid) <= tile) lo = mid;
            else hi = mid - 1;
        }
        const FillDev fd = fill_at(a, lo);
        if (RESIDENT && fd.C == kResidentChannels)
            chop_tile<NT, RESIDENT>(a, fd, lo, tile, s_bits, s_pc, s_wsum, &s_excl);
        else
            chop_tile<NT, false>(a, fd, lo, tile, s_bits, s_pc, s_wsum, &s_excl);
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) k_prepare(KArgs a) {
    __shared__ unsigned long long s_ped;
    const int nf = a.hdr ? a.hdr->n_fills : a.n_fills;
    const int64_t total = a.hdr ? a.hdr->total_tiles : a.total_tiles;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256)
        a.tile_state[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.ticket = 0;
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    for (int f = blockIdx.x; f < nf; f += gridDim.x) {
        const FillDev fd = fill_at(a, f);
        if (threadIdx.x == 0) s_ped = 0;
        __syncthreads();
        const int64_t n = fd.n < (int64_t)fd.np ? fd.n : (int64_t)fd.np;
        for (int c = wid; c < fd.C; c += 4) {
            const int16_t *row = fd.raw + (int64_t)c * fd.stride;
            int64_t P = 0;
            for (int64_t t = lane; t < n; t += 64) P += row[t];
            P = wave_sum_i64(P);
            if (lane == 0) {
                const int32_t ped = n > 0 ? (int32_t)floor_div(2 * P + n, 2 * n) : 0;
                if (fd.ped) fd.ped[c] = ped;
                atomicAdd(&s_ped, (unsigned long long)(int64_t)ped);
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            a.thr_eff[f] = (int64_t)fd.thr + (int64_t)s_ped;
            if (fd.counts) {
                fd.counts->n_islands = 0;
                fd.counts->total_len = 0;
                fd.counts->status = 0;
                fd.counts->reserved = 0;
            }
        }
        __syncthreads();
    }
}

// Two-pass gather: thread handles packed positions p0 + tid + 256 k.
__global__ void __launch_bounds__(256) k_gather(GatherArgs g) {
    constexpr int K = 8;
    const int64_t n_all = g.counts->n_islands;
    const int64_t n = n_all < g.cap ? n_all : g.cap;
    if (n <= 0) return;
    const daq_island last = g.isl[n - 1];
    const int64_t total = last.offset + (last.stop - last.start);
    if (blockIdx.x == 0 && threadIdx.x == 0 && g.counts->total_len > g.out_stride)
        atomicOr(&g.counts->status, DAQ_STATUS_OUT_STRIDE);
    const int64_t lim = total < g.out_stride ? total : g.out_stride;
    for (int64_t p0 = (int64_t)blockIdx.x * 256 * K; p0 < lim; p0 += (int64_t)gridDim.x * 256 * K) {
        int64_t src[K];
        int64_t dst[K];
#pragma unroll
        for (int k = 0; k < K; k++) {
            const int64_t pos = p0 + threadIdx.x + 256 * k;
            dst[k] = -1;
            src[k] = 0;
            if (pos < lim) {
                int64_t lo = 0, hi = n - 1;  // last island whose offset <= pos
                while (lo < hi) {
                    const int64_t mid = (lo + hi + 1) >> 1;
                    if (g.isl[mid].offset <= pos) lo = mid;
                    else hi = mid - 1;
                }
                dst[k] = pos;
                src[k] = g.isl[lo].start + (pos - g.isl[lo].offset);
            }
        }
        for (int c = 0; c < g.C; c++) {
            const int16_t *row = g.raw + (int64_t)c * g.stride;
            int16_t *orow = g.out + (int64_t)c * g.out_stride;
#pragma unroll
            for (int k = 0; k < K; k++)
                if (dst[k] >= 0) orow[dst[k]] = row[src[k]];
        }
    }
}

}  // namespace

hipError_t launch_prepare(const KArgs &a, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_prepare, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_chop(const KArgs &a, int threads, bool resident, int grid, hipStream_t s) {
    if (threads == 256) {
        if (resident) hipLaunchKernelGGL((k_chop<256, true>), dim3(grid), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_chop<256, false>), dim3(grid), dim3(256), 0, s, a);
    } else if (threads == 512) {
        if (resident) hipLaunchKernelGGL((k_chop<512, true>), dim3(grid), dim3(512), 0, s, a);
        else hipLaunchKernelGGL((k_chop<512, false>), dim3(grid), dim3(512), 0, s, a);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_gather(const GatherArgs &g, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_gather, dim3(grid), dim3(256), 0, s, g);
    return hipGetLastError();
}

int chop_max_threads(int threads, bool resident) {
    (void)resident;
    return threads;
}

}  // namespace daqk
