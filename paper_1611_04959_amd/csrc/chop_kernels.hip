// chop_kernels.hip -- gfx950 kernels of libdaqisland.
//
// T-method island chopping (Section 3, T-method paragraph; Table 2):
// pedestals, calorimeter sum, threshold, pre/post dilation, merge, island
// array and packed island samples, all in integers.
//
// k_prepare  per fill: pedestals (Table 2 pedestal row) and the effective
//            threshold thr + sum(ped); clears the look-back words.
// k_chop     the fused pass. Each thread of a work-group takes 8 consecutive
//            samples (one 16-byte load per channel row); the work-group's
//            groups cover a tile of the fill plus a halo of post + 1 samples
//            on the left and pre + 1 on the right, whose flags are recomputed
//            from the raw data (wide windows load the halo in a separate
//            loop instead). Per tile:
//              1. int32 sums per sample over all channels (Table 2 waveform-
//                 sum row), compare (threshold row) -> one flag bit per
//                 sample in an LDS bitmap;
//              2. dilation (pre/post row) as "some flag in [t - post, t + pre]"
//                 via popcount prefixes of the bitmap; island edges follow;
//              3. a decoupled look-back over the fill's earlier tiles gives
//                 the number of island samples and islands before the tile;
//              4. island records (island-array row) and, when requested, the
//                 packed raw samples of every channel (the chopped islands),
//                 staged through LDS so that the global stores are whole,
//                 aligned 16-byte chunks.
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

// Set bits of the LDS bitmap below bit x0 + j, for j = 0 .. 9 (the window
// of ten consecutive prefix counts one thread needs; x0 + 9 <= 64 * Wn).
__device__ __forceinline__ void prefix_bits10(const uint64_t *words, const uint32_t *pc, int x0,
                                              uint32_t (&out)[10]) {
    const int w = x0 >> 6;
    const int b = x0 & 63;
    const uint64_t w0 = words[w];
    const uint64_t w1 = words[w + 1];
    const uint32_t base = pc[w];
    const uint32_t all0 = (uint32_t)__popcll(w0);
#pragma unroll
    for (int j = 0; j < 10; j++) {
        const int q = b + j;
        uint32_t c;
        if (q < 64) c = (uint32_t)__popcll(q ? (w0 & ((1ull << q) - 1ull)) : 0ull);
        else c = all0 + (uint32_t)__popcll((q - 64) ? (w1 & ((1ull << (q - 64)) - 1ull)) : 0ull);
        out[j] = base + c;
    }
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

// Puts the island samples (mask mm) of one 8-sample chunk into an LDS row at
// index idx0 onwards, packed. Dense chunks use the widest aligned stores.
__device__ __forceinline__ void stage_put(int16_t *row, int idx0, uint32_t mm, const uint4 v) {
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
    if (mm == 0xFFu) {
        if ((idx0 & 7) == 0) {
            *reinterpret_cast<uint4 *>(row + idx0) = v;
        } else if ((idx0 & 1) == 0) {
#pragma unroll
            for (int i = 0; i < 4; i++) reinterpret_cast<uint32_t *>(row + idx0)[i] = w[i];
        } else {
            row[idx0] = (int16_t)(w[0] & 0xFFFFu);
            uint32_t *d = reinterpret_cast<uint32_t *>(row + idx0 + 1);
            d[0] = (w[1] << 16) | (w[0] >> 16);
            d[1] = (w[2] << 16) | (w[1] >> 16);
            d[2] = (w[3] << 16) | (w[2] >> 16);
            row[idx0 + 7] = (int16_t)(w[3] >> 16);
        }
        return;
    }
    int idx = idx0;
#pragma unroll
    for (int k = 0; k < kVec; k++) {
        if ((mm >> k) & 1u) {
            const uint32_t word = w[k >> 1];
            row[idx++] = (int16_t)((k & 1) ? (word >> 16) : (word & 0xFFFFu));
        }
    }
}

// Element offset of a row's packed position `pos` within its 16-byte line.
__device__ __forceinline__ int line_phase(const int16_t *row, int64_t pos) {
    return (int)((((uintptr_t)row >> 1) + (uint64_t)pos) & 7u);
}

// Writes `len` staged samples of up to CB channel rows [c0, c0 + CB) to the
// packed output at position m0: LDS row cl holds element j at index
// phase(row, m0) + j, so every full 16-byte LDS chunk maps onto one aligned
// 16-byte global chunk.
template <int NT, int CB>
__device__ __forceinline__ void stage_flush(const int16_t *stage, int rs, int16_t *out, int64_t ostride,
                                            int c0, int C, int64_t m0, int len) {
    const int nch = (len + 7 + 7) >> 3;
    for (int i = threadIdx.x; i < CB * nch; i += NT) {
        const int cl = i / nch;
        const int q = i - cl * nch;
        const int c = c0 + cl;
        if (c >= C) continue;
        int16_t *row = out + (int64_t)c * ostride;
        const int ph = line_phase(row, m0);
        const int j0 = q * 8 - ph;  // element of chunk lane 0
        if (j0 >= len) continue;
        const int16_t *src = stage + cl * rs + q * 8;
        const int64_t g0 = m0 + j0;
        if (j0 >= 0 && j0 + 8 <= len && g0 + 8 <= ostride) {
            *reinterpret_cast<uint4 *>(row + g0) = *reinterpret_cast<const uint4 *>(src);
        } else {
#pragma unroll
            for (int e = 0; e < 8; e++) {
                const int j = j0 + e;
                if (j >= 0 && j < len && m0 + j < ostride) row[m0 + j] = src[e];
            }
        }
    }
}

template <int NT>
struct ChopLds {
    static constexpr int kGroups = 2 * kMaxHaloGroups + NT;  // widest bitmap
    static constexpr int kWords = (kGroups + 7) / 8 + 1;
    static constexpr int kBitsBytes = kWords * 8 + (kWords + 1) * 4;
    static constexpr int kCB = NT == 256 ? 8 : 4;            // channels staged per round
    static constexpr int kRowStride = NT * kVec + 16;        // elements per staged row
    static constexpr int kStageBytes = kCB * kRowStride * 2;
    static constexpr int kBytes = kBitsBytes > kStageBytes ? kBitsBytes : kStageBytes;
};

template <int NT, bool RESIDENT>
__device__ __forceinline__ void chop_tile(const KArgs &a, const FillDev &fd, int f, int64_t tile, uint8_t *lds,
                                          uint32_t *s_wsum, uint64_t *s_excl) {
    constexpr int NW = NT / 64;
    constexpr int CR = RESIDENT ? kResidentChannels : 1;
    constexpr int CB = ChopLds<NT>::kCB;
    constexpr int RS = ChopLds<NT>::kRowStride;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;

    const int64_t lt = tile - fd.tile_base;
    const int64_t N = fd.n;
    const int C = RESIDENT ? kResidentChannels : fd.C;
    const int64_t stride = fd.stride;
    const int16_t *raw = fd.raw;
    const int gl = fd.gl;
    const int gr = fd.gr;
    const bool wide = fd.wide != 0;
    const int G = wide ? gl + NT + gr : NT;           // bitmap groups
    const int64_t t0 = lt * fd.tout;                  // first sample the tile owns
    const int64_t base = t0 - (int64_t)gl * kVec;     // sample at bitmap bit 0
    const int g = wide ? gl + tid : tid;              // this thread's group
    const bool owner = wide || (tid >= gl && tid < NT - gr);
    const int64_t p = base + (int64_t)g * kVec;       // its first sample
    int64_t te = a.thr_eff[f];
    te = te > 2147483647LL ? 2147483647LL : (te < -2147483648LL ? -2147483648LL : te);
    const int32_t thr_eff = (int32_t)te;

    uint8_t *s_bits = lds;
    uint32_t *s_pc = reinterpret_cast<uint32_t *>(lds + ChopLds<NT>::kWords * 8);
    int16_t *s_stage = reinterpret_cast<int16_t *>(lds);

    // 1. flags of this thread's 8 samples from all channel rows (Table 2
    //    waveform-sum and threshold rows); halo groups of wide windows apart
    uint4 xr[CR];
    uint32_t fb = 0;
    if (p >= 0 && p < N) {
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
    s_bits[g] = (uint8_t)fb;
    if (wide) {
        for (int h = tid; h < gl + gr; h += NT) {
            const int hg = (h < gl) ? h : (NT + h);
            const int64_t q = base + (int64_t)hg * kVec;
            uint32_t hb = 0;
            if (q >= 0 && q < N) hb = group_flags(raw + q, stride, C, thr_eff, N - q);
            s_bits[hg] = (uint8_t)hb;
        }
    }
    const int Wn = (G + 7) >> 3;  // bitmap words; word Wn stays zero
    for (int z = G + tid; z < (Wn + 1) * 8; z += NT) s_bits[z] = 0;
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

    // 2b. dilation (Table 2 pre/post row): sample t is inside an island when
    //     a flag lies in [t - post, t + pre]; masks for p-1 .. p+8
    uint32_t m10 = 0;
    if (owner) {
        const int r0 = g * kVec;
        uint32_t lo[10], hi[10];
        prefix_bits10(words, s_pc, r0 - 1 - fd.post, lo);
        prefix_bits10(words, s_pc, r0 + fd.pre, hi);
#pragma unroll
        for (int j = 0; j < 10; j++) {
            const int64_t t = p + j - 1;
            const bool in = (hi[j] != lo[j]) && t >= 0 && t < N;
            m10 |= (in ? 1u : 0u) << j;
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
    const int th_m = (int)(excl >> 16), th_i = (int)(excl & 0xFFFFu);
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

    // 4a. island records (Table 2 island-array row)
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

    // 4b. chopped islands: the packed raw samples of every channel, staged in
    //     LDS per CB channels so that global stores are aligned 16-byte lines
    if (fd.out != nullptr && tile_m > 0) {
        int16_t *out = fd.out;
        const int64_t ostride = fd.out_stride;
        const int len = (int)tile_m;
        if constexpr (RESIDENT) {
#pragma unroll
            for (int c0 = 0; c0 < kResidentChannels; c0 += CB) {
                if (mm) {
#pragma unroll
                    for (int cl = 0; cl < CB; cl++) {
                        if (c0 + cl < kResidentChannels) {
                            const int ph = line_phase(out + (int64_t)(c0 + cl) * ostride, m_before);
                            stage_put(s_stage + cl * RS, ph + th_m, mm, xr[c0 + cl]);
                        }
                    }
                }
                __syncthreads();
                stage_flush<NT, CB>(s_stage, RS, out, ostride, c0, kResidentChannels, m_before, len);
                __syncthreads();
            }
        } else {
            for (int c0 = 0; c0 < C; c0 += CB) {
                if (mm) {
                    uint4 v[CB];
#pragma unroll
                    for (int cl = 0; cl < CB; cl++)
                        if (c0 + cl < C) v[cl] = load16(raw + p + (int64_t)(c0 + cl) * stride);
#pragma unroll
                    for (int cl = 0; cl < CB; cl++) {
                        if (c0 + cl < C) {
                            const int ph = line_phase(out + (int64_t)(c0 + cl) * ostride, m_before);
                            stage_put(s_stage + cl * RS, ph + th_m, mm, v[cl]);
                        }
                    }
                }
                __syncthreads();
                stage_flush<NT, CB>(s_stage, RS, out, ostride, c0, C, m_before, len);
                __syncthreads();
            }
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

template <int NT, bool RESIDENT>
__global__ void __launch_bounds__(NT) k_chop(KArgs a) {
    __shared__ __align__(16) uint8_t s_lds[ChopLds<NT>::kBytes];
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
            chop_tile<NT, RESIDENT>(a, fd, lo, tile, s_lds, s_wsum, &s_excl);
        else
            chop_tile<NT, false>(a, fd, lo, tile, s_lds, s_wsum, &s_excl);
        __syncthreads();
    }
}

// Pedestals (Table 2 pedestal row), effective thresholds, cleared look-back
// words and counts. A block handles whole fills; its threads take
// (channel, 8-sample chunk) pairs of the pedestal window with 16-byte loads.
__global__ void __launch_bounds__(256) k_prepare(KArgs a) {
    constexpr int kChan = 512;  // channels accumulated per round
    __shared__ long long s_acc[kChan];
    __shared__ long long s_ped;
    const int nf = a.hdr ? a.hdr->n_fills : a.n_fills;
    const int64_t total = a.hdr ? a.hdr->total_tiles : a.total_tiles;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256)
        a.tile_state[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.ticket = 0;
    for (int f = blockIdx.x; f < nf; f += gridDim.x) {
        const FillDev fd = fill_at(a, f);
        const int64_t n = fd.n < (int64_t)fd.np ? fd.n : (int64_t)fd.np;
        const int64_t nch = (n + kVec - 1) / kVec;
        if (threadIdx.x == 0) s_ped = 0;
        for (int c0 = 0; c0 < fd.C; c0 += kChan) {
            const int cn = fd.C - c0 < kChan ? fd.C - c0 : kChan;
            for (int i = threadIdx.x; i < cn; i += 256) s_acc[i] = 0;
            __syncthreads();
            const int64_t items = (int64_t)cn * nch;
            for (int64_t i = threadIdx.x; i < items; i += 256) {
                const int cl = (int)(i / nch);
                const int64_t t = (i - (int64_t)cl * nch) * kVec;
                const uint4 v = load16(fd.raw + (int64_t)(c0 + cl) * fd.stride + t);
                int32_t s[kVec] = {0, 0, 0, 0, 0, 0, 0, 0};
                add8(s, v);
                int32_t part = 0;
#pragma unroll
                for (int k = 0; k < kVec; k++) part += (t + k < n) ? s[k] : 0;
                atomicAdd(reinterpret_cast<unsigned long long *>(&s_acc[cl]),
                          (unsigned long long)(long long)part);
            }
            __syncthreads();
            for (int i = threadIdx.x; i < cn; i += 256) {
                const int32_t ped = n > 0 ? (int32_t)floor_div(2 * (int64_t)s_acc[i] + n, 2 * n) : 0;
                if (fd.ped) fd.ped[c0 + i] = ped;
                atomicAdd(reinterpret_cast<unsigned long long *>(&s_ped), (unsigned long long)(long long)ped);
            }
            __syncthreads();
        }
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
