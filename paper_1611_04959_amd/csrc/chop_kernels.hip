// chop_kernels.hip -- gfx950 kernels of libdaqisland.
//
// T-method island chopping (Section 3, T-method paragraph; Table 2):
// pedestals, calorimeter sum, threshold, pre/post dilation, merge, island
// array and packed island samples, all in integers.
//
// k_prepare  per fill: pedestals (Table 2 pedestal row) and the effective
//            threshold thr + sum(ped); clears the look-back words and counts
//            (every schedule but the split one, which sums the pedestals in
//            its scan).
// k_scan_pass, k_edge_pass, k_copy_pass
//            the split schedule (the default): a streaming scan that computes
//            its fill's pedestals and writes one island-mask bit per sample
//            and tile totals; an edge pass
//            (one wave per tile: its prefix from the totals of the fill's
//            earlier tiles, the island records, a run table, the counts);
//            and a copy of the island samples in equal chunks of packed
//            positions.
// k_pipe     one persistent kernel: scan tiles (steps 1-4a below) and copy
//            chunks of finished fills, taken from shared counters.
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

// Work-group barrier for LDS traffic only. Global stores stay in flight: no
// wave of a tile reads what another wave wrote to global memory (tiles talk
// through the look-back atomics), so waiting for them would only add latency.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Global-memory views of generic pointers: descriptors arrive from memory, so
// without these the compiler would address fill data with flat instructions.
#define DAQ_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ DAQ_GLOBAL T *gbl(T *p) {
    return (DAQ_GLOBAL T *)p;
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Descriptor of fill f: from the device table, or the single fill passed in
// the kernel arguments. Returned by value so that no pointer to the kernel
// arguments is formed. f must be the same in every lane of the wave; the
// descriptor is then made wave-uniform (scalar registers).
__device__ __forceinline__ FillDev fill_at(const KArgs &a, int f) {
    if (a.table) {
        f = __builtin_amdgcn_readfirstlane(f);
        union {
            FillDev d;
            u32x4 v[sizeof(FillDev) / 16];
        } u;
        const DAQ_GLOBAL u32x4 *src = (const DAQ_GLOBAL u32x4 *)(a.table + f);
#pragma unroll
        for (int i = 0; i < (int)(sizeof(FillDev) / 16); i++) {
            const u32x4 w = src[i];
            u.v[i] = u32x4{(unsigned)__builtin_amdgcn_readfirstlane((int)w.x),
                           (unsigned)__builtin_amdgcn_readfirstlane((int)w.y),
                           (unsigned)__builtin_amdgcn_readfirstlane((int)w.z),
                           (unsigned)__builtin_amdgcn_readfirstlane((int)w.w)};
        }
        return u.d;
    }
    return a.one;
}

// Whether the launch reads its raw rows with non-temporal loads.
__device__ __forceinline__ bool stream_loads(const KArgs &a) {
    return (a.hdr ? a.hdr->stream_loads : a.stream_loads) != 0;
}

__device__ __forceinline__ int64_t tile_base_at(const KArgs &a, int f) {
    return a.table ? gbl(a.table + f)->tile_base : a.one.tile_base;
}

// The edge pass copies the descriptors of batches of at most kFdLds fills
// into LDS once per work-group, with the tile bases: a wave that meets a new
// fill then reads its descriptor from LDS instead of waiting on a global
// load. (The scan and copy passes do not: there the copy cost as much as
// the load it saves, or more.)
constexpr int kFdLds = 16;
constexpr int kFdWords = (int)(sizeof(FillDev) / 16);

// Copies the first nf descriptors of the table into s (call before the
// barrier that publishes it); false when the batch is too large or has no table.
template <int NT>
__device__ __forceinline__ bool stage_fills(const KArgs &a, int nf, u32x4 *s) {
    if (a.table == nullptr || nf > kFdLds) return false;
    const DAQ_GLOBAL u32x4 *src = (const DAQ_GLOBAL u32x4 *)a.table;
    for (int i = threadIdx.x; i < nf * kFdWords; i += NT) s[i] = src[i];
    return true;
}

// Descriptor of fill f from the LDS copy (f the same in every lane).
__device__ __forceinline__ FillDev fill_from_lds(const u32x4 *s, int f) {
    f = __builtin_amdgcn_readfirstlane(f);
    union {
        FillDev d;
        u32x4 v[kFdWords];
    } u;
#pragma unroll
    for (int i = 0; i < kFdWords; i++) {
        const u32x4 w = s[f * kFdWords + i];
        u.v[i] = u32x4{(unsigned)__builtin_amdgcn_readfirstlane((int)w.x),
                       (unsigned)__builtin_amdgcn_readfirstlane((int)w.y),
                       (unsigned)__builtin_amdgcn_readfirstlane((int)w.z),
                       (unsigned)__builtin_amdgcn_readfirstlane((int)w.w)};
    }
    return u.d;
}

typedef short s16x2 __attribute__((ext_vector_type(2)));

// Adds the eight int16 samples of one 16-byte row chunk to eight sums: one
// 2-way int16 dot product per sample (with weights (1, 0) or (0, 1)), exact.
__device__ __forceinline__ void add8(int32_t (&s)[kVec], const uint4 v) {
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
    const s16x2 lo = {1, 0};
    const s16x2 hi = {0, 1};
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const s16x2 x = __builtin_bit_cast(s16x2, w[i]);
        s[2 * i] = __builtin_amdgcn_sdot2(x, lo, s[2 * i], false);
        s[2 * i + 1] = __builtin_amdgcn_sdot2(x, hi, s[2 * i + 1], false);
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
    const u32x4 v = *(const DAQ_GLOBAL u32x4 *)p;
    return make_uint4(v.x, v.y, v.z, v.w);
}

// A 16-byte chunk of a raw row on the streaming read of a batch larger than
// the caches: non-temporal, since the summing pass uses each chunk once (its
// halo neighbours aside) and nothing of the batch would stay cached for the
// write-out anyway (150 against 162 us for the 16-fill scan). Smaller
// launches read normally, so that their rows are still cached when the
// island samples are read again.
__device__ __forceinline__ uint4 load16_stream(const int16_t *p) {
    const u32x4 v = __builtin_nontemporal_load((const DAQ_GLOBAL u32x4 *)p);
    return make_uint4(v.x, v.y, v.z, v.w);
}

// One 16-byte line of a packed output row. The packed rows are not read
// again on the device, so the store is non-temporal: the line goes out to HBM
// now, while the write-out is bound by its load chains, instead of lingering
// dirty in the caches and being written back during the next launch's
// streaming scan (where it costs scan bandwidth: 162 against 180 us).
__device__ __forceinline__ void store16(int16_t *p, const uint4 v) {
    u32x4 w;
    w.x = v.x;
    w.y = v.y;
    w.z = v.z;
    w.w = v.w;
    __builtin_nontemporal_store(w, (DAQ_GLOBAL u32x4 *)p);
}

constexpr int kQBin = 32;  // samples per decimated bin (Table 2: 560k / 17.5k)

__device__ __forceinline__ void store16_i32(int32_t *p, const uint4 v, bool stream) {
    u32x4 w;
    w.x = v.x;
    w.y = v.y;
    w.z = v.z;
    w.w = v.w;
    if (stream) __builtin_nontemporal_store(w, (DAQ_GLOBAL u32x4 *)p);
    else *(DAQ_GLOBAL u32x4 *)p = w;
}

// The same with the Q-method on the read (Section 3, Q-method paragraph;
// Table 2, decimation and fill-by-fill rows): an owner thread also adds
// x - ped[c] to the fill's accumulator rows for its 8 samples and returns the
// pedestal-subtracted calorimeter sum of its valid samples in *gsum. Every
// load of a round (raw rows, pedestals, accumulator rows) is issued before
// the round's first store.
template <int R, bool STREAM>
__device__ uint32_t group_flags_q(const FillDev &fd, int64_t p, int32_t thr_eff, int64_t valid, bool owner,
                                  int64_t ped_total, int64_t *gsum) {
    auto ld = [](const int16_t *q) { return STREAM ? load16_stream(q) : load16(q); };
    const int16_t *xr = fd.raw + p;
    int32_t *ar = (owner && fd.acc != nullptr) ? fd.acc + p : nullptr;
    const bool full = valid >= kVec;
    const int nv = full ? kVec : (int)valid;
    int32_t s[kVec] = {0, 0, 0, 0, 0, 0, 0, 0};
    auto update = [&](int c, const uint4 v, const u32x4 a0, const u32x4 a1, int32_t pc) {
        int32_t *row = ar + (int64_t)c * fd.acc_stride;
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
        uint32_t d[kVec];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            d[2 * k] = (uint32_t)((int32_t)(int16_t)(w[k] & 0xFFFFu) - pc);
            d[2 * k + 1] = (uint32_t)((int32_t)(int16_t)(w[k] >> 16) - pc);
        }
        if (full) {
            store16_i32(row, make_uint4(a0.x + d[0], a0.y + d[1], a0.z + d[2], a0.w + d[3]), STREAM);
            store16_i32(row + 4, make_uint4(a1.x + d[4], a1.y + d[5], a1.z + d[6], a1.w + d[7]), STREAM);
        } else {
            for (int k = 0; k < nv; k++) gbl(row)[k] = (int32_t)((uint32_t)gbl(row)[k] + d[k]);
        }
    };
    auto load_acc = [&](int c, u32x4 &a0, u32x4 &a1, int32_t &pc) {
        pc = *gbl(fd.ped + c);
        if (full) {
            const int32_t *row = ar + (int64_t)c * fd.acc_stride;
            a0 = *(const DAQ_GLOBAL u32x4 *)row;
            a1 = *(const DAQ_GLOBAL u32x4 *)(row + 4);
        } else {
            a0 = a1 = u32x4{0u, 0u, 0u, 0u};
        }
    };
    int c = 0;
    for (; c + R <= fd.C; c += R) {
        uint4 v[R];
        u32x4 a0[R], a1[R];
        int32_t pc[R];
#pragma unroll
        for (int u = 0; u < R; u++) v[u] = ld(xr + (int64_t)(c + u) * fd.stride);
        if (ar != nullptr) {
#pragma unroll
            for (int u = 0; u < R; u++) load_acc(c + u, a0[u], a1[u], pc[u]);
        }
#pragma unroll
        for (int u = 0; u < R; u++) {
            add8(s, v[u]);
            if (ar != nullptr) update(c + u, v[u], a0[u], a1[u], pc[u]);
        }
    }
    for (; c < fd.C; c++) {
        const uint4 v = ld(xr + (int64_t)c * fd.stride);
        add8(s, v);
        if (ar != nullptr) {
            u32x4 a0, a1;
            int32_t pc;
            load_acc(c, a0, a1, pc);
            update(c, v, a0, a1, pc);
        }
    }
    if (owner) {
#pragma unroll
        for (int k = 0; k < kVec; k++) *gsum += k < nv ? (int64_t)s[k] - ped_total : 0;
    }
    return flags8(s, thr_eff, valid);
}

// Adds the lanes' group sums (8-sample groups at p) into the decimated sums
// of their kQBin-sample bins: the first lane of each bin within the wave sums
// the bin's next lanes and makes one atomic add. Executed by whole waves.
__device__ __forceinline__ void q_bin_add(const FillDev &fd, int64_t p, int64_t gsum) {
    const int lane = threadIdx.x & 63;
    const int k = (int)((p >> 3) & (kQBin / kVec - 1));  // group index within its bin
    int64_t acc = gsum;
#pragma unroll
    for (int d = 1; d < kQBin / kVec; d++) {
        const int64_t t = __shfl_down(gsum, d, 64);
        if (lane + d < 64 && k + d < kQBin / kVec) acc += t;
    }
    if (fd.qsum != nullptr && (k == 0 || lane == 0) && acc != 0 && p >= 0 && p < fd.n)
        atomicAdd(reinterpret_cast<unsigned long long *>(fd.qsum + (p >> 5)), (unsigned long long)acc);
}

// Flags of 8 samples starting at p (all C rows read, nothing kept); R rows
// are in flight per round. STREAM: non-temporal loads.
template <int R, bool STREAM = false>
__device__ uint32_t group_flags(const int16_t *p, int64_t stride, int C, int32_t thr_eff, int64_t valid) {
    auto ld = [](const int16_t *q) { return STREAM ? load16_stream(q) : load16(q); };
    int32_t s[kVec] = {0, 0, 0, 0, 0, 0, 0, 0};
    int c = 0;
    for (; c + R <= C; c += R) {
        uint4 v[R];
#pragma unroll
        for (int u = 0; u < R; u++) v[u] = ld(p + (int64_t)(c + u) * stride);
#pragma unroll
        for (int u = 0; u < R; u++) add8(s, v[u]);
    }
    for (; c < C; c++) add8(s, ld(p + (int64_t)c * stride));
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

// Polls of a bounded look-back before it gives up.
constexpr uint32_t kLookBackSpins = 1u << 22;

// Sum of the published values of this fill's tiles [0, lt): the exclusive
// prefix of (island samples, islands). Executed by one whole wave. With
// gave_up set the wait is bounded: past kLookBackSpins polls the flag is set
// and the partial sum returned.
__device__ uint64_t look_back(uint64_t *st, int64_t lt, int lane, uint32_t *gave_up = nullptr) {
    uint64_t acc = 0;
    int64_t hi = lt - 1;
    uint32_t spins = 0;
    for (;;) {
        const int64_t j = hi - lane;
        uint64_t s = kFlagIncl;  // before the fill's first tile: empty prefix
        if (j >= 0) s = __hip_atomic_load(gbl(st + j), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t flag = s & ~kValMask;
        const uint64_t b_incl = __ballot(flag == kFlagIncl);
        const uint64_t b_none = __ballot(flag == 0);
        const uint64_t first = b_incl & (0ull - b_incl);         // lowest lane with a prefix
        const uint64_t need = b_incl ? (first | (first - 1ull)) : ~0ull;
        if (b_none & need) {  // a tile we depend on has not published yet
            if (gave_up != nullptr && ++spins > kLookBackSpins) {
                if (lane == 0) __hip_atomic_store(gave_up, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return acc;
            }
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
            store16(row + g0, *reinterpret_cast<const uint4 *>(src));
        } else {
#pragma unroll
            for (int e = 0; e < 8; e++) {
                const int j = j0 + e;
                if (j >= 0 && j < len && m0 + j < ostride) *gbl(row + m0 + j) = src[e];
            }
        }
    }
}

// Last run whose packed start is <= j, or -1 (j lies in the run open at the
// tile's first sample).
__device__ __forceinline__ int find_run(const int32_t *seg_dst, int nrun, int j) {
    int lo = 0, hi = nrun - 1, ans = -1;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        if (seg_dst[mid] <= j) {
            ans = mid;
            lo = mid + 1;
        } else {
            hi = mid - 1;
        }
    }
    return ans;
}

// Samples shift .. shift + 7 of the 16 samples held by A (0..7) and B (8..15).
__device__ __forceinline__ uint4 realign8(const uint4 A, const uint4 B, int shift) {
    const uint32_t d[8] = {A.x, A.y, A.z, A.w, B.x, B.y, B.z, B.w};
    const int h = shift >> 1;
    uint32_t e[5];
#pragma unroll
    for (int k = 0; k < 5; k++) {
        const uint32_t a0 = d[k], a1 = d[k + 1 < 8 ? k + 1 : 7], a2 = d[k + 2 < 8 ? k + 2 : 7],
                       a3 = d[k + 3 < 8 ? k + 3 : 7];
        e[k] = h == 0 ? a0 : (h == 1 ? a1 : (h == 2 ? a2 : a3));
    }
    if (shift & 1)
        return make_uint4(__builtin_amdgcn_alignbyte(e[1], e[0], 2), __builtin_amdgcn_alignbyte(e[2], e[1], 2),
                          __builtin_amdgcn_alignbyte(e[3], e[2], 2), __builtin_amdgcn_alignbyte(e[4], e[3], 2));
    return make_uint4(e[0], e[1], e[2], e[3]);
}

// ---- steps shared by every tile variant ---------------------------------------

struct TileScan {
    uint32_t mm, rise, fall;     // this thread's island mask and island edges
    int th_m, th_i;              // island samples / islands of lower threads in the tile
    int tile_m, tile_i;          // tile totals
    int64_t m_before, i_before;  // totals of the fill's earlier tiles
};

// Steps 2c and 3a of a tile, from the island-mask bits m10 of samples p - 1
// .. p + 8 of the calling thread (zero for threads that own no samples):
// island edges, work-group exclusive scan and tile totals, and the total
// published at once (the inclusive prefix for a fill's first tile); never
// waits for another tile.
template <int NT>
__device__ __forceinline__ TileScan tile_totals(const KArgs &a, const FillDev &fd, int64_t lt, uint32_t m10,
                                                uint32_t *s_wsum) {
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    TileScan r;
    r.mm = (m10 >> 1) & 0xFFu;
    r.rise = r.mm & ~(((r.mm << 1) | (m10 & 1u)) & 0xFFu);
    r.fall = r.mm & ~((r.mm >> 1) | (((m10 >> 9) & 1u) << 7));

    // 2c. work-group exclusive scan of (island samples << 16 | islands)
    const uint32_t mine = ((uint32_t)__popc(r.mm) << 16) | (uint32_t)__popc(r.rise);
    const uint32_t inc = wave_incl_scan_u32(mine, lane);
    if (lane == 63) s_wsum[wid] = inc;
    lds_barrier();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < NW; w++) {
        const uint32_t v = s_wsum[w];
        before += (w < wid) ? v : 0u;
        total += v;
    }
    const uint32_t excl = before + inc - mine;
    r.th_m = (int)(excl >> 16);
    r.th_i = (int)(excl & 0xFFFFu);
    r.tile_m = (int)(total >> 16);
    r.tile_i = (int)(total & 0xFFFFu);
    r.m_before = 0;
    r.i_before = 0;

    // 3a. publish the tile's total at once: later tiles of the fill wait for it
    if (tid == 0) {
        uint64_t *st = a.tile_state + fd.tile_base;
        const uint64_t agg = ((uint64_t)r.tile_m << 31) | (uint64_t)r.tile_i;
        __hip_atomic_store(gbl(st + lt), (lt == 0 ? kFlagIncl : kFlagAgg) | agg, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    return r;
}

// Step 2 of a tile whose flag bitmap (G groups of 8 bits, zero padding up to
// word Wn included) is in s_bits: popcount prefix, dilation of the calling
// thread's group g (owners only; its first sample is p) and work-group scan.
// Ends by publishing the tile's total (its inclusive prefix for a fill's
// first tile); never waits for another tile.
template <int NT>
__device__ __forceinline__ TileScan scan_front(const KArgs &a, const FillDev &fd, int64_t lt, int G, int g,
                                               bool owner, int64_t p, const uint8_t *s_bits, uint32_t *s_pc,
                                               uint32_t *s_wsum) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    const int64_t N = fd.n;
    const int Wn = (G + 7) >> 3;

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
    lds_barrier();

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
    return tile_totals<NT>(a, fd, lt, m10, s_wsum);
}

// Step 3b: decoupled look-back over the fill's earlier tiles (wave 0), the
// tile's inclusive prefix, and the prefix broadcast to the work-group.
__device__ __forceinline__ void scan_back(const KArgs &a, const FillDev &fd, int64_t lt, TileScan &r,
                                          uint64_t *s_excl, uint32_t *gave_up = nullptr) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    if ((tid >> 6) == 0) {
        uint64_t ex = 0;
        if (lt > 0) {
            uint64_t *st = a.tile_state + fd.tile_base;
            const uint64_t agg = ((uint64_t)r.tile_m << 31) | (uint64_t)r.tile_i;
            ex = look_back(st, lt, lane, gave_up);
            if (lane == 0)
                __hip_atomic_store(gbl(st + lt), kFlagIncl | (ex + agg), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (lane == 0) *s_excl = ex;
    }
    lds_barrier();
    const uint64_t ex = *s_excl;
    r.m_before = (int64_t)((ex >> 31) & kField);
    r.i_before = (int64_t)(ex & kField);
}

// Steps 2-3 back to back.
template <int NT>
__device__ __forceinline__ TileScan scan_tile(const KArgs &a, const FillDev &fd, int64_t lt, int G, int g,
                                              bool owner, int64_t p, const uint8_t *s_bits, uint32_t *s_pc,
                                              uint32_t *s_wsum, uint64_t *s_excl) {
    TileScan r = scan_front<NT>(a, fd, lt, G, g, owner, p, s_bits, s_pc, s_wsum);
    scan_back(a, fd, lt, r, s_excl);
    return r;
}

// Step 4a (Table 2 island-array row): the record fields this thread owns.
__device__ __forceinline__ void write_records(const FillDev &fd, const TileScan &r, int64_t p) {
    if (!(r.rise | r.fall)) return;
    DAQ_GLOBAL daq_island *isl = gbl(fd.isl);
    const int64_t cap = fd.cap;
    const int64_t mbase = r.m_before + r.th_m;
    const int64_t ibase = r.i_before + r.th_i;
#pragma unroll
    for (int k = 0; k < kVec; k++) {
        if ((r.rise >> k) & 1u) {
            const int64_t idx = ibase + __popc(r.rise & ((1u << k) - 1u));
            if (idx < cap) {
                isl[idx].start = p + k;
                isl[idx].offset = mbase + __popc(r.mm & ((1u << k) - 1u));
            }
        }
        if ((r.fall >> k) & 1u) {
            const int64_t idx = ibase + __popc(r.rise & ((2u << k) - 1u)) - 1;
            if (idx >= 0 && idx < cap) isl[idx].stop = p + k + 1;
        }
    }
}

// Step 5: totals, written by the fill's last tile (right after its scan).
// COHERENT: device-scope stores that work-groups on any XCD can read in the
// same launch.
template <bool COHERENT = false>
__device__ __forceinline__ void write_counts(const FillDev &fd, int64_t lt, const TileScan &r) {
    if (threadIdx.x != 0 || lt != fd.n_tiles - 1 || fd.counts == nullptr) return;
    const int64_t n_isl = r.i_before + r.tile_i;
    const int64_t tl = r.m_before + r.tile_m;
    int32_t status = (n_isl > fd.cap) ? DAQ_STATUS_CAPACITY : 0;
    if (fd.out != nullptr && tl > fd.out_stride) status |= DAQ_STATUS_OUT_STRIDE;
    DAQ_GLOBAL daq_counts *cnt = gbl(fd.counts);
    if constexpr (COHERENT) {
        __hip_atomic_store(&cnt->n_islands, n_isl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&cnt->total_len, tl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&cnt->status, status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&cnt->reserved, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        cnt->n_islands = n_isl;
        cnt->total_len = tl;
        cnt->status = status;
        cnt->reserved = 0;
    }
}

__device__ __forceinline__ int32_t clamp_thr(int64_t te) {
    return (int32_t)(te > 2147483647LL ? 2147483647LL : (te < -2147483648LL ? -2147483648LL : te));
}

// ---- packed write-out from a run table ----------------------------------------------

// Last run whose packed start is <= q (runs with equal starts: the later,
// non-empty one).
__device__ __forceinline__ int run_at(const int32_t *seg_dst, int nrun, int q) {
    int lo = 0, hi = nrun - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (seg_dst[mid] <= q) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Elements [0, split) of a, [split, 8) of b.
__device__ __forceinline__ uint4 blend8(const uint4 a, const uint4 b, int split) {
    auto m = [split](int k) -> uint32_t {
        return (2 * k + 1 < split) ? 0xFFFFFFFFu : (2 * k < split ? 0x0000FFFFu : 0u);
    };
    const uint32_t m0 = m(0), m1 = m(1), m2 = m(2), m3 = m(3);
    return make_uint4((a.x & m0) | (b.x & ~m0), (a.y & m1) | (b.y & ~m1), (a.z & m2) | (b.z & ~m2),
                      (a.w & m3) | (b.w & ~m3));
}

// Chopped islands copied straight from the raw rows (no staging). Run r
// moves tile samples [src_r, ...) to packed positions [dst_r, dst_{r+1})
// (tile-relative; the last run ends at tile_m). A work item is one 16-byte
// line of one channel's packed row. A line inside one run, or across the
// boundary of two runs, is read as aligned 16-byte words, realigned (and
// blended) and written with one 16-byte store; lines at the tile's ends
// (shared with the neighbouring tiles) or across three or more runs go
// sample by sample. When every row has the same line phase (out_stride a
// multiple of 8), line_run[j] holds the run of line j's first sample.
template <int NT, int U>
__device__ __forceinline__ void emit_lines(const int32_t *seg_src, const int32_t *seg_dst, const int32_t *line_run,
                                           bool uniform, int ph_all, int lines, int nrun, int tile_m,
                                           const int16_t *raw, int64_t stride, int64_t t0, int16_t *out,
                                           int64_t ostride, int C, int64_t m0) {
    const int items = C * lines;
    const int dq = NT / lines, dr = NT - dq * lines;
    int c = (int)threadIdx.x / lines, j = (int)threadIdx.x - c * lines;
    auto step = [&]() {
        j += dr;
        c += dq;
        if (j >= lines) {
            j -= lines;
            c++;
        }
    };
    // the line's tile-relative packed range [lo, hi) and its position q0
    auto span = [&](int cc, int jj, int &q0, int &lo, int &hi) {
        const int ph = uniform ? ph_all : line_phase(out + (int64_t)cc * ostride, m0);
        q0 = 8 * jj - ph;
        lo = q0 > 0 ? q0 : 0;
        hi = q0 + 8 < tile_m ? q0 + 8 : tile_m;
        if (m0 + hi > ostride) hi = (int)(ostride - m0);
    };
    for (int i0 = threadIdx.x; i0 < items; i0 += NT * U) {
        const int c_first = c, j_first = j;
        uint4 A0[U], B0[U], A1[U], B1[U];
        int meta[U];  // kind (0 none, 1 one run, 2 two runs, 3 sample by sample) | split << 2 | shifts
#pragma unroll
        for (int u = 0; u < U; u++) {
            meta[u] = 0;
            A0[u] = B0[u] = A1[u] = B1[u] = make_uint4(0, 0, 0, 0);
            if (i0 + u * NT < items) {
                int q0, lo, hi;
                span(c, j, q0, lo, hi);
                if (lo < hi) {
                    // the samples go to packed positions lo .. hi - 1; v[e] below is position lo + e
                    const int r0 = uniform ? line_run[j] : run_at(seg_dst, nrun, lo);
                    const int end0 = (r0 + 1 < nrun) ? seg_dst[r0 + 1] : tile_m;
                    const int16_t *row = raw + (int64_t)c * stride + t0;  // t0 is a multiple of 8
                    const int s0 = seg_src[r0] + lo - seg_dst[r0];
                    meta[u] = 3;
                    if (end0 >= hi) {
                        meta[u] = 1 | ((s0 & 7) << 6);
                        A0[u] = load16(row + (s0 & ~7));
                        if ((s0 & 7) + (hi - lo) > 8) B0[u] = load16(row + (s0 & ~7) + 8);
                    } else {
                        const int end1 = (r0 + 2 < nrun) ? seg_dst[r0 + 2] : tile_m;
                        if (end1 >= hi) {
                            // runs are separated by at least one sample: s1 >= s0 + 1 >= 1
                            const int sp = end0 - lo;
                            const int s1 = seg_src[r0 + 1] - sp;
                            meta[u] = 2 | (sp << 2) | ((s0 & 7) << 6) | ((s1 & 7) << 9);
                            A0[u] = load16(row + (s0 & ~7));
                            if ((s0 & 7) + sp > 8) B0[u] = load16(row + (s0 & ~7) + 8);
                            A1[u] = load16(row + (s1 & ~7));
                            if ((s1 & 7) + (hi - lo) > 8) B1[u] = load16(row + (s1 & ~7) + 8);
                        }
                    }
                }
            }
            step();
        }
        c = c_first;
        j = j_first;
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int kind = meta[u] & 3;
            if (kind != 0) {
                int q0, lo, hi;
                span(c, j, q0, lo, hi);
                int16_t *orow = out + (int64_t)c * ostride + m0;
                if (kind == 3) {
                    const int16_t *row = raw + (int64_t)c * stride + t0;
                    int r = run_at(seg_dst, nrun, lo);
                    for (int q = lo; q < hi; q++) {
                        while (r + 1 < nrun && seg_dst[r + 1] <= q) r++;
                        *gbl(orow + q) = *gbl(row + seg_src[r] + (q - seg_dst[r]));
                    }
                } else {
                    uint4 v = realign8(A0[u], B0[u], (meta[u] >> 6) & 7);
                    if (kind == 2) v = blend8(v, realign8(A1[u], B1[u], (meta[u] >> 9) & 7), (meta[u] >> 2) & 15);
                    if (lo == q0 && hi == q0 + 8) {
                        store16(orow + q0, v);
                    } else {
                        // a line shared with a neighbouring tile: this tile's samples only
                        uint32_t w[4] = {v.x, v.y, v.z, v.w};
                        for (int e = 0; e < hi - lo; e++)
                            *gbl(orow + lo + e) = (int16_t)((w[e >> 1] >> ((e & 1) * 16)) & 0xFFFFu);
                    }
                }
            }
            step();
        }
    }
}

#ifndef DAQ_EMIT_U
#define DAQ_EMIT_U 4  // lines per thread with loads in flight
#endif

// Eight consecutive int16 elements of an LDS array, starting at element e
// (any alignment): five 4-byte reads and, for odd e, byte alignment.
__device__ __forceinline__ uint4 lds_read8(const uint32_t *base, int e) {
    const uint32_t *d = base + (e >> 1);
    const uint32_t w0 = d[0], w1 = d[1], w2 = d[2], w3 = d[3], w4 = d[4];
    if (e & 1)
        return make_uint4(__builtin_amdgcn_alignbyte(w1, w0, 2), __builtin_amdgcn_alignbyte(w2, w1, 2),
                          __builtin_amdgcn_alignbyte(w3, w2, 2), __builtin_amdgcn_alignbyte(w4, w3, 2));
    return make_uint4(w0, w1, w2, w3);
}


// Descriptor of packed line j (an int4, the same for every channel when all
// rows share one line phase): x = staged element of the line's first sample
// (run r0); y = kind 2: staged element holding line element 0 of run r0 + 1
// (elements >= split are taken from there), kind 3: r0; z = lo | hi << 8
// (the line's samples, relative to 8 j - phase); w = kind (0 none, 1 one run,
// 2 two runs, 3 sample by sample) | split << 4 | full << 8.

// LDS of one packed write-out: the run table (source sample, packed position
// of every run, their staged-word prefix), per-line run and descriptor, the
// source word of every staged word, and two staging buffers of HW words.
template <int MAXRUNS, int MAXLINES, int HW_>
struct CopyLayout {
    static constexpr int kMaxRuns = MAXRUNS;
    static constexpr int kMaxLines = MAXLINES;
    static constexpr int kHW = HW_;
    static constexpr int kSrc = 0;
    static constexpr int kDst = kSrc + MAXRUNS * 4;
    static constexpr int kWb = kDst + MAXRUNS * 4;
    static constexpr int kLine = kWb + (MAXRUNS + 1) * 4;
    static constexpr int kDesc = (kLine + MAXLINES * 4 + 15) / 16 * 16;
    static constexpr int kWsrc = kDesc + MAXLINES * 16;
    static constexpr int kStage = (kWsrc + HW_ * 4 + 15) / 16 * 16;
    static constexpr int kBytes = kStage + (2 * HW_ + 1) * 16;
};

struct CopyView {
    int32_t *src, *dst, *wb, *line;
    int4 *desc;
    int32_t *wsrc;
    uint4 *stage;
};

template <class L>
__device__ __forceinline__ CopyView copy_view(uint8_t *base) {
    CopyView v;
    v.src = reinterpret_cast<int32_t *>(base + L::kSrc);
    v.dst = reinterpret_cast<int32_t *>(base + L::kDst);
    v.wb = reinterpret_cast<int32_t *>(base + L::kWb);
    v.line = reinterpret_cast<int32_t *>(base + L::kLine);
    v.desc = reinterpret_cast<int4 *>(base + L::kDesc);
    v.wsrc = reinterpret_cast<int32_t *>(base + L::kWsrc);
    v.stage = reinterpret_cast<uint4 *>(base + L::kStage);
    return v;
}

// Packed samples of every channel for positions [q0, q0 + m) of a fill from
// a run table in LDS: run r moves source samples src[r] .. (absolute) to
// packed positions dst[r] .. dst[r + 1] - 1 (relative to q0; the last run
// ends at m); consecutive runs are separated by at least one sample. Every
// packed line gets a descriptor saying where its samples sit in a staged
// channel row. For a group of channels at a time, the aligned 16-byte words
// holding the source samples are staged in LDS (two buffers: the next
// group's words are loaded while the current group is written); each
// (channel, line) is then read from LDS and written with one 16-byte store.
// Words that do not fit (very many tiny islands), or rows with different
// line phases, go through emit_lines, which reads global memory directly.
// Called by every thread of the work-group with the run table in place;
// ends with a barrier.
template <int NT, class L, int FALLBACK_U = DAQ_EMIT_U>
__device__ __forceinline__ void copy_runs(const FillDev &fd, const CopyView &v, int nrun, int m, int64_t q0) {
    constexpr int HW = L::kHW;            // words of one of the two staging buffers
    constexpr int KI = (HW + NT - 1) / NT;  // staging loads per thread and group
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    // staged words of each run: floor8(src) .. ceil8(src + len); their prefix
    if (wid == 0) {
        int carry = 0;
        for (int r0 = 0; r0 < nrun; r0 += 64) {
            const int r = r0 + lane;
            int words = 0;
            if (r < nrun) {
                const int len = ((r + 1 < nrun) ? v.dst[r + 1] : m) - v.dst[r];
                words = len > 0 ? ((v.src[r] + len + 7) >> 3) - (v.src[r] >> 3) : 0;
            }
            const uint32_t incl = wave_incl_scan_u32((uint32_t)words, lane);
            if (r < nrun) v.wb[r] = carry + (int)incl - words;
            carry += (int)__shfl(incl, 63, 64);
        }
        if (lane == 0) v.wb[nrun] = carry;
    }
    lds_barrier();
    const int W = v.wb[nrun];
    const bool uniform = (fd.out_stride & 7) == 0;
    const int ph_all = line_phase(fd.out, q0);
    const int lines = uniform ? (ph_all + m + 7) >> 3 : (m + 14) >> 3;
    const int CG = uniform ? HW / W : 0;  // channels per staging round
    if (CG < 1) {
        // direct path: run of each line's first sample, then emit_lines
        if (uniform)
            for (int jj = tid; jj < lines; jj += NT) {
                const int q = 8 * jj - ph_all;
                v.line[jj] = run_at(v.dst, nrun, q > 0 ? q : 0);
            }
        lds_barrier();
        emit_lines<NT, FALLBACK_U>(v.src, v.dst, v.line, uniform, ph_all, lines, nrun, m, fd.raw, fd.stride, 0,
                                   fd.out, fd.out_stride, fd.C, q0);
        lds_barrier();
        return;
    }
    // source word of every staged word, and the descriptor of every line
    for (int w = tid; w < W; w += NT) {
        const int r = run_at(v.wb, nrun, w);
        v.wsrc[w] = (v.src[r] >> 3) + (w - v.wb[r]);
    }
    for (int jj = tid; jj < lines; jj += NT) {
        const int qa = 8 * jj - ph_all;
        const int lo = qa > 0 ? qa : 0;
        int hi = qa + 8 < m ? qa + 8 : m;
        if (q0 + hi > fd.out_stride) hi = (int)(fd.out_stride - q0);
        int4 d = make_int4(0, 0, 0, 0);
        if (lo < hi) {
            const int r0 = run_at(v.dst, nrun, lo);
            const int end0 = (r0 + 1 < nrun) ? v.dst[r0 + 1] : m;
            const int full = (lo == qa && hi == qa + 8) ? 1 : 0;
            d.x = 8 * v.wb[r0] + (v.src[r0] & 7) + (lo - v.dst[r0]);
            d.z = (lo - qa) | ((hi - qa) << 8);
            if (end0 >= hi) {
                d.w = 1 | (full << 8);
            } else {
                const int end1 = (r0 + 2 < nrun) ? v.dst[r0 + 2] : m;
                const int sp = end0 - lo;
                if (end1 >= hi) {
                    // runs are separated by at least one sample, so this is >= 8 * wb + 1
                    d.y = 8 * v.wb[r0 + 1] + (v.src[r0 + 1] & 7) - sp;
                    d.w = 2 | (sp << 4) | (full << 8);
                } else {
                    d.y = r0;
                    d.w = 3 | (full << 8);
                }
            }
        }
        v.desc[jj] = d;
    }
    lds_barrier();
    // channel groups of CG rows, double-buffered: group g + 1's words are
    // loaded into registers while group g is written out from LDS
    const int ngroups = (fd.C + CG - 1) / CG;
    uint4 nxt[KI];
    auto load_group = [&](int grp) {
        const int c0 = grp * CG;
        const int n_it = (fd.C - c0 < CG ? fd.C - c0 : CG) * W;
        const int dq = NT / W, dr = NT - dq * W;
        int cl = tid / W, w = tid - cl * W;  // word (cl, w) of the group is slot cl * W + w
#pragma unroll
        for (int it = 0; it < KI; it++) {
            if (it * NT + tid < n_it)
                nxt[it] = load16(fd.raw + (int64_t)(c0 + cl) * fd.stride + (int64_t)v.wsrc[w] * kVec);
            w += dr;
            cl += dq;
            if (w >= W) {
                w -= W;
                cl++;
            }
        }
    };
    auto store_group = [&](uint4 *buf, int grp) {
        const int c0 = grp * CG;
        const int n_it = (fd.C - c0 < CG ? fd.C - c0 : CG) * W;
#pragma unroll
        for (int it = 0; it < KI; it++)
            if (it * NT + tid < n_it) buf[it * NT + tid] = nxt[it];
    };
    load_group(0);
    store_group(v.stage, 0);
    lds_barrier();
    for (int grp = 0; grp < ngroups; grp++) {
        if (grp + 1 < ngroups) load_group(grp + 1);
        const int c0 = grp * CG;
        const int CGn = fd.C - c0 < CG ? fd.C - c0 : CG;
        const uint32_t *stage32 = reinterpret_cast<const uint32_t *>(v.stage + (grp & 1) * HW);
        {
            const int items = CGn * lines;
            const int dq = NT / lines, dr = NT - dq * lines;
            int cl = tid / lines, j = tid - cl * lines;
            for (int i = tid; i < items; i += NT) {
                const int4 d = v.desc[j];
                const int kind = d.w & 15;
                if (kind != 0) {
                    const uint32_t *row = stage32 + cl * W * 4;
                    int16_t *orow = fd.out + (int64_t)(c0 + cl) * fd.out_stride + q0 + 8 * j - ph_all;
                    const int lo = d.z & 0xFF, hi = d.z >> 8;
                    if (kind == 3) {
                        int r = d.y;
                        for (int e = lo; e < hi; e++) {
                            const int q = 8 * j - ph_all + e;
                            while (r + 1 < nrun && v.dst[r + 1] <= q) r++;
                            const int el = 8 * v.wb[r] + (v.src[r] & 7) + (q - v.dst[r]);
                            *gbl(orow + e) = reinterpret_cast<const int16_t *>(row)[el];
                        }
                    } else {
                        uint4 v = lds_read8(row, d.x);
                        if (kind == 2) v = blend8(v, lds_read8(row, d.y), (d.w >> 4) & 15);
                        if (d.w & 256) {
                            store16(orow, v);
                        } else {
                            // a line shared with a neighbouring chunk: this chunk's samples only
                            const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
                            for (int e = lo; e < hi; e++)
                                *gbl(orow + e) = (int16_t)((wv[(e - lo) >> 1] >> (((e - lo) & 1) * 16)) & 0xFFFFu);
                        }
                    }
                }
                j += dr;
                cl += dq;
                if (j >= lines) {
                    j -= lines;
                    cl++;
                }
            }
        }
        if (grp + 1 < ngroups) store_group(v.stage + ((grp + 1) & 1) * HW, grp + 1);
        lds_barrier();
    }
}

// ---- variant 0 / 1: rows read into registers ------------------------------------

template <int NT>
struct ChopLds {
    static constexpr int kGroups = 2 * kMaxHaloGroups + NT;  // widest bitmap
    static constexpr int kWords = (kGroups + 7) / 8 + 1;
    static constexpr int kBitsBytes = kWords * 8 + (kWords + 1) * 4;
    static constexpr int kCB = NT <= 256 ? 8 : 4;            // channels staged per round
    static constexpr int kRowStride = NT * kVec + 16;        // elements per staged row
    static constexpr int kStageBytes = kCB * kRowStride * 2;
    // the re-read write-out: a run per rise of the tile plus the open run,
    // lines of any phase, two staging buffers of 512 (1024 for 512 threads) words
    using Copy = CopyLayout<NT * kVec / 2 + 2, NT + 3, NT <= 256 ? 512 : 1024>;
    static constexpr int kMax2 = kBitsBytes > kStageBytes ? kBitsBytes : kStageBytes;
    static constexpr int kBytes = kMax2 > Copy::kBytes ? kMax2 : Copy::kBytes;
};

// Geometry of a tile of NT groups of 8 samples (the halo groups included, or
// loaded apart for wide windows) as seen by one thread.
template <int NT>
struct ChopGeom {
    int64_t lt, t0, base, p;
    int G, g;
    bool owner;
    __device__ __forceinline__ ChopGeom(const FillDev &fd, int64_t tile) {
        const bool wide = fd.wide != 0;
        lt = tile - fd.tile_base;
        G = wide ? fd.gl + NT + fd.gr : NT;            // bitmap groups
        t0 = lt * fd.tout;                             // first sample the tile owns
        base = t0 - (int64_t)fd.gl * kVec;             // sample at bitmap bit 0
        g = wide ? fd.gl + (int)threadIdx.x : (int)threadIdx.x;
        owner = wide || ((int)threadIdx.x >= fd.gl && (int)threadIdx.x < NT - fd.gr);
        p = base + (int64_t)g * kVec;                  // this thread's first sample
    }
};

// Step 1 for a tile of NT groups: flags of this thread's 8 samples from all
// channel rows (Table 2 waveform-sum and threshold rows), R rows in flight,
// halo groups of wide windows loaded apart; bitmap zero padding; barrier.
template <int NT, int R, bool Q = false>
__device__ __forceinline__ void chop_flags(const FillDev &fd, const ChopGeom<NT> &q, int32_t thr_eff,
                                           uint8_t *s_bits, bool stream = false, int64_t ped_total = 0) {
    const int tid = threadIdx.x;
    const int64_t N = fd.n;
    uint32_t fb = 0;
    // waves holding halo groups read normally, so that the neighbouring
    // tile's loads of the same lines can still find them cached
    const int w = tid >> 6;
    const bool halo_wave = !fd.wide && (w == 0 || w == NT / 64 - 1);
    const bool nt = stream && !halo_wave;
    if constexpr (Q) {
        int64_t gsum = 0;
        if (q.p >= 0 && q.p < N)
            fb = nt ? group_flags_q<R, true>(fd, q.p, thr_eff, N - q.p, q.owner, ped_total, &gsum)
                    : group_flags_q<R, false>(fd, q.p, thr_eff, N - q.p, q.owner, ped_total, &gsum);
        q_bin_add(fd, q.p, gsum);
    } else {
        if (q.p >= 0 && q.p < N)
            fb = nt ? group_flags<R, true>(fd.raw + q.p, fd.stride, fd.C, thr_eff, N - q.p)
                    : group_flags<R, false>(fd.raw + q.p, fd.stride, fd.C, thr_eff, N - q.p);
    }
    s_bits[q.g] = (uint8_t)fb;
    if (fd.wide) {
        for (int h = tid; h < fd.gl + fd.gr; h += NT) {
            const int hg = (h < fd.gl) ? h : (NT + h);
            const int64_t s0 = q.base + (int64_t)hg * kVec;
            uint32_t hb = 0;
            if (s0 >= 0 && s0 < N) hb = group_flags<6>(fd.raw + s0, fd.stride, fd.C, thr_eff, N - s0);
            s_bits[hg] = (uint8_t)hb;
        }
    }
    const int Wn = (q.G + 7) >> 3;  // bitmap words; word Wn stays zero
    for (int z = q.G + tid; z < (Wn + 1) * 8; z += NT) s_bits[z] = 0;
    lds_barrier();
}

// What a re-read tile keeps between its front half (flags, scan, total
// published) and its back half (look-back, records, packed samples).
struct ReloadTile {
    TileScan r;
    int64_t lt;
    int64_t p;
};

template <int NT, int R>
__device__ __forceinline__ ReloadTile reload_front(const KArgs &a, const FillDev &fd, int32_t thr_eff, int64_t tile,
                                                   uint8_t *lds, uint32_t *s_wsum) {
    const ChopGeom<NT> q(fd, tile);
    uint8_t *s_bits = lds;
    uint32_t *s_pc = reinterpret_cast<uint32_t *>(lds + ChopLds<NT>::kWords * 8);
    chop_flags<NT, R>(fd, q, thr_eff, s_bits);
    ReloadTile t;
    t.r = scan_front<NT>(a, fd, q.lt, q.G, q.g, q.owner, q.p, s_bits, s_pc, s_wsum);
    t.lt = q.lt;
    t.p = q.p;
    return t;
}

// Back half: prefix, records, totals and the chopped islands, whose raw
// samples are read again and staged in LDS per CB channels so that global
// stores are aligned 16-byte lines.
// Back half of a re-read tile: the look-back, the island records and the
// packed samples. The tile's runs (the island open at its first owned sample,
// then one per rising edge) go into an LDS run table and copy_runs writes
// them, reading the raw rows again (recently read, so mostly from cache).
template <int NT>
__device__ __forceinline__ void reload_back(const KArgs &a, const FillDev &fd, ReloadTile &t, uint8_t *lds,
                                            uint64_t *s_excl) {
    scan_back(a, fd, t.lt, t.r, s_excl);
    const TileScan &r = t.r;
    write_records(fd, r, t.p);
    write_counts(fd, t.lt, r);
    if (fd.out == nullptr || r.tile_m == 0) return;
    using L = typename ChopLds<NT>::Copy;
    const CopyView v = copy_view<L>(lds);
    if (threadIdx.x == 0) {
        v.src[0] = (int32_t)(t.lt * fd.tout);
        v.dst[0] = 0;
    }
    if (r.rise) {
#pragma unroll
        for (int k = 0; k < kVec; k++) {
            if ((r.rise >> k) & 1u) {
                const int j = 1 + r.th_i + __popc(r.rise & ((1u << k) - 1u));
                v.src[j] = (int32_t)(t.p + k);
                v.dst[j] = r.th_m + __popc(r.mm & ((1u << k) - 1u));
            }
        }
    }
    lds_barrier();
    copy_runs<NT, L, 1>(fd, v, r.tile_i + 1, r.tile_m, r.m_before);
}

// A whole tile at once. RESIDENT keeps each thread's 54 channel chunks in
// registers for the write-out; otherwise the two halves run back to back.
template <int NT, bool RESIDENT, int kRowsInFlight>
__device__ __forceinline__ void chop_tile(const KArgs &a, const FillDev &fd, int32_t thr_eff, int64_t tile, uint8_t *lds,
                                          uint32_t *s_wsum, uint64_t *s_excl) {
    if constexpr (!RESIDENT) {
        ReloadTile t = reload_front<NT, kRowsInFlight>(a, fd, thr_eff, tile, lds, s_wsum);
        reload_back<NT>(a, fd, t, lds, s_excl);
    } else {
        constexpr int CB = ChopLds<NT>::kCB;
        constexpr int RS = ChopLds<NT>::kRowStride;
        const ChopGeom<NT> q(fd, tile);
        const int64_t N = fd.n;
        const int64_t stride = fd.stride;
        const int16_t *raw = fd.raw;
        uint8_t *s_bits = lds;
        uint32_t *s_pc = reinterpret_cast<uint32_t *>(lds + ChopLds<NT>::kWords * 8);
        int16_t *s_stage = reinterpret_cast<int16_t *>(lds);

        // 1. flags of this thread's 8 samples from all 54 rows, kept
        uint4 xr[kResidentChannels];
        uint32_t fb = 0;
        if (q.p >= 0 && q.p < N) {
#pragma unroll
            for (int c = 0; c < kResidentChannels; c++) xr[c] = load16(raw + q.p + (int64_t)c * stride);
            int32_t s[kVec] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
            for (int c = 0; c < kResidentChannels; c++) add8(s, xr[c]);
            fb = flags8(s, thr_eff, N - q.p);
        }
        s_bits[q.g] = (uint8_t)fb;
        if (fd.wide) {
            for (int h = threadIdx.x; h < fd.gl + fd.gr; h += NT) {
                const int hg = (h < fd.gl) ? h : (NT + h);
                const int64_t s0 = q.base + (int64_t)hg * kVec;
                uint32_t hb = 0;
                if (s0 >= 0 && s0 < N) hb = group_flags<6>(raw + s0, stride, kResidentChannels, thr_eff, N - s0);
                s_bits[hg] = (uint8_t)hb;
            }
        }
        const int Wn = (q.G + 7) >> 3;
        for (int z = q.G + threadIdx.x; z < (Wn + 1) * 8; z += NT) s_bits[z] = 0;
        lds_barrier();

        const TileScan r = scan_tile<NT>(a, fd, q.lt, q.G, q.g, q.owner, q.p, s_bits, s_pc, s_wsum, s_excl);
        write_records(fd, r, q.p);
        write_counts(fd, q.lt, r);

        // 4b. chopped islands from the registers, staged in LDS per CB channels
        if (fd.out != nullptr && r.tile_m > 0) {
            int16_t *out = fd.out;
            const int64_t ostride = fd.out_stride;
            const int64_t m0 = r.m_before;
            const uint32_t mm = r.mm;
#pragma unroll
            for (int c0 = 0; c0 < kResidentChannels; c0 += CB) {
                if (mm) {
#pragma unroll
                    for (int cl = 0; cl < CB; cl++) {
                        if (c0 + cl < kResidentChannels) {
                            const int ph = line_phase(out + (int64_t)(c0 + cl) * ostride, m0);
                            stage_put(s_stage + cl * RS, ph + r.th_m, mm, xr[c0 + cl]);
                        }
                    }
                }
                lds_barrier();
                stage_flush<NT, CB>(s_stage, RS, out, ostride, c0, kResidentChannels, m0, r.tile_m);
                lds_barrier();
            }
        }
    }
}

// ---- variant 2: the tile lives in LDS ---------------------------------------------

// Tile rows are DMA'd straight from HBM into LDS (no registers hold them), so
// two work-groups share a CU and overlap one another's load and compute
// phases; the write-out reads LDS.
struct StreamLds {
    static constexpr int kGroups = kStreamGroups;                       // groups per tile buffer
    static constexpr int kRow = kGroups * kVec;                         // samples per row
    static constexpr int kChunks = kResidentChannels * kGroups;         // 16-byte chunks
    static constexpr int kIters = (kChunks + kStreamThreads - 1) / kStreamThreads;
    static constexpr int kBufBytes = kIters * kStreamThreads * 16;      // last round lands in padding
    static constexpr int kWords = (kGroups + 7) / 8 + 1;
    static constexpr int kBitsOff = kBufBytes;
    static constexpr int kPcOff = kBitsOff + kWords * 8;
    static constexpr int kMaxRuns = kRow / 2 + 2;
    static constexpr int kRunOff = kPcOff + (kWords + 1) * 4;
    static constexpr int kBytes = kRunOff + 2 * kMaxRuns * 4;
};

typedef __attribute__((address_space(3))) void lds_void;

// Chopped islands of one tile straight from the LDS rows: work items are
// (channel, aligned 16-byte chunk of the packed row); a chunk whose 8 samples
// come from one run reads two aligned LDS words and realigns them, the others
// go element by element.
template <int NT>
__device__ __forceinline__ void gather_from_lds(const int16_t *buf, const int32_t *seg_src, const int32_t *seg_dst,
                                                int nrun, int own0, int16_t *out, int64_t ostride, int64_t m0,
                                                int len) {
    constexpr int C = kResidentChannels;
    constexpr int ROW = StreamLds::kRow;
    const int nch = (len + 7 + 7) >> 3;
    const int items = C * nch;
    for (int i = threadIdx.x; i < items; i += NT) {
        const int c = i / nch;
        const int q = i - c * nch;
        int16_t *orow = out + (int64_t)c * ostride;
        const int j0 = q * 8 - line_phase(orow, m0);
        if (j0 >= len) continue;
        const int16_t *brow = buf + c * ROW;
        const int jlo = j0 < 0 ? 0 : j0;
        int r = find_run(seg_dst, nrun, jlo);
        int next = (r + 1 < nrun) ? seg_dst[r + 1] : len;
        const bool full = j0 >= 0 && j0 + 8 <= len && m0 + j0 + 8 <= ostride;
        if (full && j0 + 7 < next) {  // one run: two aligned LDS words, realigned
            const int s0 = (r < 0) ? own0 + j0 : seg_src[r] + (j0 - seg_dst[r]);
            const int a0 = s0 & ~7;
            const uint4 A = *reinterpret_cast<const uint4 *>(brow + a0);
            const uint4 B = (s0 & 7) ? *reinterpret_cast<const uint4 *>(brow + a0 + 8) : make_uint4(0, 0, 0, 0);
            store16(orow + m0 + j0, realign8(A, B, s0 & 7));
            continue;
        }
        // run edges and row ends: walk the runs forward from the chunk's first
        // element, gather the values, then store them
        uint32_t v[8];
        uint32_t valid = 0;
#pragma unroll
        for (int e = 0; e < 8; e++) {
            const int j = j0 + e;
            v[e] = 0;
            if (j < 0 || j >= len || m0 + j >= ostride) continue;
            while (j >= next) {
                r++;
                next = (r + 1 < nrun) ? seg_dst[r + 1] : len;
            }
            const int sj = (r < 0) ? own0 + j : seg_src[r] + (j - seg_dst[r]);
            v[e] = (uint16_t)brow[sj];
            valid |= 1u << e;
        }
        if (valid == 0xFFu) {
            store16(orow + m0 + j0, make_uint4(v[0] | (v[1] << 16), v[2] | (v[3] << 16), v[4] | (v[5] << 16),
                                               v[6] | (v[7] << 16)));
        } else {
#pragma unroll
            for (int e = 0; e < 8; e++)
                if ((valid >> e) & 1u) *gbl(orow + m0 + j0 + e) = (int16_t)v[e];
        }
    }
}

__device__ __forceinline__ void stream_tile(const KArgs &a, const FillDev &fd, int32_t thr_eff, int64_t tile, uint8_t *lds,
                                            uint32_t *s_wsum, uint64_t *s_excl) {
    constexpr int NT = kStreamThreads;
    constexpr int G = StreamLds::kGroups;
    constexpr int C = kResidentChannels;
    constexpr int ROW = StreamLds::kRow;
    const int tid = threadIdx.x;
    const int wid = tid >> 6;

    const int64_t lt = tile - fd.tile_base;
    const int64_t N = fd.n;
    const int gl = fd.gl;
    const int gr = fd.gr;
    const int64_t t0 = lt * fd.tout;
    const int64_t base = t0 - (int64_t)gl * kVec;
    const int16_t *raw = fd.raw;
    const int64_t stride = fd.stride;
    int16_t *buf = reinterpret_cast<int16_t *>(lds);
    uint8_t *s_bits = lds + StreamLds::kBitsOff;
    uint32_t *s_pc = reinterpret_cast<uint32_t *>(lds + StreamLds::kPcOff);
    int32_t *seg_src = reinterpret_cast<int32_t *>(lds + StreamLds::kRunOff);
    int32_t *seg_dst = seg_src + StreamLds::kMaxRuns;

    // 1. every (channel, group) chunk of the tile into LDS; chunks outside
    //    the fill read the fill's first chunk instead and are never used
#pragma unroll
    for (int it = 0; it < StreamLds::kIters; it++) {
        const int k = it * NT + tid;
        const int c = k / G;
        const int g = k - c * G;
        const int64_t q = base + (int64_t)g * kVec;
        const int16_t *src = (k < StreamLds::kChunks && q >= 0 && q < N) ? raw + (int64_t)c * stride + q : raw;
        __builtin_amdgcn_global_load_lds(src, (lds_void *)(buf + (it * NT + wid * 64) * kVec), 16, 0, 0);
    }
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's chunks are in LDS
    lds_barrier();

    // 2. flags of the tile's groups from the LDS rows (Table 2 waveform-sum and
    //    threshold rows)
    if (tid < G) {
        const int64_t q = base + (int64_t)tid * kVec;
        uint32_t fb = 0;
        if (q >= 0 && q < N) {
            int32_t s[kVec] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll 6
            for (int c = 0; c < C; c++) add8(s, *reinterpret_cast<const uint4 *>(buf + c * ROW + tid * kVec));
            fb = flags8(s, thr_eff, N - q);
        }
        s_bits[tid] = (uint8_t)fb;
    }
    constexpr int Wn = (G + 7) >> 3;
    for (int z = G + tid; z < (Wn + 1) * 8; z += NT) s_bits[z] = 0;
    lds_barrier();

    const bool owner = tid >= gl && tid < G - gr;
    const int64_t p = base + (int64_t)tid * kVec;
    const TileScan r = scan_tile<NT>(a, fd, lt, G, tid, owner, p, s_bits, s_pc, s_wsum, s_excl);
    write_records(fd, r, p);
    write_counts(fd, lt, r);

    // 4b. chopped islands from the LDS rows
    if (fd.out != nullptr && r.tile_m > 0) {
        if (r.rise) {
#pragma unroll
            for (int k = 0; k < kVec; k++) {
                if ((r.rise >> k) & 1u) {
                    const int j = r.th_i + __popc(r.rise & ((1u << k) - 1u));
                    seg_src[j] = tid * kVec + k;
                    seg_dst[j] = r.th_m + __popc(r.mm & ((1u << k) - 1u));
                }
            }
        }
        lds_barrier();
        gather_from_lds<NT>(buf, seg_src, seg_dst, r.tile_i, gl * kVec, fd.out, fd.out_stride, r.m_before,
                            r.tile_m);
    }
}

// ---- the persistent kernel ------------------------------------------------------------

template <int NT, int VARIANT>
struct KernelLds {
    static constexpr int kChop = ChopLds<NT>::kBytes;
    static constexpr int kBytes = (VARIANT == kVariantStream && StreamLds::kBytes > kChop) ? StreamLds::kBytes : kChop;
};

// Fills whose first-tile indices a work-group keeps in LDS for the lookup.
constexpr int kLdsFills = 256;

template <int NT, int VARIANT>
__global__ void __launch_bounds__(NT) k_chop(KArgs a) {
    __shared__ __align__(16) uint8_t s_lds[KernelLds<NT, VARIANT>::kBytes];
    __shared__ uint32_t s_wsum[NT / 64];
    __shared__ uint64_t s_excl;
    __shared__ int64_t s_tile;
    __shared__ int64_t s_base[kLdsFills];

    const int nf = a.hdr ? a.hdr->n_fills : a.n_fills;
    const int64_t total = a.hdr ? a.hdr->total_tiles : a.total_tiles;
    const bool lds_fills = nf <= kLdsFills;
    if (lds_fills)
        for (int i = threadIdx.x; i < nf; i += NT) s_base[i] = tile_base_at(a, i);
    if (threadIdx.x == 0) s_tile = (int64_t)atomicAdd(a.ticket, 1u);
    lds_barrier();
    int64_t tile = s_tile;
    // the fill of the previous tile stays cached: consecutive tiles of a
    // work-group usually belong to the same fill
    FillDev fd{};
    int cur = -1;
    int32_t thr_eff = 0;
    // the fill owning a tile: the last one whose first tile is <= tile; the
    // previous tile's fill stays cached
    auto lookup = [&](int64_t t) {
        if (cur >= 0 && t >= fd.tile_base && t < fd.tile_base + fd.n_tiles) return;
        int lo = 0, hi = nf - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if ((lds_fills ? s_base[mid] : tile_base_at(a, mid)) <= t) lo = mid;
            else hi = mid - 1;
        }
        fd = fill_at(a, lo);
        thr_eff = clamp_thr(*gbl(a.thr_eff + lo));
        cur = lo;
    };
    constexpr bool kDeferred =
        VARIANT == kVariantReload || VARIANT == kVariantReload18 || VARIANT == kVariantReload27;
    if constexpr (kDeferred) {
        // Each tile's back half runs one tile later: by then every earlier
        // tile of its fill has published its total, so the look-back does not
        // wait, and the next tile's loads are already done.
        constexpr int R = VARIANT == kVariantReload18 ? 18 : (VARIANT == kVariantReload27 ? 27 : 6);
        FillDev fd_prev{};
        ReloadTile prev{};
        bool have_prev = false;
        while (tile < total || have_prev) {
            const bool have_cur = tile < total;
            ReloadTile now{};
            if (have_cur) {
                lookup(tile);
                now = reload_front<NT, R>(a, fd, thr_eff, tile, s_lds, s_wsum);
            }
            if (have_prev) reload_back<NT>(a, fd_prev, prev, s_lds, &s_excl);
            lds_barrier();
            // the next tile is taken only now: a dispensed tile must start at
            // once, because later tiles of its fill wait for its total
            if (threadIdx.x == 0) s_tile = have_cur ? (int64_t)atomicAdd(a.ticket, 1u) : total;
            lds_barrier();
            tile = s_tile;
            fd_prev = fd;
            prev = now;
            have_prev = have_cur;
        }
    } else {
        while (tile < total) {
            lookup(tile);
            if constexpr (VARIANT == kVariantStream && NT == kStreamThreads) {
                if (fd.mode == kModeStream) stream_tile(a, fd, thr_eff, tile, s_lds, s_wsum, &s_excl);
                else chop_tile<NT, false, 6>(a, fd, thr_eff, tile, s_lds, s_wsum, &s_excl);
            } else {
                chop_tile<NT, true, 6>(a, fd, thr_eff, tile, s_lds, s_wsum, &s_excl);  // 54-channel fills only
            }
            lds_barrier();
            // the next tile is taken only now: a dispensed tile must start at
            // once, because later tiles of its fill wait for its total
            if (threadIdx.x == 0) s_tile = (int64_t)atomicAdd(a.ticket, 1u);
            lds_barrier();
            tile = s_tile;
        }
    }
}

// ---- variant 5: scan pass, edge pass, copy pass -------------------------------------
//
// The scan pass streams the raw rows once and keeps nothing: per tile it
// writes the island-mask bits of the samples it owns and the tile's totals.
// The edge pass sums the totals of each tile's predecessors into its
// exclusive prefix and writes the island records, a run table and the
// fill's counts; the copy pass copies only the island samples. No tile
// waits for another, so the streaming pass keeps as many loads in flight as
// the CU holds.

// Fills [lo, hi) and their tiles [tile_lo, tile_hi) of the launch's part of
// the batch (the whole batch when parts <= 1).
struct PartRange {
    int lo, hi;
    int64_t tile_lo, tile_hi;
};
__device__ __forceinline__ PartRange part_range(const KArgs &a, int nf, int64_t total) {
    PartRange r{0, nf, 0, total};
    if (a.parts > 1) {
        r.lo = (int)((int64_t)nf * a.part / a.parts);
        r.hi = (int)((int64_t)nf * (a.part + 1) / a.parts);
        r.tile_lo = r.lo < nf ? tile_base_at(a, r.lo) : total;
        r.tile_hi = r.hi < nf ? tile_base_at(a, r.hi) : total;
    }
    return r;
}

#ifndef DAQ_Q_SCAN_ROWS
#define DAQ_Q_SCAN_ROWS 4  // the same with the Q-method fused (three loads per row)
#endif
#ifndef DAQ_SCAN_ROWS
#define DAQ_SCAN_ROWS 9  // channel rows each thread has in flight
#endif

// Flags and dilation of one tile (Table 2 threshold and pre/post rows): the
// island-mask bits of samples p - 1 .. p + 8 of the calling thread (zero for
// threads that own no samples).
template <int NT, int R, bool Q = false>
__device__ __forceinline__ uint32_t tile_mask10(const FillDev &fd, const ChopGeom<NT> &q, int32_t thr_eff,
                                                uint8_t *lds, bool stream, int64_t ped_total = 0) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    const int64_t N = fd.n;
    uint8_t *s_bits = lds;
    uint32_t *s_pc = reinterpret_cast<uint32_t *>(lds + ChopLds<NT>::kWords * 8);
    chop_flags<NT, R, Q>(fd, q, thr_eff, s_bits, stream, ped_total);
    const int Wn = (q.G + 7) >> 3;
    const uint64_t *words = reinterpret_cast<const uint64_t *>(s_bits);
    // windows of at most 55 samples: the flags around a group fit one 64-bit
    // word; wider ones go through popcount prefixes of the bitmap
    const bool narrow = fd.pre + fd.post <= 54;
    if (!narrow) {
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
        lds_barrier();
    }
    // sample t is marked when some flag lies in [t - post, t + pre]
    uint32_t m10 = 0;
    if (q.owner) {
        const int r0 = q.g * kVec;
        if (narrow) {
            // bits r0 - 1 - post .. r0 + 62 - post of the bitmap (r0 - 1 - post >= 0)
            const int x0 = r0 - 1 - fd.post;
            const int w = x0 >> 6, b = x0 & 63;
            const uint64_t w0 = words[w], w1 = words[w + 1];
            const uint64_t win = b ? ((w0 >> b) | (w1 << (64 - b))) : w0;
            const uint64_t span = (2ull << (fd.pre + fd.post)) - 1ull;  // pre + post + 1 ones
#pragma unroll
            for (int j = 0; j < 10; j++) {
                const int64_t t = q.p + j - 1;
                const bool in = ((win >> j) & span) != 0 && t >= 0 && t < N;
                m10 |= (in ? 1u : 0u) << j;
            }
        } else {
            uint32_t lo[10], hi[10];
            prefix_bits10(words, s_pc, r0 - 1 - fd.post, lo);
            prefix_bits10(words, s_pc, r0 + fd.pre, hi);
#pragma unroll
            for (int j = 0; j < 10; j++) {
                const int64_t t = q.p + j - 1;
                const bool in = (hi[j] != lo[j]) && t >= 0 && t < N;
                m10 |= (in ? 1u : 0u) << j;
            }
        }
    }
    return m10;
}

constexpr int kPedChannels = 512;  // channels whose pedestal sums one round accumulates in LDS

// Pedestals (Table 2 pedestal row): every channel's mean of its first
// n = min(Np, N) samples, rounded half up (floor((2 P + n) / (2 n)) of the
// int64 sum P); 0 for an empty fill. Returns their sum; writes ped[] when
// `write`. Called by a whole work-group of NT threads (barriers inside); its
// threads take (channel, 8-sample chunk) pairs with 16-byte loads, four per
// thread and round with every load issued before the adds.
template <int NT>
__device__ int64_t fill_pedestals(const FillDev &fd, bool write, long long *s_acc, long long *s_ped) {
    const int64_t n = fd.n < (int64_t)fd.np ? fd.n : (int64_t)fd.np;
    const int64_t nch = (n + kVec - 1) / kVec;
    if (threadIdx.x == 0) *s_ped = 0;
    for (int c0 = 0; c0 < fd.C; c0 += kPedChannels) {
        const int cn = fd.C - c0 < kPedChannels ? fd.C - c0 : kPedChannels;
        for (int i = threadIdx.x; i < cn; i += NT) s_acc[i] = 0;
        __syncthreads();
        const int64_t items = (int64_t)cn * nch;
        constexpr int kItems = 4;
        for (int64_t i0 = threadIdx.x; i0 < items; i0 += NT * kItems) {
            uint4 v[kItems];
            int cl[kItems];
            int64_t t[kItems];
#pragma unroll
            for (int u = 0; u < kItems; u++) {
                const int64_t i = i0 + (int64_t)u * NT;
                cl[u] = (int)(i / nch);
                t[u] = (i - (int64_t)cl[u] * nch) * kVec;
                if (i < items) v[u] = load16(fd.raw + (int64_t)(c0 + cl[u]) * fd.stride + t[u]);
            }
#pragma unroll
            for (int u = 0; u < kItems; u++) {
                if (i0 + (int64_t)u * NT >= items) break;
                int32_t s[kVec] = {0, 0, 0, 0, 0, 0, 0, 0};
                add8(s, v[u]);
                int32_t part = 0;
#pragma unroll
                for (int k = 0; k < kVec; k++) part += (t[u] + k < n) ? s[k] : 0;
                atomicAdd(reinterpret_cast<unsigned long long *>(&s_acc[cl[u]]), (unsigned long long)(long long)part);
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < cn; i += NT) {
            const int32_t ped = n > 0 ? (int32_t)floor_div(2 * (int64_t)s_acc[i] + n, 2 * n) : 0;
            if (write && fd.ped) fd.ped[c0 + i] = ped;
            atomicAdd(reinterpret_cast<unsigned long long *>(s_ped), (unsigned long long)(long long)ped);
        }
        __syncthreads();
    }
    const int64_t sum = *s_ped;
    __syncthreads();  // s_ped and s_acc are free again
    return sum;
}

// Scan pass, one tile: flags, dilation, mask bits, totals. Each wave leaves
// its totals (island samples, islands begun) in s_part; thread 0 adds them up
// and stores the tile's word after the next tile's first barrier (or after
// the work-group's last tile), so a tile ends without a barrier of its own
// and tile_state needs no clearing. Before that, thread 0 stores the word of
// the previous tile (prev_tile >= 0) from s_prev.
template <int NT>
__device__ __forceinline__ void put_tile_total(const KArgs &a, int64_t tile, const uint32_t *part) {
    uint64_t m = 0, i = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; w++) {
        m += part[w] >> 16;
        i += part[w] & 0xFFFFu;
    }
    *gbl(a.tile_state + tile) = (m << 31) | i;
}

template <int NT, int R, bool Q = false>
__device__ __forceinline__ void scan_pass_tile(const KArgs &a, const FillDev &fd, int32_t thr_eff, int64_t tile,
                                               uint8_t *lds, int64_t ped_total, uint32_t *s_part,
                                               int64_t prev_tile, const uint32_t *s_prev) {
    const int lane = threadIdx.x & 63;
    const ChopGeom<NT> q(fd, tile);
    const uint32_t m10 = tile_mask10<NT, R, Q>(fd, q, thr_eff, lds, stream_loads(a), ped_total);
    if (threadIdx.x == 0 && prev_tile >= 0) put_tile_total<NT>(a, prev_tile, s_prev);
    if (q.owner) {
        // the owned samples' mask byte: t0 is a multiple of 8
        const int64_t byte = (q.t0 >> 3) + (q.g - fd.gl);
        *gbl(fd.mbits + byte) = (uint8_t)((m10 >> 1) & 0xFFu);
    }
    const uint32_t mm = (m10 >> 1) & 0xFFu;
    const uint32_t rise = mm & ~(((mm << 1) | (m10 & 1u)) & 0xFFu);
    // the wave's totals (island samples, islands begun)
    uint32_t mine = ((uint32_t)__popc(mm) << 16) | (uint32_t)__popc(rise);
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) mine += __shfl_xor(mine, d, 64);
    if (lane == 0) s_part[threadIdx.x >> 6] = mine;
}

// PED: the work-group computes the pedestals of each fill it meets (the
// first min(Np, N) samples of every row, from L2 after the first reader) and
// the tile-0 work-group writes them out; the mask guards are cleared by the
// fill's first and last tiles. Otherwise k_prepare has done both.
template <int NT, int R, bool Q = false, bool PED = false>
__global__ void __launch_bounds__(NT) k_scan_pass(KArgs a) {
    // two bitmaps, used by alternate tiles: a wave still reading one tile's
    // bitmap never meets the next tile's writes, so tiles need no closing
    // barrier (the next-but-one tile's writes come after a barrier every
    // wave has passed)
    __shared__ __align__(16) uint8_t s_lds[2][ChopLds<NT>::kBitsBytes];
    __shared__ int64_t s_base[kLdsFills];
    __shared__ uint32_t s_part[2][NT / 64];
    __shared__ long long s_acc[kPedChannels];
    __shared__ long long s_ped;
    const int nf = a.hdr ? a.hdr->n_fills : a.n_fills;
    const int64_t total = a.hdr ? a.hdr->total_tiles : a.total_tiles;
    const bool lds_fills = nf <= kLdsFills;
    if (lds_fills)
        for (int i = threadIdx.x; i < nf; i += NT) s_base[i] = tile_base_at(a, i);
    lds_barrier();
    FillDev fd{};
    int cur = -1;
    int32_t thr_eff = 0;
    int64_t ped_total = 0;  // Q: the sum of the fill's pedestals
    int buf = 0;
    int64_t prev_tile = -1;
    const PartRange pr = part_range(a, nf, total);
    for (int64_t tile = pr.tile_lo + blockIdx.x; tile < pr.tile_hi; tile += gridDim.x) {
        if (cur < 0 || tile < fd.tile_base || tile >= fd.tile_base + fd.n_tiles) {
            int lo = 0, hi = nf - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if ((lds_fills ? s_base[mid] : tile_base_at(a, mid)) <= tile) lo = mid;
                else hi = mid - 1;
            }
            fd = fill_at(a, lo);
            int64_t te;
            if constexpr (PED) te = (int64_t)fd.thr + fill_pedestals<NT>(fd, tile == fd.tile_base, s_acc, &s_ped);
            else te = *gbl(a.thr_eff + lo);
            thr_eff = clamp_thr(te);
            ped_total = te - (int64_t)fd.thr;
            cur = lo;
        }
        if constexpr (PED) {
            const int64_t lt = tile - fd.tile_base;
            const int i = (int)threadIdx.x;
            if (i < kMaskGuard && lt == 0) fd.mbits[i - kMaskGuard] = 0;
            if (i < kMaskGuard && lt == fd.n_tiles - 1) fd.mbits[fd.n_tiles * fd.tout / kVec + i] = 0;
        }
        scan_pass_tile<NT, R, Q>(a, fd, thr_eff, tile, s_lds[buf], ped_total, s_part[buf], prev_tile, s_part[buf ^ 1]);
        prev_tile = tile;
        buf ^= 1;
    }
    lds_barrier();
    if (threadIdx.x == 0 && prev_tile >= 0) put_tile_total<NT>(a, prev_tile, s_part[buf ^ 1]);
}

// The run table entries (start, packed offset) of the islands the calling
// thread begins and, for the multiple k of kCopyChunk among its packed
// positions (at most one), the island holding packed position k; the thread
// owns samples p .. p + 7 with island mask r.mm and the prefixes of r.
// COHERENT: device-scope stores (read by other work-groups of the launch).
template <bool COHERENT = false>
__device__ __forceinline__ void write_runs(const FillDev &fd, const TileScan &r, int64_t p) {
    auto put = [](DAQ_GLOBAL int32_t *dst, int32_t v) {
        if constexpr (COHERENT) __hip_atomic_store(dst, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else *dst = v;
    };
    if (fd.out == nullptr || r.mm == 0) return;
    const int64_t mbase = r.m_before + r.th_m;
    const int64_t ibase = r.i_before + r.th_i;
    DAQ_GLOBAL int32_t *runs = gbl(fd.runs);
#pragma unroll
    for (int k = 0; k < kVec; k++) {
        if ((r.rise >> k) & 1u) {
            const int64_t idx = ibase + __popc(r.rise & ((1u << k) - 1u));
            put(runs + 2 * idx, (int32_t)(p + k));
            put(runs + 2 * idx + 1, (int32_t)(mbase + __popc(r.mm & ((1u << k) - 1u))));
        }
    }
    const int64_t q = (mbase + kCopyChunk - 1) / kCopyChunk * kCopyChunk;
    const int cnt = __popc(r.mm);
    if (q < mbase + cnt) {
        uint32_t bits = r.mm;
        for (int64_t skip = q - mbase; skip > 0; skip--) bits &= bits - 1;  // drop the lowest set bits
        const int b = __ffs(bits) - 1;
        put(gbl(fd.cmap + q / kCopyChunk), (int32_t)(ibase + __popc(r.rise & ((2u << b) - 1u)) - 1));
    }
}

// Edge pass, one tile per wave: the tile's exclusive prefix (the sum of the
// totals the scan pass wrote for the fill's earlier tiles), island edges from
// the mask bits, the island records (capacity-limited), the fill's run table
// (start, offset of every island), for every multiple k of kCopyChunk among
// the tile's packed positions the island holding packed position k, and, from
// the fill's last tile, the fill's counts. Lane l takes the tile's
// owned mask bytes 8l .. 8l + 7 (64 samples); a tile owns at most 512 bytes.
// Only wave-level scans: no barrier, and a work-group handles NT / 64 tiles
// at once.
__device__ __forceinline__ void edge_wave_tile(const KArgs &a, const FillDev &fd, int64_t tile, int lane) {
    const int64_t lt = tile - fd.tile_base;
    const int64_t t0 = lt * fd.tout;
    const int own = (int)(fd.tout / kVec);  // owned mask bytes
    const uint8_t *mb = fd.mbits + (t0 >> 3);
    const int b0 = lane * 8;
    const int nb = own - b0 < 0 ? 0 : (own - b0 < 8 ? own - b0 : 8);  // this lane's bytes
    // bytes b0 - 2 .. b0 + 13 in one 16-byte load (2-byte aligned: mbits is
    // 16-byte aligned and a tile owns an even number of bytes). It stays
    // inside the fill's mask: byte -2 and bytes up to 12 past the last tile's
    // owned bytes fall in the 16 guard bytes on either side. Byte b0 - 1 is
    // zero before the fill's first sample, byte b0 + nb after its last.
    u32x4 w = u32x4{0, 0, 0, 0};
    if (nb > 0) __builtin_memcpy(&w, (const DAQ_GLOBAL int16_t *)(mb + b0 - 2), 16);
    // the tile's exclusive prefix: the totals of the fill's earlier tiles
    // (written by the scan pass), summed by the wave; these loads are issued
    // with the mask load above, so the two wait together
    uint64_t pref = 0;
#pragma unroll 4
    for (int64_t j = lane; j < lt; j += 64) pref += *gbl(a.tile_state + fd.tile_base + j);
    pref = wave_sum_u64(pref);
    uint64_t m = 0;
    uint32_t prv = 0, nxt = 0;
    if (nb > 0) {
        const uint64_t lo = ((uint64_t)w.y << 32) | w.x;   // bytes -2 .. 5
        const uint64_t hi = ((uint64_t)w.w << 32) | w.z;   // bytes 6 .. 13
        m = (lo >> 16) | (hi << 48);                       // bytes 0 .. 7
        if (nb < 8) m &= (1ull << (8 * nb)) - 1ull;
        prv = (uint32_t)(lo >> 15) & 1u;                   // top bit of byte -1
        const int nx = nb + 2;                             // byte b0 + nb, 2 .. 10 of the load
        nxt = (uint32_t)((nx < 8 ? (lo >> (8 * nx)) : (hi >> (8 * (nx - 8)))) & 1u);
    }
    const uint64_t rise = m & ~((m << 1) | (uint64_t)prv);
    const uint64_t fall = nb > 0 ? (m & ~((m >> 1) | ((uint64_t)nxt << (8 * nb - 1)))) : 0ull;
    const uint32_t cm = (uint32_t)__popcll(m), ci = (uint32_t)__popcll(rise);
    const uint32_t mine = (cm << 16) | ci;
    const uint32_t excl = wave_incl_scan_u32(mine, lane) - mine;
    if (lt == fd.n_tiles - 1 && lane == 0 && fd.counts != nullptr) {
        // the fill's last tile writes the counts
        const uint64_t all = pref + *gbl(a.tile_state + tile);
        const int64_t n_isl = (int64_t)(all & kField);
        const int64_t tl = (int64_t)((all >> 31) & kField);
        int32_t status = (n_isl > fd.cap) ? DAQ_STATUS_CAPACITY : 0;
        if (fd.out != nullptr && tl > fd.out_stride) status |= DAQ_STATUS_OUT_STRIDE;
        DAQ_GLOBAL daq_counts *cnt = gbl(fd.counts);
        cnt->n_islands = n_isl;
        cnt->total_len = tl;
        cnt->status = status;
        cnt->reserved = 0;
    }
    const int64_t mbase = (int64_t)((pref >> 31) & kField) + (int64_t)(excl >> 16);
    const int64_t ibase = (int64_t)(pref & kField) + (int64_t)(excl & 0xFFFFu);
    const int64_t p = t0 + (int64_t)b0 * 8;  // this lane's first sample
    DAQ_GLOBAL daq_island *isl = gbl(fd.isl);
    DAQ_GLOBAL int32_t *runs = gbl(fd.runs);
    const bool copy = fd.out != nullptr;
    for (uint64_t r = rise; r; r &= r - 1) {
        const int k = __ffsll((unsigned long long)r) - 1;
        const uint64_t below = (1ull << k) - 1ull;
        const int64_t idx = ibase + __popcll(rise & below);
        const int64_t off = mbase + __popcll(m & below);
        if (idx < fd.cap) {
            isl[idx].start = p + k;
            isl[idx].offset = off;
        }
        if (copy) {
            runs[2 * idx] = (int32_t)(p + k);
            runs[2 * idx + 1] = (int32_t)off;
        }
    }
    for (uint64_t f = fall; f; f &= f - 1) {
        const int k = __ffsll((unsigned long long)f) - 1;
        const uint64_t upto = k == 63 ? ~0ull : ((2ull << k) - 1ull);
        const int64_t idx = ibase + __popcll(rise & upto) - 1;
        if (idx >= 0 && idx < fd.cap) isl[idx].stop = p + k + 1;
    }
    if (!copy || cm == 0) return;
    // at most one multiple of the chunk size among this lane's packed positions
    const int64_t q = (mbase + kCopyChunk - 1) / kCopyChunk * kCopyChunk;
    if (q < mbase + cm) {
        uint64_t bits = m;
        for (int64_t skip = q - mbase; skip > 0; skip--) bits &= bits - 1;  // drop the lowest set bits
        const int b = __ffsll((unsigned long long)bits) - 1;
        const uint64_t upto = b == 63 ? ~0ull : ((2ull << b) - 1ull);
        *gbl(fd.cmap + q / kCopyChunk) = (int32_t)(ibase + __popcll(rise & upto) - 1);
    }
}

template <int NT>
__global__ void __launch_bounds__(NT) k_edge_pass(KArgs a) {
    constexpr int NW = NT / 64;
    __shared__ int64_t s_base[kLdsFills];
    __shared__ u32x4 s_fd[kFdLds * kFdWords];
    const int nf = a.hdr ? a.hdr->n_fills : a.n_fills;
    const int64_t total = a.hdr ? a.hdr->total_tiles : a.total_tiles;
    const bool lds_fills = nf <= kLdsFills;
    if (lds_fills)
        for (int i = threadIdx.x; i < nf; i += NT) s_base[i] = tile_base_at(a, i);
    const bool fd_lds = stage_fills<NT>(a, nf, s_fd);
    lds_barrier();
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    FillDev fd{};
    int cur = -1;
    const PartRange pr = part_range(a, nf, total);
    // fills without samples have no tile: their counts and pedestals (all
    // zero) come from here, each work-group taking some of the fills
    for (int f = pr.lo + (int)blockIdx.x; f < pr.hi; f += (int)gridDim.x) {
        const FillDev *fp = a.table ? a.table + f : &a.one;
        if (fp->n_tiles != 0) continue;
        daq_counts *cnt = fp->counts;
        if (threadIdx.x == 0 && cnt != nullptr) {
            cnt->n_islands = 0;
            cnt->total_len = 0;
            cnt->status = 0;
            cnt->reserved = 0;
        }
        int32_t *ped = fp->ped;
        if (ped != nullptr)
            for (int c = (int)threadIdx.x; c < fp->C; c += NT) ped[c] = 0;
    }
    for (int64_t tile = pr.tile_lo + (int64_t)blockIdx.x * NW + wid; tile < pr.tile_hi;
         tile += (int64_t)gridDim.x * NW) {
        if (cur < 0 || tile < fd.tile_base || tile >= fd.tile_base + fd.n_tiles) {
            int lo = 0, hi = nf - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if ((lds_fills ? s_base[mid] : tile_base_at(a, mid)) <= tile) lo = mid;
                else hi = mid - 1;
            }
            fd = fd_lds ? fill_from_lds(s_fd, lo) : fill_at(a, lo);
            cur = lo;
        }
        edge_wave_tile(a, fd, tile, lane);
    }
}

// The values a copy of chunk k needs besides the run table: the fill's
// counts and the islands holding the chunk's first and last positions.
struct ChunkInfo {
    int64_t tl, n_isl;
    int32_t i0, i1;
};
__device__ __forceinline__ ChunkInfo chunk_info(const FillDev &fd, int64_t k) {
    ChunkInfo c;
    c.tl = *gbl(&fd.counts->total_len);
    c.n_isl = *gbl(&fd.counts->n_islands);
    c.i0 = k * kCopyChunk < c.tl ? *gbl(fd.cmap + k) : 0;
    c.i1 = (k + 1) * kCopyChunk < c.tl ? *gbl(fd.cmap + k + 1) : (int32_t)c.n_isl - 1;
    return c;
}

// Chunk k of fill fd's packed rows (the fill's counts, run table and chunk
// map complete; ci the same in every thread); L is a CopyLayout for
// kCopyChunk + 1 runs. COHERENT: the run table is read with device-scope
// loads (it was written in the same launch).
template <int NT, class L, bool COHERENT = false, int U = DAQ_EMIT_U>
__device__ __forceinline__ void copy_chunk(const FillDev &fd, int64_t k, const ChunkInfo &ci, const CopyView &v) {
    constexpr int P = kCopyChunk;
    const int tid = threadIdx.x;
    const int64_t q0 = k * P;
    if (q0 >= ci.tl) return;
    const int m = (int)(ci.tl - q0 < P ? ci.tl - q0 : P);
    const int nrun = ci.i1 - ci.i0 + 1;  // islands touching [q0, q0 + P], at most P + 1
    for (int r = tid; r < nrun; r += NT) {
        const DAQ_GLOBAL int32_t *e = gbl(fd.runs + 2 * (int64_t)(ci.i0 + r));
        int32_t st, of;
        if constexpr (COHERENT) {
            st = __hip_atomic_load(e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            of = __hip_atomic_load(e + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            st = e[0];
            of = e[1];
        }
        const int64_t d = (int64_t)of - q0;  // negative only for the first island
        v.dst[r] = d > 0 ? (int32_t)d : 0;
        v.src[r] = d > 0 ? st : (int32_t)(st - d);
    }
    lds_barrier();
    copy_runs<NT, L, U>(fd, v, nrun, m, q0);
}

// ---- copy pass of the split schedule ----------------------------------------------
//
// Writes the packed rows (the chopped islands of every channel) from the run
// table and chunk map of the edge pass. A work item is one wave's: a fill, a
// segment of kCopyChunk = 512 packed positions (one 16-byte word per lane)
// and a group of kCopyGroup channels. Items are numbered fill by fill; every
// work-group first computes the items of each fill from its counts (a prefix
// in LDS), so the launch needs no host-side sizes and idle waves leave at
// once. Per item the wave copies the segment's runs into its own LDS (source
// sample of the run's first packed position, packed start relative to the
// segment) and each lane finds the run holding its word's first position by
// one max-scan over the lanes (run j marks the first word that starts at or
// after its own start). Then, kCopyU channels at a time, every lane loads its
// 8 source samples with one unaligned 16-byte load per run piece (two where
// its word holds the end of one run and the start of the next), blends them
// at the run boundary and writes one 16-byte word with a non-temporal store;
// the next round's loads are issued before this round's stores, and no
// barrier is taken. A word holding pieces of three or more runs, the last
// partial word of a row and rows whose line phase differs from their
// neighbours' (out_stride not a multiple of 8 or out not 16-byte aligned) go
// sample by sample.

#ifndef DAQ_COPY_GROUP
#define DAQ_COPY_GROUP 6  // channels per work item (54 = 9 x 6)
#endif
#ifndef DAQ_COPY_U
#define DAQ_COPY_U 3  // channels with loads in flight per round
#endif
constexpr int kCopyGroup = DAQ_COPY_GROUP;
constexpr int kCopyU = DAQ_COPY_U;
constexpr int kSegRuns = kCopyChunk + 3;  // runs touching one segment, and two end marks
static_assert(kCopyChunk == 64 * kVec, "a segment is one 16-byte word per lane");

// Eight consecutive int16 samples from any element address (2-byte
// aligned): one 16-byte load, which gfx950 serves unaligned (the HSA runtime
// runs it in unaligned access mode).
__device__ __forceinline__ uint4 load16u(const int16_t *p) {
    u32x4 v;
    __builtin_memcpy(&v, (const DAQ_GLOBAL int16_t *)p, 16);
    return make_uint4(v.x, v.y, v.z, v.w);
}

// One round of the copy: the source samples of kCopyU channels starting at
// channel c, for a lane whose word is one run (kind 1: v0) or two (kind 2:
// v0, then v1 from element split on).
__device__ __forceinline__ void copy_load(const FillDev &fd, int c, int c_hi, int kind, int src0, int src1,
                                          uint4 (&v0)[kCopyU], uint4 (&v1)[kCopyU]) {
#pragma unroll
    for (int u = 0; u < kCopyU; u++) {
        if (c + u < c_hi && (kind == 1 || kind == 2)) {
            const int16_t *row = fd.raw + (int64_t)(c + u) * fd.stride;
            v0[u] = load16u(row + src0);
            if (kind == 2) v1[u] = load16u(row + src1);
        }
    }
}

__device__ __forceinline__ void copy_store(const FillDev &fd, int c, int c_hi, int kind, int split, int64_t o,
                                           const uint4 (&v0)[kCopyU], const uint4 (&v1)[kCopyU]) {
#pragma unroll
    for (int u = 0; u < kCopyU; u++) {
        if (c + u < c_hi && (kind == 1 || kind == 2)) {
            const uint4 v = kind == 2 ? blend8(v0[u], v1[u], split) : v0[u];
            store16(fd.out + (int64_t)(c + u) * fd.out_stride + o, v);
        }
    }
}

// Packed positions [q0, q0 + m) of channels [c_lo, c_hi) of fill fd; the
// segment's nrun runs are in st[] / d[] (d relative to q0, d[0] <= 0, end
// marks at nrun and nrun + 1). Executed by one whole wave.
__device__ __forceinline__ void copy_segment(const FillDev &fd, int64_t q0, int m, int c_lo, int c_hi,
                                             const int32_t *st, const int32_t *d, int32_t *slot, int nrun,
                                             int lane) {
    // run of each word's first position
    slot[lane] = -1;
    __builtin_amdgcn_wave_barrier();
    for (int j = lane; j < nrun; j += 64) {
        const int dj = d[j];
        const int w = dj <= 0 ? 0 : (dj + kVec - 1) / kVec;
        if (w < 64) atomicMax(&slot[w], j);
    }
    __builtin_amdgcn_wave_barrier();
    int R = slot[lane];
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
        const int u = __shfl_up(R, s, 64);
        if (lane >= s) R = R > u ? R : u;
    }
    const int pos = kVec * lane;                       // first packed position of this lane's word
    const int valid = m - pos < kVec ? m - pos : kVec;  // positions of the word inside the segment
    const int d0 = d[R], d1 = d[R + 1], d2 = d[R + 2];
    const int st0 = st[R], st1 = st[R + 1];
    const bool uniform = (fd.out_stride & 7) == 0 && ((uintptr_t)fd.out & 15u) == 0;
    // kind 0: nothing; 1: one run; 2: two runs; 3: sample by sample
    int kind = 0;
    if (valid > 0) {
        if (!uniform || valid < kVec) kind = 3;
        else if (d1 >= pos + kVec) kind = 1;
        else if (d2 >= pos + kVec) kind = 2;
        else kind = 3;
    }
    // run R from source sample src0 on; run R + 1 from element split on, as
    // source sample src1 + element. Every sample read lies in [src0, src0 + 8)
    // or [src1, src1 + 8), inside the row: src1 >= src0 + 1 (runs are disjoint
    // and at least one sample apart) and, for two runs, both end before the
    // word's last sample, which is a sample of the fill.
    const int src0 = st0 + (pos - d0);
    const int split = kind == 2 ? d1 - pos : kVec;
    const int src1 = st1 - split;
    const int64_t o = q0 + pos;
    uint4 a0[kCopyU], a1[kCopyU], b0[kCopyU], b1[kCopyU];
#pragma unroll
    for (int u = 0; u < kCopyU; u++) a0[u] = a1[u] = b0[u] = b1[u] = make_uint4(0, 0, 0, 0);
    // rounds of kCopyU channels, double-buffered: the next round's loads are
    // issued before this round's stores, so waiting for them never waits for
    // the stores (loads and stores share one counter)
    copy_load(fd, c_lo, c_hi, kind, src0, src1, a0, a1);
    for (int c = c_lo; c < c_hi; c += 2 * kCopyU) {
        if (c + kCopyU < c_hi) copy_load(fd, c + kCopyU, c_hi, kind, src0, src1, b0, b1);
        copy_store(fd, c, c_hi, kind, split, o, a0, a1);
        if (c + kCopyU >= c_hi) break;
        if (c + 2 * kCopyU < c_hi) copy_load(fd, c + 2 * kCopyU, c_hi, kind, src0, src1, a0, a1);
        copy_store(fd, c + kCopyU, c_hi, kind, split, o, b0, b1);
    }
    if (kind == 3) {
        for (int c = c_lo; c < c_hi; c++) {
            const int16_t *row = fd.raw + (int64_t)c * fd.stride;
            DAQ_GLOBAL int16_t *orow = gbl(fd.out + (int64_t)c * fd.out_stride + q0);
            int r = R;
            for (int e = 0; e < valid; e++) {
                const int q = pos + e;
                while (r + 1 < nrun && d[r + 1] <= q) r++;
                orow[q] = *gbl(row + st[r] + (q - d[r]));
            }
        }
    }
}

constexpr int kCopyFills = kLdsFills;  // fills per window of the item prefix

// Two consecutive int32 words (4-byte aligned) in one 8-byte load.
__device__ __forceinline__ uint64_t load8_pair(const int32_t *p) {
    uint64_t v;
    __builtin_memcpy(&v, (const DAQ_GLOBAL int32_t *)p, 8);
    return v;
}

template <int NT>
__global__ void __launch_bounds__(NT) k_copy_pass(KArgs a) {
    constexpr int NW = NT / 64;
    __shared__ int64_t s_item[kCopyFills + 1];
    __shared__ int32_t s_tl[kCopyFills], s_nisl[kCopyFills];  // each fill's counts
    __shared__ int32_t s_st[NW][kSegRuns];
    __shared__ int32_t s_d[NW][kSegRuns];
    __shared__ int32_t s_slot[NW][64];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nf = a.hdr ? a.hdr->n_fills : a.n_fills;
    const PartRange pr = part_range(a, nf, a.hdr ? a.hdr->total_tiles : a.total_tiles);
    for (int w0 = pr.lo; w0 < pr.hi; w0 += kCopyFills) {
        const int wn = pr.hi - w0 < kCopyFills ? pr.hi - w0 : kCopyFills;
        // items of each fill of the window: segments of its packed rows x channel groups
        for (int i = tid; i < wn; i += NT) {
            const FillDev *fp = a.table ? a.table + w0 + i : &a.one;
            int64_t items = 0;
            const int16_t *out = fp->out;
            if (out != nullptr) {
                const daq_counts *cnt = fp->counts;
                const int64_t tl = cnt->total_len;
                const int64_t os = fp->out_stride;
                const int64_t L = tl < os ? (tl > 0 ? tl : 0) : os;
                items = (L + kCopyChunk - 1) / kCopyChunk * ((fp->C + kCopyGroup - 1) / kCopyGroup);
                s_tl[i] = (int32_t)tl;
                s_nisl[i] = (int32_t)cnt->n_islands;
            }
            s_item[i + 1] = items;
        }
        lds_barrier();
        if (wid == 0) {  // inclusive scan of s_item[1 .. wn]
            int64_t carry = 0;
            for (int i0 = 0; i0 < wn; i0 += 64) {
                const int i = i0 + lane;
                int64_t v = i < wn ? s_item[i + 1] : 0;
#pragma unroll
                for (int s = 1; s < 64; s <<= 1) {
                    const int64_t u = __shfl_up(v, s, 64);
                    if (lane >= s) v += u;
                }
                if (i < wn) s_item[i + 1] = carry + v;
                carry += __shfl(v, 63, 64);
            }
            if (lane == 0) s_item[0] = 0;
        }
        lds_barrier();
        const int64_t total = s_item[wn];
        FillDev fd{};
        int cur = -1;
        for (int64_t g = (int64_t)blockIdx.x * NW + wid; g < total; g += (int64_t)gridDim.x * NW) {
            int lo = 0, hi = wn - 1;  // the fill: last i with s_item[i] <= g
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_item[mid] <= g) lo = mid;
                else hi = mid - 1;
            }
            if (lo != cur) {
                fd = fill_at(a, w0 + lo);
                cur = lo;
            }
            const int groups = (fd.C + kCopyGroup - 1) / kCopyGroup;
            const int64_t r = g - s_item[lo];
            const int64_t k = r / groups;
            const int cg = (int)(r - k * groups);
            const int64_t tl = __builtin_amdgcn_readfirstlane(s_tl[lo]);
            const int64_t n_isl = __builtin_amdgcn_readfirstlane(s_nisl[lo]);
            const int64_t L = tl < fd.out_stride ? tl : fd.out_stride;
            const int64_t q0 = k * kCopyChunk;
            const int m = (int)(L - q0 < kCopyChunk ? L - q0 : kCopyChunk);
            // both chunk-map words in one 8-byte load (entry k + 1 exists: the
            // map has two spare words; 4-byte alignment is enough for it)
            const uint64_t e = load8_pair(fd.cmap + k);
            const int i0 = __builtin_amdgcn_readfirstlane((int)(uint32_t)e);
            const int i1 = q0 + kCopyChunk < tl ? __builtin_amdgcn_readfirstlane((int)(uint32_t)(e >> 32))
                                                : (int)n_isl - 1;
            int nrun = i1 - i0 + 1;  // at most kCopyChunk + 1
            nrun = nrun < 1 ? 1 : (nrun > kSegRuns - 2 ? kSegRuns - 2 : nrun);
            int32_t *st = s_st[wid];
            int32_t *dd = s_d[wid];
            for (int j = lane; j < nrun; j += 64) {
                const DAQ_GLOBAL int32_t *e = gbl(fd.runs + 2 * (int64_t)(i0 + j));
                st[j] = e[0];
                dd[j] = (int32_t)((int64_t)e[1] - q0);
            }
            if (lane < 2) {
                st[nrun + lane] = 0;
                dd[nrun + lane] = 1 << 30;
            }
            __builtin_amdgcn_wave_barrier();
            const int c_lo = cg * kCopyGroup;
            const int c_hi = c_lo + kCopyGroup < fd.C ? c_lo + kCopyGroup : fd.C;
            copy_segment(fd, q0, m, c_lo, c_hi, st, dd, s_slot[wid], nrun, lane);
            __builtin_amdgcn_wave_barrier();
        }
        lds_barrier();  // the next window rewrites s_item
    }
}

// ---- variant 6: one persistent kernel, copies overlapped with the scan ----------
//
// Work-groups take two kinds of work from shared counters: scan tiles, in
// batch order, and chunks of packed rows of fills whose every tile is done.
// A scan tile streams its raw rows once, takes its exclusive prefix by the
// decoupled look-back over its fill's earlier tiles and writes its island
// records, run-table entries and chunk-map entries at once; the copy of a
// finished fill then runs beside the scan of later fills, so the copy's
// arithmetic fills the time the scan waits for memory. Chunks are taken
// before scan tiles. No work-group waits for work that was handed out after
// its own (a tile's look-back only for earlier tiles of its fill, which are
// being scanned; an idle work-group for tiles being scanned), so the launch
// always drains.
//
// Shared words: ticket[0] dispenses scan tiles; ticket[2] is the first fill
// whose chunks may remain; ticket[4] is set when a work-group gave up
// waiting. tile_pref[f] holds the finished tiles of fill f (low half) and
// its chunks handed out (high half).

#ifndef DAQ_PIPE_STAGE_WORDS
#define DAQ_PIPE_STAGE_WORDS 1024  // staged source words of a copy (two buffers)
#endif
using PipeCopyLayout = CopyLayout<kCopyChunk + 2, kCopyChunk / kVec + 3, DAQ_PIPE_STAGE_WORDS / 2>;

template <int NT>
struct PipeLds {
    static constexpr int kScan = ChopLds<NT>::kBitsBytes;
    static constexpr int kBytes = kScan > PipeCopyLayout::kBytes ? kScan : PipeCopyLayout::kBytes;
};

constexpr int64_t kJobExit = -1;         // nothing left
constexpr int64_t kJobCopy = -2;         // kJobCopy - (fill << 32 | chunk): a chunk to copy
constexpr uint32_t kPipeSpins = 1u << 20;  // idle polls before a work-group gives up

// The next work item of the calling work-group (thread 0 only): a chunk of a
// finished fill (kJobCopy - (fill << 32 | chunk), with its ChunkInfo in
// *ci), else a scan tile (>= 0), else, once every fill's chunks are handed
// out, kJobExit. Chunks are claimed with one atomic add on the fill's word
// (high half), so claims never retry. Waiting polls back off and are
// bounded: past the limit the work-group marks the launch and the waited-for
// fill as incomplete and leaves.
__device__ int64_t pipe_next(const KArgs &a, int nf, int64_t total, ChunkInfo *ci) {
    uint32_t *copy_fill = a.ticket + 2;  // first fill whose chunks may remain
    uint32_t *gave_up = a.ticket + 4;
    for (uint32_t spin = 0;; spin++) {
        int f = (int)__hip_atomic_load(copy_fill, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        while (f < nf) {
            const FillDev fc = fill_at(a, f);
            // the fill's counts, run table and chunk map were stored (device
            // scope) before its tiles were counted; they are read with
            // device-scope loads after the count is seen
            const uint64_t w = __hip_atomic_load(a.tile_pref + f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((int64_t)(uint32_t)w < fc.n_tiles) break;
            int64_t tl = 0, nch = 0;
            if (fc.out != nullptr && fc.counts != nullptr) {
                tl = __hip_atomic_load(&fc.counts->total_len, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                nch = (tl + kCopyChunk - 1) / kCopyChunk;
            }
            if ((int64_t)(w >> 32) < nch) {
                const int64_t k = (int64_t)(__hip_atomic_fetch_add(a.tile_pref + f, (uint64_t)1 << 32, __ATOMIC_RELAXED,
                                                                   __HIP_MEMORY_SCOPE_AGENT) >> 32);
                if (k < nch) {
                    const int64_t n_isl = __hip_atomic_load(&fc.counts->n_islands, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT);
                    ci->tl = tl;
                    ci->n_isl = n_isl;
                    ci->i0 = __hip_atomic_load(fc.cmap + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ci->i1 = (k + 1) * kCopyChunk < tl
                                 ? __hip_atomic_load(fc.cmap + k + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                 : (int32_t)n_isl - 1;
                    return kJobCopy - (int64_t)(((uint64_t)f << 32) | (uint64_t)k);
                }
            }
            // every chunk of fill f is handed out: move the shared pointer on
            uint32_t expect = (uint32_t)f;
            __hip_atomic_compare_exchange_strong(copy_fill, &expect, (uint32_t)(f + 1), __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            f++;
        }
        if (__hip_atomic_load(a.ticket, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (uint64_t)total) {
            const uint32_t t = atomicAdd(a.ticket, 1u);
            if ((int64_t)t < total) return (int64_t)t;
        }
        if (f >= nf) return kJobExit;
        if (__hip_atomic_load(gave_up, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u || spin >= kPipeSpins) {
            __hip_atomic_store(gave_up, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const FillDev fc = fill_at(a, f);
            if (fc.counts != nullptr)
                __hip_atomic_fetch_or(&fc.counts->status, DAQ_STATUS_INCOMPLETE, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
            return kJobExit;
        }
        // idle: poll rarely, the shared words sit on one memory channel
        if (spin < 4) __builtin_amdgcn_s_sleep(16);
        else __builtin_amdgcn_s_sleep(127);
    }
}

// One scan tile of the persistent kernel: flags, dilation, totals (published
// at once), look-back, records, counts (the fill's last tile), run table and
// chunk map; then the tile is counted as finished.
template <int NT, int R>
__device__ __forceinline__ void pipe_tile(const KArgs &a, const FillDev &fd, int f, int32_t thr_eff, int64_t tile,
                                          uint8_t *lds, uint32_t *s_wsum, uint64_t *s_excl) {
    const ChopGeom<NT> q(fd, tile);
    const uint32_t m10 = tile_mask10<NT, R>(fd, q, thr_eff, lds, stream_loads(a));
    TileScan r = tile_totals<NT>(a, fd, q.lt, m10, s_wsum);
    scan_back(a, fd, q.lt, r, s_excl, a.ticket + 4);
    write_records(fd, r, q.p);
    write_counts<true>(fd, q.lt, r);
    write_runs<true>(fd, r, q.p);
    if (threadIdx.x == 0 && fd.counts != nullptr &&
        __hip_atomic_load(a.ticket + 4, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
        __hip_atomic_fetch_or(&fd.counts->status, DAQ_STATUS_INCOMPLETE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // the counts, run table and chunk map go out as device-scope stores; each
    // wave waits until its stores are done before the tile is counted (no
    // cache write-back is needed for them)
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    lds_barrier();
    if (threadIdx.x == 0)
        __hip_atomic_fetch_add(a.tile_pref + f, (uint64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int NT, int R>
__global__ void __launch_bounds__(NT) k_pipe(KArgs a) {
    __shared__ __align__(16) uint8_t s_lds[PipeLds<NT>::kBytes];
    __shared__ uint32_t s_wsum[NT / 64];
    __shared__ uint64_t s_excl;
    __shared__ int64_t s_job;
    __shared__ ChunkInfo s_ci;
    __shared__ int64_t s_base[kLdsFills];
    const int nf = a.hdr ? a.hdr->n_fills : a.n_fills;
    const int64_t total = a.hdr ? a.hdr->total_tiles : a.total_tiles;
    const bool lds_fills = nf <= kLdsFills;
    if (lds_fills)
        for (int i = threadIdx.x; i < nf; i += NT) s_base[i] = tile_base_at(a, i);
    FillDev fd{};
    int cur = -1;
    int32_t thr_eff = 0;
    for (;;) {
        if (threadIdx.x == 0) s_job = pipe_next(a, nf, total, &s_ci);
        lds_barrier();
        const int64_t job = s_job;
        if (job == kJobExit) break;
        if (job >= 0) {
            if (cur < 0 || job < fd.tile_base || job >= fd.tile_base + fd.n_tiles) {
                int lo = 0, hi = nf - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if ((lds_fills ? s_base[mid] : tile_base_at(a, mid)) <= job) lo = mid;
                    else hi = mid - 1;
                }
                fd = fill_at(a, lo);
                thr_eff = clamp_thr(*gbl(a.thr_eff + lo));
                cur = lo;
            }
            pipe_tile<NT, R>(a, fd, cur, thr_eff, job, s_lds, s_wsum, &s_excl);
        } else {
            const uint64_t id = (uint64_t)(kJobCopy - job);
            const FillDev fc = fill_at(a, (int)(id >> 32));
            const ChunkInfo ci = s_ci;
            copy_chunk<NT, PipeCopyLayout, true>(fc, (int64_t)(uint32_t)id, ci, copy_view<PipeCopyLayout>(s_lds));
        }
        lds_barrier();
    }
}

// ---- Q-method: decimated calorimeter sum and fill-by-fill waveform sum -----------
//
// Section 3, Q-method paragraph; Table 2, decimation and fill-by-fill rows.
// Tiles of NT x 8 samples (no halo: nothing crosses a tile), grid-stride.
// Thread j takes samples p = t0 + 8 j .. p + 7 of every channel row: the raw
// 16-byte chunk is added to the thread's eight column sums and, when the
// fill has an accumulator, to the channel's eight accumulator words minus
// the channel pedestal (one 32-byte read-modify-write). The pedestal-
// subtracted column sums of four consecutive threads make one 32-sample bin.

template <int NT>
__global__ void __launch_bounds__(NT) k_q_pass(KArgs a) {
    static_assert((NT * kVec) % kQBin == 0 && kQBin % kVec == 0, "bins never cross a tile");
    constexpr int kGroupsPerBin = kQBin / kVec;
    __shared__ int64_t s_base[kLdsFills];
    const int nf = a.hdr ? a.hdr->n_fills : a.n_fills;
    const int64_t total = a.hdr ? a.hdr->total_tiles : a.total_tiles;
    const bool stream = stream_loads(a);
    const bool lds_fills = nf <= kLdsFills;
    if (lds_fills)
        for (int i = threadIdx.x; i < nf; i += NT) s_base[i] = tile_base_at(a, i);
    lds_barrier();
    const int tid = threadIdx.x;
    FillDev fd{};
    int cur = -1;
    int64_t ped_total = 0;
    for (int64_t tile = blockIdx.x; tile < total; tile += gridDim.x) {
        if (cur < 0 || tile < fd.tile_base || tile >= fd.tile_base + fd.n_tiles) {
            int lo = 0, hi = nf - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if ((lds_fills ? s_base[mid] : tile_base_at(a, mid)) <= tile) lo = mid;
                else hi = mid - 1;
            }
            fd = fill_at(a, lo);
            ped_total = *gbl(a.thr_eff + lo) - (int64_t)fd.thr;  // thr + sum of pedestals
            cur = lo;
        }
        const int64_t p = (tile - fd.tile_base) * fd.tout + (int64_t)tid * kVec;
        const int64_t valid = fd.n - p;  // samples of this thread's group inside the fill
        int64_t gsum = 0;
        if (valid > 0) {
            const int nv = valid < kVec ? (int)valid : kVec;
            int32_t s[kVec] = {0, 0, 0, 0, 0, 0, 0, 0};
            const int16_t *xr = fd.raw + p;
            int32_t *ar = fd.acc != nullptr ? fd.acc + p : nullptr;
            // one channel row: the sums, and the accumulator update with the
            // raw chunk v already loaded
            auto update = [&](int c, const uint4 v) {
                add8(s, v);
                if (ar == nullptr) return;
                const int32_t pc = *gbl(fd.ped + c);
                int32_t *row = ar + (int64_t)c * fd.acc_stride;
                const uint32_t w[4] = {v.x, v.y, v.z, v.w};
                uint32_t d[kVec];
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    d[2 * k] = (uint32_t)((int32_t)(int16_t)(w[k] & 0xFFFFu) - pc);
                    d[2 * k + 1] = (uint32_t)((int32_t)(int16_t)(w[k] >> 16) - pc);
                }
                if (nv == kVec) {
                    const u32x4 a0 = *(const DAQ_GLOBAL u32x4 *)row;
                    const u32x4 a1 = *(const DAQ_GLOBAL u32x4 *)(row + 4);
                    store16_i32(row, make_uint4(a0.x + d[0], a0.y + d[1], a0.z + d[2], a0.w + d[3]), stream);
                    store16_i32(row + 4, make_uint4(a1.x + d[4], a1.y + d[5], a1.z + d[6], a1.w + d[7]), stream);
                } else {
                    for (int k = 0; k < nv; k++) gbl(row)[k] = (int32_t)((uint32_t)gbl(row)[k] + d[k]);
                }
            };
            constexpr int R = 4;  // raw rows in flight
            int c = 0;
            for (; c + R <= fd.C; c += R) {
                uint4 v[R];
#pragma unroll
                for (int u = 0; u < R; u++) {
                    const int16_t *q = xr + (int64_t)(c + u) * fd.stride;
                    v[u] = stream ? load16_stream(q) : load16(q);
                }
#pragma unroll
                for (int u = 0; u < R; u++) update(c + u, v[u]);
            }
            for (; c < fd.C; c++) {
                const int16_t *q = xr + (int64_t)c * fd.stride;
                update(c, stream ? load16_stream(q) : load16(q));
            }
#pragma unroll
            for (int k = 0; k < kVec; k++) gsum += k < nv ? (int64_t)s[k] - ped_total : 0;
        }
        // one bin = kGroupsPerBin consecutive threads (within one wave)
#pragma unroll
        for (int d = 1; d < kGroupsPerBin; d <<= 1) gsum += __shfl_xor(gsum, d, 64);
        if (fd.qsum != nullptr && valid > 0 && (tid % kGroupsPerBin) == 0) *gbl(fd.qsum + p / kQBin) = gsum;
    }
}

// ---- 12-bit ingest ------------------------------------------------------------------
//
// Digitizer words, two 12-bit samples to three bytes (little-endian), into
// int16 rows. A work item is 8 samples of one row: 12 packed bytes (three
// aligned 32-bit words) in, one 16-byte store out; the last group of a row
// with fewer than 8 samples goes byte by byte.
__global__ void __launch_bounds__(256) k_unpack12(const uint8_t *in, int64_t in_stride, int32_t C, int64_t n,
                                                  int16_t *out, int64_t out_stride) {
    const int64_t groups = (n + kVec - 1) / kVec;
    const int64_t items = groups * C;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < items; i += (int64_t)gridDim.x * 256) {
        const int64_t c = i / groups;
        const int64_t g = i - c * groups;
        const uint8_t *row = in + c * in_stride;
        int16_t *orow = out + c * out_stride + g * kVec;
        const int64_t t0 = g * kVec;
        if (t0 + kVec <= n) {
            const uint32_t *w = reinterpret_cast<const uint32_t *>(row + 12 * g);
            const uint32_t w0 = *gbl(w), w1 = *gbl(w + 1), w2 = *gbl(w + 2);
            const uint32_t s0 = w0 & 0xFFFu, s1 = (w0 >> 12) & 0xFFFu, s2 = ((w0 >> 24) | (w1 << 8)) & 0xFFFu,
                           s3 = (w1 >> 4) & 0xFFFu, s4 = (w1 >> 16) & 0xFFFu,
                           s5 = ((w1 >> 28) | (w2 << 4)) & 0xFFFu, s6 = (w2 >> 8) & 0xFFFu,
                           s7 = (w2 >> 20) & 0xFFFu;
            u32x4 o;
            o.x = s0 | (s1 << 16);
            o.y = s2 | (s3 << 16);
            o.z = s4 | (s5 << 16);
            o.w = s6 | (s7 << 16);
            *(DAQ_GLOBAL u32x4 *)orow = o;
        } else {
            for (int64_t t = t0; t < n; t++) {
                const uint8_t *p = row + 3 * (t >> 1);
                const uint32_t v = (t & 1) ? ((uint32_t)*gbl(p + 1) >> 4) | ((uint32_t)*gbl(p + 2) << 4)
                                           : (uint32_t)*gbl(p) | (((uint32_t)*gbl(p + 1) & 0xFu) << 8);
                *gbl(orow + (t - t0)) = (int16_t)v;
            }
        }
    }
}

// Effective thresholds (thr + the sum of the pedestals), pedestals, cleared
// look-back words and counts, for the schedules whose scan does not compute
// pedestals itself. A block handles whole fills.
__global__ void __launch_bounds__(256) k_prepare(KArgs a) {
    __shared__ long long s_acc[kPedChannels];
    __shared__ long long s_ped;
    const int nf = a.hdr ? a.hdr->n_fills : a.n_fills;
    const int64_t total = a.hdr ? a.hdr->total_tiles : a.total_tiles;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256)
        a.tile_state[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x < 8) a.ticket[threadIdx.x] = 0;  // dispenser, copy cursor, flags
    for (int f = blockIdx.x; f < nf; f += gridDim.x) {
        const FillDev fd = fill_at(a, f);
        const int64_t ped_sum = fill_pedestals<256>(fd, true, s_acc, &s_ped);
        if (fd.qsum != nullptr)  // decimated sums built by atomic adds (fused Q-method)
            for (int64_t i = threadIdx.x; i < (fd.n + kQBin - 1) / kQBin; i += 256) fd.qsum[i] = 0;
        if (fd.mbits != nullptr && threadIdx.x < 2 * kMaskGuard) {
            const int64_t nbytes = fd.n_tiles * fd.tout / kVec;
            const int i = threadIdx.x;
            fd.mbits[i < kMaskGuard ? i - kMaskGuard : nbytes + (i - kMaskGuard)] = 0;
        }
        if (threadIdx.x == 0) {
            a.thr_eff[f] = (int64_t)fd.thr + ped_sum;
            if (a.tile_pref) a.tile_pref[f] = 0;  // finished tiles (pipe variant)
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

hipError_t launch_chop(const KArgs &a, int threads, int variant, int grid, hipStream_t s) {
#define DAQ_LAUNCH(NT_, V_) hipLaunchKernelGGL((k_chop<NT_, V_>), dim3(grid), dim3(NT_), 0, s, a)
#define DAQ_THREADS(V_)                      \
    do {                                     \
        if (threads == 128) DAQ_LAUNCH(128, V_); \
        else if (threads == 256) DAQ_LAUNCH(256, V_); \
        else if (threads == 512) DAQ_LAUNCH(512, V_); \
        else return hipErrorInvalidValue;    \
    } while (0)
    switch (variant) {
        case kVariantStream:
            if (threads != kStreamThreads) return hipErrorInvalidValue;
            DAQ_LAUNCH(256, kVariantStream);
            break;
        case kVariantReload: DAQ_THREADS(kVariantReload); break;
        case kVariantResident: DAQ_THREADS(kVariantResident); break;
        case kVariantReload18: DAQ_THREADS(kVariantReload18); break;
        case kVariantReload27: DAQ_THREADS(kVariantReload27); break;
        default: return hipErrorInvalidValue;
    }
#undef DAQ_THREADS
#undef DAQ_LAUNCH
    return hipGetLastError();
}

hipError_t launch_scan(const KArgs &a, int threads, int grid, hipStream_t s) {
    if (a.q_fused) {
        if (threads == 256) hipLaunchKernelGGL((k_scan_pass<256, DAQ_Q_SCAN_ROWS, true>), dim3(grid), dim3(256), 0, s, a);
        else if (threads == 512) hipLaunchKernelGGL((k_scan_pass<512, DAQ_Q_SCAN_ROWS, true>), dim3(grid), dim3(512), 0, s, a);
        else return hipErrorInvalidValue;
        return hipGetLastError();
    }
    // without the Q-method the scan computes the pedestals itself (no k_prepare)
    if (threads == 256) hipLaunchKernelGGL((k_scan_pass<256, DAQ_SCAN_ROWS, false, true>), dim3(grid), dim3(256), 0, s, a);
    else if (threads == 512) hipLaunchKernelGGL((k_scan_pass<512, DAQ_SCAN_ROWS, false, true>), dim3(grid), dim3(512), 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_emit(const KArgs &a, int threads, int edge_grid, int copy_grid, hipStream_t s) {
    // both passes stride over their work (tiles, copy items), so any grid of
    // at least one work-group covers the launch
    const int eg = edge_grid < 1 ? 1 : edge_grid;
    const int cg = copy_grid < 1 ? 1 : copy_grid;
    if (threads == 256) {
        hipLaunchKernelGGL((k_edge_pass<256>), dim3(eg), dim3(256), 0, s, a);
        hipLaunchKernelGGL((k_copy_pass<256>), dim3((int)cg), dim3(256), 0, s, a);
    } else if (threads == 512) {
        hipLaunchKernelGGL((k_edge_pass<512>), dim3(eg), dim3(512), 0, s, a);
        hipLaunchKernelGGL((k_copy_pass<512>), dim3((int)cg), dim3(512), 0, s, a);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pipe(const KArgs &a, int threads, int grid, hipStream_t s) {
    if (threads == 256) hipLaunchKernelGGL((k_pipe<256, DAQ_SCAN_ROWS>), dim3(grid), dim3(256), 0, s, a);
    else if (threads == 512) hipLaunchKernelGGL((k_pipe<512, DAQ_SCAN_ROWS>), dim3(grid), dim3(512), 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_q(const KArgs &a, int threads, int grid, hipStream_t s) {
    if (threads == 256) hipLaunchKernelGGL((k_q_pass<256>), dim3(grid), dim3(256), 0, s, a);
    else if (threads == 512) hipLaunchKernelGGL((k_q_pass<512>), dim3(grid), dim3(512), 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_unpack12(const uint8_t *in, int64_t in_stride, int32_t C, int64_t n, int16_t *out,
                           int64_t out_stride, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_unpack12, dim3(grid), dim3(256), 0, s, in, in_stride, C, n, out, out_stride);
    return hipGetLastError();
}

hipError_t launch_gather(const GatherArgs &g, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_gather, dim3(grid), dim3(256), 0, s, g);
    return hipGetLastError();
}

}  // namespace daqk
