// chop_internal.h -- structures shared by the host runtime and the kernels of
// libdaqisland (not part of the public ABI; see include/daq.h for that).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "daq.h"

namespace daqk {

// Samples per thread: one 16-byte load per channel row.
constexpr int kVec = 8;
// Halo groups on one side for the largest window (post + 1 or pre + 1).
constexpr int kMaxHaloGroups = (DAQ_MAX_WINDOW + 1 + kVec - 1) / kVec;
// Channel count of one calorimeter (a 6 x 9 crystal grid, Section 3): the
// count for which the fused kernel can keep a whole tile in registers or LDS.
constexpr int kResidentChannels = 54;
// Kernel variants (daq_schedule.variant).
constexpr int kVariantReload = 0;    // rows read into registers, read again to write out
constexpr int kVariantResident = 1;  // rows kept in registers until written out
constexpr int kVariantStream = 2;    // rows DMA'd into LDS; two work-groups per CU
constexpr int kVariantReload18 = 3;  // as kVariantReload, 18 rows in flight per round (6 there)
constexpr int kVariantReload27 = 4;  // as kVariantReload, 27 rows in flight per round
constexpr int kVariantSplit = 5;     // scan pass (mask bits, tile totals), edge and copy passes
constexpr int kVariantPipe = 6;      // one persistent kernel: scan tiles and copy chunks from shared counters
constexpr int kVariantLast = 6;
// Guard bytes around each fill's island-mask bits (read as zero past the ends).
constexpr int kMaskGuard = 16;
// Packed positions per chunk of a row: the copy pass writes one chunk of a
// channel group per wave (one 16-byte word per lane), and the edge pass
// records the island holding every multiple of it.
#ifndef DAQ_COPY_CHUNK
#define DAQ_COPY_CHUNK 512
#endif
constexpr int kCopyChunk = DAQ_COPY_CHUNK;
// Tile of the LDS variant: groups of 8 samples per row buffer, work-group size.
constexpr int kStreamGroups = 80;
constexpr int kStreamThreads = 256;
// Per-fill tile modes.
constexpr int kModeChop = 0;
constexpr int kModeStream = 1;

// Device-side view of one fill and where its results go.
struct FillDev {
    const int16_t *raw;
    int64_t n;          // samples
    int64_t stride;     // elements between channel rows
    int32_t C;
    int32_t np;         // pedestal samples
    int32_t thr;
    int32_t pre;
    int32_t post;
    int32_t gl;         // halo groups of 8 samples left of a tile: ceil((post + 1) / 8)
    int32_t gr;         // halo groups right of a tile: ceil((pre + 1) / 8)
    int32_t wide;       // 0: halo groups are ordinary thread groups of the tile;
                        // 1: extra groups loaded by a separate loop (wide windows)
    int32_t mode;       // kModeChop or kModeStream
    int32_t pad1;
    int64_t tout;       // samples a tile owns (decides and writes)
    int64_t tile_base;  // global index of the fill's first tile in the launch
    int64_t n_tiles;
    daq_island *isl;
    int64_t cap;
    daq_counts *counts;
    int32_t *ped;       // may be null
    int16_t *out;       // may be null (find only)
    int64_t out_stride;
    uint8_t *mbits;     // split variant: island-mask bits of the fill (bit t of
                        // byte t / 8), kMaskGuard zero bytes on either side
    int32_t *runs;      // split variant: (start, offset) of every island
                        // (room for the worst-case island count)
    int32_t *cmap;      // split variant: island holding packed position
                        // k * kCopyChunk, for every such position < total_len
    int64_t *qsum;      // Q-method: decimated sums, or null
    int32_t *acc;       // Q-method: fill-by-fill accumulator rows, or null
    int64_t acc_stride;
    int64_t pad2;
};
static_assert(sizeof(FillDev) % 16 == 0, "descriptors are read as 16-byte words");

// Per-launch sizes kept in device memory so that a captured graph can be
// replayed for any batch that fits the scratch it was captured with.
struct BatchHdr {
    int32_t n_fills;
    int32_t stream_loads;  // 1: the scan reads raw rows non-temporally (batches larger than the caches)
    int64_t total_tiles;
    int64_t copy_slots;  // split variant: n_fills x chunks of the longest fill
    int64_t pad2;
};
static_assert(sizeof(BatchHdr) % 16 == 0, "the descriptor table follows the header in one buffer");

struct KArgs {
    const FillDev *table;  // device table of n_fills entries, or null: use `one`
    const BatchHdr *hdr;   // device header, or null: use the three fields below
    int32_t n_fills;
    int32_t stream_loads;
    int64_t total_tiles;
    uint64_t *tile_state;  // one look-back word per tile (split variant: tile totals)
    uint32_t *ticket;      // 16 words: tile dispenser; pipe variant: copy cursor, give-up flag
    int64_t *thr_eff;      // per fill: threshold + sum of pedestals
    uint64_t *tile_pref;   // split variant: exclusive prefix of each tile; pipe variant:
                           // finished tiles of each fill (one word per fill)
    int64_t copy_slots;    // split variant, when hdr is null
    int32_t part, parts;   // split variant: this launch covers fill group `part`
                           // of `parts` equal groups of the batch
    int32_t q_fused;       // split variant: the scan pass also runs the Q-method
    int32_t pad_q;
    FillDev one;
};

struct GatherArgs {
    const int16_t *raw;
    int64_t stride;
    int32_t C;
    int32_t pad;
    const daq_island *isl;
    int64_t cap;
    daq_counts *counts;
    int16_t *out;
    int64_t out_stride;
};

// Tile geometry of one fill: halo groups, mode and the samples each tile
// owns. Halos up to a quarter of the tile's groups are ordinary groups of the
// tile; wider ones are loaded apart. The LDS variant takes 54-channel fills
// with such halos; every other fill uses the register path.
struct TileShape {
    int32_t gl, gr, wide, mode;
    int64_t tout;
};
inline TileShape tile_shape(int32_t pre, int32_t post, int32_t channels, int threads, int variant) {
    TileShape t;
    t.gl = (post + 1 + kVec - 1) / kVec;
    t.gr = (pre + 1 + kVec - 1) / kVec;
    if (variant == kVariantStream && channels == kResidentChannels && (t.gl + t.gr) * 4 <= kStreamGroups) {
        t.mode = kModeStream;
        t.wide = 0;
        t.tout = (int64_t)(kStreamGroups - t.gl - t.gr) * kVec;
        return t;
    }
    t.mode = kModeChop;
    t.wide = (t.gl + t.gr) * 4 > threads ? 1 : 0;
    t.tout = (int64_t)(t.wide ? threads : threads - t.gl - t.gr) * kVec;
    return t;
}

hipError_t launch_prepare(const KArgs &a, int blocks, hipStream_t s);
hipError_t launch_chop(const KArgs &a, int threads, int variant, int grid, hipStream_t s);
// Split variant: the scan pass, then the edge and copy passes, over the fill
// group a.part of a.parts.
hipError_t launch_scan(const KArgs &a, int threads, int grid, hipStream_t s);
hipError_t launch_emit(const KArgs &a, int threads, int edge_grid, int copy_grid, hipStream_t s);
// Work-groups per CU of the copy pass's persistent grid.
#ifndef DAQ_COPY_WGS_PER_CU
#define DAQ_COPY_WGS_PER_CU 4
#endif
constexpr int kCopyWgsPerCu = DAQ_COPY_WGS_PER_CU;
hipError_t launch_pipe(const KArgs &a, int threads, int grid, hipStream_t s);
hipError_t launch_q(const KArgs &a, int threads, int grid, hipStream_t s);
hipError_t launch_unpack12(const uint8_t *in, int64_t in_stride, int32_t C, int64_t n, int16_t *out,
                           int64_t out_stride, int grid, hipStream_t s);
// Most fill groups a split launch is cut into (one HIP stream each).
#ifndef DAQ_MAX_PARTS
#define DAQ_MAX_PARTS 4
#endif
constexpr int kMaxParts = DAQ_MAX_PARTS;
hipError_t launch_gather(const GatherArgs &g, int grid, hipStream_t s);

// Island compression: one fill's packed rows and where its stream goes.
struct ZFillDev {
    const int16_t *packed;
    int64_t stride;            // elements between packed rows
    const daq_counts *counts;  // total_len: samples per row to compress
    int64_t max_len;           // rows hold at most this many samples
    uint32_t *hdr;             // C * ceil(L / 64) block headers
    int64_t *offsets;          // C * ceil(L / 64) payload word offsets, or null
    int64_t *gofs;             // scratch: payload words of each wave of the grid
    uint32_t *words;
    int64_t cap;               // words that fit
    int64_t *n_words;          // payload words of the whole stream
    int32_t C;
    int32_t pad;
};
// Fills per launch (the descriptors travel as kernel arguments), waves per
// work-group, work-groups per fill (each wave of the pack pass sums the
// payload sizes of the waves before it: at most kZMaxGrid * kZWaves).
constexpr int kZMaxFills = 16;
constexpr int kZWaves = 4;
#ifndef DAQ_Z_MAX_GRID
#define DAQ_Z_MAX_GRID 256
#endif
constexpr int kZMaxGrid = DAQ_Z_MAX_GRID;
struct ZArgs {
    ZFillDev f[kZMaxFills];
    int32_t n;
};
hipError_t launch_z(const ZArgs &a, int grid, hipStream_t s);

// Decompression: one stream back into packed rows.
struct ZStreamDev {
    const uint32_t *hdr;
    const int64_t *offsets;
    const uint32_t *words;
    int64_t n_words;
    int16_t *out;
    int64_t out_stride;
    int64_t L;
    int32_t C;
    int32_t pad;
};
struct ZDecArgs {
    ZStreamDev f[kZMaxFills];
    int32_t n;
};
hipError_t launch_unz(const ZDecArgs &a, int grid, hipStream_t s);

}  // namespace daqk
