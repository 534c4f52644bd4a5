/*
 * chop_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded CPU statement of T-method island chopping
 * for one calorimeter fill, written from the paper (Gohn, "Data Acquisition
 * with GPUs: The DAQ for the Muon g-2 Experiment at Fermilab", ICHEP 2016):
 * Section 3 (the T-method paragraph) and Table 2 ("CUDA kernel routines used
 * to process each muon fill").
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library. The product (the HIP library) never calls it and
 * shares no code with it: no header, helper, table or constant.
 *
 * Every quantity is an integer; nothing here is approximate. Each step is the
 * plain definition, in the order Table 2 and the T-method paragraph give:
 *
 *   1. pedestal of channel c  = mean of its first Np samples (Table 2,
 *      pedestal row: Np = 100 there), rounded half up to an integer;
 *   2. calorimeter sum S[t]   = sum over channels of x[c][t] minus the sum of
 *      the channel pedestals (Table 2, waveform-sum row);
 *   3. threshold flag F[t]    = S[t] < thr, one flag per time sample
 *      (Table 2, threshold row; Section 3, T-method paragraph: one thread
 *      per sample);
 *   4. dilation               = every flagged sample t marks the window
 *      [t-pre, t+post] clipped to the fill (Table 2, pre/post-sample row);
 *   5. merging and the island array = every maximal run of marked samples is
 *      one island, so windows that overlap or touch become one island
 *      (Table 2, merge-check and island-array rows);
 *   6. chopped islands        = each island's raw samples of every channel,
 *      packed back to back (Section 3, description of the GPU thread).
 *
 * Readings where the paper is silent (all listed in the design notes):
 *   - integer pedestal: round half up of the exact mean, i.e.
 *     floor((2 P + n) / (2 n)) with n = min(Np, N); ped = 0 when N = 0;
 *   - a sample crosses the threshold when S < thr (strict);
 *   - level, not edge: every flagged sample is dilated;
 *   - windows are clipped at 0 and N-1, never dropped;
 *   - abutting windows merge (a union of marks);
 *   - island records are (start, stop, offset), stop exclusive, offset = sum
 *     of the lengths of the earlier islands, islands in increasing start;
 *   - gathered samples are the raw int16 values, not pedestal-subtracted.
 *
 * The Q-method (Section 3, Q-method paragraph; Table 2, the decimation and
 * fill-by-fill rows) integrates instead of chopping:
 *
 *   7. decimated sum Q[b]     = the pedestal-subtracted calorimeter sum S[t]
 *      summed over consecutive blocks of D samples, b = t / D (Table 2,
 *      decimation row: 17.5k threads for 560k samples, so D = 32); the last
 *      block holds the N mod D leftover samples when D does not divide N;
 *   8. fill-by-fill sum       = every channel's pedestal-subtracted waveform
 *      added sample by sample to a per-channel accumulator that persists
 *      across fills (Table 2, fill-by-fill row: 54 x 560k threads).
 *
 * Readings where the paper is silent: the pedestals are those of step 1; the
 * accumulator is int32 and wraps modulo 2^32 (exact while fewer than 2^31 /
 * 65535 = 32768 fills of arbitrary int16 data, or 524288 fills of 12-bit
 * data, have been added).
 *
 * Ingest (Section 3: 12-bit 800 MSPS digitizers, whose words the frontend
 * unpacks before the GPU thread copies a fill in): a channel row of N 12-bit
 * samples is packed two samples to three bytes, little-endian: for samples
 * a = x[2k], b = x[2k + 1], byte 3k = a & 0xFF, byte 3k + 1 = (a >> 8) |
 * (b & 0xF) << 4, byte 3k + 2 = b >> 4; an odd last sample leaves the high
 * nibble of its second byte zero and has no third byte. Unpacked samples are
 * the 12-bit values as int16 (0 .. 4095).
 *
 * Compression of the chopped islands (Section 3: the frontend's MFE thread
 * compresses the data losslessly before the event builder; the algorithm is
 * not named, this one is the reading taken): each channel's packed row of L
 * samples is cut into blocks of 64 (the last may be shorter); block b (rows
 * in order, blocks of a row in order) keeps its first sample and the
 * zigzag-coded differences z = (r << 1) ^ (r >> 31) of consecutive samples,
 * r = v[i] - v[i-1], each in w bits, w the bit length of the block's largest
 * z (0 when all are 0). Header word b = (uint16) first | w << 16; the
 * differences of block b are a little-endian bit stream (z_i at bits
 * (i-1) w .. i w - 1) in ceil((n - 1) w / 32) 32-bit words, the blocks'
 * words back to back.
 *
 * Layout: x is channel-major, x[c * stride + t], 0 <= t < N.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Mathematical floor of a / b for b > 0 (C division truncates toward 0). */
static int64_t floor_div(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b) != 0 && (a < 0))
        q -= 1;
    return q;
}

/* Step 1, Table 2 pedestal row: per-channel pedestal, the mean of the first
 * min(Np, N) samples rounded half up. */
void orc_pedestals(const int16_t *x, int32_t C, int64_t N, int64_t stride,
                   int32_t Np, int32_t *ped)
{
    int64_t n = (N < (int64_t)Np) ? N : (int64_t)Np;
    for (int32_t c = 0; c < C; c++) {
        if (n <= 0) {
            ped[c] = 0;
            continue;
        }
        int64_t P = 0;
        for (int64_t t = 0; t < n; t++)
            P += x[(int64_t)c * stride + t];
        ped[c] = (int32_t)floor_div(2 * P + n, 2 * n);
    }
}

/* Step 2, Table 2 waveform-sum row: pedestal-subtracted calorimeter sum for
 * every time sample. */
void orc_calo_sum(const int16_t *x, int32_t C, int64_t N, int64_t stride,
                  const int32_t *ped, int64_t *S)
{
    int64_t ped_total = 0;
    for (int32_t c = 0; c < C; c++)
        ped_total += ped[c];
    for (int64_t t = 0; t < N; t++) {
        int64_t s = 0;
        for (int32_t c = 0; c < C; c++)
            s += x[(int64_t)c * stride + t];
        S[t] = s - ped_total;
    }
}

/* Step 3, Table 2 threshold row: one threshold flag per time sample. */
void orc_threshold(const int64_t *S, int64_t N, int32_t thr, uint8_t *F)
{
    for (int64_t t = 0; t < N; t++)
        F[t] = (S[t] < (int64_t)thr) ? 1 : 0;
}

/* Step 4, Table 2 pre/post-sample row: every flagged sample marks pre samples
 * before it and post samples after it, clipped to the fill. */
void orc_dilate(const uint8_t *F, int64_t N, int32_t pre, int32_t post,
                uint8_t *M)
{
    memset(M, 0, (size_t)N);
    for (int64_t t = 0; t < N; t++) {
        if (!F[t])
            continue;
        int64_t lo = t - pre;
        int64_t hi = t + post;
        if (lo < 0)
            lo = 0;
        if (hi > N - 1)
            hi = N - 1;
        for (int64_t u = lo; u <= hi; u++)
            M[u] = 1;
    }
}

/* Step 5, Table 2 merge-check and island-array rows: maximal runs of marked
 * samples are the islands (so overlapping or touching windows are one
 * island), saved in increasing start with their offsets in the packed
 * output.
 * islands[3*i + 0] = start, [3*i + 1] = stop (exclusive), [3*i + 2] = offset.
 * Records past cap are counted but not stored. Returns the island count. */
int64_t orc_islands(const uint8_t *M, int64_t N, int64_t *islands,
                    int64_t cap, int64_t *total_len)
{
    int64_t n = 0;
    int64_t offset = 0;
    int64_t t = 0;
    while (t < N) {
        if (!M[t]) {
            t++;
            continue;
        }
        int64_t start = t;
        while (t < N && M[t])
            t++;
        if (n < cap) {
            islands[3 * n + 0] = start;
            islands[3 * n + 1] = t;
            islands[3 * n + 2] = offset;
        }
        offset += t - start;
        n++;
    }
    *total_len = offset;
    return n;
}

/* Step 6, Section 3 (GPU thread): every channel's raw samples of every
 * island, packed at the island's offset. */
void orc_gather(const int16_t *x, int32_t C, int64_t stride,
                const int64_t *islands, int64_t n, int16_t *out,
                int64_t out_stride)
{
    for (int64_t i = 0; i < n; i++) {
        int64_t start = islands[3 * i + 0];
        int64_t stop = islands[3 * i + 1];
        int64_t offset = islands[3 * i + 2];
        for (int32_t c = 0; c < C; c++)
            for (int64_t k = 0; k < stop - start; k++)
                out[(int64_t)c * out_stride + offset + k] =
                    x[(int64_t)c * stride + start + k];
    }
}

/* Steps 1-6 in order for one fill. out may be NULL (no gather); otherwise it
 * must hold C rows of out_stride >= total_len elements. Returns the island
 * count, or -1 when scratch memory cannot be allocated. */
int64_t orc_chop(const int16_t *x, int32_t C, int64_t N, int64_t stride,
                 int32_t Np, int32_t thr, int32_t pre, int32_t post,
                 int32_t *ped, int64_t *islands, int64_t cap,
                 int64_t *total_len, int16_t *out, int64_t out_stride)
{
    size_t n = (size_t)(N > 0 ? N : 1);
    int64_t *S = (int64_t *)malloc(n * sizeof(int64_t));
    uint8_t *F = (uint8_t *)malloc(n);
    uint8_t *M = (uint8_t *)malloc(n);
    if (!S || !F || !M) {
        free(S);
        free(F);
        free(M);
        return -1;
    }
    orc_pedestals(x, C, N, stride, Np, ped);
    orc_calo_sum(x, C, N, stride, ped, S);
    orc_threshold(S, N, thr, F);
    orc_dilate(F, N, pre, post, M);
    int64_t count = orc_islands(M, N, islands, cap, total_len);
    if (out != NULL)
        orc_gather(x, C, stride, islands, count < cap ? count : cap, out,
                   out_stride);
    free(S);
    free(F);
    free(M);
    return count;
}

/* Step 7, Table 2 decimation row: block sums of the calorimeter sum over D
 * samples; Q must hold ceil(N / D) values. */
void orc_q_decimate(const int64_t *S, int64_t N, int32_t D, int64_t *Q)
{
    int64_t nb = (N + D - 1) / D;
    for (int64_t b = 0; b < nb; b++)
        Q[b] = 0;
    for (int64_t t = 0; t < N; t++)
        Q[t / D] += S[t];
}

/* Step 8, Table 2 fill-by-fill row: acc[c][t] += x[c][t] - ped[c] for every
 * channel and sample of the fill, in int32 arithmetic modulo 2^32. */
void orc_q_accumulate(const int16_t *x, int32_t C, int64_t N, int64_t stride,
                      const int32_t *ped, int32_t *acc, int64_t acc_stride)
{
    for (int32_t c = 0; c < C; c++) {
        for (int64_t t = 0; t < N; t++) {
            int64_t v = (int64_t)x[(int64_t)c * stride + t] - ped[c];
            uint32_t a = (uint32_t)acc[(int64_t)c * acc_stride + t];
            acc[(int64_t)c * acc_stride + t] = (int32_t)(a + (uint32_t)v);
        }
    }
}

/* Steps 1, 2, 7 and 8 in order for one fill. Q (ceil(N / D) values) and acc
 * may each be NULL. Returns 0, or -1 when scratch memory cannot be
 * allocated. */
int orc_qmethod(const int16_t *x, int32_t C, int64_t N, int64_t stride,
                int32_t Np, int32_t D, int32_t *ped, int64_t *Q, int32_t *acc,
                int64_t acc_stride)
{
    orc_pedestals(x, C, N, stride, Np, ped);
    if (Q != NULL) {
        int64_t *S = (int64_t *)malloc((size_t)(N > 0 ? N : 1) * sizeof(int64_t));
        if (!S)
            return -1;
        orc_calo_sum(x, C, N, stride, ped, S);
        orc_q_decimate(S, N, D, Q);
        free(S);
    }
    if (acc != NULL)
        orc_q_accumulate(x, C, N, stride, ped, acc, acc_stride);
    return 0;
}

/* Ingest: one channel row of n samples unpacked from its 12-bit packing
 * (ceil(3 n / 2) bytes). */
void orc_unpack12_row(const uint8_t *in, int64_t n, int16_t *out)
{
    for (int64_t t = 0; t < n; t++) {
        int64_t k = t / 2;
        const uint8_t *p = in + 3 * k;
        if (t % 2 == 0)
            out[t] = (int16_t)(p[0] | ((p[1] & 0x0F) << 8));
        else
            out[t] = (int16_t)((p[1] >> 4) | (p[2] << 4));
    }
}

/* Ingest for a fill: C rows, in_stride bytes apart, into rows of out_stride
 * elements. */
void orc_unpack12(const uint8_t *in, int64_t in_stride, int32_t C, int64_t n,
                  int16_t *out, int64_t out_stride)
{
    for (int32_t c = 0; c < C; c++)
        orc_unpack12_row(in + (int64_t)c * in_stride, n, out + (int64_t)c * out_stride);
}

/* Compression: block headers and payload words of C rows of L samples.
 * Returns the number of payload words; words beyond cap are not written. */
int64_t orc_z_compress(const int16_t *x, int32_t C, int64_t L, int64_t stride,
                       uint32_t *hdr, uint32_t *words, int64_t cap)
{
    const int64_t B = 64;
    int64_t nb = (L + B - 1) / B;
    int64_t pos = 0;                      /* word offset of the next block */
    for (int32_t c = 0; c < C; c++) {
        const int16_t *row = x + (int64_t)c * stride;
        for (int64_t k = 0; k < nb; k++) {
            int64_t t0 = k * B;
            int64_t n = (L - t0 < B) ? L - t0 : B;
            uint32_t zmax = 0;
            for (int64_t i = 1; i < n; i++) {
                int32_t r = (int32_t)row[t0 + i] - (int32_t)row[t0 + i - 1];
                uint32_t z = ((uint32_t)r << 1) ^ (uint32_t)(r >> 31);
                if (z > zmax)
                    zmax = z;
            }
            uint32_t w = 0;
            while (w < 32 && (zmax >> w) != 0)
                w++;
            hdr[(int64_t)c * nb + k] = (uint32_t)(uint16_t)row[t0] | (w << 16);
            int64_t nw = ((n - 1) * (int64_t)w + 31) / 32;
            for (int64_t j = 0; j < nw; j++)
                if (pos + j < cap)
                    words[pos + j] = 0;
            for (int64_t i = 1; i < n; i++) {
                int32_t r = (int32_t)row[t0 + i] - (int32_t)row[t0 + i - 1];
                uint32_t z = ((uint32_t)r << 1) ^ (uint32_t)(r >> 31);
                for (uint32_t bit = 0; bit < w; bit++) {
                    int64_t at = (i - 1) * (int64_t)w + bit;
                    int64_t wi = pos + at / 32;
                    if (((z >> bit) & 1u) && wi < cap)
                        words[wi] |= 1u << (at % 32);
                }
            }
            pos += nw;
        }
    }
    return pos;
}

/* Decompression of orc_z_compress's output into C rows of L samples. */
void orc_z_decompress(const uint32_t *hdr, const uint32_t *words, int32_t C,
                      int64_t L, int16_t *out, int64_t stride)
{
    const int64_t B = 64;
    int64_t nb = (L + B - 1) / B;
    int64_t pos = 0;
    for (int32_t c = 0; c < C; c++) {
        int16_t *row = out + (int64_t)c * stride;
        for (int64_t k = 0; k < nb; k++) {
            int64_t t0 = k * B;
            int64_t n = (L - t0 < B) ? L - t0 : B;
            uint32_t h = hdr[(int64_t)c * nb + k];
            uint32_t w = h >> 16;
            int32_t v = (int16_t)(h & 0xFFFFu);
            row[t0] = (int16_t)v;
            for (int64_t i = 1; i < n; i++) {
                uint32_t z = 0;
                for (uint32_t bit = 0; bit < w; bit++) {
                    int64_t at = (i - 1) * (int64_t)w + bit;
                    z |= ((words[pos + at / 32] >> (at % 32)) & 1u) << bit;
                }
                int32_t r = (int32_t)(z >> 1) ^ -(int32_t)(z & 1u);
                v += r;
                row[t0 + i] = (int16_t)v;
            }
            pos += ((n - 1) * (int64_t)w + 31) / 32;
        }
    }
}
