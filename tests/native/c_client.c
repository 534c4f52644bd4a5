/* A plain C program that uses libdaqisland through include/daq.h only (HIP's
 * C runtime API for device memory, no C++ and no Python): one fill is chopped
 * with daq_chop_fill and its packed rows compressed with daq_compress_batch.
 *
 *   c_client IN OUT C N THRESHOLD PRE POST NP
 *
 * IN holds the fill as int16 [C][stride], stride = N rounded up to 8. OUT
 * receives, as little-endian binary: int64 n_islands, total_len, status;
 * int32 ped[C]; int64 islands[n_islands][3]; int16 packed[C][total_len];
 * int64 n_words; uint32 hdr[C * ceil(total_len / 64)]; uint32 words[n_words].
 * Exit status 0 on success, 2 on a usage or file error, 3 on a library or
 * runtime error (the code is printed). */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "daq.h"

#define CHECK_HIP(x)                                                        \
    do {                                                                    \
        hipError_t e_ = (x);                                                \
        if (e_ != hipSuccess) {                                             \
            fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));         \
            return 3;                                                       \
        }                                                                   \
    } while (0)
#define CHECK_DAQ(x)                                                        \
    do {                                                                    \
        int r_ = (x);                                                       \
        if (r_ != DAQ_OK) {                                                 \
            fprintf(stderr, "%s: %s (%d)\n", #x, daq_strerror(r_), r_);     \
            return 3;                                                       \
        }                                                                   \
    } while (0)

int main(int argc, char **argv) {
    if (argc != 9) {
        fprintf(stderr, "usage: c_client IN OUT C N THRESHOLD PRE POST NP\n");
        return 2;
    }
    const int32_t C = atoi(argv[3]);
    const int64_t N = atoll(argv[4]);
    const int64_t stride = (N + 7) / 8 * 8 > 8 ? (N + 7) / 8 * 8 : 8;
    const size_t raw_bytes = (size_t)C * (size_t)stride * sizeof(int16_t);
    int16_t *raw = (int16_t *)malloc(raw_bytes);
    FILE *in = fopen(argv[1], "rb");
    if (!raw || !in || fread(raw, 1, raw_bytes, in) != raw_bytes) {
        fprintf(stderr, "cannot read %s\n", argv[1]);
        return 2;
    }
    fclose(in);

    daq_ctx *ctx = NULL;
    CHECK_DAQ(daq_ctx_create(&ctx, 0));
    const int64_t cap = daq_max_islands(N, atoi(argv[6]), atoi(argv[7]));
    void *d_raw = NULL, *d_isl = NULL, *d_counts = NULL, *d_ped = NULL, *d_out = NULL;
    CHECK_HIP(hipMalloc(&d_raw, raw_bytes));
    CHECK_HIP(hipMalloc(&d_isl, (size_t)(cap > 0 ? cap : 1) * sizeof(daq_island)));
    CHECK_HIP(hipMalloc(&d_counts, sizeof(daq_counts)));
    CHECK_HIP(hipMalloc(&d_ped, (size_t)C * sizeof(int32_t)));
    CHECK_HIP(hipMalloc(&d_out, raw_bytes));
    CHECK_HIP(hipMemcpy(d_raw, raw, raw_bytes, hipMemcpyHostToDevice));

    daq_fill f = {(const int16_t *)d_raw, N, stride, C, atoi(argv[8]), atoi(argv[5]), atoi(argv[6]),
                  atoi(argv[7]), 0};
    daq_fill_out o = {(daq_island *)d_isl, cap, (daq_counts *)d_counts, (int32_t *)d_ped, (int16_t *)d_out,
                      stride};
    CHECK_DAQ(daq_chop_fill(ctx, &f, &o, NULL));

    /* compression of the packed rows, queued behind the chop on the same stream */
    const int64_t nb_max = C * ((stride + DAQ_Z_BLOCK - 1) / DAQ_Z_BLOCK);
    void *d_hdr = NULL, *d_words = NULL, *d_nw = NULL;
    CHECK_HIP(hipMalloc(&d_hdr, (size_t)nb_max * sizeof(uint32_t)));
    CHECK_HIP(hipMalloc(&d_words, (size_t)nb_max * 34 * sizeof(uint32_t)));
    CHECK_HIP(hipMalloc(&d_nw, sizeof(int64_t)));
    daq_z_fill z = {(const int16_t *)d_out, stride, (const daq_counts *)d_counts, stride, (uint32_t *)d_hdr, NULL,
                    (uint32_t *)d_words, nb_max * 34, (int64_t *)d_nw, C, 0};
    CHECK_DAQ(daq_compress_batch(ctx, &z, 1, NULL));
    CHECK_HIP(hipDeviceSynchronize());

    daq_counts cnt;
    CHECK_HIP(hipMemcpy(&cnt, d_counts, sizeof(cnt), hipMemcpyDeviceToHost));
    const int64_t n = cnt.n_islands < cap ? cnt.n_islands : cap;
    const int64_t L = cnt.total_len;
    int64_t n_words = 0;
    CHECK_HIP(hipMemcpy(&n_words, d_nw, sizeof(n_words), hipMemcpyDeviceToHost));
    const int64_t nb = C * ((L + DAQ_Z_BLOCK - 1) / DAQ_Z_BLOCK);
    int32_t *ped = (int32_t *)malloc((size_t)C * sizeof(int32_t));
    daq_island *isl = (daq_island *)malloc((size_t)(n > 0 ? n : 1) * sizeof(daq_island));
    int16_t *out = (int16_t *)malloc(raw_bytes);
    uint32_t *hdr = (uint32_t *)malloc((size_t)(nb > 0 ? nb : 1) * sizeof(uint32_t));
    uint32_t *words = (uint32_t *)malloc((size_t)(n_words > 0 ? n_words : 1) * sizeof(uint32_t));
    if (!ped || !isl || !out || !hdr || !words || n_words < 0 || n_words > nb_max * 34) {
        fprintf(stderr, "bad sizes (n_words %lld)\n", (long long)n_words);
        return 3;
    }
    CHECK_HIP(hipMemcpy(ped, d_ped, (size_t)C * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (n > 0) CHECK_HIP(hipMemcpy(isl, d_isl, (size_t)n * sizeof(daq_island), hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(out, d_out, raw_bytes, hipMemcpyDeviceToHost));
    if (nb > 0) CHECK_HIP(hipMemcpy(hdr, d_hdr, (size_t)nb * sizeof(uint32_t), hipMemcpyDeviceToHost));
    if (n_words > 0)
        CHECK_HIP(hipMemcpy(words, d_words, (size_t)n_words * sizeof(uint32_t), hipMemcpyDeviceToHost));

    FILE *fo = fopen(argv[2], "wb");
    if (!fo) return 2;
    const int64_t head[3] = {cnt.n_islands, cnt.total_len, (int64_t)cnt.status};
    fwrite(head, sizeof(int64_t), 3, fo);
    fwrite(ped, sizeof(int32_t), (size_t)C, fo);
    for (int64_t i = 0; i < n; i++) {
        const int64_t r[3] = {isl[i].start, isl[i].stop, isl[i].offset};
        fwrite(r, sizeof(int64_t), 3, fo);
    }
    for (int32_t c = 0; c < C; c++) fwrite(out + (size_t)c * (size_t)stride, sizeof(int16_t), (size_t)L, fo);
    fwrite(&n_words, sizeof(int64_t), 1, fo);
    fwrite(hdr, sizeof(uint32_t), (size_t)nb, fo);
    fwrite(words, sizeof(uint32_t), (size_t)n_words, fo);
    fclose(fo);

    hipFree(d_raw);
    hipFree(d_isl);
    hipFree(d_counts);
    hipFree(d_ped);
    hipFree(d_out);
    hipFree(d_hdr);
    hipFree(d_words);
    hipFree(d_nw);
    daq_ctx_destroy(ctx);
    free(raw);
    free(ped);
    free(isl);
    free(out);
    free(hdr);
    free(words);
    return 0;
}
