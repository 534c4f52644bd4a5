// ceiling.hip -- the plain streaming-read rate of the device, the ceiling
// the summing scan of the chop is measured against (it reads every raw sample
// once and writes almost nothing).
//
// k_read_stream reads a buffer once with 16-byte non-temporal loads (eight
// in flight per thread, grid-stride), folds the words with XOR so the loads
// cannot be dropped, and leaves one word per wave in a sink.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "daq.h"

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
#define DAQ_GLOBAL __attribute__((address_space(1)))

__global__ void __launch_bounds__(256) k_read_stream(const u32x4 *p, int64_t n16, unsigned int *sink) {
    constexpr int K = 8;  // loads in flight per thread
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const DAQ_GLOBAL u32x4 *q = (const DAQ_GLOBAL u32x4 *)p;
    u32x4 x = {0, 0, 0, 0};
    for (; i + (K - 1) * stride < n16; i += K * stride) {
        u32x4 v[K];
#pragma unroll
        for (int k = 0; k < K; k++) v[k] = __builtin_nontemporal_load(q + i + k * stride);
#pragma unroll
        for (int k = 0; k < K; k++) x ^= v[k];
    }
    for (; i < n16; i += stride) x ^= __builtin_nontemporal_load(q + i);
    unsigned int v = x.x ^ x.y ^ x.z ^ x.w;
    for (int d = 32; d > 0; d >>= 1) v ^= __shfl_xor(v, d, 64);
    if ((threadIdx.x & 63) == 0) sink[(blockIdx.x * blockDim.x + threadIdx.x) >> 6] = v;
}

}  // namespace

extern "C" int daq_read_stream(const void *d_buf, int64_t bytes, unsigned int *d_sink, int32_t blocks,
                               void *stream) {
    if (!d_buf || !d_sink || bytes < 16 || blocks < 1 || ((uintptr_t)d_buf & 15u) != 0) return DAQ_EINVAL;
    hipLaunchKernelGGL(k_read_stream, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (const u32x4 *)d_buf,
                       bytes / 16, d_sink);
    return hipGetLastError() == hipSuccess ? DAQ_OK : DAQ_EHIP;
}
