// LSH band keys over MinHash signatures (Sec. 3.2's hashmap of codes, in the
// banded form of the MMDS technique the paper cites).  One thread per
// (polygon, band): r chained SplitMix64 mixes of the band's rows.
#include "internal.hpp"

namespace polymh {

namespace {

__global__ __launch_bounds__(256) void k_band(const uint32_t *__restrict__ sig, int64_t n, int32_t k,
                                              int32_t b, int32_t r, uint64_t band_seed,
                                              uint64_t *__restrict__ keys)
{
    const int64_t total = n * b;
    for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < total;
         id += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = id / b;
        const int32_t t = (int32_t)(id - p * b);
        const uint32_t *row = sig + p * k + (int64_t)t * r;
        uint64_t f = mix64(band_seed + (uint64_t)(t + 1) * kGamma);
        for (int32_t u = 0; u < r; u++) f = mix64(f ^ (uint64_t)row[u]);
        keys[id] = f;
    }
}

}  // namespace

polymh_status launch_band(const uint32_t *sig, int64_t n, int32_t k, int32_t b, int32_t r,
                          uint64_t band_seed, uint64_t *keys, hipStream_t s)
{
    const int64_t total = n * b;
    if (total == 0) return POLYMH_OK;
    int64_t g = (total + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_band, dim3((unsigned)g), dim3(256), 0, s, sig, n, k, b, r, band_seed, keys);
    return check_launch("band");
}

}  // namespace polymh
