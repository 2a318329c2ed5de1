// Device helpers shared by the signing kernels (the per-unit walk and the
// shared-sample binned form): the lattice map of a draw and the exact
// crossing tests of Alg. 1's point-in-polygon step.
#pragma once

#include "internal.hpp"

namespace polymh {

// Lattice offset of a 32-bit half-draw: floor(h * W / 2^32).
template <bool POW2>
__device__ __forceinline__ uint32_t lattice(uint32_t h, uint32_t w, int32_t sh)
{
    if constexpr (POW2)
        return h >> sh;
    else
        return w ? __umulhi(h, w) : h;
}

// Edge record staged in LDS, oriented upward: (x_lo, y_lo, y_hi, x_hi - x_lo).
__device__ __forceinline__ int4 make_edge(int32_t x0, int32_t y0, int32_t x1, int32_t y1)
{
    return (y0 <= y1) ? make_int4(x0, y0, y1, x1 - x0) : make_int4(x1, y1, y0, x0 - x1);
}

// Crossing of the ray from (px, py) to +x with an upward edge, exact in FP64
// (edge endpoints and the sample lie in an MBR with sides < 2^26).
__device__ __forceinline__ bool crosses_fp64(int4 e, int32_t px, int32_t py)
{
    const bool straddle = (e.y <= py) & (py < e.z);
    const double t = (double)(px - e.x) * (double)(e.z - e.y);
    const double o = __fma_rn((double)e.w, (double)(py - e.y), -t);
    return straddle & (o > 0.0);
}

__device__ __forceinline__ bool crosses_i128(const int32_t *v0, const int32_t *v1, int32_t px,
                                             int32_t py)
{
    int64_t xl = v0[0], yl = v0[1], xh = v1[0], yh = v1[1];
    if (yl > yh) {
        int64_t t = xl; xl = xh; xh = t;
        t = yl; yl = yh; yh = t;
    }
    if (!(yl <= py && py < yh)) return false;
    const __int128 o = (__int128)(xh - xl) * ((int64_t)py - yl) - (__int128)((int64_t)px - xl) * (yh - yl);
    return o > 0;
}

}  // namespace polymh
