// Polygon staging (Sec. 3.1 global MBR, Alg. 1 local MBR), the sampling box
// of a polygon set, and the longest-expected-first order used by the
// persistent signing launch (expected walk length from Thm. 2).
#include "internal.hpp"

#include <cmath>

namespace polymh {

namespace {

__device__ __forceinline__ int32_t wave_min(int32_t v)
{
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int32_t wave_max(int32_t v)
{
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v)
{
    for (int o = 32; o > 0; o >>= 1) {
        uint32_t lo = __shfl_xor((uint32_t)v, o, 64);
        uint32_t hi = __shfl_xor((uint32_t)(v >> 32), o, 64);
        v += ((uint64_t)hi << 32) | lo;
    }
    return v;
}

// One wavefront per polygon: MBR by min/max reduction; twice the signed area
// as the shoelace sum of fan terms (v - v0) x (v' - v0), each exact in 128
// bits and summed modulo 2^64 (exact whenever |area2| < 2^63); collinear iff
// every fan term is zero.
__global__ __launch_bounds__(256) void k_prepare(const int32_t *__restrict__ xy,
                                                 const int64_t *__restrict__ off, int64_t n,
                                                 int32_t *__restrict__ mbr,
                                                 int64_t *__restrict__ area2,
                                                 uint32_t *__restrict__ flags)
{
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t p = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; p < n; p += nwaves) {
        const int64_t a = off[p], b = off[p + 1], m = b - a;
        if (m <= 0) {
            if (lane == 0) {
                mbr[4 * p + 0] = mbr[4 * p + 1] = mbr[4 * p + 2] = mbr[4 * p + 3] = 0;
                if (area2) area2[p] = 0;
                if (flags) flags[p] = kFlagFew | kFlagCollinear;
            }
            continue;
        }
        const int64_t x0 = xy[2 * a], y0 = xy[2 * a + 1];
        int32_t mnx = INT32_MAX, mny = INT32_MAX, mxx = INT32_MIN, mxy = INT32_MIN;
        uint64_t acc = 0;
        bool nz = false;
        for (int64_t v = a + lane; v < b; v += 64) {
            const int32_t x = xy[2 * v], y = xy[2 * v + 1];
            const int64_t w = (v + 1 == b) ? a : v + 1;
            const int64_t xn = xy[2 * w], yn = xy[2 * w + 1];
            mnx = min(mnx, x); mxx = max(mxx, x);
            mny = min(mny, y); mxy = max(mxy, y);
            const __int128 t = (__int128)((int64_t)x - x0) * (yn - y0) -
                               (__int128)(xn - x0) * ((int64_t)y - y0);
            acc += (uint64_t)t;
            nz |= (t != 0);
        }
        mnx = wave_min(mnx); mny = wave_min(mny);
        mxx = wave_max(mxx); mxy = wave_max(mxy);
        acc = wave_sum_u64(acc);
        const bool any_nz = __ballot(nz) != 0;
        if (lane == 0) {
            mbr[4 * p + 0] = mnx; mbr[4 * p + 1] = mny;
            mbr[4 * p + 2] = mxx; mbr[4 * p + 3] = mxy;
            if (area2) area2[p] = (int64_t)acc;
            if (flags) {
                uint32_t f = 0;
                if (m < 3) f |= kFlagFew;
                if (!any_nz) f |= kFlagCollinear;
                if ((int64_t)mxx - mnx >= (1ll << 26) || (int64_t)mxy - mny >= (1ll << 26)) f |= kFlagWide;
                flags[p] = f;
            }
        }
    }
}

__global__ void k_box_init(int32_t *acc)
{
    if (threadIdx.x == 0) {
        acc[0] = INT32_MAX; acc[1] = INT32_MAX; acc[2] = INT32_MIN; acc[3] = INT32_MIN;
    }
}

__global__ __launch_bounds__(256) void k_box_of(const int32_t *__restrict__ xy, int64_t nv,
                                                int32_t *__restrict__ acc)
{
    int32_t mnx = INT32_MAX, mny = INT32_MAX, mxx = INT32_MIN, mxy = INT32_MIN;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv;
         v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t x = xy[2 * v], y = xy[2 * v + 1];
        mnx = min(mnx, x); mxx = max(mxx, x);
        mny = min(mny, y); mxy = max(mxy, y);
    }
    mnx = wave_min(mnx); mny = wave_min(mny);
    mxx = wave_max(mxx); mxy = wave_max(mxy);
    if ((threadIdx.x & 63) == 0) {
        atomicMin(acc + 0, mnx); atomicMin(acc + 1, mny);
        atomicMax(acc + 2, mxx); atomicMax(acc + 3, mxy);
    }
}

constexpr int kBuckets = 64;

// Expected work of a polygon's k walks, in draw units: Thm. 2 gives
// E[draws] = 1/S_p = N_B / N_P (capped), plus the MBR-passing draws that run a
// point-in-polygon test, about (A_mbr / A_P) edges-worth each.  Bucketed by
// log2, longest first.
__device__ __forceinline__ int cost_bucket(const int64_t *off, const int32_t *mbr,
                                           const int64_t *area2, const uint32_t *flags,
                                           int64_t p, double nb, int32_t k, double cap)
{
    if (flags[p] & (kFlagFew | kFlagCollinear)) return kBuckets - 1;
    const double ap = fmax(0.5 * fabs((double)area2[p]), 0.5);
    const double amb = ((double)mbr[4 * p + 2] - mbr[4 * p] + 1) * ((double)mbr[4 * p + 3] - mbr[4 * p + 1] + 1);
    const double n = (double)(off[p + 1] - off[p]);
    const double draws = fmin(nb / ap, cap);
    const double cost = (double)k * (draws + 0.25 * n * fmin(amb / ap, draws));
    int lg = (int)floor(log2(cost + 1.0));
    lg = lg < 0 ? 0 : (lg > kBuckets - 2 ? kBuckets - 2 : lg);
    return (kBuckets - 2) - lg;  // ascending bucket = descending cost
}

__global__ void k_order_init(int32_t *counts)
{
    if (threadIdx.x < 2 * kBuckets) counts[threadIdx.x] = 0;
}

__global__ __launch_bounds__(256) void k_order_hist(const int64_t *off, const int32_t *mbr,
                                                    const int64_t *area2, const uint32_t *flags,
                                                    int64_t n, double nb, int32_t k, double cap,
                                                    int32_t *counts)
{
    __shared__ int32_t h[kBuckets];
    if (threadIdx.x < kBuckets) h[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&h[cost_bucket(off, mbr, area2, flags, p, nb, k, cap)], 1);
    __syncthreads();
    if (threadIdx.x < kBuckets && h[threadIdx.x]) atomicAdd(&counts[threadIdx.x], h[threadIdx.x]);
}

__global__ void k_order_scan(int32_t *counts)
{
    // counts[0..63] histogram -> counts[64..127] exclusive prefix (cursors)
    if (threadIdx.x == 0) {
        int32_t s = 0;
        for (int b = 0; b < kBuckets; b++) {
            counts[kBuckets + b] = s;
            s += counts[b];
        }
    }
}

// Each block reserves, per bucket, one contiguous range of the order with a
// single global atomic, then places its polygons inside it through LDS
// atomics (one block-stride slice of polygons per pass).
__global__ __launch_bounds__(256) void k_order_scatter(const int64_t *off, const int32_t *mbr,
                                                       const int64_t *area2, const uint32_t *flags,
                                                       int64_t n, double nb, int32_t k, double cap,
                                                       int32_t *counts, int32_t *order)
{
    __shared__ int32_t h[kBuckets];
    __shared__ int32_t base[kBuckets];
    for (int64_t p0 = (int64_t)blockIdx.x * blockDim.x; p0 < n; p0 += (int64_t)gridDim.x * blockDim.x) {
        if (threadIdx.x < kBuckets) h[threadIdx.x] = 0;
        __syncthreads();
        const int64_t p = p0 + threadIdx.x;
        int b = -1, rank = 0;
        if (p < n) {
            b = cost_bucket(off, mbr, area2, flags, p, nb, k, cap);
            rank = atomicAdd(&h[b], 1);
        }
        __syncthreads();
        if (threadIdx.x < kBuckets && h[threadIdx.x])
            base[threadIdx.x] = atomicAdd(&counts[kBuckets + threadIdx.x], h[threadIdx.x]);
        __syncthreads();
        if (b >= 0) order[base[b] + rank] = (int32_t)p;
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_fill_u64(unsigned long long *p, int64_t count,
                                                  unsigned long long v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

int grid_for(int64_t items, int per_block, int max_blocks)
{
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > max_blocks) g = max_blocks;
    return (int)g;
}

}  // namespace

polymh_status launch_prepare(const int32_t *xy, const int64_t *off, int64_t n, int32_t *mbr,
                             int64_t *area2, uint32_t *flags, hipStream_t s)
{
    if (n == 0) return POLYMH_OK;
    // 4 polygons (waves) per 256-thread block
    hipLaunchKernelGGL(k_prepare, dim3(grid_for(n, 4, 1 << 16)), dim3(256), 0, s, xy, off, n, mbr,
                       area2, flags);
    return check_launch("prepare");
}

polymh_status launch_box_of(const int32_t *xy, int64_t nv, int32_t *acc4, hipStream_t s)
{
    hipLaunchKernelGGL(k_box_init, dim3(1), dim3(64), 0, s, acc4);
    if (nv > 0)
        hipLaunchKernelGGL(k_box_of, dim3(grid_for(nv, 256, 4096)), dim3(256), 0, s, xy, nv, acc4);
    return check_launch("box_of");
}

polymh_status launch_sign_order(const int64_t *off, const int32_t *mbr, const int64_t *area2,
                                const uint32_t *flags, int64_t n, polymh_box box, int32_t k,
                                uint32_t cap, int32_t *counts, int32_t *order, hipStream_t s)
{
    const double nb = ((double)box.xmax - box.xmin + 1) * ((double)box.ymax - box.ymin + 1);
    hipLaunchKernelGGL(k_order_init, dim3(1), dim3(2 * kBuckets), 0, s, counts);
    const int g = grid_for(n, 256, 2048);
    hipLaunchKernelGGL(k_order_hist, dim3(g), dim3(256), 0, s, off, mbr, area2, flags, n, nb, k,
                       (double)cap, counts);
    hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(64), 0, s, counts);
    hipLaunchKernelGGL(k_order_scatter, dim3(g), dim3(256), 0, s, off, mbr, area2, flags, n, nb,
                       k, (double)cap, counts, order);
    return check_launch("sign_order");
}

polymh_status launch_fill_u64(unsigned long long *p, int64_t count, unsigned long long v,
                              hipStream_t s)
{
    if (count <= 0) return POLYMH_OK;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(count, 256, 4096)), dim3(256), 0, s, p, count, v);
    return check_launch("fill");
}

}  // namespace polymh
