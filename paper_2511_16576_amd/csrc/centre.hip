// Centring (Sec. 3.1): every polygon is translated so that its area centroid,
// rounded to the lattice, is the origin.  The centroid is the area-weighted
// mean of the signed fan triangles about the first vertex v0,
//   C - v0 = sum_i (d_i + d_{i+1}) cross(d_i, d_{i+1}) / (3 sum_i cross(d_i, d_{i+1})),
// d_i = v_i - v0, summed exactly in 128-bit integers; each coordinate is
// rounded by floor(c + 1/2), which commutes with integer translations.
#include <cmath>

#include "internal.hpp"

namespace polymh {

namespace {

using i128 = __int128;

// One DPP step of a 128-bit sum carried as two 64-bit halves: add the value
// the DPP control brings from another lane, with the carry between halves.
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ void dpp_add128(uint64_t &lo, uint64_t &hi)
{
    const uint64_t l2 = dpp::mov64<CTRL, ROWS>(0, lo), h2 = dpp::mov64<CTRL, ROWS>(0, hi);
    const uint64_t nl = lo + l2;
    hi = hi + h2 + (nl < lo ? 1u : 0u);
    lo = nl;
}

// Sum over one 16-lane DPP row (quads, then rotations by 4 and 8 within the
// row): every lane of the row receives the row's total.
__device__ __forceinline__ i128 row_sum_i128(i128 v)
{
    uint64_t lo = (uint64_t)v, hi = (uint64_t)((unsigned __int128)v >> 64);
    dpp_add128<dpp::kQuad1032>(lo, hi);
    dpp_add128<dpp::kQuad2301>(lo, hi);
    dpp_add128<dpp::kRowRor4>(lo, hi);
    dpp_add128<dpp::kRowRor8>(lo, hi);
    return (i128)(((unsigned __int128)hi << 64) | lo);
}

__device__ __forceinline__ double i128_to_f64(i128 v)
{
    const bool neg = v < 0;
    const unsigned __int128 u = neg ? (unsigned __int128)(-v) : (unsigned __int128)v;
    const double r = (double)(uint64_t)(u >> 64) * 18446744073709551616.0 + (double)(uint64_t)u;
    return neg ? -r : r;
}

// floor(num / den) for den != 0 when the quotient is far inside int64 (here
// a centroid offset inside the polygon's box): an FP64 estimate, off by at
// most one, corrected with exact 128-bit products (no 128-bit division).
__device__ __forceinline__ int64_t floor_div_small(i128 num, i128 den)
{
    if (den < 0) {
        num = -num;
        den = -den;
    }
    int64_t q = (int64_t)floor(i128_to_f64(num) / i128_to_f64(den));
    while ((i128)q * den > num) q--;
    while ((i128)(q + 1) * den <= num) q++;
    return q;
}

// One 16-lane DPP row per polygon, four polygons per wavefront: the fan
// sums are row reductions of four DPP steps, and each row divides for its own
// polygon (a whole row is active or not, so the row operations only ever read
// lanes of the same polygon).
__global__ __launch_bounds__(256) void k_centre(const int32_t *__restrict__ xy,
                                                const int64_t *__restrict__ off, int64_t n,
                                                int32_t *__restrict__ out, int32_t *__restrict__ shift,
                                                int32_t *__restrict__ range_flag)
{
    const int rl = threadIdx.x & 15;
    const int64_t nrows = ((int64_t)gridDim.x * blockDim.x) >> 4;
    for (int64_t p = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4; p < n; p += nrows) {
        const int64_t a = off[p], b = off[p + 1], m = b - a;
        int64_t sx = 0, sy = 0;
        if (m >= 3) {
            const int64_t x0 = xy[2 * a], y0 = xy[2 * a + 1];
            i128 a2 = 0, nx = 0, ny = 0;
            const int2 *v = reinterpret_cast<const int2 *>(xy + 2 * a);
            for (int64_t base = 0; base < m; base += 16) {
                const int64_t i = base + rl;
                const bool live = i < m;
                const int2 pi = v[live ? i : 0], pj = v[i + 1 < m ? i + 1 : 0];
                const int64_t dx = pi.x - x0, dy = pi.y - y0;
                const int64_t ex = pj.x - x0, ey = pj.y - y0;
                const i128 c = live ? (i128)dx * ey - (i128)ex * dy : 0;
                a2 += c;
                nx += (i128)(dx + ex) * c;
                ny += (i128)(dy + ey) * c;
            }
            a2 = row_sum_i128(a2);
            nx = row_sum_i128(nx);
            ny = row_sum_i128(ny);
            if (a2 != 0) {
                sx = x0 + floor_div_small(2 * nx + 3 * a2, 6 * a2);
                sy = y0 + floor_div_small(2 * ny + 3 * a2, 6 * a2);
            }
        }
        if (shift && rl == 0) {
            shift[2 * p] = (int32_t)sx;
            shift[2 * p + 1] = (int32_t)sy;
        }
        bool bad = false;
        for (int64_t i = rl; i < m; i += 16) {
            const int64_t x = xy[2 * (a + i)] - sx, y = xy[2 * (a + i) + 1] - sy;
            bad |= x < INT32_MIN || x > INT32_MAX || y < INT32_MIN || y > INT32_MAX;
            out[2 * (a + i)] = (int32_t)x;
            out[2 * (a + i) + 1] = (int32_t)y;
        }
        if (bad && range_flag) atomicOr(range_flag, 1);
    }
}

}  // namespace

polymh_status launch_centre(const int32_t *xy, const int64_t *off, int64_t n, int32_t *out,
                            int32_t *shift, int32_t *range_flag, hipStream_t s)
{
    if (n == 0) return POLYMH_OK;
    int64_t blocks = (n + 15) / 16;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_centre, dim3((unsigned)blocks), dim3(256), 0, s, xy, off, n, out, shift, range_flag);
    return check_launch("centre");
}

}  // namespace polymh
