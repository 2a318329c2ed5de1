// Polygons with holes and multipolygons as single rings.  Every ring of a
// shape after the first is joined to the first ring's first vertex v0 by a
// bridge walked out and back:
//   R0, v0, R1, R1[0], v0, R2, R2[0], v0, ..., Rk, Rk[0]   (closing to v0).
// The two edges of a bridge are the same segment in opposite directions, so
// they cross any ray together (the crossing parity of Alg. 1's membership
// test over all rings is unchanged), and they cancel in every boundary
// integral: the shoelace area, the centroid's fan moments and the Green's
// theorem sums of the refinement.  With filled rings counter-clockwise and
// holes clockwise, the joined ring therefore signs, refines and centres as
// the even-odd region of all the rings, and every kernel of the path takes
// it unchanged.
#include "internal.hpp"

namespace polymh {

namespace {

// One wavefront per shape.  Output offsets in closed form: shape p starts
// at ring_off[first ring] + 2 (first ring - p).  Malformed input (ring or
// vertex indices out of range, a shape without rings) raises the flag and
// is skipped; every write is checked against the output's capacity.
__global__ __launch_bounds__(256) void k_join(const int2 *__restrict__ xy, int64_t nv,
                                              const int64_t *__restrict__ roff, int64_t nr,
                                              const int64_t *__restrict__ prings, int64_t n,
                                              int2 *__restrict__ out, int64_t cap,
                                              int64_t *__restrict__ out_off, int32_t *__restrict__ bad)
{
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t p = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; p < n; p += nwaves) {
        const int64_t r0 = prings[p], r1 = prings[p + 1];
        bool ok = 0 <= r0 && r0 < r1 && r1 <= nr;
        for (int64_t r = ok ? r0 : r1; r <= r1 && ok; r++) ok = roff[r] >= 0 && roff[r] <= nv && (r == r0 || roff[r] >= roff[r - 1]);
        const int64_t base = ok ? roff[r0] + 2 * (r0 - p) : 0;
        if (lane == 0) {
            out_off[p] = base;
            if (p == n - 1) out_off[n] = ok ? roff[r1] + 2 * (r1 - n) : 0;
        }
        if (!ok) {
            if (lane == 0 && bad) atomicOr(bad, 1);
            continue;
        }
        const bool joined = r1 - r0 > 1;
        const int2 v0 = roff[r0 + 1] > roff[r0] ? xy[roff[r0]] : make_int2(0, 0);
        int64_t pos = base;
        bool short_ring = false;
        const int64_t end = base + (roff[r1] - roff[r0]) + 2 * (r1 - r0 - 1);
        if (base < 0 || end > cap) {
            if (lane == 0 && bad) atomicOr(bad, 1);
            continue;
        }
        for (int64_t r = r0; r < r1; r++) {
            const int64_t a = roff[r], len = roff[r + 1] - a;
            short_ring |= len < 3;
            for (int64_t i = lane; i < len; i += 64) out[pos + i] = xy[a + i];
            pos += len;
            if (!joined) continue;
            if (r == r0) {
                if (lane == 0) out[pos] = v0;
                pos += 1;
            } else {
                if (lane == 0) out[pos] = len > 0 ? xy[a] : v0;
                pos += 1;
                if (r + 1 < r1) {
                    if (lane == 0) out[pos] = v0;
                    pos += 1;
                }
            }
        }
        if (short_ring && lane == 0 && bad) atomicOr(bad, 1);
    }
}

}  // namespace

polymh_status launch_join_rings(const int32_t *xy, int64_t nv, const int64_t *ring_off, int64_t nr,
                                const int64_t *poly_rings, int64_t n, int32_t *out_xy, int64_t out_cap,
                                int64_t *out_off, int32_t *bad, hipStream_t s)
{
    if (n == 0) return POLYMH_OK;
    int64_t blocks = (n + 3) / 4;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_join, dim3((unsigned)blocks), dim3(256), 0, s, reinterpret_cast<const int2 *>(xy), nv, ring_off,
                       nr, poly_rings, n, reinterpret_cast<int2 *>(out_xy), out_cap, out_off, bad);
    return check_launch("join_rings");
}

}  // namespace polymh
