// Inputs of the learned candidate scorer.  Per polygon (one wavefront each):
// 12 floats, of which 6 scale-free shape features
//   ln(A)/ln(N_B), ln(P^2 / (4 pi A))/4, ln(MBR width / height)/2, ln(n)/9,
//   (area centroid - MBR centre) / sqrt(A) in x and y,
// then the area A, a pad, and the MBR as floats (x0, y0, x1 + 1, y1 + 1).
// Per (query, candidate) pair (one wavefront per row): 256 collision bits
// [h_i(q) == h_i(p)] (Thm. 1 makes each a Bernoulli(J) draw), the 6 + 6 shape
// features, ln(A_q / A_p)/4, min/max area ratio (an upper bound of J),
// MBR intersection-over-union and the collision fraction, zero-padded to 288
// columns, as BF16.
#include "internal.hpp"
#include "scorer_common.hpp"

#include <cmath>

namespace polymh {

namespace {

constexpr int kFeat = 12, kBits = 256, kCols = 288;

__device__ __forceinline__ double wsum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ int32_t wmin32(int32_t v)
{
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int32_t wmax32(int32_t v)
{
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

__global__ __launch_bounds__(256) void k_poly_feats(const int32_t *__restrict__ xy,
                                                    const int64_t *__restrict__ off, int64_t n,
                                                    double log_nb, float *__restrict__ feats)
{
    const int lane = threadIdx.x & 63;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t p = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; p < n; p += nw) {
        const int64_t a = off[p], b = off[p + 1];
        const int m = (int)(b - a);
        float *f = feats + p * kFeat;
        if (m < 3) {
            if (lane < kFeat) f[lane] = 0.f;
            continue;
        }
        const int64_t x0 = xy[2 * a], y0 = xy[2 * a + 1];
        double a2 = 0, cx = 0, cy = 0, per = 0;
        int32_t mnx = INT32_MAX, mny = INT32_MAX, mxx = INT32_MIN, mxy = INT32_MIN;
        for (int i = lane; i < m; i += 64) {
            const int j = (i + 1 == m) ? 0 : i + 1;
            const double px = (double)(xy[2 * (a + i)] - x0), py = (double)(xy[2 * (a + i) + 1] - y0);
            const double qx = (double)(xy[2 * (a + j)] - x0), qy = (double)(xy[2 * (a + j) + 1] - y0);
            const double cr = px * qy - qx * py;
            a2 += cr;
            cx += (px + qx) * cr;
            cy += (py + qy) * cr;
            per += sqrt((qx - px) * (qx - px) + (qy - py) * (qy - py));
            mnx = min(mnx, xy[2 * (a + i)]); mxx = max(mxx, xy[2 * (a + i)]);
            mny = min(mny, xy[2 * (a + i) + 1]); mxy = max(mxy, xy[2 * (a + i) + 1]);
        }
        a2 = wsum(a2); cx = wsum(cx); cy = wsum(cy); per = wsum(per);
        mnx = wmin32(mnx); mny = wmin32(mny); mxx = wmax32(mxx); mxy = wmax32(mxy);
        if (lane == 0) {
            const double A = fmax(0.5 * fabs(a2), 0.5);
            const double gx = (a2 != 0 ? cx / (3.0 * a2) : 0.0) + (double)x0;
            const double gy = (a2 != 0 ? cy / (3.0 * a2) : 0.0) + (double)y0;
            const double w = (double)mxx - mnx + 1.0, h = (double)mxy - mny + 1.0;
            const double sa = sqrt(A);
            f[0] = (float)(log(A) / log_nb);
            f[1] = (float)(log(fmax(per * per / (4.0 * M_PI * A), 1e-12)) / 4.0);
            f[2] = (float)(log(w / h) / 2.0);
            f[3] = (float)(log((double)m) / 9.0);
            f[4] = (float)((gx - 0.5 * ((double)mnx + mxx)) / sa);
            f[5] = (float)((gy - 0.5 * ((double)mny + mxy)) / sa);
            f[6] = (float)A;
            f[7] = 0.f;
            f[8] = (float)mnx; f[9] = (float)mny; f[10] = (float)mxx + 1.f; f[11] = (float)mxy + 1.f;
        }
    }
}

__global__ __launch_bounds__(256) void k_pair_feats(const uint32_t *__restrict__ lsig,
                                                    const float *__restrict__ lfeat,
                                                    const uint32_t *__restrict__ rsig,
                                                    const float *__restrict__ rfeat,
                                                    const int32_t *__restrict__ li,
                                                    const int32_t *__restrict__ ri, int64_t R,
                                                    int64_t R_pad, __bf16 *__restrict__ X)
{
    const int lane = threadIdx.x & 63;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; r < R_pad; r += nw) {
        __bf16 *row = X + r * kCols;
        // rows past R and rows of an empty head slot (negative index) are zero
        if (r >= R || li[r] < 0 || ri[r] < 0) {
            for (int c = lane; c < kCols; c += 64) row[c] = (__bf16)0.f;
            continue;
        }
        const int64_t q = li[r], p = ri[r];
        const uint32_t *sq = lsig + q * kBits, *sp = rsig + p * kBits;
        int cnt = 0;
#pragma unroll
        for (int t = 0; t < 4; t++) {
            const int i = t * 64 + lane;
            const bool eq = sq[i] == sp[i];
            row[i] = (__bf16)(eq ? 1.f : 0.f);
            cnt += __popcll(__ballot(eq));
        }
        const float *fq = lfeat + q * kFeat, *fp = rfeat + p * kFeat;
        if (lane < 32) row[kBits + lane] = (__bf16)pair_tail_feature(lane, fq, fp, cnt);
    }
}

__global__ __launch_bounds__(256) void k_csr_rows(const int64_t *__restrict__ off, int64_t nq,
                                                  int32_t *__restrict__ rows)
{
    for (int64_t q = blockIdx.x; q < nq; q += gridDim.x)
        for (int64_t c = off[q] + threadIdx.x; c < off[q + 1]; c += blockDim.x) rows[c] = (int32_t)q;
}

int grid_cap(int64_t items, int per)
{
    int64_t g = (items + per - 1) / per;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (int)g;
}

}  // namespace

polymh_status launch_poly_features(const polymh_polys *p, polymh_box box, float *feats, hipStream_t s)
{
    if (p->n == 0) return POLYMH_OK;
    const double nb = ((double)box.xmax - box.xmin + 1) * ((double)box.ymax - box.ymin + 1);
    hipLaunchKernelGGL(k_poly_feats, dim3(grid_cap(p->n, 4)), dim3(256), 0, s, p->xy, p->offsets,
                       p->n, log(fmax(nb, 2.0)), feats);
    return check_launch("poly_features");
}

polymh_status launch_pair_features(const uint32_t *lsig, const float *lfeat, const uint32_t *rsig,
                                   const float *rfeat, const int32_t *li, const int32_t *ri,
                                   int64_t R, int64_t R_pad, uint16_t *X, hipStream_t s)
{
    if (R_pad == 0) return POLYMH_OK;
    hipLaunchKernelGGL(k_pair_feats, dim3(grid_cap(R_pad, 4)), dim3(256), 0, s, lsig, lfeat, rsig,
                       rfeat, li, ri, R, R_pad, reinterpret_cast<__bf16 *>(X));
    return check_launch("pair_features");
}

polymh_status launch_csr_rows(const int64_t *off, int64_t nq, int32_t *rows, hipStream_t s)
{
    if (nq == 0) return POLYMH_OK;
    hipLaunchKernelGGL(k_csr_rows, dim3(grid_cap(nq, 1)), dim3(256), 0, s, off, nq, rows);
    return check_launch("csr_rows");
}

}  // namespace polymh
