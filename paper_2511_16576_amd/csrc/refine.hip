// Exact Jaccard refinement (Sec. 1: J = area(P n Q) / area(P u Q)).
//
// area(P n Q) by Green's theorem: the boundary of P n Q is made of the parts
// of P's edges inside Q and the parts of Q's edges inside P.  Along a straight
// edge (a, b) the integrand (x dy - y dx)/2 is the constant cross(a, b)/2, so
// an edge contributes cross(a, b)/2 times the fraction of it that lies inside
// the other polygon.  That fraction is w(a) + sum over crossings of
// s * (1 - t): w(a) is the membership of the edge's start, each crossing at
// parameter t enters (s = +1) or leaves (s = -1) the other polygon.  No
// sorting of crossings is needed, so every (edge, edge) pair is independent.
//
// Degenerate contacts (shared vertices, T-junctions, collinear overlaps) are
// resolved by a consistent symbolic perturbation: Q is translated by
// (eps, eps^2), eps -> 0+.  Every orientation predicate is then nonzero (its
// sign falls back to a fixed tie-break of the edge direction), crossings are
// proper, and the area is continuous in eps, so taking the combinatorics of
// the perturbed position with the parameters t and cross products at eps = 0
// gives exactly area(P n Q).  Orientations are exact: coordinate differences
// below 2^26 make each FP64 product exact (128-bit integers beyond that).
//
// One wavefront per candidate pair; lanes take the edges of one polygon while
// the other polygon's vertices are read at a uniform index (scalar loads).
#include "internal.hpp"

namespace polymh {

namespace {

template <bool WIDE>
struct Geo;

// Exact FP64 orientation (differences < 2^26).
template <>
struct Geo<false> {
    using C = double;
    __device__ static __forceinline__ double orient(double ax, double ay, double bx, double by,
                                                    double cx, double cy)
    {
        const double t = (by - ay) * (cx - ax);
        return __fma_rn(bx - ax, cy - ay, -t);
    }
    __device__ static __forceinline__ double conv(int64_t v) { return (double)v; }
    __device__ static __forceinline__ int sgn(double o) { return (o > 0) - (o < 0); }
    __device__ static __forceinline__ double val(double o) { return o; }
};

// Exact 128-bit orientation sign for wide pairs; the FP64 value (used only
// for crossing parameters) is rounded.
template <>
struct Geo<true> {
    using C = int64_t;
    struct O {
        __int128 v;
        double d;
    };
    __device__ static __forceinline__ O orient(int64_t ax, int64_t ay, int64_t bx, int64_t by,
                                               int64_t cx, int64_t cy)
    {
        O o;
        o.v = (__int128)(bx - ax) * (cy - ay) - (__int128)(by - ay) * (cx - ax);
        o.d = (double)(bx - ax) * (double)(cy - ay) - (double)(by - ay) * (double)(cx - ax);
        return o;
    }
    __device__ static __forceinline__ int64_t conv(int64_t v) { return v; }
    __device__ static __forceinline__ int sgn(O o) { return (o.v > 0) - (o.v < 0); }
    __device__ static __forceinline__ double val(O o) { return o.d; }
};

__device__ __forceinline__ double i128_to_double(__int128 v)
{
    const bool neg = v < 0;
    const unsigned __int128 u = neg ? (unsigned __int128)(-v) : (unsigned __int128)v;
    const double r = (double)(uint64_t)(u >> 64) * 18446744073709551616.0 + (double)(uint64_t)u;
    return neg ? -r : r;
}

// Sign of orient(a, b, X + delta) when orient(a, b, X) = 0: -sign(dy), else sign(dx).
__device__ __forceinline__ int tb_shift_point(int64_t dx, int64_t dy)
{
    return dy != 0 ? (dy > 0 ? -1 : 1) : (dx > 0 ? 1 : -1);
}
// Sign of orient(c + delta, d + delta, X) when orient(c, d, X) = 0: sign(dy'), else -sign(dx').
__device__ __forceinline__ int tb_shift_edge(int64_t dx, int64_t dy)
{
    return dy != 0 ? (dy > 0 ? 1 : -1) : (dx > 0 ? -1 : 1);
}

__device__ __forceinline__ double rcp_refined(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = __fma_rn(r, __fma_rn(-d, r, 1.0), r);
    r = __fma_rn(r, __fma_rn(-d, r, 1.0), r);
    return r;
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ int64_t wave_sum_i64(int64_t v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ int32_t wmin(int32_t v)
{
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int32_t wmax(int32_t v)
{
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

struct PairIn {
    const int32_t *P;   // data polygon vertices
    int32_t n;
    const int32_t *Q;   // query polygon vertices (uniform)
    int32_t m;
    int64_t ox, oy;     // local origin
    int32_t qmbr[4];
    int sq;             // orientation of Q (+1 counter-clockwise, -1 clockwise)
    int sp;             // orientation of P
};

// Sum over P's edges of cross(a, b) * (fraction of the edge inside Q + delta),
// plus the exact doubled area of P (shoelace about the origin).
template <bool WIDE>
__device__ void edges_in_other_P(const PairIn &in, int lane, double &sum, int64_t &area2)
{
    using G = Geo<WIDE>;
    sum = 0.0;
    area2 = 0;
    for (int e = lane; e < in.n; e += 64) {
        const int f = (e + 1 == in.n) ? 0 : e + 1;
        const int64_t ax = (int64_t)in.P[2 * e] - in.ox, ay = (int64_t)in.P[2 * e + 1] - in.oy;
        const int64_t bx = (int64_t)in.P[2 * f] - in.ox, by = (int64_t)in.P[2 * f + 1] - in.oy;
        const __int128 cr = (__int128)ax * by - (__int128)bx * ay;
        area2 += (int64_t)cr;
        if (ax == bx && ay == by) continue;
        const int64_t ex0 = min(ax, bx) + in.ox, ex1 = max(ax, bx) + in.ox;
        const int64_t ey0 = min(ay, by) + in.oy, ey1 = max(ay, by) + in.oy;
        if (ex1 < in.qmbr[0] || ex0 > in.qmbr[2] || ey1 < in.qmbr[1] || ey0 > in.qmbr[3]) continue;
        const int tbe = tb_shift_point(bx - ax, by - ay);
        const auto Ax = G::conv(ax), Ay = G::conv(ay), Bx = G::conv(bx), By = G::conv(by);
        int64_t cx = (int64_t)in.Q[0] - in.ox, cy = (int64_t)in.Q[1] - in.oy;
        auto oc = G::orient(Ax, Ay, Bx, By, G::conv(cx), G::conv(cy));
        int sc = G::sgn(oc);
        sc = sc ? sc : tbe;
        int w = 0;
        double acc = 0.0;
        for (int j = 0; j < in.m; j++) {
            const int jn = (j + 1 == in.m) ? 0 : j + 1;
            const int64_t dx = (int64_t)in.Q[2 * jn] - in.ox, dy = (int64_t)in.Q[2 * jn + 1] - in.oy;
            const auto Dx = G::conv(dx), Dy = G::conv(dy), Cx = G::conv(cx), Cy = G::conv(cy);
            auto od = G::orient(Ax, Ay, Bx, By, Dx, Dy);
            int sd = G::sgn(od);
            sd = sd ? sd : tbe;
            if (cx != dx || cy != dy) {
                const int tbf = tb_shift_edge(dx - cx, dy - cy);
                const auto oa = G::orient(Cx, Cy, Dx, Dy, Ax, Ay);
                const auto ob = G::orient(Cx, Cy, Dx, Dy, Bx, By);
                int sa = G::sgn(oa), sb = G::sgn(ob);
                sa = sa ? sa : tbf;
                sb = sb ? sb : tbf;
                // membership of a in Q + delta: half-open crossing rule
                w ^= ((cy >= ay) != (dy >= ay)) & (sa == (dy > cy ? 1 : -1));
                if ((sc != sd) & (sa != sb)) {
                    const double va = G::val(oa), vb = G::val(ob);
                    acc += (double)sb * (-vb) * rcp_refined(va - vb);
                }
            }
            cx = dx; cy = dy; sc = sd;
        }
        // crossings change Q's winding number by sb; membership = sq * winding
        sum += i128_to_double(cr) * ((double)w + (double)in.sq * acc);
    }
}

// Sum over Q's edges (shifted by delta) of cross(c, d) * (fraction inside P),
// plus the exact doubled area of Q.
template <bool WIDE>
__device__ void edges_in_other_Q(const PairIn &in, const int32_t *pmbr, int lane, double &sum,
                                 int64_t &area2)
{
    using G = Geo<WIDE>;
    sum = 0.0;
    area2 = 0;
    for (int f = lane; f < in.m; f += 64) {
        const int g = (f + 1 == in.m) ? 0 : f + 1;
        const int64_t cx = (int64_t)in.Q[2 * f] - in.ox, cy = (int64_t)in.Q[2 * f + 1] - in.oy;
        const int64_t dx = (int64_t)in.Q[2 * g] - in.ox, dy = (int64_t)in.Q[2 * g + 1] - in.oy;
        const __int128 cr = (__int128)cx * dy - (__int128)dx * cy;
        area2 += (int64_t)cr;
        if (cx == dx && cy == dy) continue;
        const int64_t fx0 = min(cx, dx) + in.ox, fx1 = max(cx, dx) + in.ox;
        const int64_t fy0 = min(cy, dy) + in.oy, fy1 = max(cy, dy) + in.oy;
        if (fx1 < pmbr[0] || fx0 > pmbr[2] || fy1 < pmbr[1] || fy0 > pmbr[3]) continue;
        const int tbf = tb_shift_edge(dx - cx, dy - cy);
        const auto Cx = G::conv(cx), Cy = G::conv(cy), Dx = G::conv(dx), Dy = G::conv(dy);
        int64_t ax = (int64_t)in.P[0] - in.ox, ay = (int64_t)in.P[1] - in.oy;
        auto oa = G::orient(Cx, Cy, Dx, Dy, G::conv(ax), G::conv(ay));
        int sa = G::sgn(oa);
        sa = sa ? sa : tbf;
        int w = 0;
        double acc = 0.0;
        for (int i = 0; i < in.n; i++) {
            const int in_ = (i + 1 == in.n) ? 0 : i + 1;
            const int64_t bx = (int64_t)in.P[2 * in_] - in.ox, by = (int64_t)in.P[2 * in_ + 1] - in.oy;
            const auto Ax = G::conv(ax), Ay = G::conv(ay), Bx = G::conv(bx), By = G::conv(by);
            auto ob = G::orient(Cx, Cy, Dx, Dy, Bx, By);
            int sb = G::sgn(ob);
            sb = sb ? sb : tbf;
            if (ax != bx || ay != by) {
                const int tbe = tb_shift_point(bx - ax, by - ay);
                const auto oc = G::orient(Ax, Ay, Bx, By, Cx, Cy);
                const auto od = G::orient(Ax, Ay, Bx, By, Dx, Dy);
                int sc = G::sgn(oc), sd = G::sgn(od);
                sc = sc ? sc : tbe;
                sd = sd ? sd : tbe;
                // membership of c + delta in P: half-open crossing rule
                w ^= ((ay > cy) != (by > cy)) & (sc == (by > ay ? 1 : -1));
                if ((sa != sb) & (sc != sd)) {
                    const double vc = G::val(oc), vd = G::val(od);
                    acc += (double)sd * (-vd) * rcp_refined(vc - vd);
                }
            }
            ax = bx; ay = by; sa = sb;
        }
        sum += i128_to_double(cr) * ((double)w + (double)in.sp * acc);
    }
}

__device__ __forceinline__ int64_t poly_area2(const int32_t *v, int32_t n, int64_t ox, int64_t oy,
                                             int lane)
{
    int64_t a = 0;
    for (int i = lane; i < n; i += 64) {
        const int j = (i + 1 == n) ? 0 : i + 1;
        const int64_t ax = (int64_t)v[2 * i] - ox, ay = (int64_t)v[2 * i + 1] - oy;
        const int64_t bx = (int64_t)v[2 * j] - ox, by = (int64_t)v[2 * j + 1] - oy;
        a += (int64_t)((__int128)ax * by - (__int128)bx * ay);
    }
    return wave_sum_i64(a);
}

__device__ __forceinline__ void poly_mbr(const int32_t *v, int32_t n, int lane, int32_t *out)
{
    int32_t mnx = INT32_MAX, mny = INT32_MAX, mxx = INT32_MIN, mxy = INT32_MIN;
    for (int i = lane; i < n; i += 64) {
        mnx = min(mnx, v[2 * i]); mxx = max(mxx, v[2 * i]);
        mny = min(mny, v[2 * i + 1]); mxy = max(mxy, v[2 * i + 1]);
    }
    out[0] = wmin(mnx); out[1] = wmin(mny); out[2] = wmax(mxx); out[3] = wmax(mxy);
}

__global__ __launch_bounds__(256) void k_refine(const int32_t *__restrict__ dxy,
                                                const int64_t *__restrict__ doff,
                                                const int32_t *__restrict__ qxy,
                                                const int64_t *__restrict__ qoff,
                                                const int64_t *__restrict__ cand_off, int64_t nq,
                                                const int32_t *__restrict__ cand_ids, int64_t n_cand,
                                                double *__restrict__ cand_j)
{
    const int lane = threadIdx.x & 63;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; c < n_cand; c += nw) {
        // query of candidate c: the last q with cand_off[q] <= c
        int64_t lo = 0, hi = nq;
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if (cand_off[mid] <= c) lo = mid;
            else hi = mid;
        }
        const int64_t q = lo;
        const int32_t p = cand_ids[c];
        PairIn in;
        const int64_t pa = doff[p], qa = qoff[q];
        in.P = dxy + 2 * pa;
        in.n = (int32_t)(doff[p + 1] - pa);
        in.Q = qxy + 2 * qa;
        in.m = (int32_t)(qoff[q + 1] - qa);
        double J = 0.0;
        if (in.n >= 3 && in.m >= 3) {
            int32_t pm[4];
            poly_mbr(in.P, in.n, lane, pm);
            poly_mbr(in.Q, in.m, lane, in.qmbr);
            const bool disjoint = pm[2] <= in.qmbr[0] || in.qmbr[2] <= pm[0] || pm[3] <= in.qmbr[1] ||
                                  in.qmbr[3] <= pm[1];
            if (!disjoint) {
                in.ox = in.Q[0];
                in.oy = in.Q[1];
                const int64_t span = max(max((int64_t)pm[2], (int64_t)in.qmbr[2]) - min((int64_t)pm[0], (int64_t)in.qmbr[0]),
                                         max((int64_t)pm[3], (int64_t)in.qmbr[3]) - min((int64_t)pm[1], (int64_t)in.qmbr[1]));
                double sa, sb;
                int64_t a2p, a2q;
                a2q = poly_area2(in.Q, in.m, in.ox, in.oy, lane);
                in.sq = a2q > 0 ? 1 : -1;
                const bool wide = span >= (1ll << 26);
                if (!wide) edges_in_other_P<false>(in, lane, sa, a2p);
                else edges_in_other_P<true>(in, lane, sa, a2p);
                a2p = wave_sum_i64(a2p);
                in.sp = a2p > 0 ? 1 : -1;
                if (a2p != 0 && a2q != 0) {
                    int64_t unused;
                    if (!wide) edges_in_other_Q<false>(in, pm, lane, sb, unused);
                    else edges_in_other_Q<true>(in, pm, lane, sb, unused);
                    sa = wave_sum(sa);
                    sb = wave_sum(sb);
                    const double inter = 0.5 * (in.sp * sa + in.sq * sb);
                    const double ap = 0.5 * fabs((double)a2p), aq = 0.5 * fabs((double)a2q);
                    const double u = ap + aq - inter;
                    J = u > 0 ? inter / u : 0.0;
                }
            }
        }
        if (lane == 0) cand_j[c] = J;
    }
}

}  // namespace

polymh_status launch_refine(const polymh_polys *data, const polymh_polys *queries,
                            const int64_t *cand_off, const int32_t *cand_ids, int64_t nq,
                            int64_t n_cand, double *cand_j, hipStream_t s)
{
    if (n_cand == 0 || nq == 0) return POLYMH_OK;
    int64_t g = (n_cand + 3) / 4;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_refine, dim3((unsigned)g), dim3(256), 0, s, data->xy, data->offsets,
                       queries->xy, queries->offsets, cand_off, nq, cand_ids, n_cand, cand_j);
    return check_launch("refine");
}

}  // namespace polymh
