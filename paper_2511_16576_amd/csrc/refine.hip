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
#include <algorithm>

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

// 1/d: the hardware reciprocal (relative error about 2^-24 on gfx950) and
// one Newton step (error about 2^-48, measured), ample for crossing
// parameters summed into areas checked to 1e-9.
__device__ __forceinline__ double rcp_refined(double d)
{
    const double r = __builtin_amdgcn_rcp(d);
    return __fma_rn(r, __fma_rn(-d, r, 1.0), r);
}

__device__ __forceinline__ double wave_sum(double v) { return wave_sum_f64(v); }
__device__ __forceinline__ int32_t wmin(int32_t v) { return wave_min32(v); }
__device__ __forceinline__ int32_t wmax(int32_t v) { return wave_max32(v); }

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

// The other ring's vertices are read 64 at a time, one per lane, by a
// wavefront whose lanes are all active, and handed to the edge loop by
// readlane: one coalesced load per 64 iterations instead of a dependent load
// in each.  Vertex (jb + lane + 1) mod m of an m-vertex ring.
__device__ __forceinline__ int2 next_vertex_block(const int32_t *V, int m, int jb, int lane)
{
    const int j = jb + lane + 1;
    const int jn = j < m ? j : (j == m ? 0 : 0);
    return *reinterpret_cast<const int2 *>(V + 2 * jn);
}

// Sum over P's edges of cross(a, b) * (fraction of the edge inside Q + delta),
// plus the exact doubled area of P (shoelace about the origin).
// Only the 64-edge blocks b0, b0 + bstride, ... of P (a split pair); (0, 1)
// takes them all.
template <bool WIDE>
__device__ void edges_in_other_P(const PairIn &in, int lane, double &sum, int64_t &area2, int b0 = 0,
                                 int bstride = 1)
{
    using G = Geo<WIDE>;
    sum = 0.0;
    area2 = 0;
    for (int eb = 64 * b0; eb < in.n; eb += 64 * bstride) {
        // every lane stays in the loop (the vertex blocks need all of them)
        const int e = eb + lane;
        const bool live = e < in.n;
        const int ei = live ? e : 0;
        const int f = (ei + 1 == in.n) ? 0 : ei + 1;
        const int64_t ax = (int64_t)in.P[2 * ei] - in.ox, ay = (int64_t)in.P[2 * ei + 1] - in.oy;
        const int64_t bx = (int64_t)in.P[2 * f] - in.ox, by = (int64_t)in.P[2 * f + 1] - in.oy;
        const __int128 cr = (__int128)ax * by - (__int128)bx * ay;
        if (live) area2 += (int64_t)cr;
        const int64_t ex0 = min(ax, bx) + in.ox, ex1 = max(ax, bx) + in.ox;
        const int64_t ey0 = min(ay, by) + in.oy, ey1 = max(ay, by) + in.oy;
        const bool act = live && !(ax == bx && ay == by) &&
                         !(ex1 < in.qmbr[0] || ex0 > in.qmbr[2] || ey1 < in.qmbr[1] || ey0 > in.qmbr[3]);
        if (__ballot(act) == 0) continue;
        const int tbe = tb_shift_point(bx - ax, by - ay);
        const auto Ax = G::conv(ax), Ay = G::conv(ay), Bx = G::conv(bx), By = G::conv(by);
        int64_t cx = (int64_t)in.Q[0] - in.ox, cy = (int64_t)in.Q[1] - in.oy;
        auto oc = G::orient(Ax, Ay, Bx, By, G::conv(cx), G::conv(cy));
        int sc = G::sgn(oc);
        sc = sc ? sc : tbe;
        int w = 0;
        double acc = 0.0;
        for (int jb = 0; jb < in.m; jb += 64) {
          const int2 blk = next_vertex_block(in.Q, in.m, jb, lane);
          const int cnt = min(64, in.m - jb);
          for (int t = 0; t < cnt; t++) {
            const int64_t dx = (int64_t)__builtin_amdgcn_readlane(blk.x, t) - in.ox;
            const int64_t dy = (int64_t)__builtin_amdgcn_readlane(blk.y, t) - in.oy;
            if (!act) {
                cx = dx; cy = dy;
                continue;
            }
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
        }
        // crossings change Q's winding number by sb; membership = sq * winding
        if (act) sum += i128_to_double(cr) * ((double)w + (double)in.sq * acc);
    }
}

// Sum over Q's edges (shifted by delta) of cross(c, d) * (fraction inside P),
// plus the exact doubled area of Q.
template <bool WIDE>
__device__ void edges_in_other_Q(const PairIn &in, const int32_t *pmbr, int lane, double &sum,
                                 int64_t &area2, int b0 = 0, int bstride = 1)
{
    using G = Geo<WIDE>;
    sum = 0.0;
    area2 = 0;
    for (int fb = 64 * b0; fb < in.m; fb += 64 * bstride) {
        // every lane stays in the loop (the vertex blocks need all of them)
        const int f = fb + lane;
        const bool live = f < in.m;
        const int fi = live ? f : 0;
        const int g = (fi + 1 == in.m) ? 0 : fi + 1;
        const int64_t cx = (int64_t)in.Q[2 * fi] - in.ox, cy = (int64_t)in.Q[2 * fi + 1] - in.oy;
        const int64_t dx = (int64_t)in.Q[2 * g] - in.ox, dy = (int64_t)in.Q[2 * g + 1] - in.oy;
        const __int128 cr = (__int128)cx * dy - (__int128)dx * cy;
        if (live) area2 += (int64_t)cr;
        const int64_t fx0 = min(cx, dx) + in.ox, fx1 = max(cx, dx) + in.ox;
        const int64_t fy0 = min(cy, dy) + in.oy, fy1 = max(cy, dy) + in.oy;
        const bool act = live && !(cx == dx && cy == dy) &&
                         !(fx1 < pmbr[0] || fx0 > pmbr[2] || fy1 < pmbr[1] || fy0 > pmbr[3]);
        if (__ballot(act) == 0) continue;
        const int tbf = tb_shift_edge(dx - cx, dy - cy);
        const auto Cx = G::conv(cx), Cy = G::conv(cy), Dx = G::conv(dx), Dy = G::conv(dy);
        int64_t ax = (int64_t)in.P[0] - in.ox, ay = (int64_t)in.P[1] - in.oy;
        auto oa = G::orient(Cx, Cy, Dx, Dy, G::conv(ax), G::conv(ay));
        int sa = G::sgn(oa);
        sa = sa ? sa : tbf;
        int w = 0;
        double acc = 0.0;
        for (int ib = 0; ib < in.n; ib += 64) {
          const int2 blk = next_vertex_block(in.P, in.n, ib, lane);
          const int cnt = min(64, in.n - ib);
          for (int t = 0; t < cnt; t++) {
            const int64_t bx = (int64_t)__builtin_amdgcn_readlane(blk.x, t) - in.ox;
            const int64_t by = (int64_t)__builtin_amdgcn_readlane(blk.y, t) - in.oy;
            if (!act) {
                ax = bx; ay = by;
                continue;
            }
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
        }
        if (act) sum += i128_to_double(cr) * ((double)w + (double)in.sp * acc);
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

// ---------------------------------------------------------------------------
// Tiled form.  The two boundaries are cut into chunks of 8 edges; only chunk
// pairs whose boxes overlap (tiles of 8 x 8 edge pairs) are tested.  Each
// crossing is found once and credited to both polygons.  The membership of
// each edge's start is not tested directly: it is the membership of the
// ring's first vertex plus the running sum of the crossing signs met along
// the ring, so with S_e the net sign of edge e's crossings,
//   sum_e cr_e * I(e) = sum_e cr_e * (w_0 + s * sum_{e' < e} S_e')
//                       + s * sum_{crossings} cr_e * sign * (1 - t).
// Q (the query) is staged once per workgroup; each wavefront stages its data
// polygon.  Pairs with a polygon beyond kTileCap edges, or coordinate spans of
// 2^26 and more, take the general per-edge form above.
//
// Work layout: overlapping tiles are compacted into a per-wavefront list and
// taken 8 at a time; lane (slot, j) keeps edge j of its tile's Q chunk in
// registers and sweeps the 8 edges of the tile's P chunk.  With e = b - a,
// f = d - c, r = c - a and X = cross(e, f) the four orientations are
//   orient(a,b,c) = cross(e, r),  orient(a,b,d) = orient(a,b,c) + X,
//   orient(c,d,a) = cross(r, f),  orient(c,d,b) = orient(c,d,a) - X,
// all exact integers in FP64 (differences < 2^26).  The symbolic tie-break is
// folded into one compare: against a threshold of -1/2 or +1/2 for P's
// edges, and for Q's edges a floating-point class test whose "positive" set
// is {+denormal, +normal, +inf}, plus both zeros when the tie resolves to +1.
// Rings are padded with copies of vertex 0, so edges past the end are
// zero-length and can never cross: no per-lane bounds checks in the sweep.

constexpr int kTileCap = 512;
constexpr int kRingLds = kTileCap + 16;   // ring vertices incl. padding
constexpr int kWavesPerBlock = 4;
constexpr int kListCap = 256;             // per-wavefront ring of tile entries (< 16 pending + 128 new)
constexpr int kCrossCap = 128;            // per-wavefront crossing buffer
constexpr int kUnitCap = 256;             // per-wavefront ring of sweep units (< 64 pending + 128 new)
constexpr int kClassPos = (1 << 7) | (1 << 8) | (1 << 9);
constexpr int kClassPosZ = kClassPos | (1 << 5) | (1 << 6);

struct RingLds {
    int2 *v;            // vertices relative to the origin; v[n..] repeat v[0]
    int4 *box;          // per 8-edge chunk: xmin, ymin, xmax, ymax
    uint32_t *S;        // P only: net crossing sign per edge, two biased 16-bit halves a word
    double *suf;        // Q only: suffix sums of the edges' cross products (see below)
};

// Crossing-sign sums are kept as 16-bit halves biased by 2^15 inside 32-bit
// words (|S| <= kTileCap, so a half never wraps and never borrows from its
// neighbour); one LDS atomic adds +-1 to either half.
constexpr uint32_t kSBias = 0x80008000u;
__device__ __forceinline__ void s_add(uint32_t *S, int e, int v)
{
    atomicAdd(&S[e >> 1], (uint32_t)v << (16 * (e & 1)));
}
__device__ __forceinline__ int s_get(const uint32_t *S, int e)
{
    return (int)((S[e >> 1] >> (16 * (e & 1))) & 0xffffu) - 0x8000;
}

// Tie-break class set of a shifted Q edge (c + delta, d + delta), f = d - c,
// for orientations of points of P: a zero counts as positive when fy > 0, or
// fy = 0 and fx < 0 (zero-length edges never cross either way).
__device__ __forceinline__ int q_edge_class(int fx, int fy)
{
    return (fy > 0 || (fy == 0 && fx < 0)) ? kClassPosZ : kClassPos;
}

// Tie-break threshold of a P edge (e = b - a) for orientations of points of
// Q + delta: a zero counts as positive when the edge points down, or is
// horizontal and points right.  Orientations are integers, so o > -1/2 is
// o >= 0 and o > +1/2 is o > 0.  fma(ey, 2^32, -ex) carries the sign of ey,
// or of -ex when ey = 0 (|ex| < 2^26), and the threshold takes that sign.
__device__ __forceinline__ double p_edge_threshold(double ex, double ey)
{
    return copysign(0.5, __fma_rn(ey, 4294967296.0, -ex));
}

__device__ __forceinline__ double orient_d(int2 a, int2 b, int2 c)
{
    const double t = (double)(b.y - a.y) * (double)(c.x - a.x);
    return __fma_rn((double)(b.x - a.x), (double)(c.y - a.y), -t);
}

__device__ __forceinline__ int sgn_tb(double o, int tb) { return o > 0 ? 1 : (o < 0 ? -1 : tb); }

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_wave_barrier();
}

// Stage a ring relative to the origin into entries [0, pad_to), entries from
// n on repeating vertex 0.
__device__ void stage_ring(const int32_t *src, int n, int pad_to, int64_t ox, int64_t oy, RingLds R,
                           int t0, int nt)
{
    for (int i = t0; i < pad_to; i += nt) {
        const int k = i < n ? i : 0;
        R.v[i] = make_int2((int)((int64_t)src[2 * k] - ox), (int)((int64_t)src[2 * k + 1] - oy));
    }
}

// Wavefront staging of a data polygon (as stage_ring) that also returns the
// MBR of its absolute coordinates (uniform), the ring's doubled area about
// the origin (exact, 64-bit; meaningful when the pair is not wide) and the
// first vertex strictly outside the box qb (-1 if none): that vertex is
// outside Q, and so is the vertex minus delta.
// Vertices i and i + 1 of the first two 64-vertex windows, fetched one
// candidate ahead (indices as the staging loop clamps them).
struct RingPrefetch {
    int2 p[2], q[2];
};

__device__ __forceinline__ void prefetch_ring(const int32_t *src, int n, int lane, RingPrefetch &pf)
{
    const int2 *v = reinterpret_cast<const int2 *>(src);
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const int i = 64 * h + lane;
        pf.p[h] = v[i < n ? i : 0];
        pf.q[h] = v[i + 1 < n ? i + 1 : 0];
    }
}

__device__ void stage_ring_mbr(const int32_t *src, int n, int pad_to, int64_t ox, int64_t oy,
                               RingLds R, int lane, const int32_t *qb, const RingPrefetch &pf, int32_t *mbr,
                               int64_t &area2, int &anchor)
{
    int x0 = INT32_MAX, y0 = INT32_MAX, x1 = INT32_MIN, y1 = INT32_MIN;
    const int2 *v = reinterpret_cast<const int2 *>(src);
    int k = -1;
    int64_t a2 = 0;
    for (int base = 0; base < pad_to; base += 64) {
        const int i = base + lane;
        const bool live = i < pad_to, edge = i < n;
        const int2 p = base == 0 ? pf.p[0] : base == 64 ? pf.p[1] : v[edge ? i : 0];
        const int2 q = base == 0 ? pf.q[0] : base == 64 ? pf.q[1] : v[i + 1 < n ? i + 1 : 0];
        // relative coordinates in 32 bits (wrapping): exact unless the pair
        // spans 2^26 or more, whose area the caller takes from elsewhere
        const int px = (int)((uint32_t)p.x - (uint32_t)ox), py = (int)((uint32_t)p.y - (uint32_t)oy);
        const int qx = (int)((uint32_t)q.x - (uint32_t)ox), qy = (int)((uint32_t)q.y - (uint32_t)oy);
        if (live) R.v[i] = make_int2(px, py);
        a2 += edge ? (int64_t)px * qy - (int64_t)qx * py : 0;
        x0 = min(x0, p.x); y0 = min(y0, p.y); x1 = max(x1, p.x); y1 = max(y1, p.y);
        const bool out = edge & ((p.x < qb[0]) | (p.x > qb[2]) | (p.y < qb[1]) | (p.y > qb[3]));
        const uint64_t mk = __ballot(out);
        if (k < 0 && mk != 0) k = base + __builtin_ctzll(mk);
    }
    mbr[0] = wave_min32(x0); mbr[1] = wave_min32(y0);
    mbr[2] = wave_max32(x1); mbr[3] = wave_max32(y1);
    area2 = wave_sum_i64(a2);
    anchor = k;
}

__device__ void chunk_boxes(RingLds R, int n, int t0, int nt)
{
    const int nc = (n + 7) >> 3;
    for (int c = t0; c < nc; c += nt) {
        int x0 = INT32_MAX, y0 = INT32_MAX, x1 = INT32_MIN, y1 = INT32_MIN;
        const int e1 = min(n, 8 * c + 8);
        for (int v = 8 * c; v <= e1; v++) {
            const int2 p = R.v[v];
            x0 = min(x0, p.x); y0 = min(y0, p.y); x1 = max(x1, p.x); y1 = max(y1, p.y);
        }
        R.box[c] = make_int4(x0, y0, x1, y1);
    }
}

// Wavefront form for P (lane = chunk, up to MAXC chunks): the chunk boxes.
// The 9 vertices of a chunk are read at once (indices clamped to the ring's
// end, which only repeats a vertex) so their LDS latencies overlap.
template <int MAXC>
__device__ void chunk_boxes_p(RingLds R, int n, int lane)
{
    const int nc = (n + 7) >> 3;
#pragma unroll
    for (int c0 = 0; c0 < MAXC; c0 += 64) {
        int c = c0 + lane;
        // recomputed here rather than hoisted out of a caller's loop over
        // pairs, where the compiler would keep 8 c + 1 and 8 c + 8 live in
        // registers (or spill them) across the whole pair
        asm volatile("" : "+v"(c));
        if (c < nc) {
            const int e1 = min(n, 8 * c + 8);
            int2 p[9];
#pragma unroll
            for (int j = 0; j < 9; j++) p[j] = R.v[min(8 * c + j, e1)];
            int x0 = p[0].x, y0 = p[0].y, x1 = p[0].x, y1 = p[0].y;
#pragma unroll
            for (int j = 1; j < 9; j++) {
                x0 = min(x0, p[j].x); y0 = min(y0, p[j].y); x1 = max(x1, p[j].x); y1 = max(y1, p[j].y);
            }
            R.box[c] = make_int4(x0, y0, x1, y1);
        }
    }
}

// Edge (c, d)'s parity term in the membership of point a + sh*delta in a
// ring (half-open crossing rule with the perturbation): sh = -1 tests
// a - delta (a vertex of P against Q + delta), sh = +1 tests a + delta (a
// vertex of Q + delta against P).  A straddling edge is never horizontal.
__device__ __forceinline__ bool flips_parity(int2 c, int2 d, int2 a, int sh)
{
    const bool st = sh < 0 ? ((c.y >= a.y) != (d.y >= a.y)) : ((c.y > a.y) != (d.y > a.y));
    const int up = d.y > c.y ? 1 : -1;
    const int tb = sh < 0 ? up : -up;   // sign of orient(c, d, a + sh*delta) when orient(c, d, a) = 0
    const double o = orient_d(c, d, a);
    const int so = o > 0 ? 1 : (o < 0 ? -1 : tb);
    return st & (so == up);
}

// The same for edge e of a ring in LDS.
__device__ __forceinline__ bool member_edge(const int2 *v, int e, int2 a, int sh)
{
    return flips_parity(v[e], v[e + 1], a, sh);
}

// Ring-start memberships of both rings in one pass: w0p for P's vertex 0
// against Q + delta, w0q for Q's vertex 0 + delta against P.
__device__ void member_starts(RingLds P, int n, RingLds Q, int m, int lane, bool need_p, bool need_q,
                              int &w0p, int &w0q)
{
    const int2 p0 = P.v[0], q0 = Q.v[0];
    bool oddp = false, oddq = false;
    const int top = max(need_p ? m : 0, need_q ? n : 0);
    for (int e = lane; e < top; e += 64) {
        const bool lq = need_p & (e < m), lp = need_q & (e < n);
        oddp ^= lq & member_edge(Q.v, lq ? e : 0, p0, -1);
        oddq ^= lp & member_edge(P.v, lp ? e : 0, q0, +1);
    }
    w0p = __popcll(__ballot(oddp)) & 1;
    w0q = __popcll(__ballot(oddq)) & 1;
}

// P's membership sum: sum_e cr_e * w_e with w_e = w0 + s * (exclusive prefix
// of S along the ring), s = Q's orientation; a per-lane partial.  Branch-free,
// so the scan runs with every lane active.
//
// Q's sum needs no pass per pair: exchanging the order of summation,
//   sum_f cr_f * (w0 + s' * sum_{f' < f} S_f') = w0 * A2Q + s' * sum_{f'} S_f' * Suf(f'),
// with Suf(f') = sum_{f > f'} cr_f fixed by Q alone (staged once per query),
// so every crossing on Q's edge f' adds its sign times Suf(f').
//
// Here the sum is split as w0 * A2P + s * T, T = sum_e cr_e * pre(e) with
// pre(e) the exclusive prefix of S; the function returns T (a per-lane
// partial) and K = pre(anchor) (uniform), so that a known membership at any
// anchor vertex fixes w0 = w(anchor) - s * K.
// Over a window of a longer ring: carry holds the crossing signs of the
// edges before the window (in and out), K is set only when the anchor's
// index (relative to the window) falls inside it, and crs gathers the
// window's cross products (per-lane partial).
__device__ double membership_term_window(RingLds P, int n, int anchor, int lane, int &carry, int &K, double &crs)
{
    double acc = 0.0;
    for (int base = 0; base < n; base += 64) {
        const int e = base + lane;
        const bool live = e < n;
        const int ee = live ? e : 0;
        const int Se = live ? s_get(P.S, ee) : 0;
        const int2 a = P.v[ee], b = P.v[ee + 1];
        const double cr = __fma_rn((double)a.x, (double)b.y, -(double)b.x * (double)a.y);
        const int incl = wave_incl_scan32(Se);
        const int excl = carry + incl - Se;
        acc += live ? cr * (double)excl : 0.0;
        crs += live ? cr : 0.0;
        if (anchor >= base && anchor < base + 64) K = __builtin_amdgcn_readlane(excl, anchor - base);
        carry += __builtin_amdgcn_readlane(incl, 63);
    }
    return acc;
}

__device__ double membership_term_p(RingLds P, int n, int anchor, int lane, int &K)
{
    int carry = 0;
    double crs = 0.0;
    K = 0;
    return membership_term_window(P, n, anchor, lane, carry, K, crs);
}

// Indices of a leftmost, a rightmost, a lowest and a highest vertex of Q
// (rb: Q's MBR relative to the origin), by one wavefront.  A pair whose P
// MBR leaves one of those sides of Q's MBR open anchors Q's memberships at
// that vertex (it lies outside P).
__device__ void q_extremes(RingLds Q, int m, int4 rb, int lane, int *ext)
{
    int k0 = -1, k1 = -1, k2 = -1, k3 = -1;
    for (int base = 0; base < m; base += 64) {
        const int i = base + lane;
        const bool live = i < m;
        const int2 p = Q.v[live ? i : 0];
        const uint64_t b0 = __ballot(live & (p.x == rb.x)), b1 = __ballot(live & (p.x == rb.z));
        const uint64_t b2 = __ballot(live & (p.y == rb.y)), b3 = __ballot(live & (p.y == rb.w));
        if (k0 < 0 && b0 != 0) k0 = base + __builtin_ctzll(b0);
        if (k1 < 0 && b1 != 0) k1 = base + __builtin_ctzll(b1);
        if (k2 < 0 && b2 != 0) k2 = base + __builtin_ctzll(b2);
        if (k3 < 0 && b3 != 0) k3 = base + __builtin_ctzll(b3);
    }
    if (lane == 0) { ext[0] = k0; ext[1] = k1; ext[2] = k2; ext[3] = k3; }
}

// Q's suffix sums Suf(f) = A2Q - sum_{f' <= f} cr_f' (exact in 64-bit
// integers), by one wavefront.
__device__ int64_t q_suffix_sums(RingLds Q, int m, int64_t a2q, int lane, int64_t carry = 0)
{
    for (int base = 0; base < m; base += 64) {
        const int e = base + lane;
        const bool live = e < m;
        const int ee = live ? e : 0;
        const int2 a = Q.v[ee], b = Q.v[ee + 1];
        const int64_t cr = live ? (int64_t)a.x * b.y - (int64_t)b.x * a.y : 0;
        const int64_t incl = carry + wave_incl_scan64(cr);
        if (live) Q.suf[e] = (double)(a2q - incl);
        carry = (int64_t)dpp::readlane64((uint64_t)incl, 63);
    }
    return carry;
}

// Crossing contributions of buffered (e, f) pairs, 64 at a time with every
// lane busy: the orientations are recomputed exactly as in the sweep, so the
// signs and parameters are the ones that detected the crossing.
__device__ void flush_crossings(RingLds P, RingLds Q, const uint32_t *buf, int count, int lane, int kq,
                                double &accP, double &accQ, double &accM, double &accK)
{
    for (int k = lane; k < count; k += 64) {
        const uint32_t ef = buf[k];
        const int e = (int)(ef >> 16), f = (int)(ef & 0xffffu);
        const int2 a = P.v[e], b = P.v[e + 1], c = Q.v[f], d = Q.v[f + 1];
        const double ax = (double)a.x, ay = (double)a.y, bx = (double)b.x, by = (double)b.y;
        const double cx = (double)c.x, cy = (double)c.y;
        const double ex = bx - ax, ey = by - ay;
        const double fx = (double)(d.x - c.x), fy = (double)(d.y - c.y);
        const double rx = cx - ax, ry = cy - ay;
        const double oc = __fma_rn(ex, ry, -(ey * rx));
        const double oa = __fma_rn(fy, rx, -(fx * ry));
        const double X = __fma_rn(ex, fy, -(ey * fx));
        const double od = oc + X, ob = oa - X;
        const bool p2 = od > p_edge_threshold(ex, ey);
        const bool p4 = __builtin_amdgcn_class(ob, q_edge_class(d.x - c.x, d.y - c.y));
        const double cre = __fma_rn(ax, by, -(bx * ay));
        const double crf = __fma_rn(cx, fy, -(fx * cy));
        accP += cre * (p4 ? 1.0 : -1.0) * (-ob) * rcp_refined(oa - ob);
        accQ += crf * (p2 ? 1.0 : -1.0) * (-od) * rcp_refined(oc - od);
        s_add(P.S, e, p4 ? 1 : -1);
        accM += (p2 ? 1.0 : -1.0) * Q.suf[f];
        accK += f < kq ? (p2 ? 1.0 : -1.0) : 0.0;
    }
}

// One sweep unit per lane: Q edge f held in registers against the 8 edges of
// P chunk cp (entry = cp << USHIFT | f).  Crossing lanes only append
// (e << 16 | f) to the wavefront's crossing buffer, which is flushed before
// it can overflow.
template <int USHIFT>
__device__ __forceinline__ void sweep_units(RingLds P, RingLds Q, int entry, int lane, uint32_t *xbuf,
                                            int &xcount, int kq, double &accP, double &accQ, double &accM,
                                            double &accK)
{
    const int cp = entry >> USHIFT, f = entry & ((1 << USHIFT) - 1);
    const int2 c = Q.v[f], d = Q.v[f + 1];
    const double cx = (double)c.x, cy = (double)c.y;
    const double fx = (double)(d.x - c.x), fy = (double)(d.y - c.y);
    const int mf = q_edge_class(d.x - c.x, d.y - c.y);
    const int e0 = 8 * cp;
    // the chunk's 9 vertices up front: the crossing-buffer stores in the
    // sweep would otherwise keep these loads from being issued early
    int2 pv[9];
#pragma unroll
    for (int i = 0; i < 9; i++) pv[i] = P.v[e0 + i];
    double ax = (double)pv[0].x, ay = (double)pv[0].y;
    double rx = cx - ax, ry = cy - ay;
    // orient(c, d, a) of the chunk's first vertex; each edge's end value
    // orient(c, d, b) = that - X is the next edge's start value (all exact
    // integers below 2^53, so carrying it equals recomputing it)
    double oa = __fma_rn(fy, rx, -(fx * ry));
#pragma unroll
    for (int i = 0; i < 8; i++) {
        const int2 b = pv[i + 1];
        const double bx = (double)b.x, by = (double)b.y;
        const double ex = bx - ax, ey = by - ay;
        const double thr = p_edge_threshold(ex, ey);
        const double oc = __fma_rn(ex, ry, -(ey * rx));
        const double X = __fma_rn(ex, fy, -(ey * fx));
        const double od = oc + X, ob = oa - X;
        const bool p1 = oc > thr, p2 = od > thr;
        const bool p3 = __builtin_amdgcn_class(oa, mf), p4 = __builtin_amdgcn_class(ob, mf);
        const bool cross = (p1 != p2) & (p3 != p4);
        const uint64_t cm = __ballot(cross);
        if (cross) {
            const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(cm >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((uint32_t)cm, 0u));
            xbuf[xcount + rank] = ((uint32_t)(e0 + i) << 16) | (uint32_t)f;
        }
        xcount += __popcll(cm);
        if (xcount > kCrossCap - 64) {
            wave_lds_sync();
            flush_crossings(P, Q, xbuf, xcount, lane, kq, accP, accQ, accM, accK);
            wave_lds_sync();
            xcount = 0;
        }
        ax = bx; ay = by;
        rx = cx - bx; ry = cy - by;
        oa = ob;
    }
}

// Expand up to 16 listed tiles (lane = tile slot x Q edge j, two slots per
// lane) into sweep units, keeping the (P chunk, Q edge) pairs whose boxes
// touch: a crossing needs the Q edge's box to meet the box of the P edge it
// crosses, inside the chunk's.
template <typename UnitT, int USHIFT>
__device__ __forceinline__ void expand_tiles(RingLds P, RingLds Q, int m, const uint16_t *tiles, int head,
                                             int count, int lane, UnitT *units, int &utail)
{
    bool keep[2];
    int entry[2];
#pragma unroll
    for (int h = 0; h < 2; h++) {
        // branch-free (see the batch loop); slots past `count` read entry 0
        const int slot = (lane >> 3) + 8 * h;
        const bool live = slot < count;
        const int t = (int)tiles[(head + (live ? slot : 0)) & (kListCap - 1)];
        const int cp = t >> 8, cq = t & 0xff;
        const int f = 8 * cq + (lane & 7);
        const int2 c = Q.v[f], d = Q.v[f + 1];
        const int4 bp = P.box[cp];
        const bool apart = (max(c.x, d.x) < bp.x) | (bp.z < min(c.x, d.x)) | (max(c.y, d.y) < bp.y) |
                           (bp.w < min(c.y, d.y));
        keep[h] = live & (f < m) & !apart;
        entry[h] = (cp << USHIFT) | f;
    }
    const uint64_t mk0 = __ballot(keep[0]), mk1 = __ballot(keep[1]);
    const int r0 = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mk0 >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mk0, 0u));
    const int r1 = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mk1 >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mk1, 0u));
    const int c0 = __popcll(mk0);
    if (keep[0]) units[(utail + r0) & (kUnitCap - 1)] = (UnitT)entry[0];
    if (keep[1]) units[(utail + c0 + r1) & (kUnitCap - 1)] = (UnitT)entry[1];
    utail += c0 + __popcll(mk1);
}

// The crossings of P's edges with the m edges of Q staged in LDS (a whole
// ring, or a window of a longer one) added to the four sums; kq is the
// anchor's index relative to the staged edges.  Sweep units are (P chunk,
// Q edge) entries packed as cp << USHIFT | f in UnitT (16 bits up to 512
// edges a side, 32 beyond).
template <typename UnitT, int USHIFT>
__device__ void tiled_accumulate(RingLds P, int n, RingLds Q, int m, int kq, int lane, uint16_t *list,
                                 UnitT *units, uint32_t *xbuf, unsigned long long *swept, double &accP,
                                 double &accQ, double &accM, double &accK)
{
    const int ncp = (n + 7) >> 3, ncq = (m + 7) >> 3;
    const int total = ncp * ncq;
    // idx -> (idx / ncq, idx % ncq) without an integer division: the float
    // quotient of idx + 1/2 is at least 1/(2 ncq) >= 1/256 away from an
    // integer (ncq <= 128) while its rounding error is below 2^-15 (the
    // quotient is below ncp <= 128 and carries two roundings of 2^-24).
    const float rq = 1.0f / (float)ncq;
    int head = 0, tail = 0, uhead = 0, utail = 0, xcount = 0;
    // two batches of 64 chunk pairs per round trip through the tile list
    for (int base = 0; base < total; base += 128) {
        int en[2];
        bool ov[2];
        // branch-free: whole boxes loaded at once, bitwise tests (no
        // short-circuit chains of dependent LDS reads)
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int i0 = base + 64 * h + lane;
            const bool live = i0 < total;
            const int idx = live ? i0 : 0;
            const int cp = (int)(((float)idx + 0.5f) * rq);
            const int cq = idx - cp * ncq;
            const int4 bp = P.box[cp], bq = Q.box[cq];
            const bool apart = (bp.z < bq.x) | (bq.z < bp.x) | (bp.w < bq.y) | (bq.w < bp.y);
            ov[h] = live & !apart;
            en[h] = (cp << 8) | cq;
        }
        const uint64_t mk0 = __ballot(ov[0]), mk1 = __ballot(ov[1]);
        const int r0 = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mk0 >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mk0, 0u));
        const int r1 = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mk1 >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mk1, 0u));
        const int c0 = __popcll(mk0);
        if (ov[0]) list[(tail + r0) & (kListCap - 1)] = (uint16_t)en[0];
        if (ov[1]) list[(tail + c0 + r1) & (kListCap - 1)] = (uint16_t)en[1];
        tail += c0 + __popcll(mk1);
        const bool last = base + 128 >= total;
        while (tail - head >= 16 || (last && tail > head)) {
            wave_lds_sync();
            const int cnt = min(16, tail - head);
            expand_tiles<UnitT, USHIFT>(P, Q, m, list, head, cnt, lane, units, utail);
            head += cnt;
            wave_lds_sync();
            while (utail - uhead >= 64) {
                sweep_units<USHIFT>(P, Q, (int)units[(uhead + lane) & (kUnitCap - 1)], lane, xbuf, xcount, kq, accP,
                                    accQ, accM, accK);
                uhead += 64;
            }
        }
    }
    if (utail > uhead) {
        // partial sweep: idle lanes take a padding edge of Q (zero length)
        const int k = utail - uhead;
        const int entry = lane < k ? (int)units[(uhead + lane) & (kUnitCap - 1)] : 8 * ncq;
        sweep_units<USHIFT>(P, Q, entry, lane, xbuf, xcount, kq, accP, accQ, accM, accK);
    }
    if (xcount > 0) {
        wave_lds_sync();
        flush_crossings(P, Q, xbuf, xcount, lane, kq, accP, accQ, accM, accK);
    }
    *swept += 8ull * (unsigned long long)utail;   // edge pairs tested (idle lanes excluded)
}

// 2 A(P n Q) from the crossing sums and the anchors' memberships (wkp at
// P's vertex kp, wkq at Q's vertex kq).
__device__ double tiled_finish(RingLds P, int n, int sp, int sq, int64_t a2p, int64_t a2q, int kp, int wkp,
                               int wkq, int lane, double accP, double accQ, double accM, double accK)
{
    // make the crossing sums visible to the whole wavefront
    wave_lds_sync();
    // 2 A = sp * (mp + sq * accP) + sq * (mq + sp * accQ) with
    //   mp = w0p * A2P + sq * T,  w0p = w(kp) - sq * pre_P(kp),
    //   mq = w0q * A2Q + sp * accM,  w0q = w(kq) - sp * pre_Q(kq), pre_Q(kq) = sum of accK
    int K;
    const double T = membership_term_p(P, n, kp, lane, K);
    const double tot = (double)(sp * sq) * (T + accP + accQ + accM - (double)a2q * accK);
    return wave_sum(tot) + (double)(sp * (wkp - sq * K)) * (double)a2p + (double)(sq * wkq) * (double)a2q;
}

// kp / kq: a vertex of P outside Q (and of Q outside P), or -1; the ring's
// memberships are anchored there (membership 0), else at vertex 0 by a
// crossing-number pass.
template <typename UnitT, int USHIFT>
__device__ double tiled_pair(RingLds P, int n, RingLds Q, int m, int sp, int sq, int64_t a2p, int64_t a2q,
                             int kp, int kq, int lane, uint16_t *list, UnitT *units, uint32_t *xbuf,
                             unsigned long long *swept)
{
    int wkp = 0, wkq = 0;
    if (kp < 0 || kq < 0) {
        int w0p, w0q;
        member_starts(P, n, Q, m, lane, kp < 0, kq < 0, w0p, w0q);
        if (kp < 0) { kp = 0; wkp = w0p; }
        if (kq < 0) { kq = 0; wkq = w0q; }
    }
    double accP = 0.0, accQ = 0.0, accM = 0.0, accK = 0.0;
    tiled_accumulate<UnitT, USHIFT>(P, n, Q, m, kq, lane, list, units, xbuf, swept, accP, accQ, accM, accK);
    return tiled_finish(P, n, sp, sq, a2p, a2q, kp, wkp, wkq, lane, accP, accQ, accM, accK);
}

// A vertex of Q strictly outside P's MBR among Q's extreme vertices, or -1.
__device__ __forceinline__ int anchor_q(const int32_t *qb, const int32_t *pb, const int *ext)
{
    if (qb[0] < pb[0]) return ext[0];
    if (qb[2] > pb[2]) return ext[1];
    if (qb[1] < pb[1]) return ext[2];
    if (qb[3] > pb[3]) return ext[3];
    return -1;
}

// One workgroup per query: Q staged once, wavefronts take its candidates.
// Heavy pairs: a pair on the general form with n m >= kHeavyMin edge pairs
// would keep one wavefront busy for a long serial run (milliseconds for a few
// thousand edges a side), so it is deferred: the wavefront records it, and a
// second launch splits each side's edges into kHeavySlices strided slices,
// one wavefront each, whose partial sums a third launch adds in a fixed
// order.  Up to kHeavyCap pairs per call are deferred; the rest run in place.
constexpr int kHeavySlices = 64;
constexpr int kHeavyCap = 8192;
constexpr int64_t kHeavyMin = 1 << 17;

struct HeavyPair {
    int64_t c;            // candidate slot of the result
    int64_t pa, qa;       // first vertex of P (data) and of Q (query)
    int64_t ox, oy;       // local origin of the pair
    int64_t a2p, a2q;     // exact doubled areas
    int32_t n, m;
    int32_t qmbr[4], pm[4];
    int32_t wide;
    int32_t pad;
};

constexpr int kStatSlots = 64;   // work counters spread over slots, folded at the end

// Wide tiled pairs: a pair with a polygon beyond kTileCap edges but none
// beyond kWideCap (and coordinate spans below 2^26) would take the general
// form, which tests all n m edge pairs; it is deferred instead, and a second
// launch runs the tiled form on it with one wavefront staging both rings.
// Up to kWideListCap pairs per call are deferred; the rest run in place.
constexpr int kWideCap = 1024;
constexpr int kWideRing = kWideCap + 16;   // ring vertices incl. padding
constexpr int kWideListCap = 1 << 20;

// A pair that spans more than two window pairs (of kWideCap edges a side) is
// split into units of one wavefront each: P windows of plen edges (128 for a
// staged polygon of kSplitFineP edges or more, else the shortest of 256, 512
// and kWideCap that keeps the units within kMultiUnits), each walking Q's
// windows, or, when Q has more than two windows, each (P window, Q window)
// alone.  k_wide_meta finds the pair's own quantities once (areas, anchors,
// Q's window carries), every unit writes its partial sums, all linear in the
// crossing signs, and k_refine_multi_finish adds them in window order.  Up
// to kMultiCap such pairs per call (the rest take all their windows on one
// wavefront).
constexpr int kMultiCap = 4096;
constexpr int kMultiUnits = 512;
constexpr int kSplitFineP = 4096;

struct SplitShape {
    int plen;             // P window length of the units
    int qs;               // units per P window (Q windows, or 1)
    int units;            // 1: the pair is not split
};

// The split of a pair whose staged polygon (P's role) has np edges and the
// other nq; deterministic, so the wide kernel and the finish recompute it.
__device__ __forceinline__ int split_plen(int np, int qs)
{
    return (np >= kSplitFineP && ((np + 127) >> 7) * qs <= kMultiUnits) ? 128
         : ((np + 255) >> 8) * qs <= kMultiUnits ? 256
         : ((np + 511) >> 9) * qs <= kMultiUnits ? 512
         : ((np + 1023) >> 10) * qs <= kMultiUnits ? 1024 : 0;
}

__device__ __forceinline__ SplitShape split_shape(int np, int nq)
{
    const int npw = (np + kWideCap - 1) / kWideCap, nqw = (nq + kWideCap - 1) / kWideCap;
    if (npw * nqw <= 2) return {kWideCap, 1, 1};
    int qs = nqw > 2 ? nqw : 1;
    int plen = split_plen(np, qs);
    if (plen == 0 && qs > 1) plen = split_plen(np, qs = 1);
    if (plen == 0) return {kWideCap, 1, 1};
    return {plen, qs, (np + plen - 1) / plen * qs};
}

struct WidePair {
    int64_t c;            // candidate slot of the result (-1: an unused entry)
    int64_t pa;           // first vertex of the data polygon
    int32_t n;            // its vertex count
    int32_t q;            // query index
    int16_t pw;           // P window of a split pair, or -1 for all windows
    int16_t qw;           // Q window of a pair split on both sides, or -1 for all
    int32_t slot;         // the split pair's slot, or -1
};

struct MultiPair {
    int64_t c;            // candidate slot (-1: the pair was not deferred)
    int64_t pa;
    int32_t n, q, units;
    int32_t first;        // list position of its first unit (k_wide_meta writes the units there)
    // the pair's own quantities, written by k_wide_meta for its units and
    // the finish (P and Q in k_refine_wide's roles)
    int64_t a2p, a2q;     // exact doubled areas
    int32_t kp, kq;       // anchors (0 where a membership pass stands in)
    int32_t wkp, wkq;     // memberships of P's vertex 0 in Q, of Q's vertex 0 in P (0 when anchored)
};

struct MultiUnit {
    double part;          // sp sq x (P window's membership term + crossing sums), summed over the wavefront
    double cr;            // sum of the P window's cross products (first Q window's unit only)
    int32_t stot;         // sum of the window's crossing signs
    int32_t kloc;         // exclusive prefix of crossing signs at the anchor, if in this window
    int64_t qpre;         // in: Q's cross-product sum before the unit's Q window (k_wide_meta)
};

struct HeavyWs {
    int32_t *count;       // [0] heavy pairs, [1] wide list entries recorded, [2] split pairs, [4] split
                          // units appended after the recorded entries (each may exceed its cap: the
                          // excess runs in place or whole), [3] wide entries taken
    HeavyPair *pairs;     // [kHeavyCap]
    double *partial;      // [kHeavyCap][2][kHeavySlices]
    unsigned long long *stat_slots;   // [kStatSlots][4]
    WidePair *wide;       // [kWideListCap]
    MultiPair *multi;     // [kMultiCap]
    MultiUnit *units;     // [kMultiCap][kMultiUnits]
};

// Records a pair for k_refine_wide as one list entry (k_expand splits the
// ones split_shape splits).  False when the list is full.
__device__ bool defer_wide(const HeavyWs &hw, int64_t c, int64_t pa, int n, int32_t q, int lane)
{
    const int slot = __builtin_amdgcn_readfirstlane(lane == 0 ? atomicAdd(hw.count + 1, 1) : 0);
    if (slot >= kWideListCap) return false;
    if (lane == 0) {
        WidePair &w = hw.wide[slot];
        w.c = c; w.pa = pa; w.n = n; w.q = q; w.pw = -1; w.qw = -1; w.slot = -1;
    }
    return true;
}

__device__ __forceinline__ double jaccard_of(double inter2, int64_t a2p, int64_t a2q)
{
    const double inter = 0.5 * inter2;
    const double ap = 0.5 * fabs((double)a2p), aq = 0.5 * fabs((double)a2q);
    const double u = ap + aq - inter;
    return u > 0 ? inter / u : 0.0;
}

__global__ __launch_bounds__(256, 4) void k_refine(const int32_t *__restrict__ dxy,
                                                const int64_t *__restrict__ doff,
                                                const int32_t *__restrict__ qxy,
                                                const int64_t *__restrict__ qoff,
                                                const int64_t *__restrict__ cand_off,
                                                const int32_t *__restrict__ cand_ids,
                                                double *__restrict__ cand_j,
                                                unsigned long long *__restrict__ stats,
                                                int slices, HeavyWs hw)
{
    __shared__ int2 sQv[kRingLds];
    __shared__ int4 sQbox[kTileCap / 8];
    __shared__ int2 sPv[kWavesPerBlock][kRingLds];
    __shared__ int4 sPbox[kWavesPerBlock][kTileCap / 8];
    __shared__ uint32_t sPS[kWavesPerBlock][kTileCap / 2];
    __shared__ double sQsuf[kTileCap];
    __shared__ uint16_t sList[kWavesPerBlock][kListCap];
    __shared__ uint16_t sUnits[kWavesPerBlock][kUnitCap];
    __shared__ uint32_t sCross[kWavesPerBlock][kCrossCap];
    __shared__ int32_t sQmbr[4];
    __shared__ long long sQa2;
    __shared__ int sQext[4];

    // `slices` workgroups share a query (small batches): slice s's wavefronts
    // take candidates s * waves + wave, stepping by slices * waves
    const int64_t q = blockIdx.x / slices;
    const int slice = (int)(blockIdx.x % slices);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t qa = qoff[q];
    const int m = (int)(qoff[q + 1] - qa);
    const int32_t *Qg = qxy + 2 * qa;
    const int64_t c0 = cand_off[q], c1 = cand_off[q + 1];
    if (c0 == c1) return;
    if (m < 3) {
        for (int64_t c = c0 + (int64_t)slice * blockDim.x + tid; c < c1; c += (int64_t)slices * blockDim.x)
            cand_j[c] = 0.0;
        return;
    }
    const int64_t ox = Qg[0], oy = Qg[1];
    const bool q_tiled = m <= kTileCap;
    if (wave == 0) {
        int32_t qm[4];
        poly_mbr(Qg, m, lane, qm);
        const int64_t a2 = poly_area2(Qg, m, ox, oy, lane);
        if (lane == 0) {
            sQmbr[0] = qm[0]; sQmbr[1] = qm[1]; sQmbr[2] = qm[2]; sQmbr[3] = qm[3];
            sQa2 = a2;
        }
    }
    if (q_tiled) {
        // Q padded by one extra chunk: the all-padding chunk ncq fills empty
        // slots of a partial tile group
        const int qpad = 8 * ((m + 7) >> 3) + 8;
        RingLds Qs{sQv, sQbox, nullptr, sQsuf};
        stage_ring(Qg, m, qpad + 1, ox, oy, Qs, tid, blockDim.x);
        __syncthreads();
        chunk_boxes(Qs, m, tid, blockDim.x);
        __syncthreads();
        if (wave == 0) {
            q_suffix_sums(Qs, m, sQa2, lane);
            const int4 rb = make_int4((int)((int64_t)sQmbr[0] - ox), (int)((int64_t)sQmbr[1] - oy),
                                      (int)((int64_t)sQmbr[2] - ox), (int)((int64_t)sQmbr[3] - oy));
            q_extremes(Qs, m, rb, lane, sQext);
        }
    }
    __syncthreads();
    const int32_t qmbr[4] = {sQmbr[0], sQmbr[1], sQmbr[2], sQmbr[3]};
    const int qext[4] = {sQext[0], sQext[1], sQext[2], sQext[3]};
    const int64_t a2q = sQa2;
    const int nwaves = (int)(blockDim.x >> 6) * slices;   // wavefronts on this query
    unsigned long long st_tiled = 0, st_swept = 0, st_general = 0, st_disjoint = 0;
    // Candidate metadata is fetched ahead: the id two candidates on and the
    // vertex range of the next one, so their latency hides behind this pair.
    int64_t c = c0 + (int64_t)slice * (blockDim.x >> 6) + wave;
    int32_t p_ahead = c < c1 ? cand_ids[c] : 0;
    int64_t pa_next = 0, pe_next = 0;
    if (c < c1) { pa_next = doff[p_ahead]; pe_next = doff[p_ahead + 1]; }
    p_ahead = (c + nwaves < c1) ? cand_ids[c + nwaves] : 0;
    // the data polygon's first 128 vertices are fetched one candidate ahead
    RingPrefetch pf_next;
    if (c < c1 && pe_next - pa_next >= 3) prefetch_ring(dxy + 2 * pa_next, (int)(pe_next - pa_next), lane, pf_next);
    for (; c < c1; c += nwaves) {
        const int64_t pa = pa_next;
        const int n = (int)(pe_next - pa_next);
        const RingPrefetch pf = pf_next;
        if (c + nwaves < c1) { pa_next = doff[p_ahead]; pe_next = doff[p_ahead + 1]; }
        p_ahead = (c + 2 * nwaves < c1) ? cand_ids[c + 2 * nwaves] : 0;
        const int32_t *Pg = dxy + 2 * pa;
        double J = 0.0;
        bool deferred = false;
        int slot = 0;
        const bool valid = n >= 3 && a2q != 0;
        const bool tiled_size = valid && q_tiled && n <= kTileCap;
        RingLds Ps{sPv[wave], sPbox[wave], sPS[wave], nullptr};
        RingLds Qs{sQv, sQbox, nullptr, sQsuf};
        const int ppad = 8 * ((n + 7) >> 3);
        int32_t pm[4] = {0, 0, 0, 0};
        // staging records the MBR of the absolute coordinates, so a wide
        // pair (whose relative coordinates do not fit) is still detected
        int kp = -1;
        int64_t a2p_staged = 0;
        if (tiled_size) stage_ring_mbr(Pg, n, ppad + 1, ox, oy, Ps, lane, qmbr, pf, pm, a2p_staged, kp);
        else if (valid) poly_mbr(Pg, n, lane, pm);
        // the next candidate's vertices, whatever this pair turns out to need
        if (c + nwaves < c1 && pe_next - pa_next >= 3)
            prefetch_ring(dxy + 2 * pa_next, (int)(pe_next - pa_next), lane, pf_next);
        if (valid) {
            const bool disjoint = pm[2] <= qmbr[0] || qmbr[2] <= pm[0] || pm[3] <= qmbr[1] || qmbr[3] <= pm[1];
            st_disjoint += disjoint;
            if (!disjoint) {
                const int64_t span = max(max((int64_t)pm[2], (int64_t)qmbr[2]) - min((int64_t)pm[0], (int64_t)qmbr[0]),
                                         max((int64_t)pm[3], (int64_t)qmbr[3]) - min((int64_t)pm[1], (int64_t)qmbr[1]));
                const bool wide = span >= (1ll << 26);
                double inter2 = 0.0;
                int64_t a2p = 0;
                if (!wide && tiled_size) {
                    for (int i = lane; i < (n + 1) >> 1; i += 64) Ps.S[i] = kSBias;
                    wave_lds_sync();
                    chunk_boxes_p<kTileCap / 8>(Ps, n, lane);
                    a2p = a2p_staged;
                    wave_lds_sync();
                    if (a2p != 0)
                        inter2 = tiled_pair<uint16_t, 10>(Ps, n, Qs, m, a2p > 0 ? 1 : -1, a2q > 0 ? 1 : -1, a2p,
                                                          a2q, kp, anchor_q(qmbr, pm, qext), lane,
                                                          sList[wave], sUnits[wave], sCross[wave], &st_swept);
                    st_tiled++;
                } else if (hw.count && !wide && defer_wide(hw, c, pa, n, (int32_t)q, lane)) {
                    // tiled form on wavefronts of the next launch
                    deferred = true;
                } else if (hw.count && (int64_t)n * m >= kHeavyMin &&
                           (a2p = poly_area2(Pg, n, ox, oy, lane)) != 0 &&
                           (slot = __builtin_amdgcn_readfirstlane(lane == 0 ? atomicAdd(hw.count, 1) : 0)) <
                               kHeavyCap) {
                    // split over many wavefronts by the next launches
                    st_general += 2ull * (unsigned long long)n * (unsigned long long)m;
                    if (lane == 0) {
                        HeavyPair &h = hw.pairs[slot];
                        h.c = c; h.pa = pa; h.qa = qa; h.ox = ox; h.oy = oy; h.a2p = a2p; h.a2q = a2q;
                        h.n = n; h.m = m; h.wide = wide; h.pad = 0;
                        for (int i = 0; i < 4; i++) { h.qmbr[i] = qmbr[i]; h.pm[i] = pm[i]; }
                    }
                    deferred = true;
                } else {
                    st_general += 2ull * (unsigned long long)n * (unsigned long long)m;
                    PairIn in;
                    in.P = Pg; in.n = n; in.Q = Qg; in.m = m; in.ox = ox; in.oy = oy;
                    in.qmbr[0] = qmbr[0]; in.qmbr[1] = qmbr[1]; in.qmbr[2] = qmbr[2]; in.qmbr[3] = qmbr[3];
                    in.sq = a2q > 0 ? 1 : -1;
                    double sa, sb;
                    if (!wide) edges_in_other_P<false>(in, lane, sa, a2p);
                    else edges_in_other_P<true>(in, lane, sa, a2p);
                    a2p = wave_sum_i64(a2p);
                    in.sp = a2p > 0 ? 1 : -1;
                    if (a2p != 0) {
                        int64_t unused;
                        if (!wide) edges_in_other_Q<false>(in, pm, lane, sb, unused);
                        else edges_in_other_Q<true>(in, pm, lane, sb, unused);
                        inter2 = wave_sum(in.sp * sa) + wave_sum(in.sq * sb);
                    }
                }
                if (a2p != 0) J = jaccard_of(inter2, a2p, a2q);
            }
        }
        if (lane == 0 && !deferred) cand_j[c] = J;
    }
    if (stats) {
        // one sum per workgroup, added to one of kStatSlots slots when the
        // workspace has them (atomics of every wavefront on four words
        // serialise at the cache), nonzero counts only
        __shared__ unsigned long long sStat[kWavesPerBlock][4];
        if (lane == 0) {
            sStat[wave][0] = st_tiled; sStat[wave][1] = st_swept;
            sStat[wave][2] = st_general; sStat[wave][3] = st_disjoint;
        }
        __syncthreads();
        if (tid < 4) {
            unsigned long long v = 0;
            for (int w = 0; w < (int)(blockDim.x >> 6); w++) v += sStat[w][tid];
            if (v) {
                if (hw.stat_slots) atomicAdd(hw.stat_slots + (blockIdx.x % kStatSlots) * 4 + tid, v);
                else atomicAdd(stats + tid, v);
            }
        }
    }
}

// Vertex i of an m-vertex ring in global memory, relative to the origin.
__device__ __forceinline__ int2 ring_vertex(const int32_t *V, int m, int i, int64_t ox, int64_t oy)
{
    const int k = i < m ? i : i - m;
    return make_int2((int)((int64_t)V[2 * k] - ox), (int)((int64_t)V[2 * k + 1] - oy));
}

// The passes below read a ring in global memory with one wavefront and
// kPassU vertices a lane in flight: a long ring costs a few round trips to
// memory rather than one per 64 vertices.
constexpr int kPassU = 8;

// One pass: the ring's MBR (absolute coordinates), twice its signed area
// about the origin (as poly_area2) and the sum of the cross products of its
// edges before edge `end`, the suffix-sum carry into a window that starts
// there (exact in 64-bit integers).
__device__ void ring_sums_global(const int32_t *V, int m, int64_t ox, int64_t oy, int end, int lane,
                                 int32_t *mbr, int64_t &a2, int64_t &pre)
{
    const int2 *W = reinterpret_cast<const int2 *>(V);
    int32_t mnx = INT32_MAX, mny = INT32_MAX, mxx = INT32_MIN, mxy = INT32_MIN;
    int64_t a = 0, p = 0;
    for (int base = 0; base < m; base += 64 * kPassU) {
        int2 v[kPassU], w[kPassU];
#pragma unroll
        for (int k = 0; k < kPassU; k++) {
            const int i = min(base + 64 * k + lane, m - 1);
            v[k] = W[i];
            w[k] = W[i + 1 == m ? 0 : i + 1];
        }
#pragma unroll
        for (int k = 0; k < kPassU; k++) {
            const int i = base + 64 * k + lane;
            if (i < m) {
                mnx = min(mnx, v[k].x); mxx = max(mxx, v[k].x);
                mny = min(mny, v[k].y); mxy = max(mxy, v[k].y);
                const int64_t ax = (int64_t)v[k].x - ox, ay = (int64_t)v[k].y - oy;
                const int64_t bx = (int64_t)w[k].x - ox, by = (int64_t)w[k].y - oy;
                const int64_t c = (int64_t)((__int128)ax * by - (__int128)bx * ay);
                a += c;
                p += i < end ? c : 0;
            }
        }
    }
    mbr[0] = wmin(mnx); mbr[1] = wmin(mny); mbr[2] = wmax(mxx); mbr[3] = wmax(mxy);
    a2 = wave_sum_i64(a);
    pre = wave_sum_i64(p);
}

// Membership of point a + sh*delta (relative coordinates) in a ring read from
// global memory: the half-open crossing rule of member_edge over every edge.
__device__ int member_point_global(const int32_t *V, int m, int64_t ox, int64_t oy, int2 a, int sh, int lane)
{
    bool odd = false;
    for (int base = 0; base < m; base += 64 * kPassU) {
        int2 cv[kPassU], dv[kPassU];
#pragma unroll
        for (int k = 0; k < kPassU; k++) {
            const int e = min(base + 64 * k + lane, m - 1);
            cv[k] = ring_vertex(V, m, e, ox, oy);
            dv[k] = ring_vertex(V, m, e + 1, ox, oy);
        }
#pragma unroll
        for (int k = 0; k < kPassU; k++) odd ^= (base + 64 * k + lane < m) & flips_parity(cv[k], dv[k], a, sh);
    }
    return __popcll(__ballot(odd)) & 1;
}

// Indices of a leftmost, a rightmost, a lowest and a highest vertex of a ring
// in global memory (mbr: its absolute MBR), as q_extremes.
__device__ void extremes_global(const int32_t *V, int m, const int32_t *mbr, int lane, int *ext)
{
    const int2 *W = reinterpret_cast<const int2 *>(V);
    int k0 = -1, k1 = -1, k2 = -1, k3 = -1;
    for (int base = 0; base < m; base += 64 * kPassU) {
        int2 v[kPassU];
#pragma unroll
        for (int k = 0; k < kPassU; k++) v[k] = W[min(base + 64 * k + lane, m - 1)];
#pragma unroll
        for (int k = 0; k < kPassU; k++) {
            const int b = base + 64 * k;
            const bool live = b + lane < m;
            const uint64_t b0 = __ballot(live & (v[k].x == mbr[0])), b1 = __ballot(live & (v[k].x == mbr[2]));
            const uint64_t b2 = __ballot(live & (v[k].y == mbr[1])), b3 = __ballot(live & (v[k].y == mbr[3]));
            if (k0 < 0 && b0 != 0) k0 = b + __builtin_ctzll(b0);
            if (k1 < 0 && b1 != 0) k1 = b + __builtin_ctzll(b1);
            if (k2 < 0 && b2 != 0) k2 = b + __builtin_ctzll(b2);
            if (k3 < 0 && b3 != 0) k3 = b + __builtin_ctzll(b3);
        }
    }
    ext[0] = k0; ext[1] = k1; ext[2] = k2; ext[3] = k3;
}

// Edges [w0, w0 + len) of an m-vertex ring staged as a chain: entry i holds
// vertex w0 + i for i <= len (vertex m is vertex 0), entries beyond len repeat
// vertex w0 + len, so edges from len on have zero length and never cross.
__device__ void stage_window(const int32_t *V, int m, int w0, int len, int pad_to, int64_t ox, int64_t oy,
                             RingLds R, int lane)
{
    for (int base = 0; base < pad_to; base += 64 * kPassU) {
        int2 v[kPassU];
#pragma unroll
        for (int k = 0; k < kPassU; k++) v[k] = ring_vertex(V, m, w0 + min(base + 64 * k + lane, len), ox, oy);
#pragma unroll
        for (int k = 0; k < kPassU; k++)
            if (base + 64 * k + lane < pad_to) R.v[base + 64 * k + lane] = v[k];
    }
}

// First vertex of a ring in global memory strictly outside the box b, or -1.
__device__ int first_outside_global(const int32_t *V, int n, const int32_t *b, int lane)
{
    const int2 *W = reinterpret_cast<const int2 *>(V);
    for (int base = 0; base < n; base += 64 * kPassU) {
        int2 v[kPassU];
#pragma unroll
        for (int k = 0; k < kPassU; k++) v[k] = W[min(base + 64 * k + lane, n - 1)];
#pragma unroll
        for (int k = 0; k < kPassU; k++) {
            const int x = v[k].x, y = v[k].y;
            const bool live = base + 64 * k + lane < n;
            const uint64_t mk = __ballot(live & ((x < b[0]) | (x > b[2]) | (y < b[1]) | (y > b[3])));
            if (mk != 0) return base + 64 * k + __builtin_ctzll(mk);
        }
    }
    return -1;
}

// The quantities of a split pair that all its units share, found once per
// pair by one workgroup (a unit used to find them itself, in four passes over
// both whole rings read from memory, and the finish again): both rings' MBRs
// and exact doubled areas, the anchors (P's first vertex strictly outside
// Q's MBR, Q's extreme vertex outside P's MBR), the memberships of the ring
// starts where there is no anchor, and Q's cross-product sum before each Q
// window, written into the units' slots as their suffix-sum carry.  All are
// exact integers, the same as the per-unit passes gave.  Rings of up to
// kMetaThreads x kMetaU vertices take one round trip to memory a pass.  The
// workgroup also writes the pair's unit entries at the list positions
// k_expand reserved (one thread each, where a thread of k_expand wrote them
// all in turn).
constexpr int kMetaThreads = 1024;
constexpr int kMetaU = 8;

__global__ __launch_bounds__(kMetaThreads) void k_wide_meta(const int32_t *__restrict__ dxy,
                                                          const int32_t *__restrict__ qxy,
                                                          const int64_t *__restrict__ qoff, HeavyWs hw)
{
    __shared__ unsigned long long sWin[kMultiUnits];   // Q's cross products per window of kWideCap edges
    __shared__ unsigned long long sA[2];               // doubled areas of Q and P
    __shared__ int32_t sBox[8];                        // MBRs of Q and P: min x, min y, max x, max y
    __shared__ int32_t sIdx[5];                        // Q's extreme vertices, P's first vertex outside
    __shared__ int32_t sOdd[2];                        // crossings of the two membership passes
    const int tid = threadIdx.x, lane = tid & 63;
    const int64_t count = min((int64_t)hw.count[2], (int64_t)kMultiCap);
    for (int64_t s = blockIdx.x; s < count; s += gridDim.x) {
        const MultiPair mp = hw.multi[s];
        if (mp.c < 0) continue;
        // the roles of k_refine_wide
        const int64_t qa = qoff[mp.q];
        const int mq = (int)(qoff[mp.q + 1] - qa);
        const bool swap = mp.n > kWideCap && mp.n > mq;
        const int2 *PW = reinterpret_cast<const int2 *>(swap ? qxy + 2 * qa : dxy + 2 * mp.pa);
        const int2 *QW = reinterpret_cast<const int2 *>(swap ? dxy + 2 * mp.pa : qxy + 2 * qa);
        const int n = swap ? mq : mp.n, m = swap ? mp.n : mq;
        const int2 o = QW[0];
        const SplitShape sh = split_shape(n, m);
        const int len = max(n, m);
        for (int i = tid; i < kMultiUnits; i += kMetaThreads) sWin[i] = 0;
        if (tid < 2) { sA[tid] = 0; sOdd[tid] = 0; }
        if (tid < 8) sBox[tid] = (tid & 3) < 2 ? INT32_MAX : INT32_MIN;
        if (tid < 5) sIdx[tid] = INT32_MAX;
        __syncthreads();
        // MBRs, areas and Q's window sums (a wavefront's 64 edges lie in one window)
        {
            int32_t b[8] = {INT32_MAX, INT32_MAX, INT32_MIN, INT32_MIN, INT32_MAX, INT32_MAX, INT32_MIN, INT32_MIN};
            int64_t aq = 0, ap = 0;
            for (int base = 0; base < len; base += kMetaThreads * kMetaU) {
                int2 qv[kMetaU], qw[kMetaU], pv[kMetaU], pw[kMetaU];
#pragma unroll
                for (int k = 0; k < kMetaU; k++) {
                    const int i = base + k * kMetaThreads + tid;
                    const int iq = min(i, m - 1), ip = min(i, n - 1);
                    qv[k] = QW[iq]; qw[k] = QW[iq + 1 == m ? 0 : iq + 1];
                    pv[k] = PW[ip]; pw[k] = PW[ip + 1 == n ? 0 : ip + 1];
                }
#pragma unroll
                for (int k = 0; k < kMetaU; k++) {
                    const int i = base + k * kMetaThreads + tid;
                    int64_t cq = 0;
                    if (i < m) {
                        b[0] = min(b[0], qv[k].x); b[1] = min(b[1], qv[k].y);
                        b[2] = max(b[2], qv[k].x); b[3] = max(b[3], qv[k].y);
                        cq = (int64_t)(qv[k].x - o.x) * (qw[k].y - o.y) - (int64_t)(qw[k].x - o.x) * (qv[k].y - o.y);
                    }
                    if (i < n) {
                        b[4] = min(b[4], pv[k].x); b[5] = min(b[5], pv[k].y);
                        b[6] = max(b[6], pv[k].x); b[7] = max(b[7], pv[k].y);
                        ap += (int64_t)(pv[k].x - o.x) * (pw[k].y - o.y) - (int64_t)(pw[k].x - o.x) * (pv[k].y - o.y);
                    }
                    aq += cq;
                    const int w0 = base + k * kMetaThreads + (tid & ~63);   // the wavefront's first edge
                    if (sh.qs > 1 && w0 < m) {
                        const int64_t ws = wave_sum_i64(cq);
                        if (lane == 0) atomicAdd(&sWin[w0 / kWideCap], (unsigned long long)ws);
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < 8; j++) b[j] = (j & 3) < 2 ? wmin(b[j]) : wmax(b[j]);
            aq = wave_sum_i64(aq);
            ap = wave_sum_i64(ap);
            if (lane == 0) {
#pragma unroll
                for (int j = 0; j < 8; j++) {
                    if ((j & 3) < 2) atomicMin(&sBox[j], b[j]);
                    else atomicMax(&sBox[j], b[j]);
                }
                atomicAdd(&sA[0], (unsigned long long)aq);
                atomicAdd(&sA[1], (unsigned long long)ap);
            }
        }
        __syncthreads();
        const int32_t qm[4] = {sBox[0], sBox[1], sBox[2], sBox[3]}, pm[4] = {sBox[4], sBox[5], sBox[6], sBox[7]};
        const int64_t a2q = (int64_t)sA[0], a2p = (int64_t)sA[1];
        int kp = 0, kq = 0, wkp = 0, wkq = 0;
        if (a2p != 0 && a2q != 0) {
            // Q's extreme vertices (the first of each side) and P's first
            // vertex strictly outside Q's MBR
            int32_t e[5] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MAX, INT32_MAX};
            for (int base = 0; base < len; base += kMetaThreads * kMetaU) {
                int2 qv[kMetaU], pv[kMetaU];
#pragma unroll
                for (int k = 0; k < kMetaU; k++) {
                    const int i = base + k * kMetaThreads + tid;
                    qv[k] = QW[min(i, m - 1)];
                    pv[k] = PW[min(i, n - 1)];
                }
#pragma unroll
                for (int k = 0; k < kMetaU; k++) {
                    const int i = base + k * kMetaThreads + tid;
                    if (i < m) {
                        if (qv[k].x == qm[0]) e[0] = min(e[0], i);
                        if (qv[k].x == qm[2]) e[1] = min(e[1], i);
                        if (qv[k].y == qm[1]) e[2] = min(e[2], i);
                        if (qv[k].y == qm[3]) e[3] = min(e[3], i);
                    }
                    const bool out = (pv[k].x < qm[0]) | (pv[k].x > qm[2]) | (pv[k].y < qm[1]) | (pv[k].y > qm[3]);
                    if (i < n && out) e[4] = min(e[4], i);
                }
            }
#pragma unroll
            for (int j = 0; j < 5; j++) e[j] = wmin(e[j]);
            if (lane == 0) {
#pragma unroll
                for (int j = 0; j < 5; j++) atomicMin(&sIdx[j], e[j]);
            }
            __syncthreads();
            const int ext[4] = {sIdx[0], sIdx[1], sIdx[2], sIdx[3]};
            kq = anchor_q(qm, pm, ext);
            kp = sIdx[4] == INT32_MAX ? -1 : sIdx[4];
            if (kp < 0 || kq < 0) {
                // without an anchor: P's vertex 0 (against Q + delta) and Q's
                // vertex 0, the origin (plus delta, against P), by the
                // crossing rule over the other ring's edges
                const int2 p0 = make_int2(PW[0].x - o.x, PW[0].y - o.y), q0 = make_int2(0, 0);
                bool op = false, oq = false;
                for (int base = 0; base < len; base += kMetaThreads * kMetaU) {
                    int2 qv[kMetaU], qw[kMetaU], pv[kMetaU], pw[kMetaU];
#pragma unroll
                    for (int k = 0; k < kMetaU; k++) {
                        const int i = base + k * kMetaThreads + tid;
                        const int iq = min(i, m - 1), ip = min(i, n - 1);
                        qv[k] = QW[iq]; qw[k] = QW[iq + 1 == m ? 0 : iq + 1];
                        pv[k] = PW[ip]; pw[k] = PW[ip + 1 == n ? 0 : ip + 1];
                    }
#pragma unroll
                    for (int k = 0; k < kMetaU; k++) {
                        const int i = base + k * kMetaThreads + tid;
                        const int2 c = make_int2(qv[k].x - o.x, qv[k].y - o.y), d = make_int2(qw[k].x - o.x, qw[k].y - o.y);
                        const int2 f = make_int2(pv[k].x - o.x, pv[k].y - o.y), g = make_int2(pw[k].x - o.x, pw[k].y - o.y);
                        op ^= kp < 0 && i < m && flips_parity(c, d, p0, -1);
                        oq ^= kq < 0 && i < n && flips_parity(f, g, q0, +1);
                    }
                }
                const int cp = __popcll(__ballot(op)), cq = __popcll(__ballot(oq));
                if (lane == 0) { atomicAdd(&sOdd[0], cp); atomicAdd(&sOdd[1], cq); }
                __syncthreads();
                if (kp < 0) { wkp = sOdd[0] & 1; kp = 0; }
                if (kq < 0) { wkq = sOdd[1] & 1; kq = 0; }
            }
        }
        if (tid == 0) {
            MultiPair &out = hw.multi[s];
            out.a2p = a2p; out.a2q = a2q; out.kp = kp; out.kq = kq; out.wkp = wkp; out.wkq = wkq;
        }
        for (int u = tid; u < mp.units; u += kMetaThreads) {
            const int qw = sh.qs > 1 ? u % sh.qs : 0;
            int64_t pre = 0;
            for (int j = 0; j < qw; j++) pre += (int64_t)sWin[j];
            hw.units[s * kMultiUnits + u].qpre = pre;
            WidePair e;
            e.c = mp.c; e.pa = mp.pa; e.n = mp.n; e.q = mp.q;
            e.pw = (int16_t)(u / sh.qs);
            e.qw = (int16_t)(sh.qs == 1 ? -1 : qw);
            e.slot = (int32_t)s;
            hw.wide[mp.first + u] = e;
        }
        // every thread is done with the LDS before the next pair clears it
        __syncthreads();
    }
}

// Splits the recorded wide entries that split_shape splits, one thread per
// entry: a split slot and the list positions of its units, appended after the
// recorded entries (k_wide_meta writes the units there; the recorded entry is
// then marked unused).  A pair stays whole when the
// split slots run out; when its units do not fit the list, the positions it
// claimed are marked unused and its slot is dropped.
__global__ __launch_bounds__(256) void k_expand(const int64_t *__restrict__ qoff, HeavyWs hw)
{
    const int64_t norig = min((int64_t)hw.count[1], (int64_t)kWideListCap);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < norig;
         i += (int64_t)gridDim.x * blockDim.x) {
        const WidePair w = hw.wide[i];
        const int mq = (int)(qoff[w.q + 1] - qoff[w.q]);
        const bool swap = w.n > kWideCap && w.n > mq;
        const SplitShape sh = split_shape(swap ? mq : w.n, swap ? w.n : mq);
        if (sh.units <= 1) continue;
        const int ms = atomicAdd(hw.count + 2, 1);
        if (ms >= kMultiCap) continue;
        MultiPair &mp = hw.multi[ms];
        const int64_t base = norig + atomicAdd(hw.count + 4, sh.units);
        if (base + sh.units > kWideListCap) {
            for (int64_t j = base; j < kWideListCap; j++) hw.wide[j].c = -1;
            mp.c = -1;
            continue;
        }
        mp.c = w.c; mp.pa = w.pa; mp.n = w.n; mp.q = w.q; mp.units = sh.units; mp.first = (int32_t)base;
        hw.wide[i].c = -1;
    }
}

// One wavefront per deferred pair (workgroups of one wavefront, so four fit a
// CU's LDS), any sizes: both rings pass through LDS in windows of up to
// kWideCap edges, P's windows in the outer loop and Q's in the inner one.
// Every sum of the tiled form adds over Q's edges, and P's membership term
// adds over P's edges once the crossing signs of the earlier windows are
// carried in, so each (P window, Q window) adds its crossings, with Q's
// suffix sums carried from window to window.  P is the data polygon, or the
// query when the data polygon has more than kWideCap edges and more than the
// query (so a polygon of at most kWideCap edges is staged once); exchanging
// the roles translates the data polygon by delta instead of the query:
// another consistent perturbation with the same limit area.
__global__ __launch_bounds__(64) void k_refine_wide(const int32_t *__restrict__ dxy,
                                                    const int32_t *__restrict__ qxy,
                                                    const int64_t *__restrict__ qoff,
                                                    double *__restrict__ cand_j, HeavyWs hw, int want_stats)
{
    __shared__ int2 sQv[kWideRing];
    __shared__ int4 sQbox[kWideCap / 8];
    __shared__ double sQsuf[kWideCap];
    __shared__ int2 sPv[kWideRing];
    __shared__ int4 sPbox[kWideCap / 8];
    __shared__ uint32_t sPS[kWideCap / 2];
    __shared__ uint16_t sList[kListCap];
    __shared__ uint32_t sUnits[kUnitCap];
    __shared__ uint32_t sCross[kCrossCap];

    const int lane = threadIdx.x;
    const int64_t norig = min((int64_t)hw.count[1], (int64_t)kWideListCap);
    const int64_t nunits = max((int64_t)0, min((int64_t)hw.count[4], (int64_t)kWideListCap - norig));
    if (norig + nunits == 0) return;   // nothing deferred (the usual case): no atomics on the counter
    unsigned long long st_pairs = 0, st_swept = 0;
    // entries are taken from a counter as wavefronts come free, the split
    // pairs' units first: costs range from one window to many
    for (;;) {
        const int64_t t = __builtin_amdgcn_readfirstlane(lane == 0 ? atomicAdd(hw.count + 3, 1) : 0);
        if (t >= norig + nunits) break;
        const WidePair w = hw.wide[t < nunits ? norig + t : t - nunits];
        if (w.c < 0) continue;
        const int64_t qa = qoff[w.q];
        const int mq = (int)(qoff[w.q + 1] - qa);
        const bool swap = w.n > kWideCap && w.n > mq;
        const int32_t *Pg = swap ? qxy + 2 * qa : dxy + 2 * w.pa;
        const int32_t *Qg = swap ? dxy + 2 * w.pa : qxy + 2 * qa;
        const int n = swap ? mq : w.n, m = swap ? w.n : mq;
        const int64_t ox = Qg[0], oy = Qg[1];
        // windows of this entry: all, or one P window (and one Q window) of
        // a split pair
        const SplitShape sh = split_shape(n, m);
        const int pfirst = w.pw < 0 ? 0 : w.pw * sh.plen;
        const int pend = w.pw < 0 ? n : min(n, pfirst + sh.plen);
        const int qfirst = w.qw < 0 ? 0 : w.qw * kWideCap;
        const int qend = w.qw < 0 ? m : min(m, qfirst + kWideCap);
        const int u = w.qw < 0 ? w.pw : w.pw * sh.qs + w.qw;   // a split pair's unit slot
        int64_t a2q, a2p, qpre;
        int kp = 0, kq = 0, wkp = 0, wkq = 0;
        if (w.pw >= 0) {
            // a split pair's unit: the pair's own quantities from k_wide_meta
            // (its ring starts' memberships are the finish's)
            const MultiPair &mp = hw.multi[w.slot];
            a2p = mp.a2p; a2q = mp.a2q; kp = mp.kp; kq = mp.kq;
            qpre = hw.units[(int64_t)w.slot * kMultiUnits + u].qpre;
        } else {
            int32_t qm[4], pm[4];
            int64_t ppre;
            ring_sums_global(Qg, m, ox, oy, 0, lane, qm, a2q, qpre);
            ring_sums_global(Pg, n, ox, oy, 0, lane, pm, a2p, ppre);
            if (a2p != 0 && a2q != 0) {
                // anchors: a vertex outside the other polygon's MBR has
                // membership 0; without one, a crossing-number pass
                int qext[4];
                extremes_global(Qg, m, qm, lane, qext);
                kq = anchor_q(qm, pm, qext);
                kp = first_outside_global(Pg, n, qm, lane);
                if (kp < 0) {
                    const int2 p0 = make_int2((int)((int64_t)Pg[0] - ox), (int)((int64_t)Pg[1] - oy));
                    wkp = member_point_global(Qg, m, ox, oy, p0, -1, lane);
                    kp = 0;
                }
                if (kq < 0) {
                    // Q's vertex 0 is the origin
                    wkq = member_point_global(Pg, n, ox, oy, make_int2(0, 0), +1, lane);
                    kq = 0;
                }
            }
        }
        double J = 0.0;
        MultiUnit unit{0.0, 0.0, 0, 0, 0};
        if (a2p != 0 && a2q != 0) {
            RingLds Qs{sQv, sQbox, nullptr, sQsuf};
            RingLds Ps{sPv, sPbox, sPS, nullptr};
            double accP = 0.0, accQ = 0.0, accM = 0.0, accK = 0.0, T = 0.0, crs = 0.0;
            int pcarry = 0, K = 0;
            const int pstep = w.pw < 0 ? kWideCap : sh.plen;
            for (int p0 = pfirst; p0 < pend; p0 += pstep) {
                const int plen = min(pstep, pend - p0);
                stage_window(Pg, n, p0, plen, 8 * ((plen + 7) >> 3) + 1, ox, oy, Ps, lane);
                for (int j = lane; j < (plen + 1) >> 1; j += 64) Ps.S[j] = kSBias;
                wave_lds_sync();
                chunk_boxes_p<kWideCap / 8>(Ps, plen, lane);
                int64_t qcarry = qpre;
                for (int w0 = qfirst; w0 < qend; w0 += kWideCap) {
                    const int len = min(kWideCap, m - w0);
                    // one all-padding chunk past the window, as for whole rings
                    stage_window(Qg, m, w0, len, 8 * ((len + 7) >> 3) + 9, ox, oy, Qs, lane);
                    wave_lds_sync();
                    chunk_boxes(Qs, len, lane, 64);
                    qcarry = q_suffix_sums(Qs, len, a2q, lane, qcarry);
                    wave_lds_sync();
                    tiled_accumulate<uint32_t, 16>(Ps, plen, Qs, len, kq - w0, lane, sList, sUnits, sCross,
                                                   &st_swept, accP, accQ, accM, accK);
                    // every lane is done with the window before the next one
                    wave_lds_sync();
                }
                T += membership_term_window(Ps, plen, kp - p0, lane, pcarry, K, crs);
                wave_lds_sync();
            }
            // as tiled_finish, with T summed over P's windows
            const int sp = a2p > 0 ? 1 : -1, sq = a2q > 0 ? 1 : -1;
            const double tot = wave_sum((double)(sp * sq) * (T + accP + accQ + accM - (double)a2q * accK));
            if (w.pw < 0) {
                const double inter2 = tot + (double)(sp * (wkp - sq * K)) * (double)a2p +
                                      (double)(sq * wkq) * (double)a2q;
                J = jaccard_of(inter2, a2p, a2q);
            } else {
                unit.part = tot;
                // the P window's cross products are the same in each of its
                // Q windows' units: the finish takes them from the first
                const double cr = wave_sum(crs);
                unit.cr = w.qw <= 0 ? cr : 0.0;
                unit.stot = pcarry;
                unit.kloc = K;
            }
        }
        st_pairs += (w.pw <= 0) & (w.qw <= 0);
        if (lane == 0) {
            if (w.pw < 0) cand_j[w.c] = J;
            else hw.units[(int64_t)w.slot * kMultiUnits + u] = unit;
        }
        // every lane is done with both rings before the next pair restages them
        wave_lds_sync();
    }
    if (want_stats && lane == 0) {
        unsigned long long *slot = hw.stat_slots + (blockIdx.x % kStatSlots) * 4;
        if (st_pairs) atomicAdd(slot + 0, st_pairs);
        if (st_swept) atomicAdd(slot + 1, st_swept);
    }
}

// One wavefront per split pair: the P windows' sums (each the sum of its Q
// windows' units, one window a lane)
// with the crossing signs of the earlier windows carried into each, added in
// a fixed order (deterministic), then J.
__global__ __launch_bounds__(256) void k_refine_multi_finish(const int64_t *__restrict__ qoff,
                                                            double *__restrict__ cand_j, HeavyWs hw)
{
    const int lane = threadIdx.x & 63;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t count = min((int64_t)hw.count[2], (int64_t)kMultiCap);
    for (int64_t s = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; s < count; s += nw) {
        const MultiPair mp = hw.multi[s];
        if (mp.c < 0) continue;
        // the roles of k_refine_wide; the pair's own quantities from k_wide_meta
        const int mq = (int)(qoff[mp.q + 1] - qoff[mp.q]);
        const bool swap = mp.n > kWideCap && mp.n > mq;
        const int n = swap ? mq : mp.n, m = swap ? mp.n : mq;
        const int64_t a2q = mp.a2q, a2p = mp.a2p;
        double J = 0.0;
        if (a2p != 0 && a2q != 0) {
            const int kp = mp.kp, wkp = mp.wkp, wkq = mp.wkq;
            const int sp = a2p > 0 ? 1 : -1, sq = a2q > 0 ? 1 : -1;
            const SplitShape sh = split_shape(n, m);
            const int pk = kp / sh.plen;
            // lanes take the P windows, 64 at a time; the carry of crossing
            // signs into each is a scan in window order
            const int qs = sh.qs, npw = mp.units / qs;
            const MultiUnit *U = hw.units + s * kMultiUnits;
            double acc = 0.0;
            int carry = 0, K = 0;
            for (int base = 0; base < npw; base += 64) {
                const int wdw = base + lane;
                const bool live = wdw < npw;
                double part = 0.0, cr = 0.0;
                int stot = 0, kloc = 0;
                if (live) {
                    cr = U[wdw * qs].cr;
                    for (int v = 0; v < qs; v++) {
                        const MultiUnit x = U[wdw * qs + v];
                        part += x.part;
                        stot += x.stot;
                        kloc += x.kloc;
                    }
                }
                const int incl = wave_incl_scan32(stot);
                const int excl = carry + incl - stot;
                acc += live ? part + (double)(sp * sq) * cr * (double)excl : 0.0;
                if (pk >= base && pk < base + 64) K = __builtin_amdgcn_readlane(excl + kloc, pk - base);
                carry += __builtin_amdgcn_readlane(incl, 63);
            }
            const double total = wave_sum(acc);
            const double inter2 = total + (double)(sp * (wkp - sq * K)) * (double)a2p + (double)(sq * wkq) * (double)a2q;
            J = jaccard_of(inter2, a2p, a2q);
        }
        if (lane == 0) cand_j[mp.c] = J;
    }
}

// One wavefront per (heavy pair, side, slice): the slice's share of that
// side's edge sums; slices past the side's last block add nothing.
__global__ __launch_bounds__(256) void k_heavy(const int32_t *__restrict__ dxy, const int32_t *__restrict__ qxy,
                                               HeavyWs hw)
{
    const int lane = threadIdx.x & 63;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t count = min(hw.count[0], kHeavyCap);
    for (int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; t < count * 2 * kHeavySlices;
         t += nw) {
        const int64_t h = t / (2 * kHeavySlices);
        const int side = (int)((t / kHeavySlices) & 1), slice = (int)(t % kHeavySlices);
        const HeavyPair &e = hw.pairs[h];
        PairIn in;
        in.P = dxy + 2 * e.pa; in.n = e.n; in.Q = qxy + 2 * e.qa; in.m = e.m; in.ox = e.ox; in.oy = e.oy;
        for (int i = 0; i < 4; i++) in.qmbr[i] = e.qmbr[i];
        in.sq = e.a2q > 0 ? 1 : -1;
        in.sp = e.a2p > 0 ? 1 : -1;
        int32_t pm[4] = {e.pm[0], e.pm[1], e.pm[2], e.pm[3]};
        double s = 0.0;
        int64_t unused;
        if (side == 0) {
            if (e.wide) edges_in_other_P<true>(in, lane, s, unused, slice, kHeavySlices);
            else edges_in_other_P<false>(in, lane, s, unused, slice, kHeavySlices);
        } else {
            if (e.wide) edges_in_other_Q<true>(in, pm, lane, s, unused, slice, kHeavySlices);
            else edges_in_other_Q<false>(in, pm, lane, s, unused, slice, kHeavySlices);
        }
        s = wave_sum(s);
        if (lane == 0) hw.partial[(h * 2 + side) * kHeavySlices + slice] = s;
    }
}

// One wavefront per heavy pair: the slices' sums in a fixed order, then J.
__global__ __launch_bounds__(256) void k_heavy_finish(HeavyWs hw, double *__restrict__ cand_j)
{
    const int lane = threadIdx.x & 63;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t count = min(hw.count[0], kHeavyCap);
    for (int64_t h = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; h < count; h += nw) {
        const HeavyPair &e = hw.pairs[h];
        const double sp = e.a2p > 0 ? 1.0 : -1.0, sq = e.a2q > 0 ? 1.0 : -1.0;
        double vp = 0.0, vq = 0.0;
        if (lane < kHeavySlices) {
            vp = hw.partial[(h * 2 + 0) * kHeavySlices + lane];
            vq = hw.partial[(h * 2 + 1) * kHeavySlices + lane];
        }
        const double inter2 = wave_sum(sp * vp) + wave_sum(sq * vq);
        if (lane == 0) cand_j[e.c] = jaccard_of(inter2, e.a2p, e.a2q);
    }
}

HeavyWs carve_heavy(Carve &cv)
{
    HeavyWs hw{};
    hw.count = cv.take<int32_t>(64);
    hw.pairs = cv.take<HeavyPair>(kHeavyCap);
    hw.partial = cv.take<double>((size_t)kHeavyCap * 2 * kHeavySlices);
    hw.stat_slots = cv.take<unsigned long long>(kStatSlots * 4);
    hw.wide = cv.take<WidePair>(kWideListCap);
    hw.multi = cv.take<MultiPair>(kMultiCap);
    hw.units = cv.take<MultiUnit>((size_t)kMultiCap * kMultiUnits);
    return hw;
}

// Clears the pair counts, the work counter and the counter slots (256 threads).
__global__ void k_zero_count(int32_t *p, unsigned long long *slots)
{
    if (threadIdx.x < 5) p[threadIdx.x] = 0;
    if (threadIdx.x < kStatSlots * 4) slots[threadIdx.x] = 0;
}

// Adds the counter slots to the caller's four counters (one wavefront).
__global__ void k_fold_stats(const unsigned long long *slots, unsigned long long *stats)
{
    const int i = threadIdx.x;
    if (i < 4) {
        unsigned long long v = 0;
        for (int s = 0; s < kStatSlots; s++) v += slots[s * 4 + i];
        if (v) atomicAdd(stats + i, v);
    }
}

}  // namespace

size_t refine_workspace_bytes()
{
    Carve cv{nullptr, 0};
    carve_heavy(cv);
    return align_up(cv.used, 256);
}

polymh_status launch_refine(const polymh_polys *data, const polymh_polys *queries,
                            const int64_t *cand_off, const int32_t *cand_ids, int64_t nq,
                            int64_t n_cand, double *cand_j, hipStream_t s,
                            unsigned long long *stats, void *ws, size_t ws_bytes)
{
    if (n_cand == 0 || nq == 0) return POLYMH_OK;
    HeavyWs hw{};
    if (ws) {
        Carve cv{static_cast<char *>(ws), ws_bytes};
        hw = carve_heavy(cv);
        if (!cv.ok) return set_error(POLYMH_ECAPACITY, "refine: workspace of %zu bytes, need %zu", ws_bytes, cv.used);
        hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(kStatSlots * 4), 0, s, hw.count, hw.stat_slots);
    }
    if (nq > 0x7fffffffLL) return set_error(POLYMH_EINVAL, "refine: too many queries");
    // a query's candidates are spread over several workgroups (each stages
    // the query once) when the batch is small or its lists are long: at
    // least 2048 workgroups, at most about 64 candidates per workgroup on
    // average (16 per wavefront: the query's staging is cheap beside them
    // and the long lists no longer set the launch's tail), at most 64
    // workgroups per query
    const int64_t by_batch = (2048 + nq - 1) / nq;
    const int64_t by_length = (n_cand + nq * 64 - 1) / (nq * 64);
    int64_t sl = std::max<int64_t>(1, std::min<int64_t>(64, std::max(by_batch, by_length)));
    if (nq * sl > 0x7fffffffLL) sl = 1;
    const int slices = (int)sl;
    hipLaunchKernelGGL(k_refine, dim3((unsigned)(nq * slices)), dim3(64 * kWavesPerBlock), 0, s, data->xy,
                       data->offsets, queries->xy, queries->offsets, cand_off, cand_ids, cand_j, stats,
                       slices, hw);
    polymh_status st = check_launch("refine");
    if (st || !ws) return st;
    hipLaunchKernelGGL(k_expand, dim3(64), dim3(256), 0, s, queries->offsets, hw);
    if ((st = check_launch("refine: split wide pairs"))) return st;
    hipLaunchKernelGGL(k_wide_meta, dim3(256), dim3(kMetaThreads), 0, s, data->xy, queries->xy, queries->offsets,
                       hw);
    if ((st = check_launch("refine: split wide pairs"))) return st;
    // deferred wide tiled pairs: four one-wavefront workgroups per CU
    hipLaunchKernelGGL(k_refine_wide, dim3(1024), dim3(64), 0, s, data->xy, queries->xy, queries->offsets, cand_j,
                       hw, stats ? 1 : 0);
    if ((st = check_launch("refine: wide pairs"))) return st;
    hipLaunchKernelGGL(k_refine_multi_finish, dim3(64), dim3(256), 0, s, queries->offsets, cand_j, hw);
    if ((st = check_launch("refine: split wide pairs"))) return st;
    // deferred heavy pairs: a grid that covers every (pair, side, slice) of a
    // full list in a few rounds, then the per-pair sums
    hipLaunchKernelGGL(k_heavy, dim3(2048), dim3(256), 0, s, data->xy, queries->xy, hw);
    if ((st = check_launch("refine: heavy pairs"))) return st;
    hipLaunchKernelGGL(k_heavy_finish, dim3(256), dim3(256), 0, s, hw, cand_j);
    if ((st = check_launch("refine: heavy pairs"))) return st;
    if (!stats) return POLYMH_OK;
    hipLaunchKernelGGL(k_fold_stats, dim3(1), dim3(64), 0, s, hw.stat_slots, stats);
    return check_launch("refine: counters");
}

}  // namespace polymh
