/*
 * PolyMinHash CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct C implementation of what the signing path
 * computes, used by the test suite, the smoke check and the CPU baseline of
 * the benchmark to check the GPU library.  It shares no code, header, table
 * or helper with the GPU library and must never be linked into it.
 *
 * Paper: "PolyMinHash: Efficient Area-Based MinHashing of Polygons for
 * Approximate Nearest Neighbor Search" (Subedi, Pokharel, Puri; SIGSPATIAL'25,
 * arXiv 2511.16576).
 *
 * Readings of the paper taken here (the paper is silent on each):
 *  - coordinates are integers on a lattice; the sampling box B (the global
 *    MBR of Sec. 3.1) is an inclusive lattice box [xmin,xmax] x [ymin,ymax];
 *  - the random source is SplitMix64 (Steele, Lea, Flood 2014): one u64 seed,
 *    hash i uses the key mix64(seed + (i+1)*GAMMA) and its j-th draw
 *    (0-based) is mix64(key + (j+1)*GAMMA);
 *  - a draw r becomes the lattice point x = xmin + floor(hi32(r) * Wx / 2^32),
 *    y = ymin + floor(lo32(r) * Wy / 2^32) (Sec. 3.2 samples x and y
 *    independently and uniformly over B);
 *  - "inside" is the crossing-number test with a half-open rule: a point on
 *    the boundary is inside iff it is inside after an infinitesimal move
 *    up and to the right;
 *  - attempts are counted from 1 (Alg. 1 increments before sampling; Fig. 2
 *    calls the 6th point's hash 6); a walk that finds no hit within `cap`
 *    draws keeps Alg. 1's initial value 0; polygons with < 3 vertices get 0;
 *  - band keys (Sec. 3.2 puts polygons in a hashmap keyed by their code; the
 *    banded form follows the MMDS banding technique cited there): band t of
 *    r rows has F0 = mix64(band_seed + (t+1)*GAMMA),
 *    F_{u+1} = mix64(F_u XOR sig[t*r+u]), key_t = F_r.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GAMMA 0x9E3779B97F4A7C15ULL

/* SplitMix64 output function (Steele, Lea, Flood 2014). */
uint64_t orc_mix64(uint64_t z)
{
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ULL;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return z;
}

/* The SplitMix64 generator itself: state += GAMMA, output mix64(state). */
void orc_splitmix64(uint64_t seed, int64_t count, uint64_t *out)
{
    uint64_t s = seed;
    for (int64_t i = 0; i < count; i++) {
        s += GAMMA;
        out[i] = orc_mix64(s);
    }
}

/* Alg. 1 initialises one generator per hash from fixed seeds: key of hash i. */
void orc_hash_keys(uint64_t seed, int32_t k, uint64_t *keys)
{
    for (int32_t i = 0; i < k; i++)
        keys[i] = orc_mix64(seed + (uint64_t)(i + 1) * GAMMA);
}

/* Sec. 3.2 / Alg. 1: sample j of the stream with key `key`, a uniform
 * lattice point of B = box[0..3] = (xmin, ymin, xmax, ymax). */
void orc_sample_point(const int32_t *box, uint64_t key, uint64_t j, int32_t *pt)
{
    uint64_t r = orc_mix64(key + (j + 1) * GAMMA);
    uint64_t wx = (uint64_t)((int64_t)box[2] - (int64_t)box[0] + 1);
    uint64_t wy = (uint64_t)((int64_t)box[3] - (int64_t)box[1] + 1);
    uint64_t hi = r >> 32, lo = r & 0xffffffffULL;
    pt[0] = (int32_t)((int64_t)box[0] + (int64_t)((hi * wx) >> 32));
    pt[1] = (int32_t)((int64_t)box[1] + (int64_t)((lo * wy) >> 32));
}

/* Alg. 1's "point (x,y) is inside polygon P": crossing number along the ray
 * to +x.  Edge (x0,y0)->(x1,y1) is crossed iff it straddles the line y=py
 * half-open ((y0>py) != (y1>py)) and the crossing lies strictly right of px,
 * i.e. the orientation o = (x1-x0)(py-y0) - (px-x0)(y1-y0) has the sign of
 * (y1-y0).  Exact in 128-bit integers. */
int orc_inside(const int32_t *xy, int64_t n, int32_t px, int32_t py)
{
    int c = 0;
    for (int64_t e = 0; e < n; e++) {
        int64_t x0 = xy[2 * e], y0 = xy[2 * e + 1];
        int64_t e1 = (e + 1 == n) ? 0 : e + 1;
        int64_t x1 = xy[2 * e1], y1 = xy[2 * e1 + 1];
        if ((y0 > py) == (y1 > py))
            continue;
        __int128 o = (__int128)(x1 - x0) * (py - y0) - (__int128)(px - x0) * (y1 - y0);
        int crosses = (y1 > y0) ? (o > 0) : (o < 0);
        c ^= crosses;
    }
    return c;
}

/* inside() for a batch of points (test helper). */
void orc_inside_points(const int32_t *xy, int64_t n, const int32_t *pts, int64_t npts, uint8_t *out)
{
    for (int64_t i = 0; i < npts; i++)
        out[i] = (uint8_t)orc_inside(xy, n, pts[2 * i], pts[2 * i + 1]);
}

/* Local MBR of one polygon (Alg. 1, "compute local MBR of P"). */
static void local_mbr(const int32_t *xy, int64_t n, int32_t *m)
{
    m[0] = m[2] = xy[0];
    m[1] = m[3] = xy[1];
    for (int64_t v = 1; v < n; v++) {
        if (xy[2 * v] < m[0]) m[0] = xy[2 * v];
        if (xy[2 * v] > m[2]) m[2] = xy[2 * v];
        if (xy[2 * v + 1] < m[1]) m[1] = xy[2 * v + 1];
        if (xy[2 * v + 1] > m[3]) m[3] = xy[2 * v + 1];
    }
}

/* Alg. 1 for one polygon: h[i] = attempts of the first sample of stream i
 * that lies inside P, 0 if none within `cap` samples.  With use_mbr the MBR
 * check rejects samples first; it never changes the result. */
static void sign_one(const int32_t *xy, int64_t n, const int32_t *box, const uint64_t *keys,
                     int32_t k, uint32_t cap, int use_mbr, uint32_t *h)
{
    for (int32_t i = 0; i < k; i++)
        h[i] = 0;
    if (n < 3)
        return;
    int32_t m[4];
    local_mbr(xy, n, m);
    for (int32_t i = 0; i < k; i++) {
        uint64_t attempts = 0;
        while (attempts < cap) {
            int32_t pt[2];
            orc_sample_point(box, keys[i], attempts, pt);
            attempts++;
            if (use_mbr && (pt[0] < m[0] || pt[0] > m[2] || pt[1] < m[1] || pt[1] > m[3]))
                continue;
            if (orc_inside(xy, n, pt[0], pt[1])) {
                h[i] = (uint32_t)attempts;
                break;
            }
        }
    }
}

/* Signatures of npoly CSR polygons: sig[p*k + i] = h_i(P_p). */
int32_t orc_sign(const int32_t *xy, const int64_t *off, int64_t npoly, const int32_t *box,
                 uint64_t seed, int32_t k, uint32_t cap, int32_t use_mbr, int32_t nthreads,
                 uint32_t *sig)
{
    uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(k > 0 ? k : 1));
    if (!keys)
        return -1;
    orc_hash_keys(seed, k, keys);
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t p = 0; p < npoly; p++)
        sign_one(xy + 2 * off[p], off[p + 1] - off[p], box, keys, k, cap, use_mbr,
                 sig + (size_t)p * (size_t)k);
    free(keys);
    return 0;
}

/* Band keys: keys[p*b + t] from rows sig[p*k + t*r .. t*r + r). */
void orc_band(const uint32_t *sig, int64_t n, int32_t k, int32_t b, int32_t r,
              uint64_t band_seed, uint64_t *keys)
{
    for (int64_t p = 0; p < n; p++)
        for (int32_t t = 0; t < b; t++) {
            uint64_t f = orc_mix64(band_seed + (uint64_t)(t + 1) * GAMMA);
            for (int32_t u = 0; u < r; u++)
                f = orc_mix64(f ^ (uint64_t)sig[(size_t)p * (size_t)k + (size_t)(t * r + u)]);
            keys[(size_t)p * (size_t)b + (size_t)t] = f;
        }
}

/* Candidates of query q: every dataset polygon sharing at least one band key
 * with it (same band), ascending id.  Brute force over all pairs.  With
 * cand_ids == NULL only cand_off (exclusive prefix, [nq+1]) is written.
 * Returns the total count, or -1 if it exceeds cand_cap. */
int64_t orc_candidates(const uint64_t *dkeys, int64_t nd, const uint64_t *qkeys, int64_t nq,
                       int32_t b, int64_t *cand_off, int32_t *cand_ids, int64_t cand_cap)
{
    int64_t total = 0;
    for (int64_t q = 0; q < nq; q++) {
        cand_off[q] = total;
        for (int64_t p = 0; p < nd; p++) {
            int hit = 0;
            for (int32_t t = 0; t < b && !hit; t++)
                hit = dkeys[(size_t)p * (size_t)b + (size_t)t] == qkeys[(size_t)q * (size_t)b + (size_t)t];
            if (hit) {
                if (cand_ids) {
                    if (total >= cand_cap)
                        return -1;
                    cand_ids[total] = (int32_t)p;
                }
                total++;
            }
        }
    }
    cand_off[nq] = total;
    return total;
}

/* ---------------- exact Jaccard (Sec. 1: J = area(P n Q) / area(P u Q)) ---- */

/* Twice the signed area (shoelace), exact. */
int64_t orc_area2(const int32_t *xy, int64_t n)
{
    __int128 s = 0;
    for (int64_t e = 0; e < n; e++) {
        int64_t e1 = (e + 1 == n) ? 0 : e + 1;
        s += (__int128)xy[2 * e] * xy[2 * e1 + 1] - (__int128)xy[2 * e1] * xy[2 * e + 1];
    }
    return (int64_t)s;
}

/* Keep the part of convex polygon `in` left of (or on) the directed line a->b
 * (one Sutherland-Hodgman step). */
static int clip_half(const double *in, int nin, const double *a, const double *b, double *out)
{
    int nout = 0;
    double ex = b[0] - a[0], ey = b[1] - a[1];
    for (int i = 0; i < nin; i++) {
        const double *p = in + 2 * i;
        const double *q = in + 2 * ((i + 1) % nin);
        double sp = ex * (p[1] - a[1]) - ey * (p[0] - a[0]);
        double sq = ex * (q[1] - a[1]) - ey * (q[0] - a[0]);
        if (sp >= 0) {
            out[2 * nout] = p[0];
            out[2 * nout + 1] = p[1];
            nout++;
        }
        if ((sp > 0 && sq < 0) || (sp < 0 && sq > 0)) {
            double t = sp / (sp - sq);
            out[2 * nout] = p[0] + t * (q[0] - p[0]);
            out[2 * nout + 1] = p[1] + t * (q[1] - p[1]);
            nout++;
        }
    }
    return nout;
}

static double poly_area_d(const double *v, int n)
{
    double s = 0;
    for (int i = 0; i < n; i++) {
        const double *p = v + 2 * i, *q = v + 2 * ((i + 1) % n);
        s += p[0] * q[1] - q[0] * p[1];
    }
    return 0.5 * s;
}

/* Area of the intersection of two counter-clockwise triangles. */
static double tri_tri_area(const double *t, const double *c)
{
    double buf0[32], buf1[32];
    int n = 3;
    memcpy(buf0, t, 6 * sizeof(double));
    double *in = buf0, *out = buf1;
    for (int e = 0; e < 3 && n > 0; e++) {
        n = clip_half(in, n, c + 2 * e, c + 2 * ((e + 1) % 3), out);
        double *tmp = in; in = out; out = tmp;
    }
    return n >= 3 ? poly_area_d(in, n) : 0.0;
}

/* Signed fan of a polygon about its first vertex: triangles (v0, v_i, v_i+1)
 * stored counter-clockwise with the sign of their orientation, so that the
 * winding number of P is the signed sum of triangle indicators.  Coordinates
 * are taken relative to (ox, oy). */
static int fan(const int32_t *xy, int64_t n, int64_t ox, int64_t oy, double *tri, int *sgn)
{
    int m = 0;
    for (int64_t i = 1; i + 1 < n; i++) {
        int64_t ax = xy[0] - ox, ay = xy[1] - oy;
        int64_t bx = xy[2 * i] - ox, by = xy[2 * i + 1] - oy;
        int64_t cx = xy[2 * i + 2] - ox, cy = xy[2 * i + 3] - oy;
        __int128 o = (__int128)(bx - ax) * (cy - ay) - (__int128)(by - ay) * (cx - ax);
        if (o == 0)
            continue;
        double *T = tri + 6 * m;
        T[0] = (double)ax; T[1] = (double)ay;
        if (o > 0) {
            T[2] = (double)bx; T[3] = (double)by; T[4] = (double)cx; T[5] = (double)cy;
            sgn[m] = 1;
        } else {
            T[2] = (double)cx; T[3] = (double)cy; T[4] = (double)bx; T[5] = (double)by;
            sgn[m] = -1;
        }
        m++;
    }
    return m;
}

static void tri_box(const double *T, double *bb)
{
    bb[0] = fmin(T[0], fmin(T[2], T[4]));
    bb[1] = fmin(T[1], fmin(T[3], T[5]));
    bb[2] = fmax(T[0], fmax(T[2], T[4]));
    bb[3] = fmax(T[1], fmax(T[3], T[5]));
}

/* area(P n Q) of two simple polygons: with 1_P = s_P * sum_i s_i 1_{T_i}
 * (signed fan decomposition), area(P n Q) = s_P s_Q sum_ij s_i s'_j
 * area(T_i n T'_j), each convex pair clipped by Sutherland-Hodgman in FP64
 * relative to P's first vertex.  Pairs with disjoint boxes contribute 0. */
double orc_intersection_area(const int32_t *P, int64_t np_, const int32_t *Q, int64_t nq_)
{
    if (np_ < 3 || nq_ < 3)
        return 0.0;
    int64_t a2p = orc_area2(P, np_), a2q = orc_area2(Q, nq_);
    if (a2p == 0 || a2q == 0)
        return 0.0;
    int32_t mp[4], mq[4];
    local_mbr(P, np_, mp);
    local_mbr(Q, nq_, mq);
    if (mp[2] < mq[0] || mq[2] < mp[0] || mp[3] < mq[1] || mq[3] < mp[1])
        return 0.0;
    int64_t ox = P[0], oy = P[1];
    double *tp = (double *)malloc(sizeof(double) * 6 * (size_t)np_);
    double *tq = (double *)malloc(sizeof(double) * 6 * (size_t)nq_);
    int *sp = (int *)malloc(sizeof(int) * (size_t)np_);
    int *sq = (int *)malloc(sizeof(int) * (size_t)nq_);
    int mP = fan(P, np_, ox, oy, tp, sp);
    int mQ = fan(Q, nq_, ox, oy, tq, sq);
    double total = 0.0;
    for (int i = 0; i < mP; i++) {
        double bi[4];
        tri_box(tp + 6 * i, bi);
        for (int j = 0; j < mQ; j++) {
            double bj[4];
            tri_box(tq + 6 * j, bj);
            if (bi[2] <= bj[0] || bj[2] <= bi[0] || bi[3] <= bj[1] || bj[3] <= bi[1])
                continue;
            total += (double)(sp[i] * sq[j]) * tri_tri_area(tp + 6 * i, tq + 6 * j);
        }
    }
    free(tp); free(tq); free(sp); free(sq);
    double s = (a2p > 0 ? 1.0 : -1.0) * (a2q > 0 ? 1.0 : -1.0);
    return s * total;
}

/* J = A_int / (A_P + A_Q - A_int); an empty union gives 0. */
double orc_jaccard(const int32_t *P, int64_t np_, const int32_t *Q, int64_t nq_)
{
    double ai = orc_intersection_area(P, np_, Q, nq_);
    double ap = 0.5 * fabs((double)orc_area2(P, np_));
    double aq = 0.5 * fabs((double)orc_area2(Q, nq_));
    double u = ap + aq - ai;
    return u > 0 ? ai / u : 0.0;
}

/* Exact J of query q against each of its candidates (CSR), all queries. */
void orc_jaccard_candidates(const int32_t *dxy, const int64_t *doff, const int32_t *qxy,
                            const int64_t *qoff, int64_t nq, const int64_t *cand_off,
                            const int32_t *cand_ids, int32_t nthreads, double *out)
{
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t q = 0; q < nq; q++) {
        const int32_t *Q = qxy + 2 * qoff[q];
        int64_t nqv = qoff[q + 1] - qoff[q];
        for (int64_t c = cand_off[q]; c < cand_off[q + 1]; c++) {
            int64_t p = cand_ids[c];
            out[c] = orc_jaccard(dxy + 2 * doff[p], doff[p + 1] - doff[p], Q, nqv);
        }
    }
}

/* Exact J of every query against every dataset polygon (brute force, Def. 1):
 * out[q*nd + p]. */
void orc_jaccard_all(const int32_t *dxy, const int64_t *doff, int64_t nd, const int32_t *qxy,
                     const int64_t *qoff, int64_t nq, int32_t nthreads, double *out)
{
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16) collapse(2)
#endif
    for (int64_t q = 0; q < nq; q++)
        for (int64_t p = 0; p < nd; p++)
            out[(size_t)q * (size_t)nd + (size_t)p] =
                orc_jaccard(dxy + 2 * doff[p], doff[p + 1] - doff[p], qxy + 2 * qoff[q], qoff[q + 1] - qoff[q]);
}

int32_t orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
