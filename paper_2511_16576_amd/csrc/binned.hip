// Shared-sample binned signing: the signatures of Alg. 1 / Def. 2, bit for
// bit, without walking every (polygon, hash) stream.  All polygons read the
// same point stream per hash (Sec. 3.2's fixed-seed generators), so the
// samples j < horizon of every hash are drawn once, in chunks of C, and each
// chunk's samples are grouped by cell of a 2^b x 2^b grid over B.  A
// (polygon, hash) unit visits the chunks in order and, in each, the samples
// of the cells its MBR meets: those inside the MBR are tested for membership
// and the smallest inside index of the first chunk that has one is the first
// hit (every sample inside the polygon lies in its MBR, hence in those
// cells).  Units with no hit below the horizon are walked from the start by
// the per-unit kernel, so every value equals Alg. 1's.
//
// Polygons whose expected walk is short (|B| / area below a threshold) are
// left to the walk altogether: a first-hit index near N_B / N_P is cheaper
// to draw than to look up.
//
// Lookup layout: one workgroup per (polygon, block of hashes), lane = hash,
// so the polygon's edges are staged once in LDS and every membership test
// reads them as broadcasts; samples inside the MBR are queued per wavefront
// and tested 64 at a time, one point per lane.
#include <cmath>

#include "internal.hpp"
#include "sign_common.hpp"

namespace polymh {

namespace {

constexpr int kBinThreads = 256;
constexpr int kMaxSpt = 16;        // samples per thread of k_bin (chunk <= 4096)
constexpr int kQueue = 128;        // per-wavefront queue of membership tests
constexpr uint32_t kNone = 0xffffffffu;

struct BinArgs {
    uint64_t seed;
    int32_t k;
    uint32_t horizon;              // samples per hash (j < horizon), <= cap
    int32_t nchunks;
    int32_t lchunk;                // chunk C = 2^lchunk samples
    int32_t bits;                  // grid side 2^bits (0..6)
    int32_t sbx, sby;              // cell of offset o: o >> sb
    uint32_t wx, wy;
    int32_t shx, shy;
    uint2 *sxy;                    // [k][nchunks][C] lattice offsets, grouped by cell
    uint16_t *sj;                  // index inside the chunk
    uint16_t *cell_off;            // [k][nchunks][cells + 1]
};

// One workgroup per (chunk, hash): draw, cell, counting sort in LDS (samples
// past the horizon go to an extra last cell that no lookup reads).  Dynamic
// LDS: counts and starts, (cells + 1) ints each.
template <bool POW2>
__global__ __launch_bounds__(kBinThreads) void k_bin(BinArgs A)
{
    extern __shared__ int s_dyn[];
    __shared__ int s_wsum[kBinThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int c = blockIdx.x, i = blockIdx.y;
    const int cells = 1 << (2 * A.bits);
    const int C = 1 << A.lchunk, spt = C / kBinThreads;
    int *s_cnt = s_dyn, *s_start = s_dyn + cells + 1;
    for (int t = tid; t <= cells; t += kBinThreads) s_cnt[t] = 0;
    __syncthreads();
    const uint64_t key = mix64(A.seed + (uint64_t)(i + 1) * kGamma);
    uint32_t ox[kMaxSpt], oy[kMaxSpt];
    int cell[kMaxSpt], rank[kMaxSpt];
#pragma unroll
    for (int q = 0; q < kMaxSpt; q++) {
        if (q < spt) {
            const uint64_t j = ((uint64_t)c << A.lchunk) + (uint64_t)(q * kBinThreads + tid);
            const uint64_t r = mix64(key + (j + 1) * kGamma);
            ox[q] = lattice<POW2>((uint32_t)(r >> 32), A.wx, A.shx);
            oy[q] = lattice<POW2>((uint32_t)r, A.wy, A.shy);
            // 64-bit shifts: a 2^32-wide side with one cell shifts by 32
            const int cx = (int)((uint64_t)ox[q] >> A.sbx), cy = (int)((uint64_t)oy[q] >> A.sby);
            cell[q] = j < A.horizon ? ((cy << A.bits) | cx) : cells;
            rank[q] = atomicAdd(&s_cnt[cell[q]], 1);
        }
    }
    __syncthreads();
    // exclusive scan of the cells + 1 counts: strips of consecutive counts per
    // thread, a wavefront scan of the strip sums, then the wavefront totals
    const int per = (cells + 1 + kBinThreads - 1) / kBinThreads;
    const int t0 = tid * per, t1 = min(t0 + per, cells + 1);
    int sum = 0;
    for (int t = t0; t < t1; t++) sum += s_cnt[t];
    const int incl = wave_incl_scan32(sum);
    if (lane == 63) s_wsum[wave] = incl;
    __syncthreads();
    int acc = incl - sum;
    for (int w = 0; w < wave; w++) acc += s_wsum[w];
    for (int t = t0; t < t1; t++) {
        s_start[t] = acc;
        acc += s_cnt[t];
    }
    __syncthreads();
    const size_t chunk = (size_t)i * A.nchunks + c;
    const size_t base = chunk << A.lchunk;
#pragma unroll
    for (int q = 0; q < kMaxSpt; q++) {
        if (q < spt) {
            const size_t pos = base + s_start[cell[q]] + rank[q];
            A.sxy[pos] = make_uint2(ox[q], oy[q]);
            A.sj[pos] = (uint16_t)(q * kBinThreads + tid);
        }
    }
    for (int t = tid; t <= cells; t += kBinThreads) A.cell_off[chunk * (cells + 1) + t] = (uint16_t)s_start[t];
}

struct LookupArgs {
    const int32_t *xy;
    const int64_t *off;
    const int32_t *mbr;
    const uint32_t *flags;
    const uint2 *sxy;
    const uint16_t *sj;
    const uint16_t *cell_off;
    uint32_t *sig;
    uint32_t *unresolved;          // [n] 1: a hash needs the walk, 2: the whole polygon is walked
    const int32_t *order;          // [n] polygons, longest lookups first (null: index order)
    int64_t n;
    int32_t k;
    uint32_t cap, horizon;
    int32_t nchunks, lchunk, bits, sbx, sby;
    int32_t bx0, by0, bx1, by1;
    int32_t lds_edges;
};

enum TestMode { kTestLds = 0, kTestStream = 1, kTestWide = 2 };

// Lane-serial crossing-number test of the lane's own point; every lane walks
// the same edge sequence, so the edge reads are broadcasts.
template <int MODE>
__device__ __forceinline__ bool inside_lane(const int4 *s_edges, const int32_t *pxy, int32_t n,
                                            int32_t px, int32_t py)
{
    bool odd = false;
    for (int e = 0; e < n; e++) {
        if constexpr (MODE == kTestLds) {
            odd ^= crosses_fp64(s_edges[e], px, py);
        } else {
            const int f = (e + 1 == n) ? 0 : e + 1;
            if constexpr (MODE == kTestStream) {
                const int2 a = *reinterpret_cast<const int2 *>(pxy + 2 * e);
                const int2 b = *reinterpret_cast<const int2 *>(pxy + 2 * f);
                odd ^= crosses_fp64(make_edge(a.x, a.y, b.x, b.y), px, py);
            } else {
                odd ^= crosses_i128(pxy + 2 * e, pxy + 2 * f, px, py);
            }
        }
    }
    return odd;
}

// Crossing-number test of each lane's point against edges read from memory
// 64 at a time, one edge per lane in one coalesced load, and handed to every
// lane by readlane (a load per edge made each step wait on memory).  Every
// lane of the wavefront takes part.
__device__ __forceinline__ bool inside_stream_block(const int32_t *pxy, int32_t n, int32_t px, int32_t py,
                                                    int lane)
{
    bool odd = false;
    for (int e0 = 0; e0 < n; e0 += 64) {
        const int e = e0 + lane < n ? e0 + lane : 0;
        const int f = (e + 1 == n) ? 0 : e + 1;
        const int2 a = *reinterpret_cast<const int2 *>(pxy + 2 * e);
        const int2 b = *reinterpret_cast<const int2 *>(pxy + 2 * f);
        const int4 ed = make_edge(a.x, a.y, b.x, b.y);
        const int cnt = min(64, n - e0);
        for (int t = 0; t < cnt; t++) {
            const int4 et = make_int4(__builtin_amdgcn_readlane(ed.x, t), __builtin_amdgcn_readlane(ed.y, t),
                                      __builtin_amdgcn_readlane(ed.z, t), __builtin_amdgcn_readlane(ed.w, t));
            odd ^= crosses_fp64(et, px, py);
        }
    }
    return odd;
}

// Test up to 64 queued points (lane = entry) and lower the owners' best index.
template <int MODE>
__device__ __forceinline__ void drain(const LookupArgs &A, const int4 *s_edges, const int32_t *pxy,
                                      int32_t n, const uint32_t *qm, const uint32_t *qx, const uint32_t *qy,
                                      int head, int count, uint32_t chunk_base, uint32_t *s_best, int lane)
{
    if constexpr (MODE == kTestStream) {
        // all lanes load the edge blocks; lanes past count test entry head
        const int q = (head + (lane < count ? lane : 0)) & (kQueue - 1);
        const uint32_t meta = qm[q];
        const int32_t px = (int32_t)((uint32_t)A.bx0 + qx[q]), py = (int32_t)((uint32_t)A.by0 + qy[q]);
        const bool in = inside_stream_block(pxy, n, px, py, lane);
        if (lane < count && in) atomicMin(&s_best[meta >> 12], chunk_base + (meta & 0xfffu));
        return;
    }
    if (lane < count) {
        const int q = (head + lane) & (kQueue - 1);
        const uint32_t meta = qm[q];
        const int32_t px = (int32_t)((uint32_t)A.bx0 + qx[q]), py = (int32_t)((uint32_t)A.by0 + qy[q]);
        if (inside_lane<MODE>(s_edges, pxy, n, px, py))
            atomicMin(&s_best[meta >> 12], chunk_base + (meta & 0xfffu));
    }
}

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_wave_barrier();
}

// Per-wavefront state of one polygon's lookup.
struct Scan {
    uint32_t mx0, my0, mx1, my1;   // MBR as lattice offsets inside B
    uint32_t *qm, *qx, *qy, *s_best;
    int head, tail;
};

// Stream the lane's samples [lo, hi) of one grid row (cells contiguous in the
// chunk's order), queue those inside the MBR, drain whenever 64 are waiting.
template <int MODE>
__device__ __forceinline__ void scan_row(const LookupArgs &A, const int4 *s_edges, const int32_t *pxy, int32_t n,
                                         Scan &S, size_t base, int lo, int hi, uint32_t chunk_base, int lane)
{
    const int cnt = hi - lo;
    const int steps = wave_max32(cnt);
    for (int s = 0; s < steps; s++) {
        bool pass = false;
        uint2 o = make_uint2(0u, 0u);
        if (s < cnt) {
            o = A.sxy[base + lo + s];
            pass = (o.x >= S.mx0) & (o.x <= S.mx1) & (o.y >= S.my0) & (o.y <= S.my1);
        }
        const uint64_t mk = __ballot(pass);
        if (pass) {
            const uint32_t jl = A.sj[base + lo + s];
            const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mk >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0u));
            const int q = (S.tail + rank) & (kQueue - 1);
            S.qm[q] = ((uint32_t)lane << 12) | jl;
            S.qx[q] = o.x;
            S.qy[q] = o.y;
        }
        S.tail += __popcll(mk);
        if (S.tail - S.head >= 64) {
            wave_sync_lds();
            drain<MODE>(A, s_edges, pxy, n, S.qm, S.qx, S.qy, S.head, 64, chunk_base, S.s_best, lane);
            S.head += 64;
            wave_sync_lds();
        }
    }
}

// Lane = hash i.  Chunks in order; a lane stops after the first chunk with a
// hit, the wavefront when all its lanes have.
template <int MODE>
__device__ void lookup_polygon(const LookupArgs &A, const int4 *s_edges, const int32_t *pxy, int32_t n,
                               Scan &S, int cx0, int cx1, int cy0, int cy1, int i, bool active, int lane,
                               uint32_t &best)
{
    const int cells = 1 << (2 * A.bits);
    const int C = 1 << A.lchunk;
    const int rows = cy1 - cy0 + 1;
    best = active ? kNone : 0u;
    for (int c = 0; c < A.nchunks; c++) {
        const bool open = active && best == kNone;
        if (__ballot(open) == 0) break;
        S.s_best[lane] = kNone;
        S.head = S.tail = 0;
        const size_t chunk = (size_t)i * A.nchunks + c;
        const uint16_t *co = A.cell_off + chunk * (cells + 1);
        const size_t base = chunk << A.lchunk;
        const uint32_t chunk_base = (uint32_t)c << A.lchunk;
        // the first four rows' ranges are loaded together
        int lo[4], hi[4];
#pragma unroll
        for (int r = 0; r < 4; r++) {
            lo[r] = hi[r] = 0;
            if (open && r < rows) {
                const int row = (cy0 + r) << A.bits;
                lo[r] = min((int)co[row | cx0], C);
                hi[r] = min((int)co[(row | cx1) + 1], C);
            }
        }
#pragma unroll
        for (int r = 0; r < 4; r++)
            if (r < rows) scan_row<MODE>(A, s_edges, pxy, n, S, base, lo[r], hi[r], chunk_base, lane);
        for (int r = 4; r < rows; r++) {
            const int row = (cy0 + r) << A.bits;
            const int l = open ? min((int)co[row | cx0], C) : 0, h = open ? min((int)co[(row | cx1) + 1], C) : 0;
            scan_row<MODE>(A, s_edges, pxy, n, S, base, l, h, chunk_base, lane);
        }
        while (S.tail > S.head) {
            wave_sync_lds();
            const int cnt = min(64, S.tail - S.head);
            drain<MODE>(A, s_edges, pxy, n, S.qm, S.qx, S.qy, S.head, cnt, chunk_base, S.s_best, lane);
            S.head += cnt;
            wave_sync_lds();
        }
        wave_sync_lds();
        if (open) best = S.s_best[lane];
    }
}

// One workgroup of 64 * W threads (W = min(4, ceil(k / 64)) wavefronts) per
// (polygon, group of 64 W hashes).
__global__ __launch_bounds__(256) void k_bin_lookup(LookupArgs A)
{
    extern __shared__ int4 s_edges[];
    __shared__ uint32_t s_qm[4][kQueue], s_qx[4][kQueue], s_qy[4][kQueue];
    __shared__ uint32_t s_best[4][64];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int per = blockDim.x;
    const int groups = (A.k + per - 1) / per;
    // workgroups start in order of their index: the order (small launches)
    // puts the longest first
    const int64_t p = A.order ? (int64_t)A.order[blockIdx.x / groups] : (int64_t)(blockIdx.x / groups);
    const int i = (int)(blockIdx.x % groups) * per + tid;
    const bool active = i < A.k;
    if (A.unresolved[p] & 2u) return;    // walked (uniform per workgroup, before any barrier)
    const int64_t a = A.off[p];
    const int32_t n = (int32_t)(A.off[p + 1] - a);
    const uint32_t fl = A.flags[p];
    const int4 mb = *reinterpret_cast<const int4 *>(A.mbr + 4 * p);
    uint32_t *out = A.sig + (size_t)p * (size_t)A.k;
    const bool empty = (fl & (kFlagFew | kFlagCollinear)) || mb.z < A.bx0 || mb.x > A.bx1 ||
                       mb.w < A.by0 || mb.y > A.by1;
    if (empty) {
        if (active) out[i] = 0u;
        return;
    }
    const int32_t *pxy = A.xy + 2 * a;
    const int mode = (fl & kFlagWide) ? kTestWide : (n <= A.lds_edges ? kTestLds : kTestStream);
    if (mode == kTestLds) {
        for (int e = tid; e < n; e += per) {
            const int f = (e + 1 == n) ? 0 : e + 1;
            const int2 u = *reinterpret_cast<const int2 *>(pxy + 2 * e);
            const int2 v = *reinterpret_cast<const int2 *>(pxy + 2 * f);
            s_edges[e] = make_edge(u.x, u.y, v.x, v.y);
        }
    }
    __syncthreads();
    Scan S;
    S.mx0 = (uint32_t)max(mb.x, A.bx0) - (uint32_t)A.bx0;
    S.my0 = (uint32_t)max(mb.y, A.by0) - (uint32_t)A.by0;
    S.mx1 = (uint32_t)min(mb.z, A.bx1) - (uint32_t)A.bx0;
    S.my1 = (uint32_t)min(mb.w, A.by1) - (uint32_t)A.by0;
    S.qm = s_qm[wave];
    S.qx = s_qx[wave];
    S.qy = s_qy[wave];
    S.s_best = s_best[wave];
    // 64-bit shifts: a 2^32-wide side with one cell shifts by 32
    const int cx0 = (int)((uint64_t)S.mx0 >> A.sbx), cx1 = (int)((uint64_t)S.mx1 >> A.sbx);
    const int cy0 = (int)((uint64_t)S.my0 >> A.sby), cy1 = (int)((uint64_t)S.my1 >> A.sby);
    // a wavefront with no hash of its own skips the lookup (uniform per wave)
    uint32_t best = 0u;
    const int ic = active ? i : 0;
    if (__ballot(active) != 0) {
        if (mode == kTestLds)
            lookup_polygon<kTestLds>(A, s_edges, pxy, n, S, cx0, cx1, cy0, cy1, ic, active, lane, best);
        else if (mode == kTestStream)
            lookup_polygon<kTestStream>(A, s_edges, pxy, n, S, cx0, cx1, cy0, cy1, ic, active, lane, best);
        else
            lookup_polygon<kTestWide>(A, s_edges, pxy, n, S, cx0, cx1, cy0, cy1, ic, active, lane, best);
    }
    if (active) {
        if (best != kNone) out[i] = best + 1;
        else if (A.horizon >= A.cap) out[i] = 0u;
        else atomicOr(&A.unresolved[p], 1u);
    }
}

// Dispatch order of the polygons for the lookup, longest first.  With
// h = C x area / |B| expected hits per chunk, a chunk has a hit with
// probability P = 1 - exp(-h); a workgroup runs until the last of its 256
// hashes has one, about ln(256) / P chunks (capped at the horizon), each a
// few round trips to memory, and tests about max(1, m) / P samples a hash
// (m = C x A_MBR / |B| samples in the MBR per chunk) against its n edges.
// Started last, the few polygons with the largest such cost set the
// launch's duration; started first, they overlap the rest.  A counting sort
// on a quantised estimate (descending; the order within a key is the
// arrival order, which affects only timing).  Walked and degenerate
// polygons, whose workgroups return at once, go last.
constexpr int kOrderCells = 4096;
constexpr int64_t kOrderMaxPolys = 65536;

__global__ __launch_bounds__(256) void k_order_count(const int64_t *__restrict__ area2,
                                                     const int64_t *__restrict__ off,
                                                     const int32_t *__restrict__ mbr,
                                                     const uint32_t *__restrict__ unresolved, int64_t n,
                                                     double box_area, double chunk, double nchunks,
                                                     uint16_t *__restrict__ key, int32_t *__restrict__ counts)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const double area = 0.5 * (double)(area2[p] < 0 ? -area2[p] : area2[p]);
        int k = kOrderCells - 1;
        if (!(unresolved[p] & 2u) && area > 0.0) {
            const int4 b = *reinterpret_cast<const int4 *>(mbr + 4 * p);
            const double a_mbr = ((double)b.z - (double)b.x + 1.0) * ((double)b.w - (double)b.y + 1.0);
            const double P = -expm1(-chunk * area / box_area);
            const double chunks = fmin(nchunks, 5.545 / P);             // ln(256) / P
            const double tests = fmax(1.0, chunk * a_mbr / box_area) / P;
            const double est = 16.0 * chunks + tests * (double)(off[p + 1] - off[p]) / 8.0;
            k = kOrderCells - 1 - (int)fmin(est, (double)(kOrderCells - 1));
        }
        key[p] = (uint16_t)k;
        // the last key (every walked polygon) is counted once a wavefront
        const bool last = k == kOrderCells - 1;
        const uint64_t m = __ballot(last);
        if (!last) atomicAdd(&counts[k], 1);
        else if ((int)(threadIdx.x & 63) == __builtin_ctzll(m)) atomicAdd(&counts[k], __popcll(m));
    }
}

// Exclusive prefix of the kOrderCells counts in place (one block of 1024).
__global__ __launch_bounds__(1024) void k_order_scan(int32_t *__restrict__ counts)
{
    constexpr int kPer = kOrderCells / 1024;
    __shared__ int sw[16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int v[kPer], sum = 0;
#pragma unroll
    for (int u = 0; u < kPer; u++) {
        v[u] = counts[kPer * tid + u];
        sum += v[u];
    }
    const int incl = wave_incl_scan32(sum);
    if (lane == 63) sw[wave] = incl;
    __syncthreads();
    int pre = incl - sum;
    for (int w = 0; w < wave; w++) pre += sw[w];
#pragma unroll
    for (int u = 0; u < kPer; u++) {
        counts[kPer * tid + u] = pre;
        pre += v[u];
    }
}

__global__ __launch_bounds__(256) void k_order_scatter(const uint16_t *__restrict__ key, int64_t n,
                                                       int32_t *__restrict__ cursor, int32_t *__restrict__ order)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const int k = key[p];
        // positions of the last key are claimed once a wavefront
        const bool last = k == kOrderCells - 1;
        const uint64_t m = __ballot(last);
        int pos;
        if (last) {
            const int leader = __builtin_ctzll(m);
            int base = 0;
            if ((int)(threadIdx.x & 63) == leader) base = atomicAdd(&cursor[k], __popcll(m));
            base = __shfl(base, leader, 64);
            pos = base + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        } else {
            pos = atomicAdd(&cursor[k], 1);
        }
        order[pos] = (int32_t)p;
    }
}

// Flags: 2 for a polygon to walk whole, else 0 (twice the area exact from
// prepare).  With walk_ratio > 0 a polygon is walked when |B| < walk_ratio x
// area, or when its walk is expected to cost less than its lookup, in edge
// tests per hash: the walk draws about |B| / area points (kDrawTests edge
// tests each) and tests the about A_mbr / area of them inside the MBR against
// its n edges; the lookup visits chunks until one has a hit (each does with
// probability P = 1 - exp(-C area / |B|)) and tests every sample of them
// that lies in the MBR, about max(1, C A_mbr / |B|) a chunk, against its n
// edges.  Either way the signature is the same.  A polygon beyond the
// lookup's LDS edge cache (walk_edges) is walked too, and in a small launch
// so is one whose lookup would test more than test_cap edges a hash: one
// lookup workgroup tests its 256 hashes' points with four wavefronts, a
// long serial run that sets a small launch's duration, where the walk
// spreads a polygon's hashes over many work items and each test over the
// lanes.  Degenerate polygons stay with the lookup, which signs them 0 at
// once.
constexpr double kDrawTests = 5.0;
constexpr double kLookupTestCap = 2048.0;

__global__ __launch_bounds__(256) void k_classify(const int64_t *__restrict__ area2,
                                                  const uint32_t *__restrict__ flags,
                                                  const int64_t *__restrict__ off,
                                                  const int32_t *__restrict__ mbr, int64_t n,
                                                  double box_area, double walk_ratio, double chunk,
                                                  double walk_edges, double test_cap,
                                                  uint32_t *__restrict__ unresolved)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const bool degenerate = (flags[p] & (kFlagFew | kFlagCollinear)) != 0;
        const double area = 0.5 * (double)(area2[p] < 0 ? -area2[p] : area2[p]);
        bool walk = false;
        if (!degenerate && walk_ratio > 0.0 && area > 0.0) {
            const int4 m = *reinterpret_cast<const int4 *>(mbr + 4 * p);
            const double a_mbr = ((double)m.z - (double)m.x + 1.0) * ((double)m.w - (double)m.y + 1.0);
            const double edges = (double)(off[p + 1] - off[p]);
            const double walk_cost = kDrawTests * box_area / area + edges * a_mbr / area;
            const double hit = -expm1(-chunk * area / box_area);         // P(a chunk has a hit)
            const double bin_cost = edges * fmax(1.0, chunk * a_mbr / box_area) / hit;
            walk = box_area < walk_ratio * area || walk_cost < bin_cost || edges > walk_edges ||
                   bin_cost > test_cap;
        }
        unresolved[p] = walk ? 2u : 0u;
    }
}

// Polygons with an unresolved hash, or walked whole, listed for the walk.
__global__ __launch_bounds__(256) void k_unresolved_list(const uint32_t *__restrict__ unresolved, int64_t n,
                                                         int32_t *__restrict__ list, int32_t *__restrict__ count)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x)
        if (unresolved[p]) list[atomicAdd(count, 1)] = (int32_t)p;
}

__global__ __launch_bounds__(256) void k_zero_words(uint32_t *p, int64_t count)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x)
        p[t] = 0u;
}


int ceil_log2(uint64_t w)
{
    int l = 0;
    while ((1ull << l) < w) l++;
    return l;
}

int grid_for(int64_t items)
{
    int64_t g = (items + 255) / 256;
    return (int)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

// Chunk of about one sample per cell, 256..4096 samples.
int chunk_log2(int32_t bits)
{
    const int l = 2 * bits;
    return l < 8 ? 8 : (l > 12 ? 12 : l);
}

struct BinnedWs {
    uint2 *sxy;
    uint16_t *sj, *cell_off;
    uint32_t *unresolved;
    int32_t *list, *count;
    int32_t *order, *cell_counts;
    uint16_t *key;
};

BinnedWs carve_binned(Carve &c, int32_t k, int64_t nchunks, int32_t bits, int64_t n)
{
    const int64_t samples = ((int64_t)k * nchunks) << chunk_log2(bits);
    const int64_t cells = ((int64_t)1 << (2 * bits)) + 1;
    BinnedWs w{};
    w.sxy = c.take<uint2>((size_t)samples);
    w.sj = c.take<uint16_t>((size_t)samples);
    w.cell_off = c.take<uint16_t>((size_t)((int64_t)k * nchunks * cells));
    w.unresolved = c.take<uint32_t>((size_t)n);
    w.list = c.take<int32_t>((size_t)n);
    w.count = c.take<int32_t>(1);
    w.order = c.take<int32_t>((size_t)n);
    w.cell_counts = c.take<int32_t>((size_t)kOrderCells);
    w.key = c.take<uint16_t>((size_t)n);
    return w;
}

}  // namespace

size_t binned_workspace_bytes(int32_t k, uint32_t horizon, int32_t bits, int64_t n)
{
    const int64_t C = (int64_t)1 << chunk_log2(bits);
    Carve c{nullptr, 0};
    carve_binned(c, k, ((int64_t)horizon + C - 1) / C, bits, n);
    return align_up(c.used, 256);
}

polymh_status launch_sign_binned(const SignLaunch &L, const int64_t *area2, uint32_t horizon, int32_t bits,
                                 double walk_ratio, void *ws, size_t ws_bytes, hipStream_t s, bool rebin)
{
    const uint64_t wx = (uint64_t)((int64_t)L.box.xmax - L.box.xmin + 1);
    const uint64_t wy = (uint64_t)((int64_t)L.box.ymax - L.box.ymin + 1);
    const int lx = ceil_log2(wx), ly = ceil_log2(wy);
    const bool pow2 = (1ull << lx) == wx && (1ull << ly) == wy && lx >= 1 && ly >= 1;
    const int lchunk = chunk_log2(bits);
    const int64_t nchunks = ((int64_t)horizon + ((int64_t)1 << lchunk) - 1) >> lchunk;
    if (nchunks > 65535) return set_error(POLYMH_EINVAL, "sign_binned: horizon too large");
    Carve cv{static_cast<char *>(ws), ws_bytes};
    BinnedWs w = carve_binned(cv, L.k, nchunks, bits, L.n);
    if (!cv.ok)
        return set_error(POLYMH_ECAPACITY, "sign_binned: workspace of %zu bytes, need %zu", ws_bytes, cv.used);
    BinArgs B{};
    B.seed = L.seed;
    B.k = L.k;
    B.horizon = horizon;
    B.nchunks = (int32_t)nchunks;
    B.lchunk = lchunk;
    B.bits = bits;
    B.sbx = lx > bits ? lx - bits : 0;
    B.sby = ly > bits ? ly - bits : 0;
    B.wx = (uint32_t)wx;
    B.wy = (uint32_t)wy;
    B.shx = pow2 ? 32 - lx : 0;
    B.shy = pow2 ? 32 - ly : 0;
    B.sxy = w.sxy;
    B.sj = w.sj;
    B.cell_off = w.cell_off;
    const size_t bin_lds = 2 * (((size_t)1 << (2 * bits)) + 1) * sizeof(int);
    // without rebin the workspace already holds these bins (an earlier call
    // with the same arguments); the lookup clamps every cell range to its
    // chunk, so bins that are not there give wrong values, never a stray read
    if (rebin) {
        if (pow2) hipLaunchKernelGGL(k_bin<true>, dim3((unsigned)nchunks, (unsigned)L.k), dim3(kBinThreads), bin_lds, s, B);
        else hipLaunchKernelGGL(k_bin<false>, dim3((unsigned)nchunks, (unsigned)L.k), dim3(kBinThreads), bin_lds, s, B);
    }
    polymh_status st = check_launch("sign_binned: bin");
    if (st) return st;
    // one workgroup per (polygon, group of up to 256 hashes)
    const int64_t waves = (L.k + 63) / 64 < 4 ? (L.k + 63) / 64 : 4;
    const int64_t per = 64 * waves, groups = (L.k + per - 1) / per;
    const int64_t units = L.n * groups;
    const double walk_edges = (double)L.cfg.lds_edges;
    // the order and the cap on a lookup's tests serve small launches, where a
    // few costly polygons set the duration; a large launch hides them
    const bool ordered = L.n <= kOrderMaxPolys;
    hipLaunchKernelGGL(k_classify, dim3(grid_for(L.n)), dim3(256), 0, s, area2, L.flags, L.off, L.mbr, L.n,
                       (double)wx * (double)wy, walk_ratio, (double)((int64_t)1 << lchunk), walk_edges,
                       ordered ? kLookupTestCap : INFINITY, w.unresolved);
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, s, reinterpret_cast<uint32_t *>(w.count), (int64_t)1);
    // the lookup's dispatch order (after the classification: walked polygons
    // last), in small launches only
    if (ordered) {
        hipLaunchKernelGGL(k_zero_words, dim3(kOrderCells / 256), dim3(256), 0, s,
                           reinterpret_cast<uint32_t *>(w.cell_counts), (int64_t)kOrderCells);
        hipLaunchKernelGGL(k_order_count, dim3(grid_for(L.n)), dim3(256), 0, s, area2, L.off, L.mbr, w.unresolved, L.n,
                           (double)wx * (double)wy, (double)((int64_t)1 << lchunk), (double)nchunks, w.key,
                           w.cell_counts);
        hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(1024), 0, s, w.cell_counts);
        hipLaunchKernelGGL(k_order_scatter, dim3(grid_for(L.n)), dim3(256), 0, s, w.key, L.n, w.cell_counts, w.order);
    }
    polymh_status st0 = check_launch("sign_binned: order");
    if (st0) return st0;
    LookupArgs A{};
    A.xy = L.xy;
    A.off = L.off;
    A.mbr = L.mbr;
    A.flags = L.flags;
    A.sxy = w.sxy;
    A.sj = w.sj;
    A.cell_off = w.cell_off;
    A.sig = L.sig;
    A.unresolved = w.unresolved;
    A.order = ordered ? w.order : nullptr;
    A.n = L.n;
    A.k = L.k;
    A.cap = L.cap;
    A.horizon = horizon;
    A.nchunks = (int32_t)nchunks;
    A.lchunk = lchunk;
    A.bits = bits;
    A.sbx = B.sbx;
    A.sby = B.sby;
    A.bx0 = L.box.xmin; A.by0 = L.box.ymin; A.bx1 = L.box.xmax; A.by1 = L.box.ymax;
    A.lds_edges = L.cfg.lds_edges;
    const int64_t grid = units;
    if (grid > 0x7fffffff) return set_error(POLYMH_EINVAL, "sign_binned: too many work items");
    const size_t lds = (size_t)L.cfg.lds_edges * sizeof(int4);
    hipLaunchKernelGGL(k_bin_lookup, dim3((unsigned)grid), dim3((unsigned)per), lds, s, A);
    if ((st = check_launch("sign_binned: lookup"))) return st;
    if (horizon >= L.cap && walk_ratio <= 0.0) return POLYMH_OK;
    // the walk for polygons with a hash unresolved below the horizon, and
    // those left to it whole
    hipLaunchKernelGGL(k_unresolved_list, dim3(grid_for(L.n)), dim3(256), 0, s, w.unresolved, L.n, w.list, w.count);
    if ((st = check_launch("sign_binned: list"))) return st;
    SignLaunch W = L;
    W.order = w.list;
    W.n_dev = w.count;
    W.cfg.persistent = 1;
    // in a small launch the few polygons left to the walk are the costly
    // ones (many edges or deep hits) and set its duration: 8 hashes a work
    // item (one a wavefront) spread one polygon's hashes over many
    // workgroups (in a large launch that only multiplies the staging of the
    // many cheap walks of large polygons)
    if (units < 32768 && (W.cfg.hash_block <= 0 || W.cfg.hash_block > 8)) W.cfg.hash_block = 8;
    return launch_sign(W, s);
}

}  // namespace polymh
