// Shared-sample binned signing: the signatures of Alg. 1 / Def. 2, bit for
// bit, without walking every (polygon, hash) stream.  All polygons read the
// same point stream per hash (Sec. 3.2's fixed-seed generators), so the
// samples j < horizon of every hash are drawn once, in chunks of 256, and
// each chunk's samples are grouped by cell of a 2^b x 2^b grid over B.  A
// (polygon, hash) unit then visits the chunks in order and, in each, the
// samples of the cells its MBR meets: those inside the MBR are tested for
// membership and the smallest inside index of the first chunk that has one
// is the first hit (every sample inside the polygon lies in its MBR, hence
// in those cells).  Units with no hit below the horizon are walked from the
// start by the per-unit kernel, so every value equals Alg. 1's.
#include "internal.hpp"
#include "sign_common.hpp"

namespace polymh {

namespace {

constexpr int kChunk = 256;        // samples per chunk (one workgroup draws a chunk)
constexpr int kQueue = 128;        // per-wavefront queue of membership tests
constexpr uint32_t kNone = 0xffffffffu;

struct BinArgs {
    uint64_t seed;
    int32_t k;
    uint32_t horizon;              // samples per hash (j < horizon), <= cap
    int32_t nchunks;
    int32_t bits;                  // grid side 2^bits (0..4)
    int32_t sbx, sby;              // cell of offset o: o >> sb
    uint32_t wx, wy;
    int32_t shx, shy;
    uint32_t *sx, *sy;             // [k][nchunks][kChunk] lattice offsets, grouped by cell
    uint8_t *sj;                   // index inside the chunk
    uint16_t *cell_off;            // [k][nchunks][cells + 1]
};

// One workgroup of 256 threads per (chunk, hash): draw, cell, counting sort
// in LDS (samples past the horizon go to an extra last cell that no lookup
// reads).
template <bool POW2>
__global__ __launch_bounds__(kChunk) void k_bin(BinArgs A)
{
    __shared__ int s_cnt[kChunk + 1];
    __shared__ int s_start[kChunk + 1];
    const int tid = threadIdx.x;
    const int c = blockIdx.x, i = blockIdx.y;
    const int cells = 1 << (2 * A.bits);
    for (int t = tid; t <= cells; t += kChunk) s_cnt[t] = 0;
    __syncthreads();
    const uint64_t j = (uint64_t)c * kChunk + tid;
    const bool valid = j < A.horizon;
    const uint64_t key = mix64(A.seed + (uint64_t)(i + 1) * kGamma);
    const uint64_t r = mix64(key + (j + 1) * kGamma);
    const uint32_t ox = lattice<POW2>((uint32_t)(r >> 32), A.wx, A.shx);
    const uint32_t oy = lattice<POW2>((uint32_t)r, A.wy, A.shy);
    // 64-bit shifts: a 2^32-wide side with one cell shifts by 32
    const int cx = (int)((uint64_t)ox >> A.sbx), cy = (int)((uint64_t)oy >> A.sby);
    const int cell = valid ? ((cy << A.bits) | cx) : cells;
    const int rank = atomicAdd(&s_cnt[cell], 1);
    __syncthreads();
    if (tid == 0) {
        // cells + 1 <= 257 counts: a serial exclusive scan is cheap beside the draws
        int acc = 0;
        for (int t = 0; t <= cells; t++) {
            s_start[t] = acc;
            acc += s_cnt[t];
        }
    }
    __syncthreads();
    const size_t chunk = (size_t)i * A.nchunks + c;
    const size_t pos = chunk * kChunk + s_start[cell] + rank;
    A.sx[pos] = ox;
    A.sy[pos] = oy;
    A.sj[pos] = (uint8_t)tid;
    for (int t = tid; t <= cells; t += kChunk) A.cell_off[chunk * (cells + 1) + t] = (uint16_t)s_start[t];
}

struct LookupArgs {
    const int32_t *xy;
    const int64_t *off;
    const int32_t *mbr;
    const uint32_t *flags;
    const uint32_t *sx, *sy;
    const uint8_t *sj;
    const uint16_t *cell_off;
    uint32_t *sig;
    uint32_t *unresolved;          // [n] set to 1 where a hash needs the walk
    int64_t n;
    int32_t k;
    uint32_t cap, horizon;
    int32_t nchunks, bits, sbx, sby;
    int32_t bx0, by0, bx1, by1;
    int32_t lds_edges;
};

enum TestMode { kTestLds = 0, kTestStream = 1, kTestWide = 2 };

// Lane-serial crossing-number test of the lane's own point (every lane walks
// the same edge sequence, so the LDS reads are broadcasts).
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

// Test up to 64 queued points (lane = entry) and lower the owners' best index.
template <int MODE>
__device__ __forceinline__ void drain(const LookupArgs &A, const int4 *s_edges, const int32_t *pxy,
                                      int32_t n, const uint32_t *qm, const uint32_t *qx, const uint32_t *qy,
                                      int head, int count, uint32_t chunk_base, uint32_t *s_best, int lane)
{
    if (lane < count) {
        const int q = (head + lane) & (kQueue - 1);
        const uint32_t meta = qm[q];
        const int32_t px = (int32_t)((uint32_t)A.bx0 + qx[q]), py = (int32_t)((uint32_t)A.by0 + qy[q]);
        if (inside_lane<MODE>(s_edges, pxy, n, px, py))
            atomicMin(&s_best[meta >> 8], chunk_base + (meta & 0xffu));
    }
}

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_wave_barrier();
}

// One workgroup (4 wavefronts, 64 hashes each) per (polygon, group of 256
// hashes).  Lane = hash.  Per chunk, the lanes stream the samples of the
// cells under the MBR; samples inside the MBR are queued and tested 64 at a
// time by all lanes; a lane stops after the first chunk with a hit.
template <int MODE>
__device__ void lookup_polygon(const LookupArgs &A, const int4 *s_edges, const int32_t *pxy, int32_t n,
                               int4 mb, int i, bool active, int lane, uint32_t *qm, uint32_t *qx,
                               uint32_t *qy, uint32_t *s_best, uint32_t &best)
{
    // MBR as lattice offsets inside B (the polygon meets B here)
    const uint32_t mx0 = (uint32_t)max(mb.x, A.bx0) - (uint32_t)A.bx0;
    const uint32_t my0 = (uint32_t)max(mb.y, A.by0) - (uint32_t)A.by0;
    const uint32_t mx1 = (uint32_t)min(mb.z, A.bx1) - (uint32_t)A.bx0;
    const uint32_t my1 = (uint32_t)min(mb.w, A.by1) - (uint32_t)A.by0;
    const int cx0 = (int)((uint64_t)mx0 >> A.sbx), cx1 = (int)((uint64_t)mx1 >> A.sbx);
    const int cy0 = (int)((uint64_t)my0 >> A.sby), cy1 = (int)((uint64_t)my1 >> A.sby);
    const int cells = 1 << (2 * A.bits);
    best = active ? kNone : 0u;
    for (int c = 0; c < A.nchunks; c++) {
        const bool open = active && best == kNone;
        if (__ballot(open) == 0) break;
        s_best[lane] = kNone;
        int head = 0, tail = 0;
        const size_t chunk = (size_t)i * A.nchunks + c;
        const uint16_t *co = A.cell_off + chunk * (cells + 1);
        const size_t sbase = chunk * kChunk;
        for (int cy = cy0; cy <= cy1; cy++) {
            for (int cx = cx0; cx <= cx1; cx++) {
                const int cell = (cy << A.bits) | cx;
                const int lo = open ? (int)co[cell] : 0;
                const int cnt = open ? (int)co[cell + 1] - lo : 0;
                const int steps = wave_max32(cnt);
                for (int s = 0; s < steps; s++) {
                    bool pass = false;
                    uint32_t ox = 0, oy = 0, jl = 0;
                    if (s < cnt) {
                        const size_t at = sbase + lo + s;
                        ox = A.sx[at];
                        oy = A.sy[at];
                        jl = A.sj[at];
                        pass = (ox >= mx0) & (ox <= mx1) & (oy >= my0) & (oy <= my1);
                    }
                    const uint64_t mk = __ballot(pass);
                    if (pass) {
                        const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mk >> 32),
                                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0u));
                        const int q = (tail + rank) & (kQueue - 1);
                        qm[q] = ((uint32_t)lane << 8) | jl;
                        qx[q] = ox;
                        qy[q] = oy;
                    }
                    tail += __popcll(mk);
                    if (tail - head >= 64) {
                        wave_sync_lds();
                        drain<MODE>(A, s_edges, pxy, n, qm, qx, qy, head, 64, (uint32_t)c * kChunk, s_best, lane);
                        head += 64;
                        wave_sync_lds();
                    }
                }
            }
        }
        while (tail > head) {
            wave_sync_lds();
            const int cnt = min(64, tail - head);
            drain<MODE>(A, s_edges, pxy, n, qm, qx, qy, head, cnt, (uint32_t)c * kChunk, s_best, lane);
            head += cnt;
            wave_sync_lds();
        }
        wave_sync_lds();
        if (open) best = s_best[lane];
    }
}

__global__ __launch_bounds__(256) void k_bin_lookup(LookupArgs A)
{
    extern __shared__ int4 s_edges[];
    __shared__ uint32_t s_qm[4][kQueue], s_qx[4][kQueue], s_qy[4][kQueue];
    __shared__ uint32_t s_best[4][64];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int groups = (A.k + 255) / 256;
    const int64_t p = blockIdx.x / groups;
    const int i = (int)(blockIdx.x % groups) * 256 + wave * 64 + lane;
    const bool active = i < A.k;
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
        for (int e = tid; e < n; e += blockDim.x) {
            const int f = (e + 1 == n) ? 0 : e + 1;
            const int2 u = *reinterpret_cast<const int2 *>(pxy + 2 * e);
            const int2 v = *reinterpret_cast<const int2 *>(pxy + 2 * f);
            s_edges[e] = make_edge(u.x, u.y, v.x, v.y);
        }
    }
    __syncthreads();
    // a wavefront with no hash of its own skips the lookup (uniform per wave)
    uint32_t best = 0u;
    const bool wave_active = __ballot(active) != 0;
    const int ic = active ? i : 0;
    if (wave_active) {
        if (mode == kTestLds)
            lookup_polygon<kTestLds>(A, s_edges, pxy, n, mb, ic, active, lane, s_qm[wave], s_qx[wave], s_qy[wave], s_best[wave], best);
        else if (mode == kTestStream)
            lookup_polygon<kTestStream>(A, s_edges, pxy, n, mb, ic, active, lane, s_qm[wave], s_qx[wave], s_qy[wave], s_best[wave], best);
        else
            lookup_polygon<kTestWide>(A, s_edges, pxy, n, mb, ic, active, lane, s_qm[wave], s_qx[wave], s_qy[wave], s_best[wave], best);
    }
    if (active) {
        if (best != kNone) out[i] = best + 1;
        else if (A.horizon >= A.cap) out[i] = 0u;
        else atomicOr(&A.unresolved[p], 1u);
    }
}

// Polygons with an unresolved hash, listed for the walk.
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

}  // namespace

size_t binned_workspace_bytes(int32_t k, uint32_t horizon, int32_t bits, int64_t n)
{
    const int64_t nchunks = ((int64_t)horizon + kChunk - 1) / kChunk;
    const int64_t samples = (int64_t)k * nchunks * kChunk;
    const int64_t cells = ((int64_t)1 << (2 * bits)) + 1;
    Carve c{nullptr, 0};
    c.take<uint32_t>((size_t)samples);
    c.take<uint32_t>((size_t)samples);
    c.take<uint8_t>((size_t)samples);
    c.take<uint16_t>((size_t)((int64_t)k * nchunks * cells));
    c.take<uint32_t>((size_t)n);        // unresolved flags
    c.take<int32_t>((size_t)n);         // their list
    c.take<int32_t>(1);                 // its length
    return align_up(c.used, 256);
}

polymh_status launch_sign_binned(const SignLaunch &L, uint32_t horizon, int32_t bits, void *ws, size_t ws_bytes,
                                 hipStream_t s)
{
    const uint64_t wx = (uint64_t)((int64_t)L.box.xmax - L.box.xmin + 1);
    const uint64_t wy = (uint64_t)((int64_t)L.box.ymax - L.box.ymin + 1);
    const int lx = ceil_log2(wx), ly = ceil_log2(wy);
    const bool pow2 = (1ull << lx) == wx && (1ull << ly) == wy && lx >= 1 && ly >= 1;
    const int64_t nchunks = ((int64_t)horizon + kChunk - 1) / kChunk;
    if (nchunks > 65535) return set_error(POLYMH_EINVAL, "sign_binned: horizon too large");
    Carve cv{static_cast<char *>(ws), ws_bytes};
    const int64_t samples = (int64_t)L.k * nchunks * kChunk;
    const int64_t cells = ((int64_t)1 << (2 * bits)) + 1;
    BinArgs B{};
    B.sx = cv.take<uint32_t>((size_t)samples);
    B.sy = cv.take<uint32_t>((size_t)samples);
    B.sj = cv.take<uint8_t>((size_t)samples);
    B.cell_off = cv.take<uint16_t>((size_t)((int64_t)L.k * nchunks * cells));
    uint32_t *unres = cv.take<uint32_t>((size_t)L.n);
    int32_t *list = cv.take<int32_t>((size_t)L.n);
    int32_t *count = cv.take<int32_t>(1);
    if (!cv.ok)
        return set_error(POLYMH_ECAPACITY, "sign_binned: workspace of %zu bytes, need %zu", ws_bytes, cv.used);
    B.seed = L.seed;
    B.k = L.k;
    B.horizon = horizon;
    B.nchunks = (int32_t)nchunks;
    B.bits = bits;
    B.sbx = lx > bits ? lx - bits : 0;
    B.sby = ly > bits ? ly - bits : 0;
    B.wx = (uint32_t)wx;
    B.wy = (uint32_t)wy;
    B.shx = pow2 ? 32 - lx : 0;
    B.shy = pow2 ? 32 - ly : 0;
    if (pow2) hipLaunchKernelGGL(k_bin<true>, dim3((unsigned)nchunks, (unsigned)L.k), dim3(kChunk), 0, s, B);
    else hipLaunchKernelGGL(k_bin<false>, dim3((unsigned)nchunks, (unsigned)L.k), dim3(kChunk), 0, s, B);
    polymh_status st = check_launch("sign_binned: bin");
    if (st) return st;
    hipLaunchKernelGGL(k_zero_words, dim3(grid_for(L.n + 1)), dim3(256), 0, s, unres, L.n);
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, s, reinterpret_cast<uint32_t *>(count), (int64_t)1);
    LookupArgs A{};
    A.xy = L.xy;
    A.off = L.off;
    A.mbr = L.mbr;
    A.flags = L.flags;
    A.sx = B.sx;
    A.sy = B.sy;
    A.sj = B.sj;
    A.cell_off = B.cell_off;
    A.sig = L.sig;
    A.unresolved = unres;
    A.n = L.n;
    A.k = L.k;
    A.cap = L.cap;
    A.horizon = horizon;
    A.nchunks = (int32_t)nchunks;
    A.bits = bits;
    A.sbx = B.sbx;
    A.sby = B.sby;
    A.bx0 = L.box.xmin; A.by0 = L.box.ymin; A.bx1 = L.box.xmax; A.by1 = L.box.ymax;
    A.lds_edges = L.cfg.lds_edges;
    const int64_t groups = (L.k + 255) / 256;
    const int64_t grid = L.n * groups;
    if (grid > 0x7fffffff) return set_error(POLYMH_EINVAL, "sign_binned: too many work items");
    const size_t lds = (size_t)L.cfg.lds_edges * sizeof(int4);
    hipLaunchKernelGGL(k_bin_lookup, dim3((unsigned)grid), dim3(256), lds, s, A);
    if ((st = check_launch("sign_binned: lookup"))) return st;
    if (horizon >= L.cap) return POLYMH_OK;
    // the walk for polygons with a hash unresolved below the horizon
    hipLaunchKernelGGL(k_unresolved_list, dim3(grid_for(L.n)), dim3(256), 0, s, unres, L.n, list, count);
    if ((st = check_launch("sign_binned: list"))) return st;
    SignLaunch W = L;
    W.order = list;
    W.n_dev = count;
    W.cfg.persistent = 1;
    return launch_sign(W, s);
}

}  // namespace polymh
