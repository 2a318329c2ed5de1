// Alg. 1 (PolyMinHash signatures) on gfx950.
//
// Work item = (polygon, block of hashes).  A workgroup stages the polygon's
// edges in LDS once; its wavefronts then take the hashes round-robin and
// walk each hash's point stream in tiles of 64 (or 128) consecutive samples:
// every lane draws one SplitMix64 sample, maps it to the lattice and applies
// the MBR check; a ballot gives the MBR-passing samples of the tile, which are
// tested in ascending sample order by an edge-parallel point-in-polygon test
// (lanes split the edges, the parity of the ballot of crossings decides);
// the first inside sample ends the walk (Def. 2: its 1-based index).
//
// The orientation test o = dx*(py - y_lo) - (px - x_lo)*dy only runs for
// samples inside the polygon's MBR on edges straddling py, so each product is
// bounded by the MBR's width * height; for sides below 2^26 the FP64 product
// and fused multiply-add are exact.  Wider polygons use 128-bit integers.
#include "internal.hpp"
#include "sign_common.hpp"

namespace polymh {

namespace {

struct SignArgs {
    const int32_t *xy;
    const int64_t *off;
    const int32_t *mbr;
    const uint32_t *flags;
    const int32_t *order;
    unsigned long long *queue;
    uint32_t *sig;
    const int32_t *n_dev;   // nullable: polygon count read on the device (persistent form only)
    uint64_t seed;
    int64_t n_items;
    int32_t k;
    int32_t hash_block;
    int32_t items_per_poly;
    int32_t lds_edges;
    uint32_t cap;
    int32_t bx0, by0, bx1, by1;
    uint32_t wx, wy;    // box widths for the multiply-shift map (0 encodes 2^32)
    int32_t shx, shy;   // power-of-two widths: shift 32 - log2(W)
};

enum EdgeMode { kLds = 0, kStream = 1, kWide = 2 };

// Edge-parallel crossing-number test of one (wave-uniform) point.
template <int MODE>
__device__ __forceinline__ bool inside_wave(const int4 *s_edges, const int32_t *pxy, int32_t n,
                                            int32_t px, int32_t py, int lane)
{
    bool odd = false;
    if constexpr (MODE == kLds) {
        for (int e = lane; e < n; e += 64) odd ^= crosses_fp64(s_edges[e], px, py);
    } else if constexpr (MODE == kStream) {
        // eight 64-edge blocks' vertices are loaded before any is tested, so a
        // long ring costs n / 512 round trips to memory instead of n / 64
        constexpr int kU = 8;
        const int2 *v = reinterpret_cast<const int2 *>(pxy);
        for (int e0 = 0; e0 < n; e0 += 64 * kU) {
            int2 a[kU], b[kU];
#pragma unroll
            for (int u = 0; u < kU; u++) {
                const int e = e0 + 64 * u + lane;
                const int ec = e < n ? e : 0;
                a[u] = v[ec];
                b[u] = v[ec + 1 == n ? 0 : ec + 1];
            }
#pragma unroll
            for (int u = 0; u < kU; u++)
                odd ^= (e0 + 64 * u + lane < n) & crosses_fp64(make_edge(a[u].x, a[u].y, b[u].x, b[u].y), px, py);
        }
    } else {
        for (int e = lane; e < n; e += 64) {
            const int f = (e + 1 == n) ? 0 : e + 1;
            odd ^= crosses_i128(pxy + 2 * e, pxy + 2 * f, px, py);
        }
    }
    return __popcll(__ballot(odd)) & 1;
}

struct PolyCtx {
    const int4 *s_edges;
    const int32_t *pxy;
    int32_t n;
    uint32_t cx, cy;    // (box origin - MBR origin) mod 2^32
    uint32_t wmx, wmy;  // MBR width - 1, height - 1
};

// One hash's walk (Alg. 1's while loop): returns the 1-based index of the
// first inside sample, 0 if none within cap samples.
template <bool POW2, int MODE, int SPL>
__device__ uint32_t walk(const SignArgs &A, const PolyCtx &C, uint64_t key, int lane)
{
    constexpr uint32_t kTile = 64u * SPL;
    uint64_t z = key + (uint64_t)(lane + 1) * kGamma;
    for (uint64_t base = 0; base < A.cap; base += kTile) {
        uint32_t ox[SPL], oy[SPL];
        uint64_t m[SPL];
#pragma unroll
        for (int s = 0; s < SPL; s++) {
            const uint64_t r = mix64(z + (uint64_t)(64 * s) * kGamma);
            ox[s] = lattice<POW2>((uint32_t)(r >> 32), A.wx, A.shx);
            oy[s] = lattice<POW2>((uint32_t)r, A.wy, A.shy);
            const uint64_t j = base + 64u * s + lane;
            const bool in = (ox[s] + C.cx <= C.wmx) & (oy[s] + C.cy <= C.wmy) & (j < A.cap);
            m[s] = __ballot(in);
        }
        z += (uint64_t)kTile * kGamma;
#pragma unroll
        for (int s = 0; s < SPL; s++) {
            uint64_t mm = m[s];
            while (mm) {
                const int c = __builtin_ctzll(mm);
                const int32_t px = A.bx0 + (int32_t)__builtin_amdgcn_readlane(ox[s], c);
                const int32_t py = A.by0 + (int32_t)__builtin_amdgcn_readlane(oy[s], c);
                if (inside_wave<MODE>(C.s_edges, C.pxy, C.n, px, py, lane))
                    return (uint32_t)(base + 64u * s + c + 1);
                mm &= mm - 1;
            }
        }
    }
    return 0u;
}

// The wavefronts of a workgroup take the item's hashes round-robin: hash
// i0 + w, i0 + w + W, ... for wave w of W.  Indices stay in [i0, i1) by
// construction, and the loop has no lane-dependent control flow around its
// cross-lane operations.
template <bool POW2, int MODE, int SPL>
__device__ void hash_loop(const SignArgs &A, const PolyCtx &C, int i0, int i1, uint32_t *out,
                          int lane, int wave, int nwaves)
{
    for (int i = i0 + wave; i < i1; i += nwaves) {
        const uint64_t key = mix64(A.seed + (uint64_t)(i + 1) * kGamma);
        const uint32_t h = walk<POW2, MODE, SPL>(A, C, key, lane);
        if (lane == 0) out[i] = h;
    }
}

template <bool POW2, int SPL>
__global__ __launch_bounds__(512) void k_sign(SignArgs A)
{
    extern __shared__ int4 s_edges[];
    __shared__ long long s_item;
    const int tid = threadIdx.x, lane = tid & 63;
    // wave index made explicitly wave-uniform (taken at entry, where control
    // flow is uniform)
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), nwaves = blockDim.x >> 6;
    int64_t it = blockIdx.x;
    const int64_t n_items = A.n_dev ? (int64_t)A.n_dev[0] * A.items_per_poly : A.n_items;
    for (;;) {
        if (A.queue) {
            __syncthreads();
            if (tid == 0) s_item = (long long)atomicAdd(A.queue, 1ull);
            __syncthreads();
            it = s_item;
        }
        if (it >= n_items) break;

        const int64_t slot = it / A.items_per_poly;
        const int32_t blk = (int32_t)(it - slot * A.items_per_poly);
        const int64_t p = A.order ? (int64_t)A.order[slot] : slot;
        const int32_t i0 = blk * A.hash_block;
        const int32_t i1 = min(A.k, i0 + A.hash_block);
        const int64_t a = A.off[p];
        const int32_t n = (int32_t)(A.off[p + 1] - a);
        const uint32_t fl = A.flags[p];
        const int4 mb = *reinterpret_cast<const int4 *>(A.mbr + 4 * p);
        uint32_t *out = A.sig + (size_t)p * (size_t)A.k;
        const bool empty = (fl & (kFlagFew | kFlagCollinear)) || mb.z < A.bx0 || mb.x > A.bx1 ||
                           mb.w < A.by0 || mb.y > A.by1;
        if (empty) {
            // no lattice point of B can be inside: every walk ends at the cap
            for (int i = i0 + tid; i < i1; i += blockDim.x) out[i] = 0u;
        } else {
            const int32_t *pxy = A.xy + 2 * a;
            int mode = (fl & kFlagWide) ? kWide : (n <= A.lds_edges ? kLds : kStream);
            if (mode == kLds) {
                for (int e = tid; e < n; e += blockDim.x) {
                    const int f = (e + 1 == n) ? 0 : e + 1;
                    const int2 u = *reinterpret_cast<const int2 *>(pxy + 2 * e);
                    const int2 v = *reinterpret_cast<const int2 *>(pxy + 2 * f);
                    s_edges[e] = make_edge(u.x, u.y, v.x, v.y);
                }
            }
            __syncthreads();
            PolyCtx C;
            C.s_edges = s_edges;
            C.pxy = pxy;
            C.n = n;
            C.cx = (uint32_t)A.bx0 - (uint32_t)mb.x;
            C.cy = (uint32_t)A.by0 - (uint32_t)mb.y;
            C.wmx = (uint32_t)mb.z - (uint32_t)mb.x;
            C.wmy = (uint32_t)mb.w - (uint32_t)mb.y;
            if (mode == kLds)
                hash_loop<POW2, kLds, SPL>(A, C, i0, i1, out, lane, wave, nwaves);
            else if (mode == kStream)
                hash_loop<POW2, kStream, SPL>(A, C, i0, i1, out, lane, wave, nwaves);
            else
                hash_loop<POW2, kWide, SPL>(A, C, i0, i1, out, lane, wave, nwaves);
            __syncthreads();
        }
        if (!A.queue) break;
    }
}

int log2_exact(uint64_t w)
{
    if (w == 0 || (w & (w - 1))) return -1;
    int l = 0;
    while ((1ull << l) < w) l++;
    return l;
}

}  // namespace

polymh_status launch_sign(const SignLaunch &L, hipStream_t s)
{
    SignArgs A{};
    A.xy = L.xy;
    A.off = L.off;
    A.mbr = L.mbr;
    A.flags = L.flags;
    A.order = L.order;
    A.queue = L.queue;
    A.sig = L.sig;
    A.n_dev = L.n_dev;
    A.seed = L.seed;
    A.k = L.k;
    A.cap = L.cap;
    A.hash_block = (L.cfg.hash_block <= 0 || L.cfg.hash_block > L.k) ? L.k : L.cfg.hash_block;
    A.items_per_poly = (L.k + A.hash_block - 1) / A.hash_block;
    A.n_items = L.n * A.items_per_poly;
    A.lds_edges = L.cfg.lds_edges;
    A.bx0 = L.box.xmin; A.by0 = L.box.ymin; A.bx1 = L.box.xmax; A.by1 = L.box.ymax;
    const uint64_t wx = (uint64_t)((int64_t)L.box.xmax - L.box.xmin + 1);
    const uint64_t wy = (uint64_t)((int64_t)L.box.ymax - L.box.ymin + 1);
    const int lx = log2_exact(wx), ly = log2_exact(wy);
    // shift form for power-of-two widths >= 2 (W = 2^32 maps hi32 unchanged)
    const bool pow2 = lx >= 1 && ly >= 1;
    A.shx = pow2 ? 32 - lx : 0;
    A.shy = pow2 ? 32 - ly : 0;
    A.wx = (uint32_t)wx;  // 2^32 wraps to 0, which the multiply-shift form maps as identity
    A.wy = (uint32_t)wy;
    if (A.n_items == 0) return POLYMH_OK;
    if (A.n_dev && !A.queue) return set_error(POLYMH_EINVAL, "sign: a device-side count needs the persistent form");
    const int bt = L.cfg.block_threads;
    const size_t lds = (size_t)L.cfg.lds_edges * sizeof(int4);
    int64_t grid = A.n_items;
    if (A.queue) {
        grid = (int64_t)L.cfg.blocks_per_cu * cu_count();
        if (grid > A.n_items) grid = A.n_items;
        polymh_status st = launch_fill_u64(A.queue, 1, 0ull, s);
        if (st) return st;
    }
    if (grid > 0x7fffffff) return set_error(POLYMH_EINVAL, "sign: too many work items for one launch");
    const bool spl2 = L.cfg.samples_per_lane == 2;
    if (pow2) {
        if (spl2) hipLaunchKernelGGL((k_sign<true, 2>), dim3((unsigned)grid), dim3(bt), lds, s, A);
        else hipLaunchKernelGGL((k_sign<true, 1>), dim3((unsigned)grid), dim3(bt), lds, s, A);
    } else {
        if (spl2) hipLaunchKernelGGL((k_sign<false, 2>), dim3((unsigned)grid), dim3(bt), lds, s, A);
        else hipLaunchKernelGGL((k_sign<false, 1>), dim3((unsigned)grid), dim3(bt), lds, s, A);
    }
    return check_launch("sign");
}

}  // namespace polymh
