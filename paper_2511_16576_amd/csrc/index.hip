// Bucket table of Sec. 3.2's hashmap: a stable LSD radix sort of the n*b
// (band key, entry index p*b + t) pairs by the 64-bit key, 8 bits per pass.
//
// Each pass: (1) every block counts the digits of its tile; (2) one block per
// digit turns the per-block counts into exclusive offsets, and a tiny kernel
// prefixes the digit totals; (3) every block re-reads its tile in order and
// scatters each entry to base[digit] + (entries of that digit before it in
// the tile), ranked inside a wavefront by ballot matching and across
// wavefronts through LDS, which keeps the sort stable.
#include "internal.hpp"

namespace polymh {

namespace {

constexpr int kRadix = 256;
constexpr int kThreads = 256;
constexpr int kItems = 16;                    // entries per thread per tile
constexpr int kTile = kThreads * kItems;      // 4096 entries per block
constexpr int kWaves = kThreads / 64;

__device__ __forceinline__ uint32_t digit_of(uint64_t key, int shift)
{
    return (uint32_t)(key >> shift) & 0xffu;
}

// Pass input: either the caller's key array (first pass; the value is the
// entry index itself) or the previous pass's ping-pong buffers.
struct PassIn {
    const uint64_t *keys;
    const int32_t *ids;   // nullptr: value = entry index
    int32_t b;
};

__device__ __forceinline__ int32_t id_of(const PassIn &in, int64_t e)
{
    return in.ids ? in.ids[e] : (int32_t)e;
}

__global__ __launch_bounds__(kThreads) void k_hist(PassIn in, int64_t m, int shift,
                                                   uint32_t *__restrict__ hist, int nblocks)
{
    __shared__ uint32_t h[kRadix];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int i = 0; i < kItems; i++) {
        const int64_t e = base + (int64_t)i * kThreads + threadIdx.x;
        if (e < m) atomicAdd(&h[digit_of(in.keys[e], shift)], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// One block per digit: exclusive prefix over blocks, total to totals[digit].
__global__ __launch_bounds__(kThreads) void k_scan_digit(uint32_t *__restrict__ hist, int nblocks,
                                                         uint32_t *__restrict__ totals)
{
    __shared__ uint32_t s[kThreads];
    uint32_t *row = hist + (int64_t)blockIdx.x * nblocks;
    uint32_t carry = 0;
    for (int c0 = 0; c0 < nblocks; c0 += kThreads) {
        const int c = c0 + threadIdx.x;
        const uint32_t v = c < nblocks ? row[c] : 0u;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < kThreads; o <<= 1) {
            const uint32_t t = threadIdx.x >= o ? s[threadIdx.x - o] : 0u;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        if (c < nblocks) row[c] = carry + s[threadIdx.x] - v;
        carry += s[kThreads - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

__global__ void k_scan_totals(uint32_t *totals)
{
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int d = 0; d < kRadix; d++) {
            const uint32_t v = totals[d];
            totals[d] = s;
            s += v;
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_scatter(PassIn in, int64_t m, int shift,
                                                      const uint32_t *__restrict__ hist,
                                                      const uint32_t *__restrict__ totals,
                                                      int nblocks, uint64_t *__restrict__ out_keys,
                                                      int32_t *__restrict__ out_ids)
{
    __shared__ uint32_t s_base[kRadix];
    __shared__ uint32_t s_wcnt[kWaves][kRadix];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    s_base[tid] = totals[tid] + hist[(int64_t)tid * nblocks + blockIdx.x];
    for (int w = 0; w < kWaves; w++) s_wcnt[w][tid] = 0;
    __syncthreads();
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int i = 0; i < kItems; i++) {
        const int64_t e = base + (int64_t)i * kThreads + tid;
        const bool valid = e < m;
        uint64_t key = 0;
        int32_t id = 0;
        uint32_t d = 0;
        if (valid) {
            key = in.keys[e];
            id = id_of(in, e);
            d = digit_of(key, shift);
        }
        // lanes of this wavefront holding the same digit
        uint64_t eq = __ballot(valid);
        for (int bit = 0; bit < 8; bit++) {
            const uint64_t bb = __ballot((d >> bit) & 1u);
            eq &= ((d >> bit) & 1u) ? bb : ~bb;
        }
        const uint32_t rank = (uint32_t)__popcll(eq & lt_mask);
        if (valid && rank == 0) s_wcnt[wave][d] = (uint32_t)__popcll(eq);
        __syncthreads();
        if (valid) {
            uint32_t pre = 0;
            for (int w = 0; w < wave; w++) pre += s_wcnt[w][d];
            const uint32_t pos = s_base[d] + pre + rank;
            out_keys[pos] = key;
            out_ids[pos] = id;
        }
        __syncthreads();
        uint32_t sum = 0;
        for (int w = 0; w < kWaves; w++) {
            sum += s_wcnt[w][tid];
            s_wcnt[w][tid] = 0;
        }
        s_base[tid] += sum;
        __syncthreads();
    }
}

}  // namespace

size_t index_workspace_bytes(int64_t m)
{
    const int64_t nblocks = (m + kTile - 1) / kTile;
    size_t bytes = 0;
    bytes += align_up((size_t)nblocks * kRadix * sizeof(uint32_t), 256);
    bytes += align_up(kRadix * sizeof(uint32_t), 256);
    bytes += align_up((size_t)m * sizeof(uint64_t), 256);
    bytes += align_up((size_t)m * sizeof(int32_t), 256);
    return bytes + 256;
}

polymh_status launch_index_build(const uint64_t *keys, int64_t n, int32_t b, void *ws,
                                 size_t ws_bytes, uint64_t *sorted_keys, int32_t *sorted_ids,
                                 hipStream_t s)
{
    const int64_t m = n * b;
    if (m == 0) return POLYMH_OK;
    if (m > 0x7fffffffLL) return set_error(POLYMH_EINVAL, "index_build: more than 2^31-1 entries");
    const int nblocks = (int)((m + kTile - 1) / kTile);
    Carve cv{static_cast<char *>(ws), ws_bytes};
    uint32_t *hist = cv.take<uint32_t>((size_t)nblocks * kRadix);
    uint32_t *totals = cv.take<uint32_t>(kRadix);
    uint64_t *tk = cv.take<uint64_t>((size_t)m);
    int32_t *ti = cv.take<int32_t>((size_t)m);
    if (!cv.ok)
        return set_error(POLYMH_ECAPACITY, "index_build: workspace of %zu bytes, need %zu", ws_bytes, cv.used);
    // 8 passes: even passes write the temporaries, odd passes the outputs, so
    // the last (8th) pass lands in the caller's arrays.
    PassIn in{keys, nullptr, b};
    for (int pass = 0; pass < 8; pass++) {
        const int shift = 8 * pass;
        uint64_t *ok_ = (pass & 1) ? sorted_keys : tk;
        int32_t *oi = (pass & 1) ? sorted_ids : ti;
        hipLaunchKernelGGL(k_hist, dim3(nblocks), dim3(kThreads), 0, s, in, m, shift, hist, nblocks);
        hipLaunchKernelGGL(k_scan_digit, dim3(kRadix), dim3(kThreads), 0, s, hist, nblocks, totals);
        hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(64), 0, s, totals);
        hipLaunchKernelGGL(k_scatter, dim3(nblocks), dim3(kThreads), 0, s, in, m, shift, hist, totals,
                           nblocks, ok_, oi);
        in = PassIn{ok_, oi, b};
    }
    return check_launch("index_build");
}

}  // namespace polymh
