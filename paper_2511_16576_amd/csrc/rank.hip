// Ordered refinement with early stop (learned candidate scorer).
//
// Each query's candidates are sorted by a predicted Jaccard (the MLP's output
// or the collision fraction of the signatures) and refined in rounds of F
// candidates in that order.  After each round the query keeps its exact top-k
// and stops once it holds k results and its k-th exact J is at least the next
// candidate's predicted J plus a margin, or when its candidates run out.
// Queries with more than kSortCap candidates are refined in their original
// order with the stop test disabled, i.e. fully (the fallback).  After the
// last round, a finishing pass refines every candidate a still-active query
// has left, so the result is always complete; the rounds and that pass keep
// their counts on the device and never wait on the host.
#include "internal.hpp"

#include <algorithm>
#include <type_traits>
#include <cfloat>

namespace polymh {

namespace {

constexpr int kSortCap = 8192;
constexpr int kTopMax = 64;

__device__ __forceinline__ bool key_before(float sa, int ia, float sb, int ib)
{
    return sa > sb || (sa == sb && ia < ib);
}

// LDS writes of a wavefront visible to its own later reads.
__device__ __forceinline__ void wave_fence_lds()
{
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_wave_barrier();
}

// One block per query: bitonic sort of (score desc, position asc) in LDS.
__global__ __launch_bounds__(1024) void k_rank_sort(const int64_t *__restrict__ off,
                                                    const float *__restrict__ score,
                                                    int32_t *__restrict__ order,
                                                    uint8_t *__restrict__ sorted_ok)
{
    __shared__ float ss[kSortCap];
    __shared__ int si[kSortCap];
    const int64_t q = blockIdx.x;
    const int64_t a = off[q];
    const int n = (int)(off[q + 1] - a);
    if (n > kSortCap) {
        for (int i = threadIdx.x; i < n; i += blockDim.x) order[a + i] = i;
        if (threadIdx.x == 0) sorted_ok[q] = 0;
        return;
    }
    int np = 1;
    while (np < n) np <<= 1;
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
        ss[i] = i < n ? score[a + i] : -FLT_MAX;
        si[i] = i < n ? i : 0x7fffffff;
    }
    __syncthreads();
    for (int k = 2; k <= np; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < np; i += blockDim.x) {
                const int l = i ^ j;
                if (l > i) {
                    const bool up = (i & k) == 0;
                    const bool before = key_before(ss[l], si[l], ss[i], si[i]);
                    if (before == up) {
                        const float t = ss[i]; ss[i] = ss[l]; ss[l] = t;
                        const int u = si[i]; si[i] = si[l]; si[l] = u;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) order[a + i] = si[i];
    if (threadIdx.x == 0) sorted_ok[q] = 1;
}


// The block's (score desc, position asc) order of the n scores it wrote to
// ss/si (entries below kSortCap), written to order[a..a+n); lists beyond
// kSortCap keep their given order and get sorted_ok 0.
__device__ __forceinline__ void order_from_lds(float *ss, int *si, int n, int64_t a, int64_t q,
                                               int32_t *__restrict__ order, uint8_t *__restrict__ sorted_ok)
{
    if (n > kSortCap) {
        for (int i = threadIdx.x; i < n; i += blockDim.x) order[a + i] = i;
        if (threadIdx.x == 0) sorted_ok[q] = 0;
        return;
    }
    int np = 1;
    while (np < n) np <<= 1;
    for (int i = n + threadIdx.x; i < np; i += blockDim.x) {
        ss[i] = -FLT_MAX;
        si[i] = 0x7fffffff;
    }
    __syncthreads();
    for (int kk = 2; kk <= np; kk <<= 1) {
        for (int j = kk >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < np; i += blockDim.x) {
                const int l = i ^ j;
                if (l > i) {
                    const bool up = (i & kk) == 0;
                    const bool before = key_before(ss[l], si[l], ss[i], si[i]);
                    if (before == up) {
                        const float t = ss[i]; ss[i] = ss[l]; ss[l] = t;
                        const int u = si[i]; si[i] = si[l]; si[l] = u;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) order[a + i] = si[i];
    if (threadIdx.x == 0) sorted_ok[q] = 1;
}

// For scores that are counts in [0, 256] (agreeing hashes, k <= 256) the
// same order comes from a stable counting sort.  Per lane, the lanes of its
// wavefront holding the same count: nine ballots, one per bit.
__device__ __forceinline__ uint64_t match_count9(int v, bool valid)
{
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 9; b++) {
        const bool bit = (v >> b) & 1;
        const uint64_t bb = __ballot(valid && bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

constexpr int kCountBins = 257;

// LDS of order_from_counts for a block of NW wavefronts.
template <int NW>
struct CountSortLds {
    static_assert(NW % 2 == 0, "the per-wavefront table is cleared as 32-bit words");
    uint16_t cs[kSortCap];                       // the counts, by position
    alignas(16) uint16_t wc[NW][kCountBins];     // per wavefront of a chunk: count of each value
    int bin[kCountBins];                         // running start of each value's slots
};

// (count desc, position asc) order of the n counts in L.cs, written to
// order[a..a+n) (n <= kSortCap): a histogram (one LDS atomic per distinct
// value a wavefront holds), the bins' starts from the largest count down,
// then, NW * 64 positions at a time, each position's slot: its bin's
// running start, plus the positions of equal count in earlier wavefronts
// of the chunk, plus those in earlier lanes of its own.  L.bin must be zero
// and L.cs complete (a barrier) before the call.
template <int NW>
__device__ void order_from_counts(CountSortLds<NW> &L, int n, int64_t a, int32_t *__restrict__ order)
{
    constexpr int NT = NW * 64;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = tid >> 6;
    const uint64_t below = (1ull << lane) - 1;
    for (int c0 = 0; c0 < n; c0 += NT) {
        const int p = c0 + tid;
        const bool valid = p < n;
        const int v = valid ? L.cs[p] : 0;
        const uint64_t m = match_count9(v, valid);
        if (valid && (m & below) == 0) atomicAdd(&L.bin[v], __popcll(m));
    }
    __syncthreads();
    if (wave == 0) {
        // exclusive prefix over the bins from 256 down, five a lane
        int h[5], sum = 0;
#pragma unroll
        for (int j = 0; j < 5; j++) {
            const int d = 5 * lane + j;
            h[j] = d < kCountBins ? L.bin[kCountBins - 1 - d] : 0;
            sum += h[j];
        }
        int pre = wave_incl_scan32(sum) - sum;
#pragma unroll
        for (int j = 0; j < 5; j++) {
            const int d = 5 * lane + j;
            if (d < kCountBins) L.bin[kCountBins - 1 - d] = pre;
            pre += h[j];
        }
    }
    __syncthreads();
    for (int c0 = 0; c0 < n; c0 += NT) {
        uint32_t *wz = reinterpret_cast<uint32_t *>(&L.wc[0][0]);
        for (int t = tid; t < NW * kCountBins / 2; t += NT) wz[t] = 0;
        __syncthreads();
        const int p = c0 + tid;
        const bool valid = p < n;
        const int v = valid ? L.cs[p] : 0;
        const uint64_t m = match_count9(v, valid);
        if (valid && (m & below) == 0) L.wc[wave][v] = (uint16_t)__popcll(m);
        __syncthreads();
        if (valid) {
            int slot = L.bin[v] + __popcll(m & below);
            for (int w = 0; w < wave; w++) slot += L.wc[w][v];
            order[a + slot] = p;
        }
        __syncthreads();
        if (c0 + NT < n) {
            for (int t = tid; t < kCountBins; t += NT) {
                int s = 0;
                for (int w = 0; w < NW; w++) s += L.wc[w][t];
                L.bin[t] += s;
            }
            __syncthreads();
        }
    }
}

// One block per query: the collision fraction of every candidate (the
// unbiased estimate of J of Thm. 1: the share of the k hashes on which the
// two signatures agree), written to score[], then the (score desc, position
// asc) order as k_rank_sort.  One wavefront per candidate; with k a multiple
// of 4 and at most 1024 and both tables 16-byte aligned (`vec`), a lane keeps
// its 16-byte slices of the query's signature in registers and reads the
// candidate's with 16-byte loads.  With k <= 256 (kCount) the order comes
// from the counting sort, otherwise from the bitonic sort of the scores.
struct BitonicLds {
    float ss[kSortCap];
    int si[kSortCap];
};

template <bool kCount>
__global__ __launch_bounds__(1024, 8) void k_rank_jhat_sort(const uint32_t *__restrict__ qsig,
                                                         const uint32_t *__restrict__ dsig, int32_t k,
                                                         int vec, const int64_t *__restrict__ off,
                                                         const int32_t *__restrict__ cand_ids,
                                                         float *__restrict__ score,
                                                         int32_t *__restrict__ order,
                                                         uint8_t *__restrict__ sorted_ok)
{
    __shared__ typename std::conditional<kCount, CountSortLds<16>, BitonicLds>::type L;
    // the score of position i, for the sort
    auto record = [&](int i, int cnt, float sc) {
        if constexpr (kCount) {
            if (i < kSortCap) L.cs[i] = (uint16_t)cnt;
        } else {
            if (i < kSortCap) {
                L.ss[i] = sc;
                L.si[i] = i;
            }
        }
    };
    if constexpr (kCount) {
        for (int v = threadIdx.x; v < kCountBins; v += blockDim.x) L.bin[v] = 0;
    }
    const int64_t q = blockIdx.x;
    const int64_t a = off[q];
    const int n = (int)(off[q + 1] - a);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int nwave = (int)(blockDim.x >> 6);
    const uint32_t *sq = qsig + q * (int64_t)k;
    const float inv_k = 1.0f / (float)k;
    uint4 qv[4];
#pragma unroll
    for (int t = 0; t < 4; t++) {
        const int h = 4 * lane + 256 * t;
        qv[t] = (vec && h < k) ? *reinterpret_cast<const uint4 *>(sq + h) : make_uint4(0, 0, 0, 0);
    }
    if (vec && k <= 256) {
        // the common case (k <= 256): a wavefront takes eight candidates at
        // a time, their eight 16-byte slices a lane loaded together
        constexpr int kU = 8;
        const bool in = 4 * lane < k;
        // the candidate ids of a wavefront's next eight are loaded while the
        // current eight's signatures are in flight
        int32_t idn[kU];
#pragma unroll
        for (int u = 0; u < kU; u++) {
            const int i = min(wave * kU + u, n - 1);
            idn[u] = n > 0 ? cand_ids[a + i] : 0;
        }
        for (int i0 = wave * kU; i0 < n; i0 += nwave * kU) {
            uint4 pv[kU];
#pragma unroll
            for (int u = 0; u < kU; u++) {
                const uint32_t *sp = dsig + (int64_t)idn[u] * k;
                pv[u] = in ? *reinterpret_cast<const uint4 *>(sp + 4 * lane) : make_uint4(0, 0, 0, 0);
            }
#pragma unroll
            for (int u = 0; u < kU; u++) idn[u] = cand_ids[a + min(i0 + nwave * kU + u, n - 1)];
#pragma unroll
            for (int u = 0; u < kU; u++) {
                const int i = i0 + u;
                const int cnt = __popcll(__ballot(in && pv[u].x == qv[0].x)) + __popcll(__ballot(in && pv[u].y == qv[0].y)) +
                                __popcll(__ballot(in && pv[u].z == qv[0].z)) + __popcll(__ballot(in && pv[u].w == qv[0].w));
                const float sc = (float)cnt * inv_k;
                if (lane == 0 && i < n) {
                    score[a + i] = sc;
                    record(i, cnt, sc);
                }
            }
        }
    } else {
        for (int i = wave; i < n; i += nwave) {
            const uint32_t *sp = dsig + (int64_t)cand_ids[a + i] * k;
            int cnt = 0;
            if (vec) {
#pragma unroll
                for (int t = 0; t < 4; t++) {
                    const int h = 4 * lane + 256 * t;
                    if (256 * t < k) {   // wave-uniform
                        const bool in = h < k;
                        const uint4 pv = in ? *reinterpret_cast<const uint4 *>(sp + h) : make_uint4(0, 0, 0, 0);
                        cnt += __popcll(__ballot(in && pv.x == qv[t].x)) + __popcll(__ballot(in && pv.y == qv[t].y)) +
                               __popcll(__ballot(in && pv.z == qv[t].z)) + __popcll(__ballot(in && pv.w == qv[t].w));
                    }
                }
            } else {
                for (int h0 = 0; h0 < k; h0 += 64) {
                    const int h = h0 + lane;
                    cnt += __popcll(__ballot(h < k && sq[h] == sp[h]));
                }
            }
            const float sc = (float)cnt * inv_k;
            if (lane == 0) {
                score[a + i] = sc;
                record(i, cnt, sc);
            }
        }
    }
    if constexpr (kCount) {
        __syncthreads();
        if (n > kSortCap) {
            for (int i = threadIdx.x; i < n; i += blockDim.x) order[a + i] = i;
            if (threadIdx.x == 0) sorted_ok[q] = 0;
            return;
        }
        order_from_counts<16>(L, n, a, order);
        if (threadIdx.x == 0) sorted_ok[q] = 1;
    } else {
        order_from_lds(L.ss, L.si, n, a, q, order, sorted_ok);
    }
}

// Saturated signature table: value i of signature r as min(value, 65535),
// 16 bits, so 2k bytes a row (whole 128-byte lines at k = 256) instead of
// 4k.  Two values are equal exactly when their saturated copies are equal
// and below 65535, or both copies are 65535 and the full values are equal;
// first hits average 1/S_p draws (Thm. 2), so at the configured data sets'
// shares almost every value lies below 65535 and the full table is read
// only for the rare hashes where both the query's and the candidate's value
// saturate.
__device__ __forceinline__ uint32_t sat16(uint32_t v) { return v < 0xffffu ? v : 0xffffu; }

// Lane l saturates values 4l .. 4l+3 of a row; a wavefront takes a row.
__global__ __launch_bounds__(256) void k_sig_pack(const uint32_t *__restrict__ sig, int64_t n, int32_t k,
                                                  uint16_t *__restrict__ packed)
{
    const int lane = threadIdx.x & 63;
    const bool in = 4 * lane < k;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; r < n; r += nw) {
        if (!in) continue;
        const uint4 v = *reinterpret_cast<const uint4 *>(sig + r * k + 4 * lane);
        *reinterpret_cast<uint2 *>(packed + r * k + 4 * lane) =
            make_uint2(sat16(v.x) | (sat16(v.y) << 16), sat16(v.z) | (sat16(v.w) << 16));
    }
}

// k_rank_jhat_sort on the saturated table (k a multiple of 4, at most 256):
// a lane compares 4 hashes from 8 bytes of the candidate's row; the full
// table `dsig` is read only where the query's and the candidate's copies
// both saturate.
__global__ __launch_bounds__(1024, 8) void k_rank_jhat_packed(const uint32_t *__restrict__ qsig,
                                                              const uint16_t *__restrict__ packed,
                                                              const uint32_t *__restrict__ dsig, int32_t k,
                                                              const int64_t *__restrict__ off,
                                                              const int32_t *__restrict__ cand_ids,
                                                              float *__restrict__ score,
                                                              int32_t *__restrict__ order,
                                                              uint8_t *__restrict__ sorted_ok)
{
    __shared__ CountSortLds<16> L;
    const int64_t q = blockIdx.x;
    const int64_t a = off[q];
    const int n = (int)(off[q + 1] - a);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int nwave = (int)(blockDim.x >> 6);
    for (int v = threadIdx.x; v < kCountBins; v += blockDim.x) L.bin[v] = 0;
    const float inv_k = 1.0f / (float)k;
    const bool in = 4 * lane < k;
    const uint4 qv = in ? *reinterpret_cast<const uint4 *>(qsig + q * (int64_t)k + 4 * lane) : make_uint4(0, 0, 0, 0);
    const uint32_t qs0 = sat16(qv.x) | (sat16(qv.y) << 16), qs1 = sat16(qv.z) | (sat16(qv.w) << 16);
    // hashes whose query value saturates: equal copies need the full values
    const uint32_t qsat = (uint32_t)(qv.x >= 0xffffu) | ((uint32_t)(qv.y >= 0xffffu) << 1) |
                          ((uint32_t)(qv.z >= 0xffffu) << 2) | ((uint32_t)(qv.w >= 0xffffu) << 3);
    constexpr int kU = 8;
    int32_t idn[kU];
#pragma unroll
    for (int u = 0; u < kU; u++) {
        const int i = min(wave * kU + u, n - 1);
        idn[u] = n > 0 ? cand_ids[a + i] : 0;
    }
    for (int i0 = wave * kU; i0 < n; i0 += nwave * kU) {
        uint2 cv[kU];
        int32_t idc[kU];
#pragma unroll
        for (int u = 0; u < kU; u++) {
            cv[u] = in ? *reinterpret_cast<const uint2 *>(packed + (int64_t)idn[u] * k + 4 * lane) : make_uint2(0, 0);
            idc[u] = idn[u];
        }
#pragma unroll
        for (int u = 0; u < kU; u++) idn[u] = cand_ids[a + min(i0 + nwave * kU + u, n - 1)];
#pragma unroll
        for (int u = 0; u < kU; u++) {
            const int i = i0 + u;
            const uint32_t d0 = cv[u].x ^ qs0, d1 = cv[u].y ^ qs1;
            uint32_t eq = (uint32_t)((d0 & 0xffffu) == 0) | ((uint32_t)((d0 >> 16) == 0) << 1) |
                          ((uint32_t)((d1 & 0xffffu) == 0) << 2) | ((uint32_t)((d1 >> 16) == 0) << 3);
            if (!in) eq = 0;
            // both copies saturated: compare the full values
            const uint32_t need = eq & qsat;
            if (__ballot(need != 0)) {
                if (need) {
                    const uint4 fv = *reinterpret_cast<const uint4 *>(dsig + (int64_t)idc[u] * k + 4 * lane);
                    const uint32_t ne = (uint32_t)(fv.x != qv.x) | ((uint32_t)(fv.y != qv.y) << 1) |
                                        ((uint32_t)(fv.z != qv.z) << 2) | ((uint32_t)(fv.w != qv.w) << 3);
                    eq &= ~(need & ne);
                }
            }
            const int cnt = __popcll(__ballot(eq & 1u)) + __popcll(__ballot(eq & 2u)) +
                            __popcll(__ballot(eq & 4u)) + __popcll(__ballot(eq & 8u));
            if (lane == 0 && i < n) {
                score[a + i] = (float)cnt * inv_k;
                if (i < kSortCap) L.cs[i] = (uint16_t)cnt;
            }
        }
    }
    __syncthreads();
    if (n > kSortCap) {
        for (int i = threadIdx.x; i < n; i += blockDim.x) order[a + i] = i;
        if (threadIdx.x == 0) sorted_ok[q] = 0;
        return;
    }
    // scores are counts over k <= 256: the same order by counting
    order_from_counts<16>(L, n, a, order);
    if (threadIdx.x == 0) sorted_ok[q] = 1;
}

__global__ void k_rank_init(int64_t nq, int32_t topk, int64_t *__restrict__ cursor,
                            uint8_t *__restrict__ active, int32_t *__restrict__ top_ids,
                            double *__restrict__ top_j)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nq;
         q += (int64_t)gridDim.x * blockDim.x) {
        cursor[q] = 0;
        active[q] = 1;
        for (int t = 0; t < topk; t++) {
            top_ids[q * topk + t] = -1;
            top_j[q * topk + t] = 0.0;
        }
    }
}

// The round's per-query pair counts (active queries: min(F, left), or all
// left for F <= 0) and their exclusive prefix into roff[0..nq], in one
// block: tiles of 8192 queries, 8 consecutive ones a thread, a wavefront
// scan of the thread sums and a pass over the 16 wavefront totals.
__global__ __launch_bounds__(1024) void k_round_offsets(const int64_t *__restrict__ off, int64_t nq,
                                                        const int64_t *__restrict__ cursor,
                                                        const uint8_t *__restrict__ active, int32_t F,
                                                        int64_t *__restrict__ roff)
{
    constexpr int kPer = 8;
    __shared__ int64_t s_w[16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t carry = 0;
    for (int64_t t0 = 0; t0 < nq; t0 += 1024 * kPer) {
        const int64_t base = t0 + (int64_t)threadIdx.x * kPer;
        int64_t v[kPer];
        int64_t sum = 0;
#pragma unroll
        for (int u = 0; u < kPer; u++) {
            const int64_t q = base + u;
            v[u] = 0;
            if (q < nq && active[q]) {
                const int64_t left = (off[q + 1] - off[q]) - cursor[q];
                v[u] = (F <= 0 || left < F) ? left : F;
            }
            sum += v[u];
        }
        const int64_t incl = wave_incl_scan64(sum);
        if (lane == 63) s_w[wave] = incl;
        __syncthreads();
        int64_t pre = carry + incl - sum, tot = 0;
#pragma unroll
        for (int w = 0; w < 16; w++) {
            const int64_t x = s_w[w];
            pre += w < wave ? x : 0;
            tot += x;
        }
#pragma unroll
        for (int u = 0; u < kPer; u++) {
            if (base + u < nq) roff[base + u] = pre;
            pre += v[u];
        }
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) roff[nq] = carry;
}

__global__ void k_round_fill(const int64_t *__restrict__ off, const int32_t *__restrict__ cand_ids,
                             const int32_t *__restrict__ order, const int64_t *__restrict__ cursor,
                             const int64_t *__restrict__ roff, int64_t nq,
                             int32_t *__restrict__ rids, int32_t *__restrict__ rpos)
{
    for (int64_t q = blockIdx.x; q < nq; q += gridDim.x) {
        const int64_t b = roff[q], cnt = roff[q + 1] - b;
        for (int64_t t = threadIdx.x; t < cnt; t += blockDim.x) {
            const int32_t pos = order[off[q] + cursor[q] + t];
            rpos[b + t] = pos;
            rids[b + t] = cand_ids[off[q] + pos];
        }
    }
}

// One wavefront per query: merge the round's exact results into the top-k
// and apply the stop test.  Lane t holds entry t of the (J desc, id asc)
// list (topk <= 64); the round's results are read 64 at a time, those that
// beat the list's last entry are inserted one after another (the first lane
// they beat takes them, the lanes behind it shift down by one).
__global__ __launch_bounds__(256) void k_round_merge(const int64_t *__restrict__ off, const float *__restrict__ score,
                              const int32_t *__restrict__ order, const uint8_t *__restrict__ sorted_ok,
                              const int64_t *__restrict__ roff, const int32_t *__restrict__ rids,
                              const double *__restrict__ rj, int64_t nq, int32_t topk, float margin,
                              int64_t *__restrict__ cursor, uint8_t *__restrict__ active,
                              int32_t *__restrict__ top_ids, double *__restrict__ top_j,
                              int32_t *__restrict__ n_active, unsigned long long *__restrict__ counters,
                              int finishing)
{
    __shared__ int s_left[4];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    // counters[0] += pairs refined in this round; counters[1] += queries the
    // finishing pass had to complete
    if (counters && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&counters[0], (unsigned long long)roff[nq]);
    int left = 0;                               // queries of this wavefront still active
    const int64_t nw = (int64_t)gridDim.x * 4;
    for (int64_t q = (int64_t)blockIdx.x * 4 + wave; q < nq; q += nw) {
        if (!active[q]) continue;               // uniform per wavefront
        const int64_t r0 = roff[q], r1 = roff[q + 1];
        if (finishing && counters && r1 > r0 && lane == 0) atomicAdd(&counters[1], 1ull);
        int32_t *ti = top_ids + q * topk;
        double *tj = top_j + q * topk;
        int32_t li = lane < topk ? ti[lane] : -1;
        double lj = lane < topk ? tj[lane] : 0.0;
        for (int64_t c0 = r0; c0 < r1; c0 += 64) {
            const int64_t c = c0 + lane;
            const int32_t id = c < r1 ? rids[c] : -1;
            const double j = c < r1 ? rj[c] : 0.0;
            const int32_t wid = __shfl(li, topk - 1, 64);
            const double wj = __shfl(lj, topk - 1, 64);
            uint64_t m = __ballot(c < r1 && (wid < 0 || j > wj || (j == wj && id < wid)));
            while (m) {
                const int src = __builtin_ctzll(m);
                m &= m - 1;
                const int32_t cid = __shfl(id, src, 64);
                const double cj = __shfl(j, src, 64);
                const uint64_t bm = __ballot(lane < topk && (li < 0 || cj > lj || (cj == lj && cid < li)));
                if (bm == 0) continue;
                const int at = __builtin_ctzll(bm);
                const int32_t ui = __shfl_up(li, 1, 64);
                const double uj = __shfl_up(lj, 1, 64);
                if (lane == at) {
                    li = cid;
                    lj = cj;
                } else if (lane > at && lane < topk) {
                    li = ui;
                    lj = uj;
                }
            }
        }
        if (lane < topk) {
            ti[lane] = li;
            tj[lane] = lj;
        }
        const int64_t cur = cursor[q] + (r1 - r0);
        const int64_t nq_c = off[q + 1] - off[q];
        bool stop = cur >= nq_c;
        const int32_t last_id = __shfl(li, topk - 1, 64);
        const double last_j = __shfl(lj, topk - 1, 64);
        if (!stop && sorted_ok[q] && last_id >= 0) {
            const float next = score[off[q] + order[off[q] + cur]];
            stop = last_j >= (double)next + (double)margin;
        }
        if (lane == 0) {
            cursor[q] = cur;
            if (stop) active[q] = 0;
        }
        left += stop ? 0 : 1;
    }
    if (n_active) {
        // one atomic per workgroup
        if (lane == 0) s_left[wave] = left;
        __syncthreads();
        if (threadIdx.x == 0) {
            const int t = s_left[0] + s_left[1] + s_left[2] + s_left[3];
            if (t) atomicAdd(n_active, t);
        }
    }
}

__global__ void k_zero_i32(int32_t *p) { if (threadIdx.x == 0) p[0] = 0; }

// Head of each query's order: the first min(M, C_q) candidates, as (row of
// the query, candidate index) pairs in a CSR of per-query counts.
__global__ void k_head_count(const int64_t *__restrict__ off, int64_t nq, int32_t M,
                             int64_t *__restrict__ counts)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nq;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = off[q + 1] - off[q];
        counts[q] = c < M ? c : M;
    }
}

__global__ void k_head_fill(const int64_t *__restrict__ off, const int32_t *__restrict__ cand_ids,
                            const int32_t *__restrict__ order, const int64_t *__restrict__ hoff,
                            int64_t nq, int32_t *__restrict__ hq, int64_t *__restrict__ hc,
                            int32_t *__restrict__ hid)
{
    for (int64_t q = blockIdx.x; q < nq; q += gridDim.x) {
        const int64_t b = hoff[q], cnt = hoff[q + 1] - b;
        for (int64_t t = threadIdx.x; t < cnt; t += blockDim.x) {
            const int64_t c = off[q] + order[off[q] + t];
            hq[b + t] = (int32_t)q;
            hc[b + t] = c;
            hid[b + t] = cand_ids[c];
        }
    }
}


// Head of each query's order in fixed slots: slot q*M + t holds the t-th
// best candidate (t < min(M, C_q)) as its global index and data polygon, or
// -1 in both (an empty slot).  Sizes are known before the lookup's counts,
// so the call needs no host read.
__global__ void k_head_fixed(const int64_t *__restrict__ off, const int32_t *__restrict__ cand_ids,
                             const int32_t *__restrict__ order, int64_t nq, int32_t M,
                             int32_t *__restrict__ hq, int64_t *__restrict__ hc,
                             int32_t *__restrict__ hid)
{
    const int64_t total = nq * (int64_t)M;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < total;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = s / M;
        const int t = (int)(s - q * M);
        const int64_t a = off[q], n = off[q + 1] - a;
        hq[s] = (int32_t)q;
        if (t < n) {
            const int64_t c = a + order[a + t];
            hc[s] = c;
            hid[s] = cand_ids[c];
        } else {
            hc[s] = -1;
            hid[s] = -1;
        }
    }
}

// One wavefront per query: the order after the first h = min(M, C_q)
// candidates of an order sorted by the old scores were given new scores (the
// rest keep theirs).  The h re-scored candidates are sorted among themselves
// (bitonic over the lanes), then merged with the unchanged rest, which is
// still sorted: a candidate's new place is its place in its own sequence
// plus the number of the other sequence's candidates ordered before it (a
// binary search).  The result equals a sort of all candidates by (score
// desc, position asc).  Queries left unsorted (sorted_ok 0) are copied.
__global__ __launch_bounds__(256) void k_reorder_head(const int64_t *__restrict__ off, int64_t nq,
                                                      const float *__restrict__ score,
                                                      const int32_t *__restrict__ order_in, int32_t M,
                                                      const uint8_t *__restrict__ sorted_ok,
                                                      int32_t *__restrict__ order_out)
{
    __shared__ float hs[4][64];
    __shared__ int hp[4][64];
    __shared__ int hc[4][65];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t q = (int64_t)blockIdx.x * 4 + wave;
    if (q >= nq) return;                       // wavefront-uniform
    const int64_t a = off[q];
    const int n = (int)(off[q + 1] - a);
    if (!sorted_ok[q]) {
        for (int i = lane; i < n; i += 64) order_out[a + i] = order_in[a + i];
        return;
    }
    const int h = n < M ? n : M;
    // the re-scored head, one per lane, padded with keys after everything
    int p = lane < h ? order_in[a + lane] : 0x7fffffff;
    float sc = lane < h ? score[a + p] : -FLT_MAX;
    for (int k = 2; k <= 64; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            const float so = __shfl_xor(sc, j, 64);
            const int po = __shfl_xor(p, j, 64);
            const bool lower = (lane & j) == 0;          // keeps the earlier key of the pair if ascending
            const bool asc = (lane & k) == 0;
            const bool other_first = key_before(so, po, sc, p);
            if (other_first == (lower == asc)) {
                sc = so;
                p = po;
            }
        }
    }
    hs[wave][lane] = sc;
    hp[wave][lane] = p;
    hc[wave][lane] = 0;
    if (lane == 0) hc[wave][64] = 0;
    wave_fence_lds();
    const int tail = n - h;
    // tail element j (the unchanged, sorted rest) goes to j + lo_j, lo_j the
    // head elements before it (a search of the head in LDS); its order
    // entries and scores are loaded eight a lane ahead, so a list costs a few
    // round trips to memory.  Head element i goes to i + the tail elements
    // before it, those with lo_j <= i: counted per lo_j, then summed.
    constexpr int kU = 8;
    for (int j0 = 0; j0 < tail; j0 += 64 * kU) {
        int pt[kU];
        float st[kU];
#pragma unroll
        for (int u = 0; u < kU; u++) {
            const int j = j0 + 64 * u + lane;
            pt[u] = j < tail ? order_in[a + h + j] : 0;
        }
#pragma unroll
        for (int u = 0; u < kU; u++) {
            const int j = j0 + 64 * u + lane;
            st[u] = j < tail ? score[a + pt[u]] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < kU; u++) {
            const int j = j0 + 64 * u + lane;
            if (j < tail) {
                int lo = 0, hi = h;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (key_before(hs[wave][mid], hp[wave][mid], st[u], pt[u])) lo = mid + 1;
                    else hi = mid;
                }
                order_out[a + j + lo] = pt[u];
                atomicAdd(&hc[wave][lo], 1);
            }
        }
    }
    wave_fence_lds();
    // head element `lane`: lane + (tail elements with lo_j <= lane)
    const int c = hc[wave][lane];
    const int before = wave_incl_scan32(c);
    if (lane < h) order_out[a + lane + before] = p;
}

__global__ void k_scatter_scores(const int64_t *__restrict__ idx, const float *__restrict__ val,
                                 int64_t n, float *__restrict__ score)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        if (idx[i] >= 0) score[idx[i]] = val[i];
}

__global__ __launch_bounds__(256) void k_jhat(const uint32_t *__restrict__ lsig,
                                              const uint32_t *__restrict__ rsig,
                                              const int32_t *__restrict__ li,
                                              const int32_t *__restrict__ ri, int64_t R, int32_t k,
                                              float *__restrict__ out)
{
    const int lane = threadIdx.x & 63;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; r < R; r += nw) {
        const uint32_t *a = lsig + (int64_t)li[r] * k, *b = rsig + (int64_t)ri[r] * k;
        int cnt = 0;
        for (int i = lane; i < k; i += 64) cnt += a[i] == b[i];
        for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
        if (lane == 0) out[r] = (float)cnt / (float)k;
    }
}

int g_of(int64_t items, int per)
{
    int64_t g = (items + per - 1) / per;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (int)g;
}

}  // namespace

int32_t rank_sort_cap() { return kSortCap; }

polymh_status launch_head_select(const int64_t *off, const int32_t *cand_ids, int64_t nq,
                                 const int32_t *order, int32_t M, int64_t *hoff, int32_t *hq,
                                 int64_t *hc, int32_t *hid, hipStream_t s)
{
    if (nq == 0) return POLYMH_OK;
    hipLaunchKernelGGL(k_head_count, dim3(g_of(nq, 256)), dim3(256), 0, s, off, nq, M, hoff);
    polymh_status st = launch_offsets(hoff, nq, s);
    if (st) return st;
    hipLaunchKernelGGL(k_head_fill, dim3(g_of(nq, 1)), dim3(64), 0, s, off, cand_ids, order, hoff, nq,
                       hq, hc, hid);
    return check_launch("head_select");
}

polymh_status launch_head_fixed(const int64_t *off, const int32_t *cand_ids, int64_t nq, const int32_t *order,
                                int32_t M, int32_t *hq, int64_t *hc, int32_t *hid, hipStream_t s)
{
    if (nq == 0) return POLYMH_OK;
    hipLaunchKernelGGL(k_head_fixed, dim3(g_of(nq * (int64_t)M, 256)), dim3(256), 0, s, off, cand_ids, order, nq,
                       M, hq, hc, hid);
    return check_launch("head_fixed");
}

polymh_status launch_rank_jhat_sort(const uint32_t *qsig, const uint32_t *dsig, int32_t k, const int64_t *off,
                                    const int32_t *cand_ids, int64_t nq, float *score, int32_t *order,
                                    uint8_t *sorted_ok, hipStream_t s)
{
    if (nq == 0) return POLYMH_OK;
    if (nq > 0x7fffffffLL) return set_error(POLYMH_EINVAL, "rank_jhat: too many queries");
    const int vec = (k & 3) == 0 && k <= 1024 && (reinterpret_cast<uintptr_t>(qsig) & 15) == 0 &&
                    (reinterpret_cast<uintptr_t>(dsig) & 15) == 0;
    if (k <= 256)   // counts of at most 256 agreeing hashes: the counting sort
        hipLaunchKernelGGL(k_rank_jhat_sort<true>, dim3((unsigned)nq), dim3(1024), 0, s, qsig, dsig, k, vec, off,
                           cand_ids, score, order, sorted_ok);
    else
        hipLaunchKernelGGL(k_rank_jhat_sort<false>, dim3((unsigned)nq), dim3(1024), 0, s, qsig, dsig, k, vec, off,
                           cand_ids, score, order, sorted_ok);
    return check_launch("rank_jhat");
}

polymh_status launch_sig_pack(const uint32_t *sig, int64_t n, int32_t k, uint16_t *packed, hipStream_t s)
{
    if (n == 0) return POLYMH_OK;
    const int64_t blocks = std::min<int64_t>((n + 3) / 4, 1 << 20);
    hipLaunchKernelGGL(k_sig_pack, dim3((unsigned)blocks), dim3(256), 0, s, sig, n, k, packed);
    return check_launch("sig_pack");
}

polymh_status launch_rank_jhat_packed(const uint32_t *qsig, const uint16_t *packed, const uint32_t *dsig, int32_t k,
                                      const int64_t *off, const int32_t *cand_ids, int64_t nq, float *score,
                                      int32_t *order, uint8_t *sorted_ok, hipStream_t s)
{
    if (nq == 0) return POLYMH_OK;
    if (nq > 0x7fffffffLL) return set_error(POLYMH_EINVAL, "rank_jhat_packed: too many queries");
    hipLaunchKernelGGL(k_rank_jhat_packed, dim3((unsigned)nq), dim3(1024), 0, s, qsig, packed, dsig, k, off,
                       cand_ids, score, order, sorted_ok);
    return check_launch("rank_jhat_packed");
}

polymh_status launch_reorder_head(const int64_t *off, int64_t nq, const float *score, const int32_t *order_in,
                                 int32_t M, const uint8_t *sorted_ok, int32_t *order_out, hipStream_t s)
{
    if (nq == 0) return POLYMH_OK;
    hipLaunchKernelGGL(k_reorder_head, dim3(g_of(nq, 4)), dim3(256), 0, s, off, nq, score, order_in, M, sorted_ok,
                       order_out);
    return check_launch("reorder_head");
}

polymh_status launch_scatter_scores(const int64_t *idx, const float *val, int64_t n, float *score,
                                    hipStream_t s)
{
    if (n == 0) return POLYMH_OK;
    hipLaunchKernelGGL(k_scatter_scores, dim3(g_of(n, 256)), dim3(256), 0, s, idx, val, n, score);
    return check_launch("scatter_scores");
}

polymh_status launch_rank_sort(const int64_t *off, int64_t nq, const float *score, int32_t *order,
                               uint8_t *sorted_ok, hipStream_t s)
{
    if (nq == 0) return POLYMH_OK;
    hipLaunchKernelGGL(k_rank_sort, dim3((unsigned)nq), dim3(1024), 0, s, off, score, order, sorted_ok);
    return check_launch("rank_sort");
}

polymh_status launch_rank_init(int64_t nq, int32_t topk, int64_t *cursor, uint8_t *active,
                               int32_t *top_ids, double *top_j, hipStream_t s)
{
    if (nq == 0) return POLYMH_OK;
    hipLaunchKernelGGL(k_rank_init, dim3(g_of(nq, 256)), dim3(256), 0, s, nq, topk, cursor, active,
                       top_ids, top_j);
    return check_launch("rank_init");
}

polymh_status launch_round_offsets(const int64_t *off, int64_t nq, const int64_t *cursor,
                                   const uint8_t *active, int32_t F, int64_t *roff, hipStream_t s)
{
    hipLaunchKernelGGL(k_round_offsets, dim3(1), dim3(1024), 0, s, off, nq, cursor, active, F, roff);
    return check_launch("round_offsets");
}

polymh_status launch_round_fill(const int64_t *off, const int32_t *cand_ids, const int32_t *order,
                                const int64_t *cursor, const int64_t *roff, int64_t nq,
                                int32_t *rids, int32_t *rpos, hipStream_t s)
{
    hipLaunchKernelGGL(k_round_fill, dim3(g_of(nq, 1)), dim3(64), 0, s, off, cand_ids, order, cursor,
                       roff, nq, rids, rpos);
    return check_launch("round_fill");
}

polymh_status launch_round_merge(const int64_t *off, const float *score, const int32_t *order,
                                 const uint8_t *sorted_ok, const int64_t *roff, const int32_t *rids,
                                 const double *rj, int64_t nq, int32_t topk, float margin,
                                 int64_t *cursor, uint8_t *active, int32_t *top_ids, double *top_j,
                                 int32_t *n_active, unsigned long long *counters, int finishing, hipStream_t s)
{
    if (n_active) hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, n_active);
    const int64_t g = std::min<int64_t>(std::max<int64_t>((nq + 3) / 4, 1), 1024);
    hipLaunchKernelGGL(k_round_merge, dim3((unsigned)g), dim3(256), 0, s, off, score, order,
                       sorted_ok, roff, rids, rj, nq, topk, margin, cursor, active, top_ids, top_j,
                       n_active, counters, finishing);
    return check_launch("round_merge");
}

polymh_status launch_jhat(const uint32_t *lsig, const uint32_t *rsig, const int32_t *li,
                          const int32_t *ri, int64_t R, int32_t k, float *out, hipStream_t s)
{
    if (R == 0) return POLYMH_OK;
    hipLaunchKernelGGL(k_jhat, dim3(g_of(R, 4)), dim3(256), 0, s, lsig, rsig, li, ri, R, k, out);
    return check_launch("jhat");
}

}  // namespace polymh
