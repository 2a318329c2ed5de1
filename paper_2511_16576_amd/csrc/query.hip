// Candidate generation (Sec. 3.2: a query's candidates are the polygons in
// its buckets).  Each (query, band) key is looked up by binary search in the
// sorted bucket table and every entry of the bucket that belongs to the same
// band sets its polygon's bit in the query's bitmap; a query's candidate list is then its set bits in ascending
// id order, which deduplicates across bands without any sort.
#include "internal.hpp"

namespace polymh {

namespace {

__global__ __launch_bounds__(256) void k_zero_u32(uint32_t *p, int64_t count)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// First index in a[lo, hi) whose value is >= v, by a 64-way search: each
// round the lanes sample 64 evenly spaced positions and the count of samples
// below v (a ballot) narrows the range by a factor of 64.  All lanes of the
// wavefront take part; the result is uniform.
__device__ __forceinline__ int64_t lower_bound_wave(const uint64_t *a, int64_t lo, int64_t hi, uint64_t v,
                                                    int lane)
{
    while (hi - lo > 64) {
        const int64_t step = (hi - lo + 63) >> 6;
        const int64_t p = lo + (int64_t)lane * step;
        const bool valid = p < hi;
        const bool less = valid && a[valid ? p : lo] < v;
        const int c = __popcll(__ballot(less));
        const int nvalid = __popcll(__ballot(valid));
        const int64_t nlo = c > 0 ? lo + (int64_t)(c - 1) * step + 1 : lo;
        const int64_t nhi = c < nvalid ? lo + (int64_t)c * step : hi;
        lo = nlo;
        hi = nhi;
    }
    const int64_t p = lo + lane;
    const bool less = p < hi && a[p < hi ? p : lo] < v;
    return lo + __popcll(__ballot(less));
}

// One wavefront per (query, band): find the bucket, lanes mark its entries.
// The bucket's end is found by scanning forward 64 entries at a time (a
// bucket holds the polygons sharing one 64-bit key: a handful).
__global__ __launch_bounds__(256) void k_mark(const uint64_t *__restrict__ skeys,
                                              const int32_t *__restrict__ sids, int64_t n_entries,
                                              const uint64_t *__restrict__ qkeys, int64_t nq,
                                              int32_t b, uint32_t *__restrict__ bitmap, int64_t words)
{
    const int lane = threadIdx.x & 63;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; w < nq * b; w += nw) {
        const uint64_t key = qkeys[w];
        const int32_t t = (int32_t)(w % b);
        uint32_t *row = bitmap + (w / b) * words;
        int64_t e0 = lower_bound_wave(skeys, 0, n_entries, key, lane);
        while (e0 < n_entries) {
            const int64_t e = e0 + lane;
            const bool in = e < n_entries && skeys[e < n_entries ? e : 0] == key;
            const uint64_t mk = __ballot(in);
            if (in) {
                const int32_t ent = sids[e];          // entry p*b + t'
                const int32_t id = ent / b;
                if (ent - id * b == t) atomicOr(&row[id >> 5], 1u << (id & 31));
            }
            if (mk != ~0ull) break;                   // the bucket ended inside this window
            e0 += 64;
        }
    }
}

// One block per query: popcount of its bitmap row.
__global__ __launch_bounds__(256) void k_count(const uint32_t *__restrict__ bitmap, int64_t words,
                                               int64_t *__restrict__ counts)
{
    __shared__ int64_t s[256];
    const uint32_t *row = bitmap + (int64_t)blockIdx.x * words;
    int64_t c = 0;
    for (int64_t i = threadIdx.x; i < words; i += blockDim.x) c += __popc(row[i]);
    s[threadIdx.x] = c;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[blockIdx.x] = s[0];
}

// Exclusive prefix of counts[0..nq) into off[0..nq], single block.
__global__ __launch_bounds__(1024) void k_offsets(int64_t *__restrict__ off, int64_t nq)
{
    __shared__ int64_t s[1024];
    int64_t carry = 0;
    for (int64_t c0 = 0; c0 < nq; c0 += 1024) {
        const int64_t c = c0 + threadIdx.x;
        const int64_t v = c < nq ? off[c] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int64_t t = threadIdx.x >= (unsigned)o ? s[threadIdx.x - o] : 0;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        if (c < nq) off[c] = carry + s[threadIdx.x] - v;
        carry += s[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) off[nq] = carry;
}

// One block per query: write its set bits in ascending order.
__global__ __launch_bounds__(256) void k_emit(const uint32_t *__restrict__ bitmap, int64_t words,
                                              const int64_t *__restrict__ off,
                                              int32_t *__restrict__ ids)
{
    __shared__ uint32_t s[256];
    const int64_t q = blockIdx.x;
    const uint32_t *row = bitmap + q * words;
    int64_t base = off[q];
    for (int64_t w0 = 0; w0 < words; w0 += 256) {
        const int64_t w = w0 + threadIdx.x;
        uint32_t bits = w < words ? row[w] : 0u;
        const uint32_t c = __popc(bits);
        s[threadIdx.x] = c;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {
            const uint32_t t = threadIdx.x >= (unsigned)o ? s[threadIdx.x - o] : 0u;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        int64_t pos = base + s[threadIdx.x] - c;
        while (bits) {
            const int bit = __builtin_ctz(bits);
            ids[pos++] = (int32_t)(w * 32 + bit);
            bits &= bits - 1;
        }
        base += s[255];
        __syncthreads();
    }
}

// Capacity guard for graph-captured lookups: if the candidates do not fit,
// raise the flag and empty every query's range so later stages see none.
__global__ __launch_bounds__(256) void k_cap_guard(int64_t *__restrict__ off, int64_t nq, int64_t cap,
                                                   int32_t *__restrict__ overflow)
{
    const int64_t total = off[nq];
    if (total <= cap) {
        if (blockIdx.x == 0 && threadIdx.x == 0) overflow[0] = 0;
        return;
    }
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q <= nq;
         q += (int64_t)gridDim.x * blockDim.x)
        off[q] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) overflow[0] = 1;
}

int blocks_for(int64_t items, int per_block)
{
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (int)g;
}

}  // namespace

polymh_status launch_query_capped(const uint64_t *skeys, const int32_t *sids, int64_t n_entries,
                                  int64_t n_data, const uint64_t *qkeys, int64_t nq, int32_t b,
                                  void *ws, size_t ws_bytes, int64_t *cand_off, int32_t *cand_ids,
                                  int64_t cand_cap, int32_t *overflow, hipStream_t s)
{
    const int64_t words = (n_data + 31) / 32;
    Carve cv{static_cast<char *>(ws), ws_bytes};
    uint32_t *bitmap = cv.take<uint32_t>((size_t)(nq * words));
    if (!cv.ok)
        return set_error(POLYMH_ECAPACITY, "query_capped: workspace of %zu bytes, need %zu", ws_bytes, cv.used);
    if (nq > 0x7fffffffLL) return set_error(POLYMH_EINVAL, "query_capped: too many queries");
    if (nq * words > 0)
        hipLaunchKernelGGL(k_zero_u32, dim3(blocks_for(nq * words, 256)), dim3(256), 0, s, bitmap, nq * words);
    if (n_entries > 0 && words > 0 && nq > 0)
        hipLaunchKernelGGL(k_mark, dim3(blocks_for(nq * b, 4)), dim3(256), 0, s, skeys, sids, n_entries,
                           qkeys, nq, b, bitmap, words);
    if (nq > 0) hipLaunchKernelGGL(k_count, dim3((unsigned)nq), dim3(256), 0, s, bitmap, words, cand_off);
    hipLaunchKernelGGL(k_offsets, dim3(1), dim3(1024), 0, s, cand_off, nq);
    hipLaunchKernelGGL(k_cap_guard, dim3(blocks_for(nq + 1, 256)), dim3(256), 0, s, cand_off, nq, cand_cap, overflow);
    if (nq > 0) hipLaunchKernelGGL(k_emit, dim3((unsigned)nq), dim3(256), 0, s, bitmap, words, cand_off, cand_ids);
    return check_launch("query_capped");
}

polymh_status launch_offsets(int64_t *off, int64_t nq, hipStream_t s)
{
    hipLaunchKernelGGL(k_offsets, dim3(1), dim3(1024), 0, s, off, nq);
    return check_launch("offsets");
}

size_t query_workspace_bytes(int64_t n_data, int64_t nq)
{
    const int64_t words = (n_data + 31) / 32;
    return align_up((size_t)(nq * words) * sizeof(uint32_t), 256) + 256;
}

polymh_status launch_query(const uint64_t *skeys, const int32_t *sids, int64_t n_entries,
                           int64_t n_data, const uint64_t *qkeys, int64_t nq, int32_t b, void *ws,
                           size_t ws_bytes, int64_t *cand_off, int32_t *cand_ids, hipStream_t s)
{
    const int64_t words = (n_data + 31) / 32;
    Carve cv{static_cast<char *>(ws), ws_bytes};
    uint32_t *bitmap = cv.take<uint32_t>((size_t)(nq * words));
    if (!cv.ok)
        return set_error(POLYMH_ECAPACITY, "query: workspace of %zu bytes, need %zu", ws_bytes, cv.used);
    if (nq == 0) {
        hipLaunchKernelGGL(k_offsets, dim3(1), dim3(1024), 0, s, cand_off, (int64_t)0);
        return check_launch("query");
    }
    if (nq * words > 0)
        hipLaunchKernelGGL(k_zero_u32, dim3(blocks_for(nq * words, 256)), dim3(256), 0, s, bitmap, nq * words);
    if (n_entries > 0 && words > 0)
        hipLaunchKernelGGL(k_mark, dim3(blocks_for(nq * b, 4)), dim3(256), 0, s, skeys, sids, n_entries,
                           qkeys, nq, b, bitmap, words);
    if (!cand_ids) {
        if (nq > 0x7fffffffLL) return set_error(POLYMH_EINVAL, "query: too many queries");
        hipLaunchKernelGGL(k_count, dim3((unsigned)nq), dim3(256), 0, s, bitmap, words, cand_off);
        hipLaunchKernelGGL(k_offsets, dim3(1), dim3(1024), 0, s, cand_off, nq);
    } else {
        hipLaunchKernelGGL(k_emit, dim3((unsigned)nq), dim3(256), 0, s, bitmap, words, cand_off, cand_ids);
    }
    return check_launch("query");
}

}  // namespace polymh
