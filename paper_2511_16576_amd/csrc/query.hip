// Candidate generation (Sec. 3.2: a query's candidates are the polygons in
// its buckets).  Each (query, band) key is looked up by binary search in the
// sorted bucket table; a query's candidate list is the ids of the bucket
// entries that belong to the same band, in ascending order without repeats.
// A query whose buckets hold at most kSparseCap entries gathers them in LDS
// and sorts them there (work in proportion to its entries); a larger one
// sets its polygons' bits in a bitmap row of the data set's size and reads
// its set bits in order.  Both give the same list.
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
                                              int32_t b, uint32_t *__restrict__ bitmap, int64_t words,
                                              const int32_t *__restrict__ dense)
{
    const int lane = threadIdx.x & 63;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; w < nq * b; w += nw) {
        if (!dense[w / b]) continue;
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

// One block per query whose list is too long for LDS: clear its bitmap row.
__global__ __launch_bounds__(256) void k_zero_rows(uint32_t *__restrict__ bitmap, int64_t words,
                                                   const int32_t *__restrict__ dense)
{
    if (!dense[blockIdx.x]) return;
    uint32_t *row = bitmap + (int64_t)blockIdx.x * words;
    for (int64_t i = threadIdx.x; i < words; i += blockDim.x) row[i] = 0u;
}

constexpr int kSparseCap = 4096;

__device__ __forceinline__ void wave_lds_fence()
{
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_wave_barrier();
}

// One wavefront per query (four per block): its bucket entries of the same
// band gathered in LDS, sorted (bitonic, padded to a power of two with
// INT32_MAX) and kept without repeats in the query's own bitmap row, which
// the list leaves unused (rows hold at least kSparseCap words).  dense[q] =
// 1 when they do not fit (the bitmap takes the query), else 0 and counts[q]
// = the list's length.
__global__ __launch_bounds__(256) void k_sparse(const uint64_t *__restrict__ skeys,
                                                const int32_t *__restrict__ sids, int64_t n_entries,
                                                const uint64_t *__restrict__ qkeys, int64_t nq, int32_t b,
                                                int32_t *__restrict__ dense, int64_t *__restrict__ counts,
                                                uint32_t *__restrict__ bitmap, int64_t words)
{
    __shared__ int32_t lists[4][kSparseCap];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t q = (int64_t)blockIdx.x * 4 + wave;
    if (q >= nq) return;                       // wavefront-uniform; no block barriers below
    int32_t *L = lists[wave];
    int cnt = 0;
    // lane = band: every lane searches its own key, then the lanes walk their
    // buckets one entry per step
    for (int32_t t0 = 0; t0 < b && cnt <= kSparseCap; t0 += 64) {
        const int32_t t = t0 + lane;
        bool live = t < b && n_entries > 0;
        const uint64_t key = live ? qkeys[q * b + t] : 0ull;
        int64_t e = 0;
        if (live) {
            int64_t hi = n_entries;
            while (e < hi) {
                const int64_t mid = (e + hi) >> 1;
                if (skeys[mid] < key) e = mid + 1;
                else hi = mid;
            }
        }
        while (__ballot(live) != 0 && cnt <= kSparseCap) {
            const bool in = live && e < n_entries && skeys[e < n_entries ? e : 0] == key;
            int32_t id = 0;
            bool ok = false;
            if (in) {
                const int32_t ent = sids[e];          // entry p*b + t'
                id = ent / b;
                ok = ent - id * b == t;
            }
            const uint64_t om = __ballot(ok);
            const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(om >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((uint32_t)om, 0u));
            if (ok && cnt + rank < kSparseCap) L[cnt + rank] = id;
            cnt += __popcll(om);
            live = in;
            e++;
        }
    }
    const bool over = cnt > kSparseCap;
    if (lane == 0) dense[q] = over ? 1 : 0;
    if (over) return;
    int P = 64;
    while (P < cnt) P <<= 1;
    for (int i = cnt + lane; i < P; i += 64) L[i] = INT32_MAX;
    wave_lds_fence();
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = lane; i < P; i += 64) {
                const int x = i ^ j;
                if (x > i) {
                    const int32_t a = L[i], c = L[x];
                    if ((a > c) == ((i & k) == 0)) { L[i] = c; L[x] = a; }
                }
            }
            wave_lds_fence();
        }
    }
    int32_t *row = reinterpret_cast<int32_t *>(bitmap + q * words);
    int u = 0;
    for (int i0 = 0; i0 < cnt; i0 += 64) {
        const int i = i0 + lane;
        const bool live = i < cnt;
        const int32_t v = live ? L[i] : 0;
        const bool first = live && (i == 0 || L[i - 1] != v);
        const uint64_t fm = __ballot(first);
        if (first) {
            const int r = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(fm >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)fm, 0u));
            row[u + r] = v;
        }
        u += __popcll(fm);
    }
    if (lane == 0) counts[q] = u;
}

// One wavefront per query taken by k_sparse: its list copied from its row to
// off[q] (nothing when the capacity flag is raised).
__global__ __launch_bounds__(256) void k_sparse_emit(const uint32_t *__restrict__ bitmap, int64_t words,
                                                     const int32_t *__restrict__ dense, int64_t nq,
                                                     const int64_t *__restrict__ off, int32_t *__restrict__ ids,
                                                     const int32_t *__restrict__ overflow)
{
    const int lane = threadIdx.x & 63;
    const int64_t q = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (q >= nq || dense[q] || (overflow && overflow[0])) return;
    const int32_t *row = reinterpret_cast<const int32_t *>(bitmap + q * words);
    const int64_t base = off[q], n = off[q + 1] - base;
    for (int64_t i = lane; i < n; i += 64) ids[base + i] = row[i];
}

// One block per dense query: popcount of its bitmap row.
__global__ __launch_bounds__(256) void k_count(const uint32_t *__restrict__ bitmap, int64_t words,
                                               int64_t *__restrict__ counts, const int32_t *__restrict__ dense)
{
    if (!dense[blockIdx.x]) return;
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

// One block per dense query: write its set bits in ascending order (nothing
// when the capacity flag is raised).
__global__ __launch_bounds__(256) void k_emit(const uint32_t *__restrict__ bitmap, int64_t words,
                                              const int64_t *__restrict__ off,
                                              int32_t *__restrict__ ids, const int32_t *__restrict__ dense,
                                              const int32_t *__restrict__ overflow)
{
    __shared__ uint32_t s[256];
    const int64_t q = blockIdx.x;
    if (!dense[q] || (overflow && overflow[0])) return;
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


// Workspace: dense flags [nq], counts [nq], bitmap rows [nq][words].
struct QueryWs {
    int32_t *dense;
    int64_t *counts;
    uint32_t *bitmap;
};

QueryWs carve_query(Carve &cv, int64_t nq, int64_t words)
{
    QueryWs w{};
    w.dense = cv.take<int32_t>((size_t)nq);
    w.counts = cv.take<int64_t>((size_t)nq);
    w.bitmap = cv.take<uint32_t>((size_t)(nq * words));
    return w;
}

// Lengths of every query's list into counts (the sparse pass, then the
// bitmap rows of the dense queries).
// The bitmap is cleared, counted and read whole: once it passes 1 GiB (with
// rows of 16 KB and more) that costs more than gathering and sorting the
// queries' lists, and the lists are taken on chip where they fit.
constexpr int64_t kSparseMinBytes = (int64_t)1 << 30;
constexpr int64_t kSparseMinWords = 1 << 12;
static_assert(kSparseMinWords >= kSparseCap, "a sparse list is kept in its query's bitmap row");

__host__ __device__ inline bool use_sparse(int64_t nq, int64_t words)
{
    return words >= kSparseMinWords && nq * words * 4 >= kSparseMinBytes;
}

__global__ __launch_bounds__(256) void k_fill_i32(int32_t *p, int64_t count, int32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

void lookup_counts(const uint64_t *skeys, const int32_t *sids, int64_t n_entries, int64_t words,
                   const uint64_t *qkeys, int64_t nq, int32_t b, const QueryWs &w, int64_t *counts, hipStream_t s)
{
    if (use_sparse(nq, words))
        hipLaunchKernelGGL(k_sparse, dim3((unsigned)((nq + 3) / 4)), dim3(256), 0, s, skeys, sids, n_entries,
                           qkeys, nq, b, w.dense, counts, w.bitmap, words);
    else
        hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(nq, 256)), dim3(256), 0, s, w.dense, nq, 1);
    if (words > 0) {
        hipLaunchKernelGGL(k_zero_rows, dim3((unsigned)nq), dim3(256), 0, s, w.bitmap, words, w.dense);
        if (n_entries > 0)
            hipLaunchKernelGGL(k_mark, dim3(blocks_for(nq * b, 4)), dim3(256), 0, s, skeys, sids, n_entries,
                               qkeys, nq, b, w.bitmap, words, w.dense);
    }
    // also with no data (a zero count per query)
    hipLaunchKernelGGL(k_count, dim3((unsigned)nq), dim3(256), 0, s, w.bitmap, words, counts, w.dense);
}

void lookup_emit(const uint64_t *skeys, const int32_t *sids, int64_t n_entries, int64_t words,
                 const uint64_t *qkeys, int64_t nq, int32_t b, const QueryWs &w, int64_t *off, int32_t *ids,
                 const int32_t *overflow, hipStream_t s)
{
    if (use_sparse(nq, words))
        hipLaunchKernelGGL(k_sparse_emit, dim3((unsigned)((nq + 3) / 4)), dim3(256), 0, s, w.bitmap, words, w.dense,
                           nq, off, ids, overflow);
    if (words > 0)
        hipLaunchKernelGGL(k_emit, dim3((unsigned)nq), dim3(256), 0, s, w.bitmap, words, off, ids, w.dense,
                           overflow);
}

}  // namespace

polymh_status launch_query_capped(const uint64_t *skeys, const int32_t *sids, int64_t n_entries,
                                  int64_t n_data, const uint64_t *qkeys, int64_t nq, int32_t b,
                                  void *ws, size_t ws_bytes, int64_t *cand_off, int32_t *cand_ids,
                                  int64_t cand_cap, int32_t *overflow, hipStream_t s)
{
    const int64_t words = (n_data + 31) / 32;
    Carve cv{static_cast<char *>(ws), ws_bytes};
    const QueryWs w = carve_query(cv, nq, words);
    if (!cv.ok)
        return set_error(POLYMH_ECAPACITY, "query_capped: workspace of %zu bytes, need %zu", ws_bytes, cv.used);
    if (nq > 0x7fffffffLL) return set_error(POLYMH_EINVAL, "query_capped: too many queries");
    if (nq > 0) lookup_counts(skeys, sids, n_entries, words, qkeys, nq, b, w, cand_off, s);
    hipLaunchKernelGGL(k_offsets, dim3(1), dim3(1024), 0, s, cand_off, nq);
    hipLaunchKernelGGL(k_cap_guard, dim3(blocks_for(nq + 1, 256)), dim3(256), 0, s, cand_off, nq, cand_cap, overflow);
    if (nq > 0) lookup_emit(skeys, sids, n_entries, words, qkeys, nq, b, w, cand_off, cand_ids, overflow, s);
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
    Carve cv{nullptr, 0};
    carve_query(cv, nq, words);
    return align_up(cv.used, 256) + 256;
}

polymh_status launch_query(const uint64_t *skeys, const int32_t *sids, int64_t n_entries,
                           int64_t n_data, const uint64_t *qkeys, int64_t nq, int32_t b, void *ws,
                           size_t ws_bytes, int64_t *cand_off, int32_t *cand_ids, hipStream_t s)
{
    const int64_t words = (n_data + 31) / 32;
    Carve cv{static_cast<char *>(ws), ws_bytes};
    const QueryWs w = carve_query(cv, nq, words);
    if (!cv.ok)
        return set_error(POLYMH_ECAPACITY, "query: workspace of %zu bytes, need %zu", ws_bytes, cv.used);
    if (nq == 0) {
        hipLaunchKernelGGL(k_offsets, dim3(1), dim3(1024), 0, s, cand_off, (int64_t)0);
        return check_launch("query");
    }
    if (nq > 0x7fffffffLL) return set_error(POLYMH_EINVAL, "query: too many queries");
    if (!cand_ids) {
        lookup_counts(skeys, sids, n_entries, words, qkeys, nq, b, w, cand_off, s);
        hipLaunchKernelGGL(k_offsets, dim3(1), dim3(1024), 0, s, cand_off, nq);
    } else {
        // the offsets are the caller's from the first phase; the lengths go
        // to the workspace
        lookup_counts(skeys, sids, n_entries, words, qkeys, nq, b, w, w.counts, s);
        lookup_emit(skeys, sids, n_entries, words, qkeys, nq, b, w, cand_off, cand_ids, nullptr, s);
    }
    return check_launch("query");
}

}  // namespace polymh
