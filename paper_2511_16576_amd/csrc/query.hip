// Candidate generation (Sec. 3.2: a query's candidates are the polygons in
// its buckets).  Each (query, band) key is looked up by binary search in the
// sorted bucket table; a query's candidate list is the ids of the bucket
// entries that belong to the same band, in ascending order without repeats.
// For large data sets a query's same-band bucket entries are gathered into
// its own bitmap row (work in proportion to its entries), then sorted and
// kept without repeats on chip (one wavefront for up to kSparseCap entries,
// a block for up to kBigCap); a query with more entries sets its polygons'
// bits in the bitmap row and reads its set bits in order.  Every way gives
// the same list.
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

// First index in a[0, n) whose value is >= key.  Band keys are SplitMix64
// outputs, uniform over 64 bits, so a probe placed by linear interpolation
// between the bracket's end values lands near the answer (about log log n
// probes): the first five probes interpolate, then interpolation
// alternates with bisection, which bounds the probes by about 5 + 2 log2 n
// on any key set (long runs of equal keys included).  On 2^25 uniform keys
// the probes average 5.4, against 8.9 when alternating from the first.
__device__ __forceinline__ int64_t lower_bound_interp(const uint64_t *__restrict__ a, int64_t n, uint64_t key)
{
    int64_t lo = 0, hi = n;                 // answer in [lo, hi]
    uint64_t klo = 0, khi = ~0ull;          // a[lo - 1] < key <= a[hi] (or the ends of the key range)
    int step = 0;
    while (lo < hi) {
        int64_t p = (lo + hi) >> 1;
        const bool interp = step < 5 || (step & 1);
        if (interp && khi > klo) {
            const double f = (double)(key - klo) / (double)(khi - klo);
            const int64_t g = lo + (int64_t)(f * (double)(hi - lo));
            p = g < lo ? lo : (g >= hi ? hi - 1 : g);
        }
        step++;
        const uint64_t v = a[p];
        if (v < key) {
            lo = p + 1;
            klo = v;
        } else {
            hi = p;
            khi = v;
        }
    }
    return lo;
}

// Sorts L[0, cnt) in place (bitonic, padded with INT32_MAX to a power of
// two of at most kSparseCap) and keeps each value once; returns the new
// length.  One wavefront.
__device__ int sort_unique(int32_t *L, int cnt, int lane)
{
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
    // in place: a chunk's values are read before any of its writes, and
    // writes land at or below the positions already read
    int u = 0;
    for (int i0 = 0; i0 < cnt; i0 += 64) {
        const int i = i0 + lane;
        const bool live = i < cnt;
        const int32_t v = live ? L[i] : 0;
        const bool first = live && (i == 0 || L[i - 1] != v);
        wave_lds_fence();
        const uint64_t fm = __ballot(first);
        if (first) {
            const int r = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(fm >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)fm, 0u));
            L[u + r] = v;
        }
        u += __popcll(fm);
        wave_lds_fence();
    }
    return u;
}

// Bitonic sort of 64 R values held R to a lane (element i = R lane + r, a
// blocked layout), ascending, in registers: steps within a lane swap
// registers, steps across lanes exchange with __shfl_xor.  R is 16 or 32.
template <int R>
__device__ __forceinline__ void sort_regs(int32_t (&v)[R], int lane)
{
#pragma unroll
    for (int k = 2; k <= 64 * R; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= R) {
                const int lj = j / R;                   // partner lane offset
                const bool lower = (lane & lj) == 0;
#pragma unroll
                for (int r = 0; r < R; r++) {
                    const bool up = ((R * lane + r) & k) == 0;
                    const int32_t o = __shfl_xor(v[r], lj, 64);
                    const int32_t lo = min(v[r], o), hi = max(v[r], o);
                    v[r] = (lower == up) ? lo : hi;
                }
            } else {
#pragma unroll
                for (int r = 0; r < R; r++) {
                    if ((r & j) == 0) {
                        const bool up = ((R * lane + r) & k) == 0;
                        const int32_t a = v[r], b = v[r | j];
                        const int32_t lo = min(a, b), hi = max(a, b);
                        v[r] = up ? lo : hi;
                        v[r | j] = up ? hi : lo;
                    }
                }
            }
        }
    }
}

constexpr int kBigCap = 16384;

// Gather pass, one wavefront per query (four per block): the query's
// same-band bucket entries, in bucket order with repeats, written to the
// start of its own bitmap row; raw[q] = their number.  A query with more
// than min(kBigCap, words) entries gets dense[q] = 1 (the bitmap takes it).
//
// Lane t takes band t's key: an interpolation search gives its bucket's
// first entry, a galloping search (probes 1, 2, 4, ... entries on, then a
// binary search between the last two) its end.  The bucket lengths' prefix
// sum then spreads every entry of the 64 buckets over the lanes, 64 entries
// a step with independent loads, so the walk takes (entries / 64) steps
// instead of as many as the longest bucket holds.
__global__ __launch_bounds__(256) void k_sparse(const uint64_t *__restrict__ skeys,
                                                const int32_t *__restrict__ sids, int64_t n_entries,
                                                const uint64_t *__restrict__ qkeys, int64_t nq, int32_t b,
                                                int32_t *__restrict__ dense, int64_t *__restrict__ raw,
                                                uint32_t *__restrict__ bitmap, int64_t words)
{
    __shared__ int32_t sbase[4][65];     // exclusive prefix of the bucket lengths, then the total
    __shared__ int64_t slo[4][64];       // each lane's bucket start
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t q = (int64_t)blockIdx.x * 4 + wave;
    if (q >= nq) return;                       // wavefront-uniform; no block barriers below
    const int cap = (int)(words < kBigCap ? words : kBigCap);
    int32_t *row = reinterpret_cast<int32_t *>(bitmap + q * words);
    int32_t *base = sbase[wave];
    int64_t *los = slo[wave];
    int cnt = 0;
    bool over = false;
    for (int32_t t0 = 0; t0 < b && !over; t0 += 64) {
        const int32_t t = t0 + lane;
        const bool live = t < b && n_entries > 0;
        const uint64_t key = live ? qkeys[q * b + t] : 0ull;
        int64_t lo = 0, hi = 0;
        if (live) {
            lo = lower_bound_interp(skeys, n_entries, key);
            hi = lo;
            if (lo < n_entries && skeys[lo] == key) {
                // gallop: skeys[last] == key, probe = lo + step is the next test
                int64_t last = lo, step = 1;
                while (lo + step < n_entries && skeys[lo + step] == key) {
                    last = lo + step;
                    step <<= 1;
                }
                int64_t a = last + 1, c = lo + step < n_entries ? lo + step : n_entries;
                while (a < c) {
                    const int64_t mid = (a + c) >> 1;
                    if (skeys[mid] == key) a = mid + 1;
                    else c = mid;
                }
                hi = a;
            }
        }
        // a bucket longer than the list sends the query to the bitmap (which
        // is exact in every case)
        const int64_t len64 = hi - lo;
        if (__ballot(len64 > cap) != 0) {
            over = true;
            break;
        }
        const int len = (int)len64;
        // inclusive scan over the wavefront (64 x 16384 fits an int)
        int inc = len;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(inc, o, 64);
            if (lane >= o) inc += v;
        }
        base[lane] = inc - len;
        los[lane] = lo;
        const int total = __shfl(inc, 63, 64);
        if (lane == 63) base[64] = total;
        wave_lds_fence();
        // every entry of the 64 buckets, one per lane per step (band lane
        // tl of entry j is the last with base[tl] <= j); the entries of
        // kWalk steps are loaded before any is used, so the walk costs
        // total / (64 kWalk) round trips to memory
        constexpr int kWalk = 8;
        for (int j00 = 0; j00 < total && !over; j00 += 64 * kWalk) {
            int32_t ent[kWalk];
            int band[kWalk];
#pragma unroll
            for (int u = 0; u < kWalk; u++) {
                const int j = j00 + 64 * u + lane;
                ent[u] = -1;
                band[u] = 0;
                if (j < total) {
                    int l = 0, h = 63;         // base[l] <= j < base[h + 1]
                    while (l < h) {
                        const int mid = (l + h + 1) >> 1;
                        if (base[mid] <= j) l = mid;
                        else h = mid - 1;
                    }
                    ent[u] = sids[los[l] + (j - base[l])];   // entry p*b + t'
                    band[u] = t0 + l;
                }
            }
#pragma unroll
            for (int u = 0; u < kWalk; u++) {
                const int32_t id = ent[u] >= 0 ? ent[u] / b : 0;
                const bool ok = ent[u] >= 0 && ent[u] - id * b == band[u];
                const uint64_t om = __ballot(ok);
                const int n_new = __popcll(om);
                if (cnt + n_new > cap) {       // wavefront-uniform
                    over = true;
                    break;
                }
                const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(om >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)om, 0u));
                if (ok) row[cnt + rank] = id;
                cnt += n_new;
            }
        }
        wave_lds_fence();                      // base/los are rewritten by the next band chunk
    }
    if (lane == 0) {
        dense[q] = over ? 1 : 0;
        raw[q] = over ? 0 : cnt;
    }
}

// Multiplicative hash of a polygon id to a slot of a 2^bits table.
__device__ __forceinline__ int id_slot(int32_t id, int bits)
{
    return (int)(((uint32_t)id * 2654435761u) >> (32 - bits));
}

// Inserts v into an open-addressing set T of 2^bits slots (-1 = empty) by
// linear probing; returns true if v was not there yet.  Needs an empty slot.
__device__ __forceinline__ bool set_insert(int32_t *T, int bits, int32_t v)
{
    int h = id_slot(v, bits);
    const int mask = (1 << bits) - 1;
    for (;;) {
        const int32_t old = atomicCAS(&T[h], -1, v);
        if (old == -1) return true;
        if (old == v) return false;
        h = (h + 1) & mask;
    }
}

constexpr int kSetBits = 12;                 // wavefront pass: 4096 slots
constexpr int kSetMax = 3072;                // ... filled to at most 3/4
constexpr int kBigSetBits = 14;              // block pass: 16384 slots
constexpr int kBigSetMax = 12288;
static_assert((1 << kSetBits) == kSparseCap && (1 << kBigSetBits) == kBigCap, "set sizes");

// Sort pass for short lists, one wavefront per query (four per block): a
// query's raw list of at most kSparseCap entries, read from its row 64 at a
// time, goes into an LDS hash set (each polygon once); the set's members
// are moved to its front, sorted (bitonic) and written back; counts[q] =
// the list's length.  A list with more than kSetMax distinct polygons is
// sorted whole instead (its repeats dropped after the sort).
__global__ __launch_bounds__(256) void k_sparse_sort(const int32_t *__restrict__ dense, int64_t nq,
                                                     int64_t *__restrict__ counts, uint32_t *__restrict__ bitmap,
                                                     int64_t words)
{
    __shared__ int32_t lists[4][kSparseCap];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t q = (int64_t)blockIdx.x * 4 + wave;
    if (q >= nq || dense[q]) return;           // wavefront-uniform
    const int cnt = (int)counts[q];            // the raw count of the gather pass
    if (cnt > kSparseCap) return;              // the block pass takes it
    int32_t *T = lists[wave];
    int32_t *row = reinterpret_cast<int32_t *>(bitmap + q * words);
    for (int i = lane; i < kSparseCap; i += 64) T[i] = -1;
    wave_lds_fence();
    int uniq = 0;
    bool whole = false;
    // eight of a lane's entries are loaded together, then inserted
    for (int i0 = 0; i0 < cnt && !whole; i0 += 8 * 64) {
        int32_t v[8];
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const int i = i0 + 64 * u + lane;
            v[u] = i < cnt ? row[i] : -1;
        }
#pragma unroll
        for (int u = 0; u < 8; u++) {
            if (uniq + 64 > kSetMax) {         // wavefront-uniform: keep the set below 3/4 full
                whole = true;
                break;
            }
            const bool fresh = v[u] >= 0 && set_insert(T, kSetBits, v[u]);
            uniq += __popcll(__ballot(fresh));
        }
    }
    wave_lds_fence();
    int u;
    if (whole) {
        for (int i = lane; i < cnt; i += 64) T[i] = row[i];
        wave_lds_fence();
        u = sort_unique(T, cnt, lane);
    } else {
        // members to the front, in place (a chunk reads before it writes,
        // and writes land at or below what it read)
        int m = 0;
        for (int i0 = 0; i0 < kSparseCap; i0 += 64) {
            const int32_t v = T[i0 + lane];
            const bool keep = v != -1;
            wave_lds_fence();
            const uint64_t km = __ballot(keep);
            if (keep) {
                const int r = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(km >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u));
                T[m + r] = v;
            }
            m += __popcll(km);
            wave_lds_fence();
        }
        // the members are distinct: sorted in registers when they fit
        // (1,024 or 2,048 of them), else in LDS
        if (m <= 1024) {
            int32_t v[16];
#pragma unroll
            for (int r = 0; r < 16; r++) v[r] = 16 * lane + r < m ? T[16 * lane + r] : INT32_MAX;
            sort_regs<16>(v, lane);
#pragma unroll
            for (int r = 0; r < 16; r++)
                if (16 * lane + r < m) row[16 * lane + r] = v[r];
            if (lane == 0) counts[q] = m;
            return;
        }
        if (m <= 2048) {
            int32_t v[32];
#pragma unroll
            for (int r = 0; r < 32; r++) v[r] = 32 * lane + r < m ? T[32 * lane + r] : INT32_MAX;
            sort_regs<32>(v, lane);
#pragma unroll
            for (int r = 0; r < 32; r++)
                if (32 * lane + r < m) row[32 * lane + r] = v[r];
            if (lane == 0) counts[q] = m;
            return;
        }
        u = sort_unique(T, m, lane);
    }
    for (int i = lane; i < u; i += 64) row[i] = T[i];
    if (lane == 0) counts[q] = u;
}

// Bitonic sort of 4096 values over a 1024-thread block, thread t holding
// positions 4t .. 4t + 3: partners in the same thread are swapped in
// registers, partners in the same wavefront exchanged by shuffles, and the
// ten steps whose partners sit in another wavefront go through L (a write,
// a barrier, a read, a barrier).
__device__ void sort_block4096(int32_t (&v)[4], int32_t *L, int tid)
{
    const int lane = tid & 63;
    for (int k = 2; k <= 4096; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= 256) {
#pragma unroll
                for (int r = 0; r < 4; r++) L[4 * tid + r] = v[r];
                __syncthreads();
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int i = 4 * tid + r;
                    const int32_t o = L[i ^ j];
                    const bool keep_min = ((i & j) == 0) == ((i & k) == 0);
                    v[r] = keep_min ? min(v[r], o) : max(v[r], o);
                }
                __syncthreads();
            } else if (j >= 4) {
                const int lj = j >> 2;
                const bool lower = (lane & lj) == 0;
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const bool up = ((4 * tid + r) & k) == 0;
                    const int32_t o = __shfl_xor(v[r], lj, 64);
                    v[r] = (lower == up) ? min(v[r], o) : max(v[r], o);
                }
            } else {
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    if ((r & j) == 0) {
                        const bool up = ((4 * tid + r) & k) == 0;
                        const int32_t x = v[r], y = v[r | j];
                        v[r] = up ? min(x, y) : max(x, y);
                        v[r | j] = up ? max(x, y) : min(x, y);
                    }
                }
            }
        }
    }
}

// Block-wide exclusive prefix of one int per thread (1024 threads); *total
// gets the sum.  sw holds 16 ints.
__device__ __forceinline__ int block_excl_scan1024(int x, int *sw, int tid, int *total)
{
    const int lane = tid & 63, wave = tid >> 6;
    const int incl = wave_incl_scan32(x);
    if (lane == 63) sw[wave] = incl;
    __syncthreads();
    int pre = incl - x, tot = 0;
#pragma unroll
    for (int w = 0; w < 16; w++) {
        const int y = sw[w];
        pre += w < wave ? y : 0;
        tot += y;
    }
    *total = tot;
    return pre;
}

// Sort pass for long lists, one block of 1024 threads per query with more
// than kSparseCap raw entries (at most kBigCap): the raw list is loaded
// whole (16 entries a thread, all in flight together), inserted into an LDS
// hash set of 16384 slots (each polygon once), the set's members moved to
// the front (a block-wide scan places them) and sorted: up to 4096 of them
// in registers, more in LDS.  More than kBigSetMax distinct polygons: the
// raw list is sorted whole in LDS and its repeats dropped.
__global__ __launch_bounds__(1024) void k_sparse_sort_big(const int32_t *__restrict__ dense,
                                                          int64_t *__restrict__ counts,
                                                          uint32_t *__restrict__ bitmap, int64_t words)
{
    __shared__ int32_t L[kBigCap];
    __shared__ int sw[16];
    __shared__ int s_uniq;
    const int64_t q = blockIdx.x;
    if (dense[q]) return;
    const int cnt = (int)counts[q];
    if (cnt <= kSparseCap) return;             // the wavefront pass took it
    const int tid = threadIdx.x, lane = tid & 63;
    int32_t *row = reinterpret_cast<int32_t *>(bitmap + q * words);
    int32_t raw[kBigCap / 1024];
#pragma unroll
    for (int u = 0; u < kBigCap / 1024; u++) {
        const int i = u * 1024 + tid;
        raw[u] = i < cnt ? row[i] : -1;
    }
    for (int i = tid; i < kBigCap; i += 1024) L[i] = -1;
    if (tid == 0) s_uniq = 0;
    __syncthreads();
    bool whole = false;
#pragma unroll
    for (int u = 0; u < kBigCap / 1024; u++) {
        if (u * 1024 >= cnt) break;             // block-uniform
        if (s_uniq + 1024 > kBigSetMax) {     // block-uniform (read after a barrier)
            whole = true;
            break;
        }
        const bool fresh = raw[u] >= 0 && set_insert(L, kBigSetBits, raw[u]);
        const int nf = __popcll(__ballot(fresh));
        if (lane == 0 && nf) atomicAdd(&s_uniq, nf);
        __syncthreads();
    }
    __syncthreads();
    int n;                                      // entries to sort at the front of L
    if (whole) {
        for (int i = tid; i < cnt; i += 1024) L[i] = row[i];
        n = cnt;
    } else {
        // members to the front: thread tid owns slots [16 tid, 16 tid + 16)
        int32_t v[16];
        int mine = 0;
#pragma unroll
        for (int k = 0; k < 16; k++) {
            v[k] = L[16 * tid + k];
            mine += v[k] != -1;
        }
        int at = block_excl_scan1024(mine, sw, tid, &n);
        __syncthreads();                        // every slot read before any is rewritten
#pragma unroll
        for (int k = 0; k < 16; k++)
            if (v[k] != -1) L[at++] = v[k];
        __syncthreads();
        if (n <= 4096) {
            // distinct ids: sorted in registers and written out as they are
            int32_t w[4];
#pragma unroll
            for (int r = 0; r < 4; r++) w[r] = 4 * tid + r < n ? L[4 * tid + r] : INT32_MAX;
            __syncthreads();                    // L is reused by the sort's cross-wavefront steps
            sort_block4096(w, L, tid);
#pragma unroll
            for (int r = 0; r < 4; r++)
                if (4 * tid + r < n) row[4 * tid + r] = w[r];
            if (tid == 0) counts[q] = n;
            return;
        }
    }
    int P = 1;
    while (P < n) P <<= 1;
    for (int i = n + tid; i < P; i += 1024) L[i] = INT32_MAX;
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < P; i += 1024) {
                const int x = i ^ j;
                if (x > i) {
                    const int32_t a = L[i], c = L[x];
                    if ((a > c) == ((i & k) == 0)) { L[i] = c; L[x] = a; }
                }
            }
            __syncthreads();
        }
    }
    // thread tid owns positions [tid * per, (tid + 1) * per); the first of
    // each run of equal values is kept
    const int per = (n + 1023) / 1024;
    const int i0 = tid * per, i1 = min(n, i0 + per);
    int mine = 0;
    for (int i = i0; i < i1; i++) mine += (i == 0 || L[i - 1] != L[i]) ? 1 : 0;
    int total;
    int u = block_excl_scan1024(mine, sw, tid, &total);
    for (int i = i0; i < i1; i++)
        if (i == 0 || L[i - 1] != L[i]) row[u++] = L[i];
    if (tid == 0) counts[q] = total;
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
    // eight independent loads in flight a thread
    int64_t i = threadIdx.x;
    for (; i + 7 * 256 < words; i += 8 * 256) {
        uint32_t v[8];
#pragma unroll
        for (int u = 0; u < 8; u++) v[u] = row[i + u * 256];
#pragma unroll
        for (int u = 0; u < 8; u++) c += __popc(v[u]);
    }
    for (; i < words; i += blockDim.x) c += __popc(row[i]);
    s[threadIdx.x] = c;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[blockIdx.x] = s[0];
}

// Exclusive prefix of counts[0..nq) into off[0..nq], single block, in
// tiles of 8192: each thread adds 8 consecutive counts, a wavefront scan of
// those sums and a pass over the 16 wavefront totals place every thread.
__global__ __launch_bounds__(1024) void k_offsets(int64_t *__restrict__ off, int64_t nq)
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
            v[u] = base + u < nq ? off[base + u] : 0;
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
            if (base + u < nq) off[base + u] = pre;
            pre += v[u];
        }
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) off[nq] = carry;
}

// One block per dense query: write its set bits in ascending order (nothing
// when the capacity flag is raised).  The row is read in tiles of 4096
// words, 16 consecutive words a thread: one block-wide scan of the threads'
// bit counts per tile places every thread's output.
__global__ __launch_bounds__(256) void k_emit(const uint32_t *__restrict__ bitmap, int64_t words,
                                              const int64_t *__restrict__ off,
                                              int32_t *__restrict__ ids, const int32_t *__restrict__ dense,
                                              const int32_t *__restrict__ overflow)
{
    constexpr int kPer = 16;
    __shared__ uint32_t s[256];
    const int64_t q = blockIdx.x;
    if (!dense[q] || (overflow && overflow[0])) return;
    const uint32_t *row = bitmap + q * words;
    int64_t base = off[q];
    for (int64_t w0 = 0; w0 < words; w0 += 256 * kPer) {
        const int64_t w = w0 + (int64_t)threadIdx.x * kPer;
        uint32_t bits[kPer];
        uint32_t c = 0;
#pragma unroll
        for (int i = 0; i < kPer; i++) {
            bits[i] = w + i < words ? row[w + i] : 0u;
            c += __popc(bits[i]);
        }
        s[threadIdx.x] = c;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {
            const uint32_t t = threadIdx.x >= (unsigned)o ? s[threadIdx.x - o] : 0u;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        int64_t pos = base + s[threadIdx.x] - c;
#pragma unroll
        for (int i = 0; i < kPer; i++) {
            uint32_t v = bits[i];
            while (v) {
                const int bit = __builtin_ctz(v);
                ids[pos++] = (int32_t)((w + i) * 32 + bit);
                v &= v - 1;
            }
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
static_assert(kBigCap <= 16384 && kSparseCap <= kBigCap, "list caps");

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
    if (use_sparse(nq, words)) {
        hipLaunchKernelGGL(k_sparse, dim3((unsigned)((nq + 3) / 4)), dim3(256), 0, s, skeys, sids, n_entries,
                           qkeys, nq, b, w.dense, counts, w.bitmap, words);
        hipLaunchKernelGGL(k_sparse_sort, dim3((unsigned)((nq + 3) / 4)), dim3(256), 0, s, w.dense, nq, counts,
                           w.bitmap, words);
        hipLaunchKernelGGL(k_sparse_sort_big, dim3((unsigned)nq), dim3(1024), 0, s, w.dense, counts, w.bitmap,
                           words);
    } else
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
