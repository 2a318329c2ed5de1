// Internal declarations shared by the libpolymh translation units (device
// helpers, kernel launchers, error reporting).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/polymh.h"

namespace polymh {

// SplitMix64 increment (the golden-ratio constant of Steele, Lea, Flood).
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

// SplitMix64 output function: the per-hash key and every draw of Alg. 1's
// fixed-seed point streams go through it.
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z;
}

// ---- wavefront reductions and scans over DPP ------------------------------
// Data-parallel-primitive moves read a neighbour lane's register inside the
// VALU, without the LDS crossbar that a shuffle goes through.  GFX9 controls:
// quad permutes, row (16-lane) rotates and shifts, and the two broadcasts of
// lane 15 of each row into the next row and of lane 31 into rows 2 and 3.
// Every lane of the wavefront must be active.
namespace dpp {
constexpr int kQuad1032 = 0xB1;
constexpr int kQuad2301 = 0x4E;
constexpr int kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr3 = 0x113, kRowShr4 = 0x114,
              kRowShr8 = 0x118;
constexpr int kRowRor4 = 0x124, kRowRor8 = 0x128;
constexpr int kRowBcast15 = 0x142, kRowBcast31 = 0x143;

template <int CTRL, int ROWS = 0xf, int BANKS = 0xf>
__device__ __forceinline__ int mov(int old, int src)
{
    return __builtin_amdgcn_update_dpp(old, src, CTRL, ROWS, BANKS, false);
}
template <int CTRL, int ROWS = 0xf, int BANKS = 0xf>
__device__ __forceinline__ uint64_t mov64(uint64_t old, uint64_t src)
{
    const uint32_t lo = (uint32_t)mov<CTRL, ROWS, BANKS>((int)(uint32_t)old, (int)(uint32_t)src);
    const uint32_t hi = (uint32_t)mov<CTRL, ROWS, BANKS>((int)(uint32_t)(old >> 32), (int)(uint32_t)(src >> 32));
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t readlane64(uint64_t v, int lane)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}
}  // namespace dpp

// Reduction of a 32-bit value over the wavefront; the result is uniform.
// Quads, then rows (rotate by 4 and 8: every lane holds its row's total),
// then rows 1/3 take rows 0/2 and rows 2-3 take lane 31: lane 63 ends with
// the total.
template <class Op>
__device__ __forceinline__ int wave_reduce32(int x, int id, Op op)
{
    x = op(x, dpp::mov<dpp::kQuad1032>(id, x));
    x = op(x, dpp::mov<dpp::kQuad2301>(id, x));
    x = op(x, dpp::mov<dpp::kRowRor4>(id, x));
    x = op(x, dpp::mov<dpp::kRowRor8>(id, x));
    x = op(x, dpp::mov<dpp::kRowBcast15, 0xa>(id, x));
    x = op(x, dpp::mov<dpp::kRowBcast31, 0xc>(id, x));
    return __builtin_amdgcn_readlane(x, 63);
}
__device__ __forceinline__ int wave_min32(int x)
{
    return wave_reduce32(x, INT32_MAX, [](int a, int b) { return a < b ? a : b; });
}
__device__ __forceinline__ int wave_max32(int x)
{
    return wave_reduce32(x, INT32_MIN, [](int a, int b) { return a > b ? a : b; });
}
__device__ __forceinline__ int64_t wave_sum_i64(int64_t v)
{
    uint64_t x = (uint64_t)v;
    x += dpp::mov64<dpp::kQuad1032>(0, x);
    x += dpp::mov64<dpp::kQuad2301>(0, x);
    x += dpp::mov64<dpp::kRowRor4>(0, x);
    x += dpp::mov64<dpp::kRowRor8>(0, x);
    x += dpp::mov64<dpp::kRowBcast15, 0xa>(0, x);
    x += dpp::mov64<dpp::kRowBcast31, 0xc>(0, x);
    return (int64_t)dpp::readlane64(x, 63);
}
__device__ __forceinline__ double wave_sum_f64(double v)
{
    auto step = [](double x, uint64_t moved) { return x + __longlong_as_double((long long)moved); };
    const uint64_t z = (uint64_t)__double_as_longlong(0.0);
    v = step(v, dpp::mov64<dpp::kQuad1032>(z, (uint64_t)__double_as_longlong(v)));
    v = step(v, dpp::mov64<dpp::kQuad2301>(z, (uint64_t)__double_as_longlong(v)));
    v = step(v, dpp::mov64<dpp::kRowRor4>(z, (uint64_t)__double_as_longlong(v)));
    v = step(v, dpp::mov64<dpp::kRowRor8>(z, (uint64_t)__double_as_longlong(v)));
    v = step(v, dpp::mov64<dpp::kRowBcast15, 0xa>(z, (uint64_t)__double_as_longlong(v)));
    v = step(v, dpp::mov64<dpp::kRowBcast31, 0xc>(z, (uint64_t)__double_as_longlong(v)));
    return __longlong_as_double((long long)dpp::readlane64((uint64_t)__double_as_longlong(v), 63));
}
// Inclusive prefix sum of a 32-bit value over the wavefront (lane 63 holds
// the total): within each row by shifts of 1, 2, 3, then 4 (lanes 4-15) and
// 8 (lanes 8-15), then across rows by the two broadcasts.
__device__ __forceinline__ int wave_incl_scan32(int x)
{
    int s = x;
    s += dpp::mov<dpp::kRowShr1>(0, x);
    s += dpp::mov<dpp::kRowShr2>(0, x);
    s += dpp::mov<dpp::kRowShr3>(0, x);
    s += dpp::mov<dpp::kRowShr4, 0xf, 0xe>(0, s);
    s += dpp::mov<dpp::kRowShr8, 0xf, 0xc>(0, s);
    s += dpp::mov<dpp::kRowBcast15, 0xa>(0, s);
    s += dpp::mov<dpp::kRowBcast31, 0xc>(0, s);
    return s;
}

// The same inclusive prefix sum for 64-bit integers.
__device__ __forceinline__ int64_t wave_incl_scan64(int64_t x)
{
    uint64_t s = (uint64_t)x;
    const uint64_t u = (uint64_t)x;
    s += dpp::mov64<dpp::kRowShr1>(0, u);
    s += dpp::mov64<dpp::kRowShr2>(0, u);
    s += dpp::mov64<dpp::kRowShr3>(0, u);
    s += dpp::mov64<dpp::kRowShr4, 0xf, 0xe>(0, s);
    s += dpp::mov64<dpp::kRowShr8, 0xf, 0xc>(0, s);
    s += dpp::mov64<dpp::kRowBcast15, 0xa>(0, s);
    s += dpp::mov64<dpp::kRowBcast31, 0xc>(0, s);
    return (int64_t)s;
}

// Per-polygon flag bits written by the staging kernel.
constexpr uint32_t kFlagFew = 1u;        // fewer than 3 vertices
constexpr uint32_t kFlagCollinear = 2u;  // all vertices on one line
constexpr uint32_t kFlagWide = 4u;       // MBR side >= 2^26: 128-bit orientation

polymh_status set_error(polymh_status st, const char *fmt, ...);
polymh_status check_launch(const char *what);
int cu_count();

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Bump allocator over a caller workspace.
struct Carve {
    char *base;
    size_t cap;
    size_t used = 0;
    bool ok = true;
    template <class T>
    T *take(size_t count)
    {
        size_t off = align_up(used, 256);
        size_t need = off + count * sizeof(T);
        if (need > cap || base == nullptr) {
            ok = false;
            used = need;
            return nullptr;
        }
        used = need;
        return reinterpret_cast<T *>(base + off);
    }
};

// ---- launchers (each defined next to its kernels) -------------------------

// prepare.hip
polymh_status launch_prepare(const int32_t *xy, const int64_t *off, int64_t n, int32_t *mbr,
                             int64_t *area2, uint32_t *flags, hipStream_t s);
polymh_status launch_box_of(const int32_t *xy, int64_t n_vertices, int32_t *acc4, hipStream_t s);
polymh_status launch_sign_order(const int64_t *off, const int32_t *mbr, const int64_t *area2,
                                const uint32_t *flags, int64_t n, polymh_box box, int32_t k,
                                uint32_t cap, int32_t *bucket_counts, int32_t *order,
                                hipStream_t s);
// centre.hip
polymh_status launch_centre(const int32_t *xy, const int64_t *off, int64_t n, int32_t *out,
                            int32_t *shift, int32_t *range_flag, hipStream_t s);

// sign.hip
struct SignLaunch {
    const int32_t *xy;
    const int64_t *off;
    const int32_t *mbr;
    const uint32_t *flags;
    const int32_t *order;     // nullable: identity
    unsigned long long *queue;  // nullable: plain grid
    uint32_t *sig;
    const int32_t *n_dev;     // nullable: the first *n_dev entries of `order` (n bounds it)
    int64_t n;
    polymh_box box;
    uint64_t seed;
    int32_t k;
    uint32_t cap;
    polymh_sign_config cfg;
};
polymh_status launch_sign(const SignLaunch &L, hipStream_t s);

// rings.hip
polymh_status launch_join_rings(const int32_t *xy, int64_t nv, const int64_t *ring_off, int64_t nr,
                                const int64_t *poly_rings, int64_t n, int32_t *out_xy, int64_t out_cap,
                                int64_t *out_off, int32_t *bad, hipStream_t s);

// binned.hip
size_t binned_workspace_bytes(int32_t k, uint32_t horizon, int32_t bits, int64_t n);
polymh_status launch_sign_binned(const SignLaunch &L, const int64_t *area2, uint32_t horizon, int32_t bits,
                                 double walk_ratio, void *ws, size_t ws_bytes, hipStream_t s, bool rebin = true);

// band.hip
polymh_status launch_band(const uint32_t *sig, int64_t n, int32_t k, int32_t b, int32_t r,
                          uint64_t band_seed, uint64_t *keys, hipStream_t s);

// index.hip
size_t index_workspace_bytes(int64_t m);
polymh_status launch_index_build(const uint64_t *keys, int64_t n, int32_t b, void *ws,
                                 size_t ws_bytes, uint64_t *sorted_keys, int32_t *sorted_ids,
                                 hipStream_t s);

// query.hip
size_t query_workspace_bytes(int64_t n_data, int64_t nq);
polymh_status launch_query(const uint64_t *skeys, const int32_t *sids, int64_t n_entries,
                           int64_t n_data, const uint64_t *qkeys, int64_t nq, int32_t b, void *ws,
                           size_t ws_bytes, int64_t *cand_off, int32_t *cand_ids, hipStream_t s);

// refine.hip
size_t refine_workspace_bytes();
polymh_status launch_refine(const polymh_polys *data, const polymh_polys *queries,
                            const int64_t *cand_off, const int32_t *cand_ids, int64_t nq,
                            int64_t n_cand, double *cand_j, hipStream_t s,
                            unsigned long long *stats = nullptr, void *ws = nullptr, size_t ws_bytes = 0);

// topk.hip
polymh_status launch_topk(const int64_t *off, const int32_t *ids, const double *js, int64_t nq,
                          int32_t k, int32_t *top_ids, double *top_j, hipStream_t s);

// mlp.hip
int64_t mlp_param_count();
int64_t mlp_bf16_count();
size_t mlp_acts_bytes_aligned(int64_t B);
size_t mlp_backward_scratch_bytes(int64_t B);
polymh_status launch_mlp_sync_bf16(const float *params, uint16_t *wbf16, hipStream_t s);
polymh_status launch_mlp_forward(const uint16_t *X, int64_t B, const float *params,
                                 const uint16_t *wbf16, float *y, void *acts, hipStream_t s);
polymh_status launch_mlp_backward(const uint16_t *X, int64_t B, const float *params,
                                  const uint16_t *wbf16, void *acts, const float *label,
                                  float *grad, float *loss, void *scratch, hipStream_t s);
polymh_status launch_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t step,
                              float lr, float b1, float b2, float eps, uint16_t *wbf16, hipStream_t s);
polymh_status launch_gemm_bf16(const uint16_t *A, int64_t sai, int64_t sak, const uint16_t *B,
                               int64_t sbj, int64_t sbk, int64_t M, int64_t N, int64_t K, float *C,
                               hipStream_t s);

// features.hip
polymh_status launch_poly_features(const polymh_polys *p, polymh_box box, float *feats, hipStream_t s);
polymh_status launch_pair_features(const uint32_t *lsig, const float *lfeat, const uint32_t *rsig,
                                   const float *rfeat, const int32_t *li, const int32_t *ri,
                                   int64_t R, int64_t R_pad, uint16_t *X, hipStream_t s);
polymh_status launch_csr_rows(const int64_t *off, int64_t nq, int32_t *rows, hipStream_t s);

// rank.hip
int32_t rank_sort_cap();
polymh_status launch_head_select(const int64_t *off, const int32_t *cand_ids, int64_t nq,
                                 const int32_t *order, int32_t M, int64_t *hoff, int32_t *hq,
                                 int64_t *hc, int32_t *hid, hipStream_t s);
polymh_status launch_scatter_scores(const int64_t *idx, const float *val, int64_t n, float *score,
                                    hipStream_t s);
polymh_status launch_rank_sort(const int64_t *off, int64_t nq, const float *score, int32_t *order,
                               uint8_t *sorted_ok, hipStream_t s);
polymh_status launch_rank_init(int64_t nq, int32_t topk, int64_t *cursor, uint8_t *active,
                               int32_t *top_ids, double *top_j, hipStream_t s);
// roff[0..nq]: exclusive prefix of the round's per-query pair counts
polymh_status launch_round_offsets(const int64_t *off, int64_t nq, const int64_t *cursor,
                                   const uint8_t *active, int32_t F, int64_t *roff, hipStream_t s);
polymh_status launch_round_fill(const int64_t *off, const int32_t *cand_ids, const int32_t *order,
                                const int64_t *cursor, const int64_t *roff, int64_t nq,
                                int32_t *rids, int32_t *rpos, hipStream_t s);
polymh_status launch_round_merge(const int64_t *off, const float *score, const int32_t *order,
                                 const uint8_t *sorted_ok, const int64_t *roff, const int32_t *rids,
                                 const double *rj, int64_t nq, int32_t topk, float margin,
                                 int64_t *cursor, uint8_t *active, int32_t *top_ids, double *top_j,
                                 int32_t *n_active, unsigned long long *counters, int finishing, hipStream_t s);
polymh_status launch_reorder_head(const int64_t *off, int64_t nq, const float *score, const int32_t *order_in,
                                 int32_t M, const uint8_t *sorted_ok, int32_t *order_out, hipStream_t s);
// score.hip
polymh_status launch_score_pairs(const uint32_t *lsig, const float *lfeat, const uint32_t *rsig, const float *rfeat,
                                 const int32_t *li, const int32_t *ri, const int64_t *out_idx, int64_t R,
                                 const float *params, const uint16_t *wbf16, float *out, hipStream_t s);
polymh_status launch_head_fixed(const int64_t *off, const int32_t *cand_ids, int64_t nq, const int32_t *order,
                                int32_t M, int32_t *hq, int64_t *hc, int32_t *hid, hipStream_t s);
polymh_status launch_rank_jhat_sort(const uint32_t *qsig, const uint32_t *dsig, int32_t k, const int64_t *off,
                                    const int32_t *cand_ids, int64_t nq, float *score, int32_t *order,
                                    uint8_t *sorted_ok, hipStream_t s);
polymh_status launch_sig_pack(const uint32_t *sig, int64_t n, int32_t k, uint16_t *packed, hipStream_t s);
polymh_status launch_rank_jhat_packed(const uint32_t *qsig, const uint16_t *packed, const uint32_t *dsig, int32_t k,
                                      const int64_t *off, const int32_t *cand_ids, int64_t nq, float *score,
                                      int32_t *order, uint8_t *sorted_ok, hipStream_t s);
polymh_status launch_jhat(const uint32_t *lsig, const uint32_t *rsig, const int32_t *li,
                          const int32_t *ri, int64_t R, int32_t k, float *out, hipStream_t s);
polymh_status launch_offsets(int64_t *off, int64_t nq, hipStream_t s);
polymh_status launch_query_capped(const uint64_t *skeys, const int32_t *sids, int64_t n_entries,
                                  int64_t n_data, const uint64_t *qkeys, int64_t nq, int32_t b,
                                  void *ws, size_t ws_bytes, int64_t *cand_off, int32_t *cand_ids,
                                  int64_t cand_cap, int32_t *overflow, hipStream_t s);

// util
polymh_status launch_fill_u64(unsigned long long *p, int64_t count, unsigned long long v,
                              hipStream_t s);

}  // namespace polymh
