// Learned scorer inference in one persistent launch: for a list of pairs,
// each pair's input row (256 collision bits and 32 feature columns, as
// k_pair_feats builds it) is assembled on chip, both hidden layers run on
// v_mfma_f32_32x32x16_bf16 with FP32 accumulation, the output layer and the
// sigmoid follow, and the prediction is written where the caller asks (for
// the ranked search: into the candidate's score).  Nothing between the
// signatures and the prediction goes through memory.
//
// Layout: a workgroup of 8 wavefronts owns the network; wavefront w owns
// hidden units 32w .. 32w + 31 of both layers and keeps its slices of W1
// (18 k-steps) and W2 (16 k-steps) in registers for the whole launch.  Pairs
// are taken 32 at a time (one MFMA row tile): the 32 input rows are built in
// LDS by the 8 wavefronts (four rows each: a 16-byte load of each signature
// per lane), layer 1 reads its A operand from that tile, writes GELU(z1) as
// BF16 into a second LDS tile, layer 2 reads it; each wavefront reduces its
// 32 columns of GELU(z2) * w3 per row, and the 8 partial sums of a row are
// added in wavefront order.  The tiles are software-pipelined: while a tile
// runs on the matrix cores, the next tile's signature slices and features
// are in flight (and the indices of the one after), and they are written
// into the other of two input buffers once the tile is done.
//
// MFMA operand layout (one wavefront, 32 x 32 output tile, k-step 16): lane
// l supplies row l % 32 of A and column l % 32 of B at k = 8 (l / 32) .. +7;
// result element r of lane l is row 8 (r / 4) + 4 (l / 32) + r % 4, column
// l % 32.
#include "internal.hpp"
#include "scorer_common.hpp"

#include <algorithm>

namespace polymh {

namespace {

constexpr int kTileRows = 32;
constexpr int kWaves = kScorerHid / 32;          // 8: one 32-unit slice each
constexpr int kXStride = kScorerIn + 8;          // LDS row strides in BF16 (16-byte multiples)
constexpr int kHStride = kScorerHid + 8;
constexpr int kK1 = kScorerIn / 16, kK2 = kScorerHid / 16;

// Offsets in the FP32 parameter block: W1 [256][288], b1, W2 [256][256], b2, w3, b3.
constexpr int64_t kPB1 = (int64_t)kScorerHid * kScorerIn;
constexpr int64_t kPW2 = kPB1 + kScorerHid;
constexpr int64_t kPB2 = kPW2 + (int64_t)kScorerHid * kScorerHid;
constexpr int64_t kPW3 = kPB2 + kScorerHid;
constexpr int64_t kPB3 = kPW3 + kScorerHid;

// Pair rows of one tile still in registers: the signature slices of the
// wavefront's four rows, the rows' 12 + 12 polygon features (lane f < 12
// holds the left polygon's feature f, lane 12 + f the right one's).
struct TileRegs {
    int32_t qi[kTileRows / kWaves], pi[kTileRows / kWaves];
    uint4 sa[kTileRows / kWaves], sb[kTileRows / kWaves];
    float fv[kTileRows / kWaves];
};

__device__ __forceinline__ void load_indices(const int32_t *li, const int32_t *ri, int64_t R, int64_t r0, int wave,
                                             int32_t *qi, int32_t *pi)
{
#pragma unroll
    for (int u = 0; u < kTileRows / kWaves; u++) {
        const int64_t r = r0 + wave + kWaves * u;
        qi[u] = r0 >= 0 && r < R ? li[r] : -1;
        pi[u] = r0 >= 0 && r < R ? ri[r] : -1;
    }
}

__device__ __forceinline__ void load_rows(const uint32_t *lsig, const float *lfeat, const uint32_t *rsig,
                                          const float *rfeat, int lane, TileRegs &T)
{
#pragma unroll
    for (int u = 0; u < kTileRows / kWaves; u++) {
        const bool ok = T.qi[u] >= 0 && T.pi[u] >= 0;
        T.sa[u] = ok ? *reinterpret_cast<const uint4 *>(lsig + (int64_t)T.qi[u] * kScorerBits + 4 * lane)
                     : make_uint4(0, 0, 0, 0);
        T.sb[u] = ok ? *reinterpret_cast<const uint4 *>(rsig + (int64_t)T.pi[u] * kScorerBits + 4 * lane)
                     : make_uint4(1, 1, 1, 1);
        const float *f = lane < kPolyFeat ? lfeat + (int64_t)T.qi[u] * kPolyFeat + lane
                                          : rfeat + (int64_t)T.pi[u] * kPolyFeat + (lane - kPolyFeat);
        T.fv[u] = ok && lane < 2 * kPolyFeat ? *f : 0.f;
    }
}

// The wavefront's four rows of the tile into the LDS input buffer X: the
// collision bits and the 32 feature columns (all zero for an empty row).
__device__ __forceinline__ void build_rows(const TileRegs &T, __bf16 *X, int wave, int lane)
{
#pragma unroll
    for (int u = 0; u < kTileRows / kWaves; u++) {
        __bf16 *xr = X + (wave + kWaves * u) * kXStride;
        const bool ok = T.qi[u] >= 0 && T.pi[u] >= 0;   // wavefront-uniform
        const bool e0 = T.sa[u].x == T.sb[u].x, e1 = T.sa[u].y == T.sb[u].y, e2 = T.sa[u].z == T.sb[u].z,
                   e3 = T.sa[u].w == T.sb[u].w;         // all false on an empty row
        xr[4 * lane + 0] = (__bf16)(e0 ? 1.f : 0.f);
        xr[4 * lane + 1] = (__bf16)(e1 ? 1.f : 0.f);
        xr[4 * lane + 2] = (__bf16)(e2 ? 1.f : 0.f);
        xr[4 * lane + 3] = (__bf16)(e3 ? 1.f : 0.f);
        const int cnt = __popcll(__ballot(e0)) + __popcll(__ballot(e1)) + __popcll(__ballot(e2)) +
                        __popcll(__ballot(e3));
        float fq[kPolyFeat], fp[kPolyFeat];
#pragma unroll
        for (int f = 0; f < kPolyFeat; f++) {
            fq[f] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, T.fv[u]), f));
            fp[f] = __builtin_bit_cast(float,
                                       __builtin_amdgcn_readlane(__builtin_bit_cast(int, T.fv[u]), kPolyFeat + f));
        }
        if (lane < 32) xr[kScorerBits + lane] = ok ? (__bf16)pair_tail_feature(lane, fq, fp, cnt) : (__bf16)0.f;
    }
}

__global__ __launch_bounds__(512) void k_score_pairs(const uint32_t *__restrict__ lsig,
                                                     const float *__restrict__ lfeat,
                                                     const uint32_t *__restrict__ rsig,
                                                     const float *__restrict__ rfeat,
                                                     const int32_t *__restrict__ li,
                                                     const int32_t *__restrict__ ri,
                                                     const int64_t *__restrict__ out_idx, int64_t R,
                                                     const float *__restrict__ params,
                                                     const __bf16 *__restrict__ wbf16,
                                                     float *__restrict__ out)
{
    __shared__ __attribute__((aligned(16))) __bf16 X[2][kTileRows * kXStride];
    __shared__ __attribute__((aligned(16))) __bf16 H[kTileRows * kHStride];
    __shared__ float part[kWaves][kTileRows];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int col = 32 * wave + (lane & 31);    // this lane's hidden unit (B column, output column)
    const int kl = 8 * (lane >> 5);
    const int64_t tiles = (R + kTileRows - 1) / kTileRows;
    const int64_t G = gridDim.x;
    int64_t t = blockIdx.x;
    if (t >= tiles) return;                      // workgroup-uniform, before any barrier
    // the first tile's rows, and the next tile's indices, are requested
    // before the weights so their latencies overlap
    TileRegs T;
    int32_t nqi[kTileRows / kWaves], npi[kTileRows / kWaves];
    load_indices(li, ri, R, t * kTileRows, wave, T.qi, T.pi);
    load_rows(lsig, lfeat, rsig, rfeat, lane, T);
    load_indices(li, ri, R, t + G < tiles ? (t + G) * kTileRows : -1, wave, nqi, npi);
    const __bf16 *W1 = wbf16;
    const __bf16 *W2 = wbf16 + (int64_t)kScorerHid * kScorerIn;
    bf16x8 w1[kK1], w2[kK2];
#pragma unroll
    for (int ks = 0; ks < kK1; ks++)
        w1[ks] = *reinterpret_cast<const bf16x8 *>(W1 + (int64_t)col * kScorerIn + 16 * ks + kl);
#pragma unroll
    for (int ks = 0; ks < kK2; ks++)
        w2[ks] = *reinterpret_cast<const bf16x8 *>(W2 + (int64_t)col * kScorerHid + 16 * ks + kl);
    const float b1c = params[kPB1 + col], b2c = params[kPB2 + col], w3c = params[kPW3 + col];
    const float b3 = params[kPB3];
    build_rows(T, X[0], wave, lane);
    int buf = 0;
    for (; t < tiles; t += G, buf ^= 1) {
        const int64_t r0 = t * kTileRows;
        // -- the next tile's rows are requested now and land while this
        // tile runs on the matrix cores; the tile after it, its indices
        const bool more = t + G < tiles;
#pragma unroll
        for (int u = 0; u < kTileRows / kWaves; u++) {
            T.qi[u] = nqi[u];
            T.pi[u] = npi[u];
        }
        if (more) load_rows(lsig, lfeat, rsig, rfeat, lane, T);
        load_indices(li, ri, R, t + 2 * G < tiles ? (t + 2 * G) * kTileRows : -1, wave, nqi, npi);
        __syncthreads();                          // X[buf] complete
        // -- layer 1: z1 = X W1^T + b1, H = BF16(GELU(z1))
        f32x16 acc = {};
        const __bf16 *xa = X[buf] + (lane & 31) * kXStride + kl;
#pragma unroll
        for (int ks = 0; ks < kK1; ks++)
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(*reinterpret_cast<const bf16x8 *>(xa + 16 * ks), w1[ks],
                                                          acc, 0, 0, 0);
#pragma unroll
        for (int e = 0; e < 16; e++) {
            const int row = 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
            H[row * kHStride + col] = (__bf16)gelu(acc[e] + b1c);
        }
        __syncthreads();
        // -- layer 2: z2 = H W2^T + b2; partial output sums of this slice
        acc = f32x16{};
        const __bf16 *ha = H + (lane & 31) * kHStride + kl;
#pragma unroll
        for (int ks = 0; ks < kK2; ks++)
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(*reinterpret_cast<const bf16x8 *>(ha + 16 * ks), w2[ks],
                                                          acc, 0, 0, 0);
#pragma unroll
        for (int e = 0; e < 16; e++) {
            // h2 is BF16 between the layers, as in the training forward pass
            float v = (float)(__bf16)gelu(acc[e] + b2c) * w3c;
#pragma unroll
            for (int o = 16; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);   // the 32 columns of a half
            if ((lane & 31) == 0) part[wave][8 * (e >> 2) + 4 * (lane >> 5) + (e & 3)] = v;
        }
        __syncthreads();
        if (threadIdx.x < kTileRows) {
            const int64_t r = r0 + threadIdx.x;
            if (r < R && li[r] >= 0 && ri[r] >= 0) {
                float s = 0.f;
#pragma unroll
                for (int w = 0; w < kWaves; w++) s += part[w][threadIdx.x];
                const float y = 1.0f / (1.0f + expf(-(s + b3)));
                const int64_t o = out_idx ? out_idx[r] : r;
                if (o >= 0) out[o] = y;
            }
        }
        // -- the next tile's rows into the other input buffer (its last
        // readers, layer 1 of the previous tile, are past two barriers)
        if (more) build_rows(T, X[buf ^ 1], wave, lane);
    }
}

}  // namespace

polymh_status launch_score_pairs(const uint32_t *lsig, const float *lfeat, const uint32_t *rsig, const float *rfeat,
                                 const int32_t *li, const int32_t *ri, const int64_t *out_idx, int64_t R,
                                 const float *params, const uint16_t *wbf16, float *out, hipStream_t s)
{
    if (R == 0) return POLYMH_OK;
    const int64_t tiles = (R + kTileRows - 1) / kTileRows;
    const int64_t grid = std::min<int64_t>(tiles, (int64_t)cu_count());
    hipLaunchKernelGGL(k_score_pairs, dim3((unsigned)grid), dim3(64 * kWaves), 0, s, lsig, lfeat, rsig, rfeat, li, ri,
                       out_idx, R, params, reinterpret_cast<const __bf16 *>(wbf16), out);
    return check_launch("score_pairs");
}

}  // namespace polymh
