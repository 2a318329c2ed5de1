// Learned candidate scorer: a 288 -> 256 -> 256 -> 1 MLP (GELU, GELU,
// sigmoid) with BF16 weights and activations on the MFMA units, FP32
// accumulation, MSE loss and Adam on FP32 master weights.
//
// Products run on v_mfma_f32_32x32x16_bf16: one wavefront owns a 32 x 32 tile
// of the output and walks K in steps of 16.  Operand fragments: lane l holds
// row (l % 32) of A and column (l % 32) of B, for the 8 consecutive k values
// 8*(l / 32) .. 8*(l / 32) + 7 of the step; result element r of lane l is
// row 8*(r / 4) + 4*(l / 32) + r % 4, column l % 32.  Operands are read with
// arbitrary strides so the forward (X W^T), the input gradient (dZ W) and the
// weight gradient (dZ^T H) share the kernel; when k is the contiguous index
// a lane reads its 8 values with one 16-byte load.
#include "internal.hpp"
#include "scorer_common.hpp"

#include <algorithm>
#include <cmath>

namespace polymh {

namespace {

constexpr int kIn = kScorerIn, kHid = kScorerHid;

__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }

struct Operand {
    const __bf16 *p;
    int64_t si;  // stride of the row (A) / column (B) index
    int64_t sk;  // stride of the reduction index
};

template <bool KC>
__device__ __forceinline__ bf16x8 frag(const Operand &o, int64_t row, int64_t k)
{
    const __bf16 *q = o.p + row * o.si + k * o.sk;
    if constexpr (KC) {
        return *reinterpret_cast<const bf16x8 *>(q);
    } else {
        bf16x8 v;
#pragma unroll
        for (int t = 0; t < 8; t++) v[t] = q[t * o.sk];
        return v;
    }
}

enum Epi { kStoreF32 = 0, kBiasGelu = 1, kGeluGrad = 2, kAccF32 = 3 };

struct GemmArgs {
    Operand A, B;
    int64_t M, N, K;   // M, N multiples of 32; K multiple of 16
    int epi;
    float *outf;       // kStoreF32/kAccF32: C; kBiasGelu: z; kGeluGrad: dz (fp32)
    __bf16 *outb;      // kBiasGelu: h = gelu(z); kGeluGrad: dz (bf16)
    const float *bias; // kBiasGelu
    const float *zin;  // kGeluGrad: the pre-activation z
    int64_t ldo;       // leading dimension of the outputs
};

template <bool AKC, bool BKC>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g)
{
    const int lane = threadIdx.x & 63;
    const int64_t tiles_n = g.N / 32;
    const int64_t tile = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (tile >= (g.M / 32) * tiles_n) return;
    const int64_t i0 = (tile / tiles_n) * 32, j0 = (tile % tiles_n) * 32;
    const int64_t row = i0 + (lane & 31), col = j0 + (lane & 31);
    const int64_t kl = 8 * (lane >> 5);
    f32x16 acc = {};
    for (int64_t k0 = 0; k0 < g.K; k0 += 16) {
        const bf16x8 a = frag<AKC>(g.A, row, k0 + kl);
        const bf16x8 b = frag<BKC>(g.B, col, k0 + kl);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 16; r++) {
        const int64_t i = i0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int64_t o = i * g.ldo + col;
        const float c = acc[r];
        if (g.epi == kStoreF32) {
            g.outf[o] = c;
        } else if (g.epi == kAccF32) {
            g.outf[o] += c;
        } else if (g.epi == kBiasGelu) {
            const float z = c + g.bias[col];
            g.outf[o] = z;
            g.outb[o] = to_bf16(gelu(z));
        } else {
            const float d = c * gelu_grad(g.zin[o]);
            g.outf[o] = d;
            g.outb[o] = to_bf16(d);
        }
    }
}

// Split-K form of the product for the weight gradients, whose M x N output
// is a few dozen tiles while K is the whole batch (one wavefront a tile
// would leave the chip nearly idle): split s (blockIdx.y) reduces over
// [s kc, min(K, (s + 1) kc)) and writes its partial tile to part[s][M][N];
// k_split_sum then adds the splits in order, so the result is deterministic.
template <bool AKC, bool BKC>
__global__ __launch_bounds__(256) void k_gemm_part(GemmArgs g, int64_t kc, float *__restrict__ part)
{
    const int lane = threadIdx.x & 63;
    const int64_t tiles_n = g.N / 32;
    const int64_t tile = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (tile >= (g.M / 32) * tiles_n) return;
    const int64_t i0 = (tile / tiles_n) * 32, j0 = (tile % tiles_n) * 32;
    const int64_t row = i0 + (lane & 31), col = j0 + (lane & 31);
    const int64_t kl = 8 * (lane >> 5);
    const int64_t k_lo = (int64_t)blockIdx.y * kc, k_hi = min(g.K, k_lo + kc);
    f32x16 acc = {};
    for (int64_t k0 = k_lo; k0 < k_hi; k0 += 16) {
        const bf16x8 a = frag<AKC>(g.A, row, k0 + kl);
        const bf16x8 b = frag<BKC>(g.B, col, k0 + kl);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    float *out = part + (int64_t)blockIdx.y * g.M * g.N;
#pragma unroll
    for (int r = 0; r < 16; r++) {
        const int64_t i = i0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        out[i * g.N + col] = acc[r];
    }
}

__global__ __launch_bounds__(256) void k_split_sum(const float *__restrict__ part, int nsplit, int64_t M,
                                                   int64_t N, float *__restrict__ out, int64_t ldo)
{
    const int64_t mn = M * N;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < mn;
         e += (int64_t)gridDim.x * blockDim.x) {
        float v = 0.f;
        for (int s = 0; s < nsplit; s++) v += part[s * mn + e];
        const int64_t i = e / N;
        out[i * ldo + (e - i * N)] = v;
    }
}

// Output layer and loss gradient: y = sigmoid(h2 . w3 + b3); with labels,
// dz3 = 2 (y - J) / B * y (1 - y) and dH2 = dz3 w3^T (bf16, before GELU').
__global__ __launch_bounds__(256) void k_head(const __bf16 *__restrict__ h2, const float *__restrict__ w3,
                                              const float *__restrict__ b3, int64_t B,
                                              float *__restrict__ y, const float *__restrict__ label,
                                              float *__restrict__ dz3, float *__restrict__ loss)
{
    const int lane = threadIdx.x & 63;
    const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (r >= B) return;
    float s = 0.f;
    for (int j = lane; j < kHid; j += 64) s += (float)h2[r * kHid + j] * w3[j];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    const float yy = 1.0f / (1.0f + expf(-(s + b3[0])));
    if (lane == 0) {
        y[r] = yy;
        if (label) {
            const float e = yy - label[r];
            dz3[r] = 2.0f * e / (float)B * yy * (1.0f - yy);
            atomicAdd(loss, e * e / (float)B);
        }
    }
}

// dH2[r, j] = dz3[r] * w3[j] as bf16 (operand of the next product is the
// GELU' scaling, fused into the elementwise pass below).
__global__ __launch_bounds__(256) void k_head_back(const float *__restrict__ dz3, const float *__restrict__ w3,
                                                   const float *__restrict__ z2, int64_t B,
                                                   float *__restrict__ dz2f, __bf16 *__restrict__ dz2b)
{
    const int64_t total = B * kHid;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / kHid;
        const int j = (int)(i - r * kHid);
        const float d = dz3[r] * w3[j] * gelu_grad(z2[i]);
        dz2f[i] = d;
        dz2b[i] = to_bf16(d);
    }
}

// Column sums over the batch: out[j] = sum_r M[r, j] (bias gradients) and,
// for the output layer, dw3[j] = sum_r dz3[r] h2[r, j].
__global__ __launch_bounds__(256) void k_colsum(const float *__restrict__ m, int64_t B, int ncol,
                                                float *__restrict__ out)
{
    const int j = blockIdx.x;
    float s = 0.f;
    for (int64_t r = threadIdx.x; r < B; r += blockDim.x) s += m[r * ncol + j];
    __shared__ float sh[256];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = sh[0];
}

__global__ __launch_bounds__(256) void k_head_grads(const float *__restrict__ dz3, const __bf16 *__restrict__ h2,
                                                    int64_t B, float *__restrict__ dw3, float *__restrict__ db3)
{
    const int j = blockIdx.x;  // 0..kHid (kHid = the bias)
    float s = 0.f;
    for (int64_t r = threadIdx.x; r < B; r += blockDim.x) s += dz3[r] * (j < kHid ? (float)h2[r * kHid + j] : 1.0f);
    __shared__ float sh[256];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (j < kHid) dw3[j] = sh[0];
        else db3[0] = sh[0];
    }
}

__global__ __launch_bounds__(256) void k_adam(float *__restrict__ p, const float *__restrict__ g,
                                              float *__restrict__ m, float *__restrict__ v, int64_t n,
                                              float lr, float b1, float b2, float eps, float c1, float c2)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

__global__ __launch_bounds__(256) void k_to_bf16(const float *__restrict__ x, __bf16 *__restrict__ y, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = to_bf16(x[i]);
}

__global__ void k_zero_f32(float *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.f;
}

int grid_of(int64_t items, int per)
{
    int64_t g = (items + per - 1) / per;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (int)g;
}

polymh_status gemm(const GemmArgs &g, hipStream_t s)
{
    const int64_t tiles = (g.M / 32) * (g.N / 32);
    if (tiles == 0) return POLYMH_OK;
    if (tiles > (int64_t)0x7fffffff / 4) return set_error(POLYMH_EINVAL, "mlp: product too large");
    const dim3 grid((unsigned)((tiles + 3) / 4)), block(256);
    const bool akc = g.A.sk == 1, bkc = g.B.sk == 1;
    if (akc && bkc) hipLaunchKernelGGL((k_gemm<true, true>), grid, block, 0, s, g);
    else if (akc) hipLaunchKernelGGL((k_gemm<true, false>), grid, block, 0, s, g);
    else if (bkc) hipLaunchKernelGGL((k_gemm<false, true>), grid, block, 0, s, g);
    else hipLaunchKernelGGL((k_gemm<false, false>), grid, block, 0, s, g);
    return check_launch("mlp gemm");
}

// At most kMaxSplit splits of at least kMinSplitK reduction steps each.
constexpr int kMaxSplit = 64, kMinSplitK = 256;

// The product as split-K with plain FP32 stores (the weight gradients);
// part holds kMaxSplit x M x N floats.
polymh_status gemm_split(const GemmArgs &g, float *part, hipStream_t s)
{
    const int64_t tiles = (g.M / 32) * (g.N / 32);
    if (tiles == 0) return POLYMH_OK;
    int64_t kc = (g.K + kMaxSplit - 1) / kMaxSplit;
    kc = std::max<int64_t>(kMinSplitK, (kc + 15) / 16 * 16);
    const int nsplit = (int)std::max<int64_t>(1, (g.K + kc - 1) / kc);
    const dim3 grid((unsigned)((tiles + 3) / 4), (unsigned)nsplit), block(256);
    const bool akc = g.A.sk == 1, bkc = g.B.sk == 1;
    if (akc && bkc) hipLaunchKernelGGL((k_gemm_part<true, true>), grid, block, 0, s, g, kc, part);
    else if (akc) hipLaunchKernelGGL((k_gemm_part<true, false>), grid, block, 0, s, g, kc, part);
    else if (bkc) hipLaunchKernelGGL((k_gemm_part<false, true>), grid, block, 0, s, g, kc, part);
    else hipLaunchKernelGGL((k_gemm_part<false, false>), grid, block, 0, s, g, kc, part);
    polymh_status st = check_launch("mlp gemm (split)");
    if (st) return st;
    hipLaunchKernelGGL(k_split_sum, dim3(grid_of(g.M * g.N, 256)), dim3(256), 0, s, part, nsplit, g.M, g.N,
                       g.outf, g.ldo);
    return check_launch("mlp gemm (split sum)");
}

}  // namespace

// Parameter block (FP32 master): W1[256][288], b1[256], W2[256][256], b2[256], w3[256], b3.
constexpr int64_t kOffW1 = 0, kOffB1 = kOffW1 + (int64_t)kHid * kIn, kOffW2 = kOffB1 + kHid,
                  kOffB2 = kOffW2 + (int64_t)kHid * kHid, kOffW3 = kOffB2 + kHid, kOffB3 = kOffW3 + kHid,
                  kNParams = kOffB3 + 1;
// BF16 copies: W1 then W2.
constexpr int64_t kNBf16 = (int64_t)kHid * kIn + (int64_t)kHid * kHid;

int64_t mlp_param_count() { return kNParams; }
int64_t mlp_bf16_count() { return kNBf16; }

size_t mlp_acts_bytes(int64_t B)
{
    // z1, z2 (f32), h1, h2 (bf16), y (f32)
    return (size_t)B * kHid * (4 + 4 + 2 + 2) + (size_t)B * 4 + 1024;
}

struct Acts {
    float *z1, *z2, *y;
    __bf16 *h1, *h2;
};

static Acts carve_acts(void *p, int64_t B)
{
    char *c = static_cast<char *>(p);
    Acts a;
    a.z1 = reinterpret_cast<float *>(c);
    c += align_up((size_t)B * kHid * 4, 256);
    a.z2 = reinterpret_cast<float *>(c);
    c += align_up((size_t)B * kHid * 4, 256);
    a.h1 = reinterpret_cast<__bf16 *>(c);
    c += align_up((size_t)B * kHid * 2, 256);
    a.h2 = reinterpret_cast<__bf16 *>(c);
    c += align_up((size_t)B * kHid * 2, 256);
    a.y = reinterpret_cast<float *>(c);
    return a;
}

size_t mlp_acts_bytes_aligned(int64_t B)
{
    return 4 * align_up((size_t)B * kHid * 4, 256) + align_up((size_t)B * 4, 256) + 256;
}

polymh_status launch_mlp_sync_bf16(const float *params, uint16_t *wbf16, hipStream_t s)
{
    __bf16 *w = reinterpret_cast<__bf16 *>(wbf16);
    hipLaunchKernelGGL(k_to_bf16, dim3(grid_of((int64_t)kHid * kIn, 256)), dim3(256), 0, s,
                       params + kOffW1, w, (int64_t)kHid * kIn);
    hipLaunchKernelGGL(k_to_bf16, dim3(grid_of((int64_t)kHid * kHid, 256)), dim3(256), 0, s,
                       params + kOffW2, w + (int64_t)kHid * kIn, (int64_t)kHid * kHid);
    return check_launch("mlp bf16 copy");
}

polymh_status launch_mlp_forward(const uint16_t *X, int64_t B, const float *params,
                                 const uint16_t *wbf16, float *y, void *acts, hipStream_t s)
{
    if (B == 0) return POLYMH_OK;
    Acts a = carve_acts(acts, B);
    const __bf16 *x = reinterpret_cast<const __bf16 *>(X);
    const __bf16 *w1 = reinterpret_cast<const __bf16 *>(wbf16);
    const __bf16 *w2 = w1 + (int64_t)kHid * kIn;
    GemmArgs g{};
    // z1 = X W1^T + b1, h1 = gelu(z1)
    g.A = Operand{x, kIn, 1};
    g.B = Operand{w1, kIn, 1};
    g.M = B; g.N = kHid; g.K = kIn;
    g.epi = kBiasGelu; g.outf = a.z1; g.outb = a.h1; g.bias = params + kOffB1; g.ldo = kHid;
    polymh_status st = gemm(g, s);
    if (st) return st;
    // z2 = h1 W2^T + b2, h2 = gelu(z2)
    g.A = Operand{a.h1, kHid, 1};
    g.B = Operand{w2, kHid, 1};
    g.K = kHid; g.outf = a.z2; g.outb = a.h2; g.bias = params + kOffB2;
    if ((st = gemm(g, s))) return st;
    hipLaunchKernelGGL(k_head, dim3(grid_of(B, 4)), dim3(256), 0, s, a.h2, params + kOffW3,
                       params + kOffB3, B, y ? y : a.y, (const float *)nullptr, (float *)nullptr,
                       (float *)nullptr);
    return check_launch("mlp head");
}

// Loss and parameter gradient of one batch (the forward must have run on the
// same X and acts).  grad [kNParams] is overwritten; loss (device float) is
// overwritten with the batch MSE.  scratch: dz3 [B], dz2/dz1 fp32 and bf16,
// the weight gradients' split-K partials.
size_t mlp_backward_scratch_bytes(int64_t B)
{
    return align_up((size_t)B * 4, 256) + 2 * align_up((size_t)B * kHid * 4, 256) +
           2 * align_up((size_t)B * kHid * 2, 256) + align_up((size_t)kMaxSplit * kHid * kIn * 4, 256) + 256;
}

polymh_status launch_mlp_backward(const uint16_t *X, int64_t B, const float *params,
                                  const uint16_t *wbf16, void *acts, const float *label,
                                  float *grad, float *loss, void *scratch, hipStream_t s)
{
    if (B == 0) return POLYMH_OK;
    Acts a = carve_acts(acts, B);
    char *c = static_cast<char *>(scratch);
    float *dz3 = reinterpret_cast<float *>(c); c += align_up((size_t)B * 4, 256);
    float *dz2f = reinterpret_cast<float *>(c); c += align_up((size_t)B * kHid * 4, 256);
    float *dz1f = reinterpret_cast<float *>(c); c += align_up((size_t)B * kHid * 4, 256);
    __bf16 *dz2b = reinterpret_cast<__bf16 *>(c); c += align_up((size_t)B * kHid * 2, 256);
    __bf16 *dz1b = reinterpret_cast<__bf16 *>(c); c += align_up((size_t)B * kHid * 2, 256);
    float *part = reinterpret_cast<float *>(c);
    const __bf16 *x = reinterpret_cast<const __bf16 *>(X);
    const __bf16 *w2 = reinterpret_cast<const __bf16 *>(wbf16) + (int64_t)kHid * kIn;

    hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(64), 0, s, loss, (int64_t)1);
    hipLaunchKernelGGL(k_head, dim3(grid_of(B, 4)), dim3(256), 0, s, a.h2, params + kOffW3,
                       params + kOffB3, B, a.y, label, dz3, loss);
    hipLaunchKernelGGL(k_head_grads, dim3(kHid + 1), dim3(256), 0, s, dz3, a.h2, B,
                       grad + kOffW3, grad + kOffB3);
    hipLaunchKernelGGL(k_head_back, dim3(grid_of(B * kHid, 256)), dim3(256), 0, s, dz3,
                       params + kOffW3, a.z2, B, dz2f, dz2b);
    polymh_status st = check_launch("mlp head backward");
    if (st) return st;
    GemmArgs g{};
    // dW2 = dz2^T h1 : (out i, in j), reduction over rows r
    g.A = Operand{dz2b, 1, kHid};
    g.B = Operand{a.h1, 1, kHid};
    g.M = kHid; g.N = kHid; g.K = B; g.epi = kStoreF32; g.outf = grad + kOffW2; g.ldo = kHid;
    if ((st = gemm_split(g, part, s))) return st;
    hipLaunchKernelGGL(k_colsum, dim3(kHid), dim3(256), 0, s, dz2f, B, kHid, grad + kOffB2);
    // dz1 = (dz2 W2) * gelu'(z1)
    g.A = Operand{dz2b, kHid, 1};
    g.B = Operand{w2, 1, kHid};
    g.M = B; g.N = kHid; g.K = kHid; g.epi = kGeluGrad; g.outf = dz1f; g.outb = dz1b;
    g.zin = a.z1; g.ldo = kHid;
    if ((st = gemm(g, s))) return st;
    // dW1 = dz1^T X : (out i, in j) over rows r
    g.A = Operand{dz1b, 1, kHid};
    g.B = Operand{x, 1, kIn};
    g.M = kHid; g.N = kIn; g.K = B; g.epi = kStoreF32; g.outf = grad + kOffW1; g.ldo = kIn;
    if ((st = gemm_split(g, part, s))) return st;
    hipLaunchKernelGGL(k_colsum, dim3(kHid), dim3(256), 0, s, dz1f, B, kHid, grad + kOffB1);
    return check_launch("mlp backward");
}

polymh_status launch_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t step,
                              float lr, float b1, float b2, float eps, uint16_t *wbf16, hipStream_t s)
{
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(grid_of(kNParams, 256)), dim3(256), 0, s, params, grad, m, v,
                       kNParams, lr, b1, b2, eps, c1, c2);
    polymh_status st = check_launch("mlp adam");
    if (st) return st;
    return launch_mlp_sync_bf16(params, wbf16, s);
}

polymh_status launch_gemm_bf16(const uint16_t *A, int64_t sai, int64_t sak, const uint16_t *B,
                               int64_t sbj, int64_t sbk, int64_t M, int64_t N, int64_t K, float *C,
                               hipStream_t s)
{
    GemmArgs g{};
    g.A = Operand{reinterpret_cast<const __bf16 *>(A), sai, sak};
    g.B = Operand{reinterpret_cast<const __bf16 *>(B), sbj, sbk};
    g.M = M; g.N = N; g.K = K; g.epi = kStoreF32; g.outf = C; g.ldo = N;
    return gemm(g, s);
}

}  // namespace polymh
