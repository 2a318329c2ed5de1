// Device helpers of the learned candidate scorer shared by its kernels (the
// training products, the input rows and the fused inference): BF16 MFMA
// operand types, the tanh form of GELU, and the 32 columns after the 256
// collision bits of a pair's input row.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace polymh {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int kScorerIn = 288, kScorerHid = 256, kScorerBits = 256, kPolyFeat = 12;

constexpr float kGeluC = 0.7978845608028654f;  // sqrt(2 / pi)
constexpr float kGeluA = 0.044715f;

__device__ __forceinline__ float gelu(float z)
{
    return 0.5f * z * (1.0f + tanhf(kGeluC * (z + kGeluA * z * z * z)));
}
__device__ __forceinline__ float gelu_grad(float z)
{
    const float t = tanhf(kGeluC * (z + kGeluA * z * z * z));
    return 0.5f * (1.0f + t) + 0.5f * z * (1.0f - t * t) * kGeluC * (1.0f + 3.0f * kGeluA * z * z);
}

// Column 256 + c (0 <= c < 32) of the input row of a pair whose polygons
// have the per-polygon features fq, fp (12 floats each: 6 shape values, the
// area, a pad, the MBR) and agree on `cnt` of the 256 hashes: the 6 + 6
// shape values, ln(A_q / A_p) / 4, min/max area ratio (an upper bound of J),
// MBR intersection-over-union, the collision fraction, then zeros.
__device__ __forceinline__ float pair_tail_feature(int c, const float *fq, const float *fp, int cnt)
{
    if (c < 6) return fq[c];
    if (c < 12) return fp[c - 6];
    if (c >= 16) return 0.f;
    const float aq = fmaxf(fq[6], 0.5f), ap = fmaxf(fp[6], 0.5f);
    if (c == 12) return logf(aq / ap) / 4.f;
    if (c == 13) return fminf(aq, ap) / fmaxf(aq, ap);
    if (c == 14) {
        const float ix = fmaxf(0.f, fminf(fq[10], fp[10]) - fmaxf(fq[8], fp[8]));
        const float iy = fmaxf(0.f, fminf(fq[11], fp[11]) - fmaxf(fq[9], fp[9]));
        const float in = ix * iy;
        const float u = (fq[10] - fq[8]) * (fq[11] - fq[9]) + (fp[10] - fp[8]) * (fp[11] - fp[9]) - in;
        return u > 0 ? in / u : 0.f;
    }
    return (float)cnt / (float)kScorerBits;
}

}  // namespace polymh
