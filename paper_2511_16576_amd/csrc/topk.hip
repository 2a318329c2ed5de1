// Per-query top-k by (J descending, id ascending): Def. 1's K nearest
// neighbours under the Jaccard distance 1 - J.  One block per query; round r
// selects, by a block-wide reduction, the best candidate strictly after the
// (r-1)-th selection in that total order.
#include "internal.hpp"

#include <cfloat>

namespace polymh {

namespace {

__device__ __forceinline__ bool better(double ja, int32_t ia, double jb, int32_t ib)
{
    return ja > jb || (ja == jb && ia < ib);
}

__global__ __launch_bounds__(256) void k_topk(const int64_t *__restrict__ off,
                                              const int32_t *__restrict__ ids,
                                              const double *__restrict__ js, int32_t k,
                                              int32_t *__restrict__ top_ids,
                                              double *__restrict__ top_j)
{
    __shared__ double s_j[256];
    __shared__ int32_t s_i[256];
    const int64_t q = blockIdx.x;
    const int64_t a = off[q], b = off[q + 1];
    double pj = DBL_MAX;
    int32_t pi = -1;
    for (int r = 0; r < k; r++) {
        double bj = -DBL_MAX;
        int32_t bi = -1;
        for (int64_t c = a + threadIdx.x; c < b; c += blockDim.x) {
            const double j = js[c];
            const int32_t i = ids[c];
            const bool after = j < pj || (j == pj && i > pi);
            if (after && (bi < 0 || better(j, i, bj, bi))) {
                bj = j;
                bi = i;
            }
        }
        s_j[threadIdx.x] = bj;
        s_i[threadIdx.x] = bi;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (threadIdx.x < o) {
                const double oj = s_j[threadIdx.x + o];
                const int32_t oi = s_i[threadIdx.x + o];
                if (oi >= 0 && (s_i[threadIdx.x] < 0 || better(oj, oi, s_j[threadIdx.x], s_i[threadIdx.x]))) {
                    s_j[threadIdx.x] = oj;
                    s_i[threadIdx.x] = oi;
                }
            }
            __syncthreads();
        }
        pj = s_j[0];
        pi = s_i[0];
        if (threadIdx.x == 0) {
            top_ids[q * k + r] = pi;
            top_j[q * k + r] = pi >= 0 ? pj : 0.0;
        }
        __syncthreads();
        if (pi < 0) {
            for (int rr = r + 1 + threadIdx.x; rr < k; rr += blockDim.x) {
                top_ids[q * k + rr] = -1;
                top_j[q * k + rr] = 0.0;
            }
            break;
        }
    }
}

}  // namespace

polymh_status launch_topk(const int64_t *off, const int32_t *ids, const double *js, int64_t nq,
                          int32_t k, int32_t *top_ids, double *top_j, hipStream_t s)
{
    if (nq == 0) return POLYMH_OK;
    if (nq > 0x7fffffffLL) return set_error(POLYMH_EINVAL, "topk: too many queries");
    hipLaunchKernelGGL(k_topk, dim3((unsigned)nq), dim3(256), 0, s, off, ids, js, k, top_ids, top_j);
    return check_launch("topk");
}

}  // namespace polymh
