// fem_jacobian.hip -- the input of the NOJAC variant (section 4): detJ and the 9 entries of J^{-1}
// for every element at every Gauss point, written on the device in one FP64 pass over the
// vertices (the paper computes them on the host and transfers them). Record of point q of
// element e: 10 doubles at out + 10 (b_off ? b_off[e] : e Nq) + 10 q, q = q1 + n q2 + n^2 q3.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fem_geometry.h"
#include "fem_jacobian.h"

namespace fem {

namespace {

__device__ inline void write_point(const JacArgs &a, int64_t e, int p, int q, int64_t rec)
{
    const int n = p + 1;
    const double *X = a.geom + e * 24;
    double tc[24];
#pragma unroll
    for (int t = 0; t < 24; ++t) tc[t] = trilinear_coeff(X, t / 8, t % 8);
    const double *x = a.xq[p];
    double Ji[3][3];
    const double det = jacobian_terms(tc, x[q % n], x[(q / n) % n], x[q / (n * n)], Ji);
    double *o = a.out + rec * 10;
    o[0] = det;
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int k = 0; k < 3; ++k) o[1 + 3 * m + k] = Ji[m][k];
}

// One thread per point, grid-stride. Uniform degree: point t belongs to element t / Nq. Mixed:
// to the last element e with b_off[e] <= t (a binary search over the scan; elements without
// points never match); records whose degree or index do not fit are left unwritten.
__global__ void __launch_bounds__(256) k_jacobian_terms(JacArgs a)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a.p > 0) {
        const int n = a.p + 1, nq = n * n * n;
        const int64_t total = a.nel * nq;
        for (int64_t t = t0; t < total; t += stride) write_point(a, t / nq, a.p, (int)(t % nq), t);
        return;
    }
    const int64_t total = a.b_off[a.nel];
    for (int64_t t = t0; t < total; t += stride) {
        int64_t lo = 0, hi = a.nel - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) / 2;
            if (a.b_off[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        const int p = a.degree[lo];
        if (p < 1 || p > 7) continue;
        const int64_t q = t - a.b_off[lo];
        if (q < 0 || q >= (int64_t)(p + 1) * (p + 1) * (p + 1)) continue;
        write_point(a, lo, p, (int)q, t);
    }
}

}  // namespace

hipError_t jacobian_terms_launch(const JacArgs &a, hipStream_t s, int64_t cus)
{
    const int64_t cap = cus * 16;  // enough resident waves to hide the scattered reads
    int64_t blocks = cap;
    if (a.p > 0) {
        const int64_t n = a.p + 1, total = a.nel * n * n * n;
        blocks = (total + 255) / 256 < cap ? (total + 255) / 256 : cap;
    }
    hipLaunchKernelGGL(k_jacobian_terms, dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace fem
