// fem_transpose.hip -- the lower blocks of the elasticity element matrix from the upper ones.
// The isotropic tensor has the major symmetry c_ijkl = c_klij (section 5.1), so block (k, i)
// of the 3 x 3 block matrix is the transpose of block (i, k); for i < k it is copied transposed
// instead of integrated. One workgroup per 32 x 32 tile of one block of one element, staged
// through LDS so that reads and writes are both row-contiguous.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fem_transpose.h"

namespace fem {

namespace {

constexpr int TT = 32;  // tile edge
constexpr int TR = 8;   // rows per thread pass (256 threads)
constexpr int TG = 4;   // tiles per work item: their loads are all in flight before the barrier

template <typename T>
__global__ void __launch_bounds__(TT * TR) k_transpose_blocks(T *A, int64_t nel, int ns)
{
    __shared__ T tile[TG][TT][TT + 1];
    const int tiles = (ns + TT - 1) / TT;
    const int groups = (tiles * tiles + TG - 1) / TG;
    const int64_t per_el = 3LL * groups;  // three block pairs (0,1) (0,2) (1,2)
    const int tx = threadIdx.x % TT, ty = threadIdx.x / TT;
    const int64_t nsq = (int64_t)ns * ns;
    for (int64_t w = blockIdx.x; w < nel * per_el; w += gridDim.x) {
        const int64_t e = w / per_el;
        const int rem = (int)(w % per_el);
        const int pair = rem / groups, t0 = (rem % groups) * TG;
        const int i = pair < 2 ? 0 : 1, k = pair == 0 ? 1 : 2;
        const T *src = A + (e * 9 + 3 * i + k) * nsq;
        T *dst = A + (e * 9 + 3 * k + i) * nsq;
        __syncthreads();  // the previous tiles have left LDS
#pragma unroll
        for (int g = 0; g < TG; ++g) {
            const int t = t0 + g;
            if (t >= tiles * tiles) break;
            const int r0 = (t / tiles) * TT, c0 = (t % tiles) * TT;
#pragma unroll
            for (int y = ty; y < TT; y += TR) {
                const int r = r0 + y, c = c0 + tx;
                if (r < ns && c < ns) tile[g][y][tx] = src[(int64_t)r * ns + c];
            }
        }
        __syncthreads();
        // dst[c][r] = src[r][c]: row c0 + y of the destination holds column c0 + y of a tile
#pragma unroll
        for (int g = 0; g < TG; ++g) {
            const int t = t0 + g;
            if (t >= tiles * tiles) break;
            const int r0 = (t / tiles) * TT, c0 = (t % tiles) * TT;
#pragma unroll
            for (int y = ty; y < TT; y += TR) {
                const int r = c0 + y, c = r0 + tx;
                if (r < ns && c < ns) dst[(int64_t)r * ns + c] = tile[g][tx][y];
            }
        }
    }
}

}  // namespace

hipError_t transpose_elastic_blocks(void *A, bool fp64, int64_t nel, int ns, hipStream_t s, int64_t cus)
{
    const int tiles = (ns + TT - 1) / TT;
    const int64_t work = nel * 3 * ((tiles * tiles + TG - 1) / TG);
    const int64_t cap = cus * 8;
    const int64_t grid = work < cap ? work : cap;
    if (grid <= 0) return hipSuccess;
    if (fp64)
        hipLaunchKernelGGL(k_transpose_blocks<double>, dim3((unsigned)grid), dim3(TT * TR), 0, s,
                           static_cast<double *>(A), nel, ns);
    else
        hipLaunchKernelGGL(k_transpose_blocks<float>, dim3((unsigned)grid), dim3(TT * TR), 0, s,
                           static_cast<float *>(A), nel, ns);
    return hipGetLastError();
}

}  // namespace fem
