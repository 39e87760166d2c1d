// fem_transpose.hip -- the lower blocks of the elasticity element matrix from the upper ones.
// The isotropic tensor has the major symmetry c_ijkl = c_klij (section 5.1), so block (k, i)
// of the 3 x 3 block matrix is the transpose of block (i, k); for i < k it is copied transposed
// instead of integrated. Blocks that fit in LDS are moved whole by one workgroup; larger ones in
// 32 x 32 tiles. Either way reads and writes are row-contiguous.
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

// Small blocks (ns (ns + 1) values in at most 20 KiB of LDS, p <= 3): one workgroup per block,
// read and written as two contiguous streams. (Whole 125 x 125 blocks at p = 4 leave too few
// workgroups per CU in flight; the tiles are faster there.)
template <typename T>
__global__ void __launch_bounds__(256) k_transpose_small_blocks(T *A, int64_t nel, int ns)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *blk = reinterpret_cast<T *>(smem_raw);
    const int64_t nsq = (int64_t)ns * ns;
    const int n2 = ns * ns;
    for (int64_t w = blockIdx.x; w < nel * 3; w += gridDim.x) {
        const int64_t e = w / 3;
        const int pair = (int)(w % 3);
        const int i = pair < 2 ? 0 : 1, k = pair == 0 ? 1 : 2;
        const T *src = A + (e * 9 + 3 * i + k) * nsq;
        T *dst = A + (e * 9 + 3 * k + i) * nsq;
        __syncthreads();  // the previous block has left LDS
        for (int f = threadIdx.x; f < n2; f += blockDim.x) blk[(f / ns) * (ns + 1) + f % ns] = src[f];
        __syncthreads();
        // dst[r][c] = src[c][r]
        for (int f = threadIdx.x; f < n2; f += blockDim.x) dst[f] = blk[(f % ns) * (ns + 1) + f / ns];
    }
}

}  // namespace

hipError_t transpose_elastic_blocks(void *A, bool fp64, int64_t nel, int ns, hipStream_t s, int64_t cus)
{
    const size_t small = size_t(ns) * (ns + 1) * (fp64 ? 8 : 4);
    if (small <= 20480) {  // p <= 3: many small blocks in flight per CU
        const int64_t work = nel * 3, cap = cus * 8;
        const int64_t grid = work < cap ? work : cap;
        if (grid <= 0) return hipSuccess;
        if (fp64)
            hipLaunchKernelGGL(k_transpose_small_blocks<double>, dim3((unsigned)grid), dim3(256), small, s,
                               static_cast<double *>(A), nel, ns);
        else
            hipLaunchKernelGGL(k_transpose_small_blocks<float>, dim3((unsigned)grid), dim3(256), small, s,
                               static_cast<float *>(A), nel, ns);
        return hipGetLastError();
    }
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
