// fem_transpose.hip -- the lower blocks of the elasticity element matrix from the upper ones.
// The isotropic tensor has the major symmetry c_ijkl = c_klij (section 5.1), so block (k, i)
// of the 3 x 3 block matrix is the transpose of block (i, k); for i < k it is copied transposed
// instead of integrated. Each block is Ns x Ns, row-major and contiguous (element e's block
// (i, k) at (9 e + 3 i + k) Ns^2).
//
// Large blocks (p >= 4) go in panels: a workgroup produces PW whole rows of the destination
// block, which lie back to back in memory (one linear write stream), from the same PW columns
// of the source, read as PW-wide row segments with many loads in flight per thread. Small
// blocks (p = 2) are moved whole, one per workgroup pass. Both stage through LDS with an odd
// row pitch, so the transposed LDS accesses of a wave fall in distinct banks.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fem_transpose.h"

namespace fem {

namespace {

constexpr int NT = 256;                // threads of a small-block workgroup
constexpr int NTP = 512;               // threads of a panel workgroup
constexpr int CH = 16;                 // panel loads each thread has in flight before its LDS writes
constexpr int CU_LDS = 160 * 1024;     // LDS of one CU
constexpr int CU_THREADS = 2048;       // resident threads of one CU (32 waves)
constexpr int PANEL_LDS = 80 * 1024;   // bytes of LDS per panel workgroup, at most (two per CU)

__host__ __device__ inline int odd_pitch(int ns) { return ns | 1; }

// Panel width for a block edge and entry size: the widest power of two up to 64 whose staged
// panel (pw x odd_pitch(ns) entries) fits in PANEL_LDS.
inline int panel_width(int ns, int bytes)
{
    int pw = 64;
    while (pw > 1 && size_t(pw) * odd_pitch(ns) * bytes > size_t(PANEL_LDS)) pw /= 2;
    return pw;
}

// Work item w = 3 e + pair; pair 0, 1, 2 = blocks (0, 1), (0, 2), (1, 2) of element e.
__device__ inline int64_t src_block(int64_t e, int pair) { return e * 9 + (pair == 2 ? 5 : 1 + pair); }
__device__ inline int64_t dst_block(int64_t e, int pair) { return e * 9 + (pair == 0 ? 3 : (pair == 1 ? 6 : 7)); }

// Panels: work item w = (3 e + pair) np + panel (np panels per block), lg = log2(pw). A thread
// reads one column c of the panel (pw divides NTP), every (NTP / pw)-th row, CH loads at a
// time held in registers; the write phase walks the panel's destination rows linearly with
// incremental (row, column) carries, so no entry needs a division.
template <typename T>
__global__ void __launch_bounds__(NTP) k_transpose_panels(T *A, int64_t nel, int ns, int lg)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *pan = reinterpret_cast<T *>(smem_raw);  // [pw][pitch]: pan[c][r] = src[r][c0 + c]
    const int pw = 1 << lg;
    const int pitch = odd_pitch(ns);
    const int np = (ns + pw - 1) / pw;
    const int64_t nsq = (int64_t)ns * ns;
    const int tid = threadIdx.x;
    const int rc = tid & (pw - 1), rr0 = tid >> lg, rstep = NTP >> lg;  // read phase
    const int wc0 = tid / ns, wr0 = tid - wc0 * ns;                     // write phase
    const int dq = NTP / ns, dr = NTP - dq * ns;
    for (int64_t w = blockIdx.x; w < nel * 3 * np; w += gridDim.x) {
        const int64_t item = w / np;
        const int panel = (int)(w - item * np);
        const int64_t e = item / 3;
        const int pair = (int)(item - e * 3);
        const int c0 = panel * pw;
        const int wcols = ns - c0 < pw ? ns - c0 : pw;  // columns of this panel
        const T *src = A + src_block(e, pair) * nsq + c0 + rc;
        T *dst = A + dst_block(e, pair) * nsq + (int64_t)c0 * ns;
        __syncthreads();  // the previous panel has left LDS
        if (rc < wcols) {
            for (int r = rr0; r < ns; r += rstep * CH) {
                T v[CH];
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    const int q = r + u * rstep;
                    v[u] = q < ns ? src[(int64_t)q * ns] : T(0);
                }
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    const int q = r + u * rstep;
                    if (q < ns) pan[rc * pitch + q] = v[u];
                }
            }
        }
        __syncthreads();
        // destination rows c0 .. c0 + wcols lie back to back: wcols ns entries
        const int nwrite = wcols * ns;
        int c = wc0, r = wr0;
#pragma unroll 4
        for (int f = tid; f < nwrite; f += NTP) {
            dst[f] = pan[c * pitch + r];
            r += dr;
            c += dq;
            if (r >= ns) {
                r -= ns;
                ++c;
            }
        }
    }
}

// Small blocks (n2 = ns^2 <= 4 NT entries, p = 2): one block per workgroup pass, read and
// written as two contiguous streams, each thread's four entries loaded before its LDS writes.
template <typename T>
__global__ void __launch_bounds__(NT) k_transpose_small_blocks(T *A, int64_t nel, int ns)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *blk = reinterpret_cast<T *>(smem_raw);  // [ns][pitch]
    const int pitch = odd_pitch(ns);
    const int64_t nsq = (int64_t)ns * ns;
    const int n2 = ns * ns;
    const int tid = threadIdx.x;
    // (row, column) of entries tid + u NT, u = 0..3
    int row[4], col[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int g = tid + u * NT;
        row[u] = g / ns;
        col[u] = g - row[u] * ns;
    }
    for (int64_t w = blockIdx.x; w < nel * 3; w += gridDim.x) {
        const int64_t e = w / 3;
        const int pair = (int)(w - e * 3);
        const T *src = A + src_block(e, pair) * nsq;
        T *dst = A + dst_block(e, pair) * nsq;
        __syncthreads();  // the previous block has left LDS
        T v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = tid + u * NT < n2 ? src[tid + u * NT] : T(0);
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (tid + u * NT < n2) blk[row[u] * pitch + col[u]] = v[u];
        __syncthreads();
        // dst[row][col] = src[col][row]
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (tid + u * NT < n2) dst[tid + u * NT] = blk[col[u] * pitch + row[u]];
    }
}

template <typename T>
hipError_t launch_transpose(T *A, int64_t nel, int ns, hipStream_t s, int64_t cus)
{
    if (ns * ns <= 4 * NT) {  // p = 2: whole blocks
        const size_t lds = size_t(ns) * odd_pitch(ns) * sizeof(T);
        const int64_t work = nel * 3, cap = cus * 8;
        const int64_t grid = work < cap ? work : cap;
        if (grid <= 0) return hipSuccess;
        hipLaunchKernelGGL(k_transpose_small_blocks<T>, dim3((unsigned)grid), dim3(NT), lds, s, A, nel, ns);
        return hipGetLastError();
    }
    const int pw = panel_width(ns, (int)sizeof(T));
    int lg = 0;
    while ((1 << lg) < pw) ++lg;
    const size_t lds = size_t(pw) * odd_pitch(ns) * sizeof(T);
    int64_t per_cu = CU_LDS / lds;  // workgroups one CU holds
    if (per_cu > CU_THREADS / NTP) per_cu = CU_THREADS / NTP;
    const int64_t work = nel * 3 * ((ns + pw - 1) / pw), cap = cus * per_cu;
    const int64_t grid = work < cap ? work : cap;
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_transpose_panels<T>, dim3((unsigned)grid), dim3(NTP), lds, s, A, nel, ns, lg);
    return hipGetLastError();
}

}  // namespace

hipError_t transpose_prepare()
{
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_transpose_panels<float>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, PANEL_LDS);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_transpose_panels<double>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, PANEL_LDS);
}

hipError_t transpose_elastic_blocks(void *A, bool fp64, int64_t nel, int ns, hipStream_t s, int64_t cus)
{
    if (fp64) return launch_transpose(static_cast<double *>(A), nel, ns, s, cus);
    return launch_transpose(static_cast<float *>(A), nel, ns, s, cus);
}

}  // namespace fem
