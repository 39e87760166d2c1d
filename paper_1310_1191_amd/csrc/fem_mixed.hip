// fem_mixed.hip -- device-side degree classification and output offsets (fem_mixed.h).
#include "fem_mixed.h"

namespace fem {

namespace {

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 4;
constexpr int64_t SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

// Workspace layout (bytes): [0, 128) seg[8][2] int64; [256, 288) cursor[8] int32;
// [512, ...) elist[nel] int32; then scan partials [2][nblocks] int64.
constexpr size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
constexpr int64_t scan_blocks(int64_t nel) { return (nel + 1 + SCAN_TILE - 1) / SCAN_TILE; }
constexpr size_t off_elist() { return 512; }
constexpr size_t off_partials(int64_t nel) { return off_elist() + align256(size_t(nel) * 4); }
constexpr size_t workspace_bytes(int64_t nel) { return off_partials(nel) + align256(size_t(scan_blocks(nel)) * 16); }

// Workspace of the allocation-free entry point: one copy per device, held until the process
// ends, sized for NOALLOC_MAX_NEL elements (about 16 MiB). Host code never passes this name to a
// kernel (on the host it is only a stand-in for the symbol); it takes the device address from
// mixed_scratch_address instead.
static __device__ __align__(256) unsigned char scratch[workspace_bytes(NOALLOC_MAX_NEL)];

__device__ inline int64_t ns_of_deg(int d)
{
    return (d >= 1 && d <= 7) ? int64_t(d + 1) * (d + 1) * (d + 1) : 0;
}

__global__ void k_clear(int64_t *seg, int32_t *cursor)
{
    const int t = threadIdx.x;
    if (t < 16) seg[t] = 0;
    if (t < 8) cursor[t] = 0;
}

__global__ void k_histogram(int64_t nel, const int8_t *degree, int64_t *seg)
{
    __shared__ int cnt[8];
    if (threadIdx.x < 8) cnt[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nel;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int d = degree[e];
        if (d >= 1 && d <= 7) atomicAdd(&cnt[d], 1);
    }
    __syncthreads();
    if (threadIdx.x >= 1 && threadIdx.x < 8 && cnt[threadIdx.x])
        atomicAdd((unsigned long long *)&seg[2 * threadIdx.x + 1], (unsigned long long)cnt[threadIdx.x]);
}

// starts: heaviest degree first in elist (7, 6, ..., 1)
__global__ void k_starts(int64_t *seg)
{
    if (threadIdx.x == 0) {
        int64_t s = 0;
        for (int d = 7; d >= 1; --d) {
            seg[2 * d] = s;
            s += seg[2 * d + 1];
        }
    }
}

__global__ void k_scatter(int64_t nel, const int8_t *degree, const int64_t *seg, int32_t *cursor,
                          int32_t *elist)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nel;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int d = degree[e];
        if (d >= 1 && d <= 7) {
            const int pos = atomicAdd(&cursor[d], 1);
            elist[seg[2 * d] + pos] = (int32_t)e;
        }
    }
}

// Exclusive scan of (Ns^2, Ns) over elements: tile sums, scan of the tile sums, tile scans.
__global__ void k_tile_sums(int64_t nel, const int8_t *degree, int64_t *part)
{
    __shared__ int64_t sa[SCAN_BLOCK], sb[SCAN_BLOCK];
    const int64_t base = blockIdx.x * SCAN_TILE;
    int64_t ta = 0, tb = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const int64_t e = base + threadIdx.x * SCAN_ITEMS + k;
        if (e < nel) {
            const int64_t ns = ns_of_deg(degree[e]);
            ta += ns * ns;
            tb += ns;
        }
    }
    sa[threadIdx.x] = ta;
    sb[threadIdx.x] = tb;
    __syncthreads();
    for (int off = SCAN_BLOCK / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            sa[threadIdx.x] += sa[threadIdx.x + off];
            sb[threadIdx.x] += sb[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sa[0];
        part[2 * blockIdx.x + 1] = sb[0];
    }
}

__global__ void k_scan_partials(int64_t nb, int64_t *part)
{
    // one block: sequential chunks, Hillis-Steele inside each chunk
    __shared__ int64_t sa[SCAN_BLOCK], sb[SCAN_BLOCK];
    int64_t carry_a = 0, carry_b = 0;
    for (int64_t c0 = 0; c0 < nb; c0 += SCAN_BLOCK) {
        const int64_t i = c0 + threadIdx.x;
        const int64_t va = i < nb ? part[2 * i] : 0, vb = i < nb ? part[2 * i + 1] : 0;
        sa[threadIdx.x] = va;
        sb[threadIdx.x] = vb;
        __syncthreads();
        for (int off = 1; off < SCAN_BLOCK; off <<= 1) {
            int64_t xa = 0, xb = 0;
            if (threadIdx.x >= off) {
                xa = sa[threadIdx.x - off];
                xb = sb[threadIdx.x - off];
            }
            __syncthreads();
            sa[threadIdx.x] += xa;
            sb[threadIdx.x] += xb;
            __syncthreads();
        }
        if (i < nb) {  // exclusive
            part[2 * i] = carry_a + sa[threadIdx.x] - va;
            part[2 * i + 1] = carry_b + sb[threadIdx.x] - vb;
        }
        const int64_t ta = sa[SCAN_BLOCK - 1], tb = sb[SCAN_BLOCK - 1];
        __syncthreads();
        carry_a += ta;
        carry_b += tb;
    }
}

__global__ void k_tile_scan(int64_t nel, const int8_t *degree, const int64_t *part, int64_t *a_off,
                            int64_t *b_off)
{
    __shared__ int64_t sa[SCAN_BLOCK], sb[SCAN_BLOCK];
    const int64_t base = blockIdx.x * SCAN_TILE;
    int64_t va[SCAN_ITEMS], vb[SCAN_ITEMS], ta = 0, tb = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const int64_t e = base + threadIdx.x * SCAN_ITEMS + k;
        const int64_t ns = e < nel ? ns_of_deg(degree[e]) : 0;
        va[k] = ns * ns;
        vb[k] = ns;
        ta += va[k];
        tb += vb[k];
    }
    sa[threadIdx.x] = ta;
    sb[threadIdx.x] = tb;
    __syncthreads();
    for (int off = 1; off < SCAN_BLOCK; off <<= 1) {
        int64_t xa = 0, xb = 0;
        if (threadIdx.x >= off) {
            xa = sa[threadIdx.x - off];
            xb = sb[threadIdx.x - off];
        }
        __syncthreads();
        sa[threadIdx.x] += xa;
        sb[threadIdx.x] += xb;
        __syncthreads();
    }
    int64_t ra = part[2 * blockIdx.x] + sa[threadIdx.x] - ta;
    int64_t rb = part[2 * blockIdx.x + 1] + sb[threadIdx.x] - tb;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const int64_t e = base + threadIdx.x * SCAN_ITEMS + k;
        if (e <= nel) {  // entry nel holds the totals
            a_off[e] = ra;
            b_off[e] = rb;
        }
        ra += va[k];
        rb += vb[k];
    }
}

}  // namespace

size_t mixed_workspace_bytes(int64_t nel) { return workspace_bytes(nel); }

hipError_t mixed_scratch_address(void **ptr)
{
    *ptr = nullptr;
    return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch));
}

hipError_t mixed_prepare() { return hipSuccess; }

hipError_t mixed_offsets(int64_t nel, const int8_t *degree, int64_t *a_off, int64_t *b_off,
                         void *workspace, hipStream_t s)
{
    unsigned char *ws = static_cast<unsigned char *>(workspace);
    int64_t *part = reinterpret_cast<int64_t *>(ws + off_partials(nel));
    const int64_t nb = scan_blocks(nel);
    hipLaunchKernelGGL(k_tile_sums, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, nel, degree, part);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(SCAN_BLOCK), 0, s, nb, part);
    hipLaunchKernelGGL(k_tile_scan, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, nel, degree, part,
                       a_off, b_off);
    return hipGetLastError();
}

hipError_t mixed_bucket(int64_t nel, const int8_t *degree, void *workspace, hipStream_t s,
                        MixedPlan *plan)
{
    unsigned char *ws = static_cast<unsigned char *>(workspace);
    int64_t *seg = reinterpret_cast<int64_t *>(ws);
    int32_t *cursor = reinterpret_cast<int32_t *>(ws + 256);
    int32_t *elist = reinterpret_cast<int32_t *>(ws + off_elist());
    const int64_t blocks64 = (nel + 255) / 256;
    const unsigned blocks = (unsigned)(blocks64 < 4096 ? (blocks64 > 0 ? blocks64 : 1) : 4096);
    hipLaunchKernelGGL(k_clear, dim3(1), dim3(64), 0, s, seg, cursor);
    hipLaunchKernelGGL(k_histogram, dim3(blocks), dim3(256), 0, s, nel, degree, seg);
    hipLaunchKernelGGL(k_starts, dim3(1), dim3(64), 0, s, seg);
    hipLaunchKernelGGL(k_scatter, dim3(blocks), dim3(256), 0, s, nel, degree, seg, cursor, elist);
    plan->elist = elist;
    plan->seg = seg;
    return hipGetLastError();
}

}  // namespace fem
