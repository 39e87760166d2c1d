// fem_timestep.hip -- device-side time stepping of the coefficient fields (fem_field_advance) and
// the gather of a step's sampled element matrices (fem_gather_sample).
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fem {

namespace {

__global__ void k_field_advance(double *field, const double *deltas, int32_t nsteps, int32_t *step)
{
    const int t = *step;  // every thread reads the counter before thread 0 moves it on
    const bool active = t >= 0 && t < nsteps;
    const int m = threadIdx.x;  // one thread per (field, mode)
    if (active && m < 35) {
        const double two_pi = 6.283185307179586476925286766559;
        double th = field[m * 5 + 4] + deltas[(int64_t)t * 35 + m];
        th = fmod(th, two_pi);
        if (th < 0.0) th += two_pi;
        field[m * 5 + 4] = th;
    }
    __syncthreads();
    if (active && m == 0) *step = t + 1;
}

// One workgroup per selected element: its destination offset is the sum of the sizes of the
// selections before it (a workgroup reduction over at most nsel entries), then a word copy.
// Selections outside [0, nel) and words past the capacity are skipped.
constexpr int GATHER_NT = 256;

__device__ int64_t gather_prefix(const int32_t *s, int64_t i, int64_t nel, const int64_t *off,
                                 int64_t *red)
{
    int64_t acc = 0;
    for (int64_t j = threadIdx.x; j < i; j += GATHER_NT) {
        const int32_t e = s[j];
        if (e >= 0 && e < nel) acc += off[e + 1] - off[e];
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = GATHER_NT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    const int64_t r = red[0];
    __syncthreads();
    return r;
}

__device__ void gather_copy(const uint32_t *src, uint32_t *dst, int64_t words)
{
    for (int64_t k = threadIdx.x; k < words; k += GATHER_NT) dst[k] = src[k];
}

__global__ void __launch_bounds__(GATHER_NT)
k_gather_sample(int64_t nsel, const int32_t *sel, int32_t nrows, const int32_t *step, int64_t nel,
                const int64_t *a_off, const int64_t *b_off, const uint32_t *A, const uint32_t *b,
                uint32_t *out_A, int64_t cap_A, uint32_t *out_b, int64_t cap_b, int32_t wpe)
{
    __shared__ int64_t red[GATHER_NT];
    const int64_t i = blockIdx.x;
    int64_t row = 0;
    if (step) {
        const int64_t t = (int64_t)*step - 1;
        row = ((t % nrows) + nrows) % nrows;
    }
    const int32_t *s = sel + row * nsel;
    const int32_t e = s[i];
    const bool ok = e >= 0 && e < nel;
    {
        const int64_t at = gather_prefix(s, i, nel, a_off, red);
        if (ok) {
            int64_t n = a_off[e + 1] - a_off[e];
            n = at >= cap_A ? 0 : (at + n > cap_A ? cap_A - at : n);
            gather_copy(A + a_off[e] * wpe, out_A + at * wpe, n * wpe);
        }
    }
    if (b && out_b) {
        const int64_t at = gather_prefix(s, i, nel, b_off, red);
        if (ok) {
            int64_t n = b_off[e + 1] - b_off[e];
            n = at >= cap_b ? 0 : (at + n > cap_b ? cap_b - at : n);
            gather_copy(b + b_off[e] * wpe, out_b + at * wpe, n * wpe);
        }
    }
}

}  // namespace

hipError_t gather_sample(int64_t nsel, const int32_t *sel, int32_t nrows, const int32_t *step, int64_t nel,
                         const int64_t *a_off, const int64_t *b_off, const void *A, const void *b,
                         void *out_A, int64_t cap_A, void *out_b, int64_t cap_b, int32_t entry_bytes,
                         hipStream_t s)
{
    if (nsel <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_sample, dim3((unsigned)nsel), dim3(GATHER_NT), 0, s, nsel, sel, nrows,
                       step, nel, a_off, b_off, static_cast<const uint32_t *>(A),
                       static_cast<const uint32_t *>(b), static_cast<uint32_t *>(out_A), cap_A,
                       static_cast<uint32_t *>(out_b), cap_b, entry_bytes / 4);
    return hipGetLastError();
}

hipError_t field_advance(double *field, const double *deltas, int32_t nsteps, int32_t *step,
                         hipStream_t s)
{
    hipLaunchKernelGGL(k_field_advance, dim3(1), dim3(64), 0, s, field, deltas, nsteps, step);
    return hipGetLastError();
}

}  // namespace fem
