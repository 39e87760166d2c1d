// fem_timestep.hip -- device-side time stepping of the coefficient fields (fem_field_advance).
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

}  // namespace

hipError_t field_advance(double *field, const double *deltas, int32_t nsteps, int32_t *step,
                         hipStream_t s)
{
    hipLaunchKernelGGL(k_field_advance, dim3(1), dim3(64), 0, s, field, deltas, nsteps, step);
    return hipGetLastError();
}

}  // namespace fem
