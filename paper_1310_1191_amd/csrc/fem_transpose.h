// fem_transpose.h -- the lower elasticity blocks as transposes of the upper ones.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fem {

// A: [nel][3][3][ns][ns] (FP64 when fp64, else FP32); writes block (k, i) = block (i, k)^T for
// (i, k) in {(0, 1), (0, 2), (1, 2)}. Asynchronous on s; allocates nothing.
hipError_t transpose_elastic_blocks(void *A, bool fp64, int64_t nel, int ns, hipStream_t s, int64_t cus);

// Once per device, before the first transpose: allows the kernels' LDS staging above 64 KiB.
hipError_t transpose_prepare();

}  // namespace fem
