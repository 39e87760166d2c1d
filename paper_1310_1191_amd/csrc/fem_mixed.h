// fem_mixed.h -- mixed-degree support: element classification by degree (section 4.2 of the
// paper: the host manager classifies elements into sets of equal degree) and output offsets,
// both computed on the device so that a mixed-degree call never synchronises with the host.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fem {

struct MixedPlan {
    const int32_t *elist;  // element ids grouped by degree
    const int64_t *seg;    // [8][2]: {start, count} of degree p's ids in elist
};

size_t mixed_workspace_bytes(int64_t nel);
hipError_t mixed_prepare();
// Element capacity of the library's static device scratch (the workspace of the allocation-free
// entry point) and the device address of that scratch on the current device.
constexpr int64_t NOALLOC_MAX_NEL = int64_t(1) << 22;
hipError_t mixed_scratch_address(void **ptr);
// a_off[e] = sum_{e' < e} Ns(e')^2, b_off[e] = sum_{e' < e} Ns(e'), nel + 1 entries.
hipError_t mixed_offsets(int64_t nel, const int8_t *degree, int64_t *a_off, int64_t *b_off,
                         void *workspace, hipStream_t s);
// Counting sort of element ids by degree into the workspace.
hipError_t mixed_bucket(int64_t nel, const int8_t *degree, void *workspace, hipStream_t s,
                        MixedPlan *plan);

}  // namespace fem
