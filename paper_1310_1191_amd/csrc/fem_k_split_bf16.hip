// Kernel instances of the split-BF16 contraction path: every compiled variant for p = 1..7.
#include "fem_launch.h"

namespace fem {
hipError_t prepare_split_bf16() { return prepare_all<PREC_SPLIT_BF16>(); }
hipError_t launch_split_bf16(int p, int v, const KArgs &a, hipStream_t s, int64_t cus) { return launch_p<PREC_SPLIT_BF16>(p, v, a, s, cus); }
int variants_split_bf16(int p) { return variants_p<PREC_SPLIT_BF16>(p); }
}  // namespace fem
