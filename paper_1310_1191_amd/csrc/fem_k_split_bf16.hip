// Kernel instances of the SPLIT_BF16 contraction path, p = 1..7.
#include "fem_launch.h"

namespace fem {
hipError_t prepare_split_bf16() { return prepare_all<PREC_SPLIT_BF16>(); }
hipError_t launch_split_bf16(int p, const KArgs &a, hipStream_t s, int64_t cap) { return launch_p<PREC_SPLIT_BF16>(p, a, s, cap); }
}  // namespace fem
