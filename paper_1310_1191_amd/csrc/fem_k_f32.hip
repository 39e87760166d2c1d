// Kernel instances of the F32 contraction path, p = 1..7.
#include "fem_launch.h"

namespace fem {
hipError_t prepare_f32() { return prepare_all<PREC_F32>(); }
hipError_t launch_f32(int p, const KArgs &a, hipStream_t s, int64_t cap) { return launch_p<PREC_F32>(p, a, s, cap); }
}  // namespace fem
