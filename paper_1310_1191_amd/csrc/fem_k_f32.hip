// Kernel instances of the F32 contraction path: every compiled variant for p = 1..7.
#include "fem_launch.h"

namespace fem {
hipError_t prepare_f32() { return prepare_all<PREC_F32>(); }
hipError_t launch_f32(int p, int v, const KArgs &a, hipStream_t s, int64_t cus) { return launch_p<PREC_F32>(p, v, a, s, cus); }
int variants_f32(int p) { return variants_p<PREC_F32>(p); }
}  // namespace fem
