// Kernel instances of the F64 contraction path, p = 1..7.
#include "fem_launch.h"

namespace fem {
hipError_t prepare_f64() { return prepare_all<PREC_F64>(); }
hipError_t launch_f64(int p, const KArgs &a, hipStream_t s, int64_t cap) { return launch_p<PREC_F64>(p, a, s, cap); }
}  // namespace fem
