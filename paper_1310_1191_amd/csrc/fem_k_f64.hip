// Kernel instances of the F64 contraction path: every compiled variant for p = 1..7.
#include "fem_launch.h"

namespace fem {
hipError_t prepare_f64() { return prepare_all<PREC_F64>(); }
hipError_t launch_f64(int p, int v, const KArgs &a, hipStream_t s, int64_t cus) { return launch_p<PREC_F64>(p, v, a, s, cus); }
int variants_f64(int p) { return variants_p<PREC_F64>(p); }
}  // namespace fem
