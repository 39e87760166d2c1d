// Kernel instances of the F64 contraction path: every compiled variant for p = 1..7 and the
// single-launch mixed-degree kernel.
#include "fem_launch.h"

namespace fem {
hipError_t prepare_f64()
{
    const hipError_t e = prepare_all<PREC_F64>();
    return e != hipSuccess ? e : MixedInst<PREC_F64>::prepare();
}
hipError_t launch_f64(int p, int v, const KArgs &a, hipStream_t s, int64_t cus) { return launch_p<PREC_F64>(p, v, a, s, cus); }
hipError_t launch_mixed_f64(const MixedKArgs &m, int64_t nel, hipStream_t s, int64_t cus)
{
    return MixedInst<PREC_F64>::launch(m, nel, s, (int)cus);
}
int variants_f64(int p) { return variants_p<PREC_F64>(p); }
}  // namespace fem
