// Kernel instances of the F32 contraction path: every compiled variant for p = 1..7 and the
// single-launch mixed-degree kernel.
#include "fem_launch.h"

namespace fem {
hipError_t prepare_f32()
{
    const hipError_t e = prepare_all<PREC_F32>();
    return e != hipSuccess ? e : MixedInst<PREC_F32>::prepare();
}
hipError_t launch_f32(int p, int v, const KArgs &a, hipStream_t s, int64_t cus) { return launch_p<PREC_F32>(p, v, a, s, cus); }
hipError_t launch_mixed_f32(const MixedKArgs &m, int64_t nel, hipStream_t s, int64_t cus)
{
    return MixedInst<PREC_F32>::launch(m, nel, s, (int)cus);
}
int variants_f32(int p) { return variants_p<PREC_F32>(p); }
}  // namespace fem
