// Kernel instances of the BF16 contraction path: every compiled variant for p = 1..7 and the
// single-launch mixed-degree kernel.
#include "fem_launch.h"

namespace fem {
hipError_t prepare_bf16()
{
    const hipError_t e = prepare_all<PREC_BF16>();
    return e != hipSuccess ? e : MixedInst<PREC_BF16>::prepare();
}
hipError_t launch_bf16(int p, int v, const KArgs &a, hipStream_t s, int64_t cus) { return launch_p<PREC_BF16>(p, v, a, s, cus); }
hipError_t launch_mixed_bf16(const MixedKArgs &m, int64_t nel, hipStream_t s, int64_t cus)
{
    return MixedInst<PREC_BF16>::launch(m, nel, s, (int)cus);
}
int variants_bf16(int p) { return variants_p<PREC_BF16>(p); }
}  // namespace fem
