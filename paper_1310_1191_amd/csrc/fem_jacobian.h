// fem_jacobian.h -- launch of the kernel that writes the supplied Jacobian terms (NOJAC input).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fem {

struct JacArgs {
    int64_t nel;
    int32_t p;              // uniform degree 1..7, or 0: per-element degree[] with the b_off scan
    const double *geom;     // [nel][8][3]
    const int8_t *degree;   // [nel], p == 0 only
    const int64_t *b_off;   // [nel + 1] exclusive scan of Nq, p == 0 only
    const double *xq[8];    // Gauss points of degree p at index p
    double *out;            // [sum Nq][10]
};

hipError_t jacobian_terms_launch(const JacArgs &a, hipStream_t s, int64_t cus);

}  // namespace fem
