// fem_geometry.h -- the element maps in FP64 (the trilinear hexahedron; the prism, linear in the
// triangle and in the vertical direction): points and the Jacobian terms (J, detJ, J^{-1}).
// Shared by the integration prologue and by the kernel that writes the supplied-terms (NOJAC)
// input, so both produce the same values.
#pragma once
#include <hip/hip_runtime.h>

namespace fem {

// x_c(xi) = sum_S tc[8c + S] prod_{d in S} xi_d over the subsets S of {1,2,3} (bit d-1 of S);
// tc[8c + S] = 1/8 sum_v X[v][c] prod_{d in S} s_vd with s_vd = +-1 the vertex's side. `sub` is S.
__device__ inline double trilinear_coeff(const double *X, int coord, int sub)
{
    double acc = 0.0;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const int neg_bits = __popc(sub & ~v);
        const double x = X[v * 3 + coord];
        acc += (neg_bits & 1) ? -x : x;
    }
    return 0.125 * acc;
}

// Position of the point (x1, x2, x3) under the trilinear form tc[24].
__device__ inline void trilinear_point(const double *tc, double x1, double x2, double x3, double xq[3])
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double *k = tc + c * 8;
        xq[c] = k[0] + k[1] * x1 + k[2] * x2 + k[4] * x3 + x1 * (k[3] * x2 + k[5] * x3) +
                x2 * x3 * (k[6] + k[7] * x1);
    }
}

// J[c][d] = dx_c/dxi_d at (x1, x2, x3); returns detJ and writes J^{-1} = adj(J) / detJ.
__device__ inline double jacobian_terms(const double *tc, double x1, double x2, double x3,
                                        double Ji[3][3])
{
    double J[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double *k = tc + c * 8;
        J[c][0] = k[1] + k[3] * x2 + k[5] * x3 + k[7] * x2 * x3;
        J[c][1] = k[2] + k[3] * x1 + k[6] * x3 + k[7] * x1 * x3;
        J[c][2] = k[4] + k[5] * x1 + k[6] * x2 + k[7] * x1 * x2;
    }
    Ji[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    Ji[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    Ji[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double det = J[0][0] * Ji[0][0] + J[0][1] * Ji[1][0] + J[0][2] * Ji[2][0];
    Ji[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    Ji[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    Ji[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    Ji[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    Ji[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    Ji[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const double id = 1.0 / det;
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int n = 0; n < 3; ++n) Ji[m][n] *= id;
    return det;
}

// ---- the prism map (vertex v = t + 3h at triangle vertex t = (0,0), (1,0), (0,1) and
// zeta = -1 (h = 0) or +1 (h = 1); X holds [6][3]):
//   x(xi1, xi2, zeta) = sum_h (1 + s_h zeta)/2 [X_0h + xi1 (X_1h - X_0h) + xi2 (X_2h - X_0h)] ----
__device__ inline void prism_point(const double *X, double x1, double x2, double z, double xq[3])
{
    const double fb = 0.5 * (1.0 - z), ft = 0.5 * (1.0 + z);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double bot = X[c] + x1 * (X[3 + c] - X[c]) + x2 * (X[6 + c] - X[c]);
        const double top = X[9 + c] + x1 * (X[12 + c] - X[9 + c]) + x2 * (X[15 + c] - X[9 + c]);
        xq[c] = fb * bot + ft * top;
    }
}

// J[c][d] = dx_c/dxi_d (xi_3 = zeta) of the prism map; returns detJ and writes J^{-1}.
__device__ inline double prism_jacobian_terms(const double *X, double x1, double x2, double z,
                                              double Ji[3][3])
{
    const double fb = 0.5 * (1.0 - z), ft = 0.5 * (1.0 + z);
    const double l0 = 1.0 - x1 - x2;
    double J[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        J[c][0] = fb * (X[3 + c] - X[c]) + ft * (X[12 + c] - X[9 + c]);
        J[c][1] = fb * (X[6 + c] - X[c]) + ft * (X[15 + c] - X[9 + c]);
        J[c][2] = 0.5 * (l0 * (X[9 + c] - X[c]) + x1 * (X[12 + c] - X[3 + c]) + x2 * (X[15 + c] - X[6 + c]));
    }
    Ji[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    Ji[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    Ji[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double det = J[0][0] * Ji[0][0] + J[0][1] * Ji[1][0] + J[0][2] * Ji[2][0];
    Ji[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    Ji[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    Ji[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    Ji[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    Ji[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    Ji[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const double id = 1.0 / det;
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int n = 0; n < 3; ++n) Ji[m][n] *= id;
    return det;
}

}  // namespace fem
