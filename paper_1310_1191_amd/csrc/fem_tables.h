// fem_tables.h -- host-side reference-element tables of libfem (FP64, built once in fem_init).
//
// For each degree p the library needs (section 2 of the paper: xi^Q, w^Q and the reference
// shape-function values and derivatives phi^Q, precomputed once and kept in device memory,
// section 4.1):
//   * the (p+1)-point Gauss-Legendre points and weights on [-1,1];
//   * the 1-D Lagrange polynomials on the p+1 Gauss-Lobatto-Legendre nodes and their
//     derivatives, evaluated at the Gauss points: L[q][a], D[q][a];
//   * the row operand of the contraction A = B^T blockdiag(D_q) B, i.e. B^T with
//     B[(q, r)][i] = (phi_i, dphi_i/dxi_1, dphi_i/dxi_2, dphi_i/dxi_3)(xi_q), stored in the exact
//     per-lane order that the MFMA instructions read it (see fem_layout.h).
#pragma once
#include <cstddef>
#include <cstdint>
#include <vector>

namespace fem {

struct HostDegreeTables {
    int p = 0, n = 0, ns = 0;
    std::vector<double> xq, wq;   // [n]
    std::vector<double> L, D;     // [n][n]: (gauss point q, node a)
    double bmax = 0.0;            // max over (q, j) of sum_r |B[(q, r)][j]|
};

// Gauss-Legendre rule on [-1,1] with n points, ascending.
void gauss_legendre_rule(int n, double *x, double *w);
// The p+1 Gauss-Lobatto-Legendre nodes, ascending.
void lobatto_nodes(int p, double *x);
// Tables of degree p.
HostDegreeTables make_degree_tables(int p);
// B[(q, r)][i] in FP64 for the whole reference element, [nq][4][ns].
std::vector<double> reference_operand(const HostDegreeTables &t);

}  // namespace fem
