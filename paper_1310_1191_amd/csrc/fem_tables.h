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

// The prism of degree p (section 2, Tables 1-2): triangle lattice times GLL nodes, the
// symmetric degree-2p triangle rule times the (p+1)-point Gauss-Legendre rule.
struct HostPrismTables {
    int p = 0, n = 0, nt = 0, ns = 0, ntq = 0, nq = 0;
    std::vector<double> pts;  // [nq][4]: xi1, xi2, zeta, weight; q = qt + ntq qz
    std::vector<double> B;    // [nq][4][ns]: value and d/dxi1, d/dxi2, d/dzeta; i = t + nt c
    std::vector<double> phi;  // [nq][ns]: the values alone (load vector)
    double bmax = 0.0;        // max over (q, j) of sum_r |B[(q, r)][j]|
};
// Points (xi1, xi2) and weights of the degree-2p triangle rule; false if the refinement fails.
bool prism_triangle_rule(int p, std::vector<double> &x, std::vector<double> &y, std::vector<double> &w);
bool make_prism_tables(int p, HostPrismTables &t);

}  // namespace fem
