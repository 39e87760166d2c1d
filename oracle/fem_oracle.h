/*
 * fem_oracle.h -- FP64 CPU oracle for element stiffness-matrix and load-vector integration.
 *
 * TEST INFRASTRUCTURE. This library exists to check the HIP path; it is not part of it.
 * Only the test-suite, the package's smoke check and the benchmark's CPU-baseline leg load it.
 * It shares no source, header, table or helper with the GPU library.
 *
 * What it computes (Banas, Plaszewski, Maciol, "Numerical integration on GPUs for higher order
 * finite elements", section 2, Algorithm 1 and Algorithm 2; element entry as in eq. (sum_int)
 * of section 5.1), specialised to one scalar unknown (N_E = 1) and a convection-diffusion-
 * reaction form:
 *
 *   A[i][j] = sum_q w_q detJ_q [ sum_kl K_kl d_k phi_i d_l phi_j
 *                                + phi_i sum_k b_k d_k phi_j + c phi_i phi_j ]
 *   b[i]    = sum_q w_q detJ_q f phi_i
 *
 * Conventions (readings where the paper is silent):
 *   reference cube [-1,1]^3; vertex v = v1 + 2 v2 + 4 v3 sits at xi = (2v1-1, 2v2-1, 2v3-1);
 *   geometry is trilinear from the 8 vertices; shape functions are tensor-product Lagrange
 *   polynomials on the p+1 Gauss-Lobatto-Legendre nodes, node i = a + n b + n^2 c (n = p+1);
 *   quadrature is the (p+1)^3 Gauss-Legendre rule, point q = q1 + n q2 + n^2 q3;
 *   J[a][b] = dx_a/dxi_b, physical gradient = J^{-T} times reference gradient;
 *   row i of A is the test function, column j the trial function.
 *
 * Coefficient records (FP64):
 *   ELEMENT mode: 14 per element = K (3x3 row-major), b (3), c, f
 *   FIELD mode:   10 per element = Q (3x3 row-major), f; plus a shared field descriptor of
 *                 7 fields x 5 modes x (a, k1, k2, k3, theta). Field s at x is
 *                 g_s(x) = sum_m a_sm sin(2 pi (k_sm . x) + theta_sm); then
 *                 K = Q diag(10^g0, 10^g1, 10^g2) Q^T, b = (g3, g4, g5), c = (1 + g6)/2.
 */
#ifndef FEM_ORACLE_H
#define FEM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_COEF_ELEMENT 0
#define ORACLE_COEF_FIELD 1
#define ORACLE_COEF_ELASTIC 2 /* prisms: the elastostatics of section 5.1, records [5] */
#define ORACLE_FLAG_DETJ 1     /* detJ <= 0 at one or more quadrature points */
#define ORACLE_FLAG_NONFINITE 2 /* non-finite input or output */

/* Gauss-Legendre rule with n points on [-1,1], ascending. Returns 0, or -1 if n < 1 or n > 64. */
int oracle_gauss_legendre(int n, double *x, double *w);

/* The p+1 Gauss-Lobatto-Legendre nodes on [-1,1], ascending. Returns 0, or -1 if p < 1 or p > 63. */
int oracle_gll_nodes(int p, double *x);

/* Values and first derivatives at x of the n Lagrange polynomials on the given nodes. */
void oracle_lagrange(int n, const double *nodes, double x, double *val, double *der);

/* The 7 field values g_s at point x (FIELD mode descriptor layout above). */
void oracle_field_eval(const double *field, const double *x, double *g);

/* Integrate nel elements.
 *   p        uniform degree 1..7, used when degree == NULL
 *   degree   per-element degree (1..7) or NULL
 *   geom     [nel][8][3]
 *   coef     [nel][14] (ELEMENT) or [nel][10] (FIELD)
 *   field    175 doubles, FIELD mode only
 *   a_off    [nel+1] element offsets into out_A, or NULL for e * Ns^2 (uniform p only)
 *   b_off    [nel+1] element offsets into out_b, or NULL for e * Ns (uniform p only)
 *   out_A    row-major Ns x Ns per element
 *   out_b    Ns per element, may be NULL
 *   flags    [nel] ORACLE_FLAG_* bits per element, may be NULL
 *   nthreads OpenMP threads, 0 = the runtime default
 * Returns 0, or -1 on an argument error (nothing is written). */
int oracle_integrate(int64_t nel, int p, const int8_t *degree, const double *geom, int mode,
                     const double *coef, const double *field, const int64_t *a_off,
                     const int64_t *b_off, double *out_A, double *out_b, int32_t *flags,
                     int nthreads);

/* Linear elastostatics (section 5.1, eq. (sum_int) with the isotropic tensor c_ijkl of the
 * element's Young modulus and Poisson ratio), uniform degree p = 1..7.
 *   coef   [nel][5] = E, nu, f1, f2, f3 (body force, constant per element)
 *   out_A  [nel][3][3][Ns][Ns]: block (i, k) couples test component i with trial component k,
 *          entry [s][r] = sum_q c_ijkl (d phi_r/d x_l)(d phi_s/d x_j) detJ w_q
 *   out_b  [nel][3][Ns]: b[i][s] = sum_q f_i phi_s detJ w_q, may be NULL
 *   flags  as for oracle_integrate, may be NULL
 * Returns 0, or -1 on an argument error. */
int oracle_integrate_elastic(int64_t nel, int p, const double *geom, const double *coef,
                             double *out_A, double *out_b, int32_t *flags, int nthreads);

/* Jacobian terms of the NOJAC variant (section 4: the determinant and the 9 entries of the
 * inverse Jacobian for every element and quadrature point, supplied instead of recomputed):
 *   out[q][0] = detJ(xi_q), out[q][1 + 3a + b] = (J^{-1})[a][b], J[a][b] = dx_a / dxi_b, for
 *   q = q1 + n q2 + n^2 q3 of the element's Gauss-Legendre rule. Element e's Nq = Ns records start
 *   at out + 10 * (degree ? b_off[e] : e * Ns); degree == NULL selects the uniform p.
 * Returns 0, or -1 on an argument error. */
int oracle_jacobian_terms(int64_t nel, int p, const int8_t *degree, const int64_t *b_off,
                          const double *geom, double *out, int nthreads);

/* oracle_integrate with the Jacobian terms read from jac (layout of oracle_jacobian_terms;
 * mixed degree then needs b_off even without out_b) instead of computed from the vertices.
 * geom supplies x_q in FIELD mode and may be NULL in ELEMENT mode. */
int oracle_integrate_nojac(int64_t nel, int p, const int8_t *degree, const double *jac,
                           const double *geom, int mode, const double *coef, const double *field,
                           const int64_t *a_off, const int64_t *b_off, double *out_A,
                           double *out_b, int32_t *flags, int nthreads);

/* oracle_integrate_elastic with the Jacobian terms read from jac ([nel][Ns][10]). */
int oracle_integrate_elastic_nojac(int64_t nel, int p, const double *jac, const double *coef,
                                   double *out_A, double *out_b, int32_t *flags, int nthreads);

/* ---- prismatic elements (fem_oracle_prism.c; the reference element of section 2, Tables 1-2) ----
 * Reference prism T x [-1,1] (T the unit right triangle), vertices v = t + 3h (triangle vertex t at
 * (0,0), (1,0), (0,1); h = 0 bottom, zeta = -1; h = 1 top), geometry linear in the triangle and in
 * zeta. Shape function i = t + Nt c: Lagrange basis of the degree-p polynomials on the triangle's
 * principal lattice (node t = (a/p, b/p), a + b <= p, b outer, a inner) times the 1-D Lagrange
 * polynomial of GLL node c in zeta; Ns = (p+1)^2 (p+2)/2. Quadrature point q = qt + ntq qz: the
 * caller's triangle rule tri[ntq][3] = (xi1, xi2, weight) times the (p+1)-point Gauss-Legendre
 * rule in zeta. */

/* Ns of the degree-p prism, or -1. */
int oracle_prism_ns(int p);

/* phi[i][0..3] = value and reference derivatives (d/dxi1, d/dxi2, d/dzeta) of every prism shape
 * function at one point. Returns 0, or -1 on a bad argument. */
int oracle_prism_shape(int p, double xi1, double xi2, double zeta, double *phi);

/* Integrate nel prisms of degree p (Algorithm 2 of section 2, eq. (sum_int) of section 5.1).
 *   geom  [nel][6][3]
 *   mode  ORACLE_COEF_ELEMENT (coef [nel][14]), ORACLE_COEF_FIELD (coef [nel][10], field [175])
 *         or ORACLE_COEF_ELASTIC (coef [nel][5] = E, nu, f1, f2, f3)
 *   out_A [nel][Ns][Ns] (elastostatics: [nel][3][3][Ns][Ns], block (i, k) = test component i,
 *         trial component k); out_b [nel][Ns] ([nel][3][Ns]), may be NULL
 * Returns 0, or -1 on an argument error. */
int oracle_integrate_prism(int64_t nel, int p, const double *geom, int mode, const double *coef,
                           const double *field, int ntq, const double *tri, double *out_A,
                           double *out_b, int32_t *flags, int nthreads);

/* Number of OpenMP threads a call with nthreads = 0 uses. */
int oracle_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif
