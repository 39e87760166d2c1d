/*
 * fem_oracle.c -- FP64 CPU oracle for element integration (declarations and conventions in
 * fem_oracle.h).
 *
 * TEST INFRASTRUCTURE: only the tests, the package's smoke check and the benchmark's
 * CPU-baseline leg load this code. It is deliberately plain: one element at a time, loops in
 * the order of Algorithm 2 (quadrature points outermost, section 2), no blocking, no fusion,
 * no precomputed tables shared between elements, OpenMP over elements only (the CPU
 * parallelisation the paper measures against, section 5.2).
 */
#include "fem_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAX_N 8 /* p <= 7 */
#define MAX_NS (MAX_N * MAX_N * MAX_N)

/* Legendre polynomial P_n(x) and P_{n-1}(x) by the three-term recurrence
 * (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}. */
static void legendre_pair(int n, double x, double *pn, double *pnm1)
{
    double p0 = 1.0, p1 = x;
    if (n == 0) {
        *pn = 1.0;
        *pnm1 = 0.0;
        return;
    }
    for (int k = 1; k < n; ++k) {
        double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
    }
    *pn = p1;
    *pnm1 = p0;
}

/* Quadrature points and weights xi^Q, w^Q (section 2). The paper asks for a Gaussian rule; the
 * reading used here is Gauss-Legendre with n = p+1 points per direction. Roots of P_n by Newton
 * from x0 = cos(pi (k - 1/4) / (n + 1/2)); weight 2 / ((1 - x^2) P_n'(x)^2). */
int oracle_gauss_legendre(int n, double *x, double *w)
{
    if (n < 1 || n > 64)
        return -1;
    for (int k = 1; k <= n; ++k) {
        double r = cos(M_PI * (k - 0.25) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double pn, pnm1;
            legendre_pair(n, r, &pn, &pnm1);
            dp = n * (r * pn - pnm1) / (r * r - 1.0);
            double dx = pn / dp;
            r -= dx;
            if (fabs(dx) < 1e-16)
                break;
        }
        {
            double pn, pnm1;
            legendre_pair(n, r, &pn, &pnm1);
            dp = n * (r * pn - pnm1) / (r * r - 1.0);
        }
        /* k = 1 gives the largest root: store descending from the top, i.e. ascending. */
        x[n - k] = r;
        w[n - k] = 2.0 / ((1.0 - r * r) * dp * dp);
    }
    return 0;
}

/* Gauss-Lobatto-Legendre nodes: -1, the p-1 roots of P_p', +1. Newton on P_p' with
 * P_p'' = (2 x P_p' - p(p+1) P_p) / (1 - x^2), started from the Chebyshev-Gauss-Lobatto points. */
int oracle_gll_nodes(int p, double *x)
{
    if (p < 1 || p > 63)
        return -1;
    x[0] = -1.0;
    x[p] = 1.0;
    for (int k = 1; k < p; ++k) {
        double r = -cos(M_PI * k / p);
        for (int it = 0; it < 100; ++it) {
            double pn, pnm1;
            legendre_pair(p, r, &pn, &pnm1);
            double d1 = p * (r * pn - pnm1) / (r * r - 1.0);
            double d2 = (2.0 * r * d1 - p * (p + 1.0) * pn) / (1.0 - r * r);
            double dx = d1 / d2;
            r -= dx;
            if (fabs(dx) < 1e-16)
                break;
        }
        x[k] = r;
    }
    return 0;
}

/* Lagrange polynomials l_a(x) = prod_{b != a} (x - x_b)/(x_a - x_b) and their derivatives
 * l_a'(x) = sum_{m != a} 1/(x_a - x_m) prod_{b != a, m} (x - x_b)/(x_a - x_b). */
void oracle_lagrange(int n, const double *nodes, double x, double *val, double *der)
{
    for (int a = 0; a < n; ++a) {
        double v = 1.0;
        for (int b = 0; b < n; ++b)
            if (b != a)
                v *= (x - nodes[b]) / (nodes[a] - nodes[b]);
        val[a] = v;
        double d = 0.0;
        for (int m = 0; m < n; ++m) {
            if (m == a)
                continue;
            double t = 1.0 / (nodes[a] - nodes[m]);
            for (int b = 0; b < n; ++b)
                if (b != a && b != m)
                    t *= (x - nodes[b]) / (nodes[a] - nodes[b]);
            d += t;
        }
        der[a] = d;
    }
}

/* g_s(x) = sum_m a_sm sin(2 pi (k_sm . x) + theta_sm), s = 0..6, m = 0..4. */
void oracle_field_eval(const double *field, const double *x, double *g)
{
    for (int s = 0; s < 7; ++s) {
        double acc = 0.0;
        for (int m = 0; m < 5; ++m) {
            const double *md = field + (s * 5 + m) * 5;
            double arg = 2.0 * M_PI * (md[1] * x[0] + md[2] * x[1] + md[3] * x[2]) + md[4];
            acc += md[0] * sin(arg);
        }
        g[s] = acc;
    }
}

/* The problem-dependent coefficients at one quadrature point (Algorithm 2, the step that forms
 * c^Q[i_Q] from c). Out: K row-major 3x3, b, c, f. */
static void point_coefficients(int mode, const double *rec, const double *field, const double *xq,
                               double *K, double *bv, double *c, double *f)
{
    if (mode == ORACLE_COEF_ELEMENT) {
        for (int t = 0; t < 9; ++t)
            K[t] = rec[t];
        for (int t = 0; t < 3; ++t)
            bv[t] = rec[9 + t];
        *c = rec[12];
        *f = rec[13];
        return;
    }
    double g[7];
    oracle_field_eval(field, xq, g);
    double lam[3] = {pow(10.0, g[0]), pow(10.0, g[1]), pow(10.0, g[2])};
    const double *Q = rec;
    for (int r = 0; r < 3; ++r)
        for (int s = 0; s < 3; ++s) {
            double acc = 0.0;
            for (int t = 0; t < 3; ++t)
                acc += Q[r * 3 + t] * lam[t] * Q[s * 3 + t];
            K[r * 3 + s] = acc;
        }
    bv[0] = g[3];
    bv[1] = g[4];
    bv[2] = g[5];
    *c = 0.5 * (1.0 + g[6]);
    *f = rec[9];
}

/* The trilinear map at xi: position x, Jacobian J[a][b] = dx_a / dxi_b, determinant and inverse
 * (adjugate / det). X is the element's [8][3] vertex array. */
static void trilinear_jacobian(const double *X, const double *xi, double *x, double J[3][3],
                               double *det, double Ji[3][3])
{
    for (int a = 0; a < 3; ++a) {
        x[a] = 0.0;
        for (int b = 0; b < 3; ++b)
            J[a][b] = 0.0;
    }
    for (int v = 0; v < 8; ++v) {
        const double s1 = (v & 1) ? 1.0 : -1.0;
        const double s2 = (v & 2) ? 1.0 : -1.0;
        const double s3 = (v & 4) ? 1.0 : -1.0;
        const double f1 = 1.0 + s1 * xi[0], f2 = 1.0 + s2 * xi[1], f3 = 1.0 + s3 * xi[2];
        const double Nv = f1 * f2 * f3 / 8.0;
        const double dN[3] = {s1 * f2 * f3 / 8.0, f1 * s2 * f3 / 8.0, f1 * f2 * s3 / 8.0};
        for (int a = 0; a < 3; ++a) {
            x[a] += X[v * 3 + a] * Nv;
            for (int b = 0; b < 3; ++b)
                J[a][b] += X[v * 3 + a] * dN[b];
        }
    }
    const double d = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                     J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                     J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / d;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / d;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / d;
    Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / d;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / d;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / d;
    Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / d;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / d;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / d;
    *det = d;
}

/* The Jacobian terms (detJ and J^{-1}) at point q = q1 + n q2 + n^2 q3 with coordinates xi:
 * computed from the vertices X when jt == NULL, else read from jt[q][0] (detJ) and jt[q][1..9]
 * (J^{-1} row-major). xq receives the physical point when X is given (zeros otherwise).
 * Returns ORACLE_FLAG_* bits for the point. */
static int point_jacobian(const double *X, const double *jt, int q, const double *xi, double *xq,
                          double *det, double Ji[3][3])
{
    int flags = 0;
    double J[3][3];
    xq[0] = xq[1] = xq[2] = 0.0;
    if (X)
        trilinear_jacobian(X, xi, xq, J, det, Ji);
    if (jt) {
        const double *r = jt + (size_t)q * 10;
        *det = r[0];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                Ji[a][b] = r[1 + 3 * a + b];
        for (int t = 0; t < 10; ++t)
            if (!isfinite(r[t]))
                flags |= ORACLE_FLAG_NONFINITE;
    }
    if (!(*det > 0.0))
        flags |= ORACLE_FLAG_DETJ;
    return flags;
}

/* One element, following Algorithm 2 of section 2: read coefficients and geometry, zero A^e,
 * then for each quadrature point read the reference shape functions, compute the Jacobian, its
 * determinant and inverse, the physical derivatives psi, the point coefficients, and update every
 * (i, j) entry. Returns ORACLE_FLAG_* bits.
 * With jt != NULL (the NOJAC variant of section 4) the determinant and inverse at point q are
 * read from jt[q][0] and jt[q][1..9] (J^{-1} row-major) instead; X then only supplies the
 * physical point x_q for FIELD mode and may be NULL otherwise. */
static int integrate_one(int p, const double *X, const double *jt, int mode, const double *rec,
                         const double *field, double *A, double *bvec)
{
    const int n = p + 1;
    const int ns = n * n * n;
    double gx[MAX_N], gw[MAX_N], nodes[MAX_N];
    double L[MAX_N][MAX_N], D[MAX_N][MAX_N]; /* [point][node] */
    double phi[MAX_NS][4], psi[MAX_NS][4];
    int flags = 0;

    oracle_gauss_legendre(n, gx, gw);
    oracle_gll_nodes(p, nodes);
    for (int q = 0; q < n; ++q)
        oracle_lagrange(n, nodes, gx[q], L[q], D[q]);

    if (X)
        for (int t = 0; t < 24; ++t)
            if (!isfinite(X[t]))
                flags |= ORACLE_FLAG_NONFINITE;

    memset(A, 0, sizeof(double) * (size_t)ns * ns);
    if (bvec)
        memset(bvec, 0, sizeof(double) * (size_t)ns);

    for (int q3 = 0; q3 < n; ++q3)
        for (int q2 = 0; q2 < n; ++q2)
            for (int q1 = 0; q1 < n; ++q1) {
                const double xi[3] = {gx[q1], gx[q2], gx[q3]};
                const double wq = gw[q1] * gw[q2] * gw[q3];

                /* reference values and derivatives phi^Q[i_Q] */
                for (int c = 0; c < n; ++c)
                    for (int b = 0; b < n; ++b)
                        for (int a = 0; a < n; ++a) {
                            int i = a + n * b + n * n * c;
                            phi[i][0] = L[q1][a] * L[q2][b] * L[q3][c];
                            phi[i][1] = D[q1][a] * L[q2][b] * L[q3][c];
                            phi[i][2] = L[q1][a] * D[q2][b] * L[q3][c];
                            phi[i][3] = L[q1][a] * L[q2][b] * D[q3][c];
                        }

                /* Jacobian terms: computed from the trilinear map of the vertices, or read */
                double Ji[3][3], det, xq[3];
                flags |= point_jacobian(X, jt, q1 + n * q2 + n * n * q3, xi, xq, &det, Ji);

                /* physical derivatives psi^Q[i_Q]: d_k phi = sum_m (J^{-1})_{mk} d phi / d xi_m */
                for (int i = 0; i < ns; ++i) {
                    psi[i][0] = phi[i][0];
                    for (int k = 0; k < 3; ++k)
                        psi[i][1 + k] = Ji[0][k] * phi[i][1] + Ji[1][k] * phi[i][2] +
                                        Ji[2][k] * phi[i][3];
                }

                /* coefficients at the point, c^Q[i_Q] */
                double K[9], bv[3], cc, ff;
                point_coefficients(mode, rec, field, xq, K, bv, &cc, &ff);

                /* update every entry (i_DOF, j_DOF) with det * w * c^Q * psi * psi */
                const double dw = det * wq;
                for (int i = 0; i < ns; ++i) {
                    for (int j = 0; j < ns; ++j) {
                        double s = cc * psi[i][0] * psi[j][0];
                        for (int k = 0; k < 3; ++k)
                            s += psi[i][0] * bv[k] * psi[j][1 + k];
                        for (int k = 0; k < 3; ++k)
                            for (int l = 0; l < 3; ++l)
                                s += K[k * 3 + l] * psi[i][1 + k] * psi[j][1 + l];
                        A[(size_t)i * ns + j] += dw * s;
                    }
                    if (bvec)
                        bvec[i] += dw * ff * psi[i][0];
                }
            }

    for (size_t t = 0; t < (size_t)ns * ns; ++t)
        if (!isfinite(A[t]))
            flags |= ORACLE_FLAG_NONFINITE;
    return flags;
}

/* Element e's Jacobian terms start at jac + 10 * (b_off ? b_off[e] : e * Nq) (Nq = Ns). */
static int integrate_all(int64_t nel, int p, const int8_t *degree, const double *geom,
                         const double *jac, int mode, const double *coef, const double *field,
                         const int64_t *a_off, const int64_t *b_off, double *out_A, double *out_b,
                         int32_t *flags, int nthreads)
{
    if (nel < 0)
        return -1;
    if (nel == 0)
        return 0;
    if (!coef || !out_A || (!geom && !jac))
        return -1;
    if (mode != ORACLE_COEF_ELEMENT && mode != ORACLE_COEF_FIELD)
        return -1;
    if (mode == ORACLE_COEF_FIELD && (!field || !geom))
        return -1;
    if (degree) {
        if (!a_off || ((out_b || jac) && !b_off))
            return -1;
        for (int64_t e = 0; e < nel; ++e)
            if (degree[e] < 1 || degree[e] > 7)
                return -1;
    } else if (p < 1 || p > 7) {
        return -1;
    }
    const int rec_len = (mode == ORACLE_COEF_ELEMENT) ? 14 : 10;

#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t e = 0; e < nel; ++e) {
        const int pe = degree ? degree[e] : p;
        const int64_t ns = (int64_t)(pe + 1) * (pe + 1) * (pe + 1);
        const int64_t ao = a_off ? a_off[e] : e * ns * ns;
        const int64_t bo = b_off ? b_off[e] : e * ns;
        int fl = integrate_one(pe, geom ? geom + e * 24 : NULL, jac ? jac + 10 * bo : NULL, mode,
                               coef + e * rec_len, field, out_A + ao, out_b ? out_b + bo : NULL);
        if (flags)
            flags[e] = fl;
    }
    return 0;
}

int oracle_integrate(int64_t nel, int p, const int8_t *degree, const double *geom, int mode,
                     const double *coef, const double *field, const int64_t *a_off,
                     const int64_t *b_off, double *out_A, double *out_b, int32_t *flags,
                     int nthreads)
{
    if (nel > 0 && !geom)
        return -1;
    return integrate_all(nel, p, degree, geom, NULL, mode, coef, field, a_off, b_off, out_A, out_b,
                         flags, nthreads);
}

int oracle_integrate_nojac(int64_t nel, int p, const int8_t *degree, const double *jac,
                           const double *geom, int mode, const double *coef, const double *field,
                           const int64_t *a_off, const int64_t *b_off, double *out_A,
                           double *out_b, int32_t *flags, int nthreads)
{
    if (nel > 0 && !jac)
        return -1;
    return integrate_all(nel, p, degree, geom, jac, mode, coef, field, a_off, b_off, out_A, out_b,
                         flags, nthreads);
}

int oracle_jacobian_terms(int64_t nel, int p, const int8_t *degree, const int64_t *b_off,
                          const double *geom, double *out, int nthreads)
{
    if (nel < 0)
        return -1;
    if (nel == 0)
        return 0;
    if (!geom || !out || (degree && !b_off) || (!degree && (p < 1 || p > 7)))
        return -1;
    if (degree)
        for (int64_t e = 0; e < nel; ++e)
            if (degree[e] < 1 || degree[e] > 7)
                return -1;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t e = 0; e < nel; ++e) {
        const int n = (degree ? degree[e] : p) + 1;
        const int64_t bo = degree ? b_off[e] : e * (int64_t)n * n * n;
        double gx[MAX_N], gw[MAX_N];
        oracle_gauss_legendre(n, gx, gw);
        for (int q3 = 0; q3 < n; ++q3)
            for (int q2 = 0; q2 < n; ++q2)
                for (int q1 = 0; q1 < n; ++q1) {
                    const double xi[3] = {gx[q1], gx[q2], gx[q3]};
                    double x[3], J[3][3], Ji[3][3], det;
                    trilinear_jacobian(geom + e * 24, xi, x, J, &det, Ji);
                    double *r = out + 10 * (bo + q1 + n * q2 + n * n * q3);
                    r[0] = det;
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b)
                            r[1 + 3 * a + b] = Ji[a][b];
                }
    }
    return 0;
}

/* ---------------------------------------------------------------------------------------------
 * Vector problem of section 5.1: linear elastostatics, d = 3 components, the same shape
 * functions for every component. Element entry (eq. (sum_int)) for test function s of
 * component i and trial function r of component k:
 *
 *   A[(i,s)][(k,r)] = sum_q c_ijkl (d phi_r / d x_l) (d phi_s / d x_j) detJ w_q
 *
 * with the isotropic tensor from the element's Young modulus E and Poisson ratio nu (the two
 * material parameters of section 5.1):
 *   lambda = E nu / ((1 + nu)(1 - 2 nu)),  mu = E / (2 (1 + nu)),
 *   c_ijkl = lambda delta_ij delta_kl + mu (delta_ik delta_jl + delta_il delta_jk).
 * Load vector (body force f, constant per element): b[(i,s)] = sum_q f_i phi_s detJ w_q.
 * ------------------------------------------------------------------------------------------- */
static int integrate_elastic_one(int p, const double *X, const double *jt, const double *rec,
                                 double *A, double *bvec)
{
    const int n = p + 1;
    const int ns = n * n * n;
    double gx[MAX_N], gw[MAX_N], nodes[MAX_N];
    double L[MAX_N][MAX_N], D[MAX_N][MAX_N]; /* [point][node] */
    double phi[MAX_NS][4], psi[MAX_NS][4];
    int flags = 0;

    oracle_gauss_legendre(n, gx, gw);
    oracle_gll_nodes(p, nodes);
    for (int q = 0; q < n; ++q)
        oracle_lagrange(n, nodes, gx[q], L[q], D[q]);
    if (X)
        for (int t = 0; t < 24; ++t)
            if (!isfinite(X[t]))
                flags |= ORACLE_FLAG_NONFINITE;

    const double E = rec[0], nu = rec[1];
    const double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    const double mu = E / (2.0 * (1.0 + nu));
    double c[3][3][3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l)
                    c[i][j][k][l] = lam * (i == j) * (k == l) + mu * ((i == k) * (j == l) + (i == l) * (j == k));

    memset(A, 0, sizeof(double) * 9 * (size_t)ns * ns);
    if (bvec)
        memset(bvec, 0, sizeof(double) * 3 * (size_t)ns);

    for (int q3 = 0; q3 < n; ++q3)
        for (int q2 = 0; q2 < n; ++q2)
            for (int q1 = 0; q1 < n; ++q1) {
                const double xi[3] = {gx[q1], gx[q2], gx[q3]};
                const double wq = gw[q1] * gw[q2] * gw[q3];
                for (int cc = 0; cc < n; ++cc)
                    for (int bb = 0; bb < n; ++bb)
                        for (int aa = 0; aa < n; ++aa) {
                            int r = aa + n * bb + n * n * cc;
                            phi[r][0] = L[q1][aa] * L[q2][bb] * L[q3][cc];
                            phi[r][1] = D[q1][aa] * L[q2][bb] * L[q3][cc];
                            phi[r][2] = L[q1][aa] * D[q2][bb] * L[q3][cc];
                            phi[r][3] = L[q1][aa] * L[q2][bb] * D[q3][cc];
                        }
                double Ji[3][3], det, xq[3];
                flags |= point_jacobian(X, jt, q1 + n * q2 + n * n * q3, xi, xq, &det, Ji);
                /* d phi / d x_l = sum_m (d phi / d xi_m)(d xi_m / d x_l), a column of J^{-1} */
                for (int r = 0; r < ns; ++r) {
                    psi[r][0] = phi[r][0];
                    for (int l = 0; l < 3; ++l)
                        psi[r][1 + l] = Ji[0][l] * phi[r][1] + Ji[1][l] * phi[r][2] + Ji[2][l] * phi[r][3];
                }
                const double dw = det * wq;
                for (int i = 0; i < 3; ++i)
                    for (int k = 0; k < 3; ++k) {
                        double *blk = A + (size_t)(3 * i + k) * ns * ns;
                        for (int s = 0; s < ns; ++s)
                            for (int r = 0; r < ns; ++r) {
                                double t = 0.0;
                                for (int j = 0; j < 3; ++j)
                                    for (int l = 0; l < 3; ++l)
                                        t += c[i][j][k][l] * psi[r][1 + l] * psi[s][1 + j];
                                blk[(size_t)s * ns + r] += dw * t;
                            }
                    }
                if (bvec)
                    for (int i = 0; i < 3; ++i)
                        for (int s = 0; s < ns; ++s)
                            bvec[(size_t)i * ns + s] += dw * rec[2 + i] * psi[s][0];
            }
    for (size_t t = 0; t < 9 * (size_t)ns * ns; ++t)
        if (!isfinite(A[t]))
            flags |= ORACLE_FLAG_NONFINITE;
    return flags;
}

static int integrate_elastic_all(int64_t nel, int p, const double *geom, const double *jac,
                                 const double *coef, double *out_A, double *out_b, int32_t *flags,
                                 int nthreads)
{
    if (nel < 0)
        return -1;
    if (nel == 0)
        return 0;
    if ((!geom && !jac) || !coef || !out_A || p < 1 || p > 7)
        return -1;
    const int64_t ns = (int64_t)(p + 1) * (p + 1) * (p + 1);
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t e = 0; e < nel; ++e) {
        int fl = integrate_elastic_one(p, geom ? geom + e * 24 : NULL, jac ? jac + e * 10 * ns : NULL,
                                       coef + e * 5, out_A + e * 9 * ns * ns,
                                       out_b ? out_b + e * 3 * ns : NULL);
        if (flags)
            flags[e] = fl;
    }
    return 0;
}

int oracle_integrate_elastic(int64_t nel, int p, const double *geom, const double *coef,
                             double *out_A, double *out_b, int32_t *flags, int nthreads)
{
    if (nel > 0 && !geom)
        return -1;
    return integrate_elastic_all(nel, p, geom, NULL, coef, out_A, out_b, flags, nthreads);
}

int oracle_integrate_elastic_nojac(int64_t nel, int p, const double *jac, const double *coef,
                                   double *out_A, double *out_b, int32_t *flags, int nthreads)
{
    if (nel > 0 && !jac)
        return -1;
    return integrate_elastic_all(nel, p, NULL, jac, coef, out_A, out_b, flags, nthreads);
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
