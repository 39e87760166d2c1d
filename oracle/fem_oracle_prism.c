/*
 * fem_oracle_prism.c -- FP64 CPU oracle for prismatic elements (declarations in fem_oracle.h).
 *
 * TEST INFRASTRUCTURE: only the tests, the package's smoke check and the benchmark's CPU-baseline
 * leg load this code; it shares nothing with the GPU library.
 *
 * The element is the paper's reference element of section 2 (Tables 1 and 2): a prism whose
 * shape functions are products of the complete polynomials of degree p on the triangle and the
 * 1-D polynomials of degree p in the vertical direction, integrated with a Gaussian rule. Readings
 * where the paper is silent:
 *   reference prism  T x [-1,1], T = {xi1 >= 0, xi2 >= 0, xi1 + xi2 <= 1};
 *   vertices         v = t + 3 h: triangle vertex t at (0,0), (1,0), (0,1), h = 0 at zeta = -1,
 *                    h = 1 at zeta = +1; geometry x = sum_v lambda_t(xi) (1 + (2h-1) zeta)/2 X_v
 *                    with barycentrics lambda = (1 - xi1 - xi2, xi1, xi2);
 *   shape functions  i = t + Nt c (Nt = (p+1)(p+2)/2): the Lagrange basis of the degree-p
 *                    polynomials on the triangle's principal lattice (a/p, b/p), a + b <= p,
 *                    t enumerated with b outer and a inner, times the 1-D Lagrange polynomial of
 *                    GLL node c in zeta;
 *   quadrature       q = qt + NTQ qz: a fully symmetric triangle rule of degree 2p with NTQ points
 *                    (Table 1's N_Q / (p+1): 3, 6, 12, 16, 25, 33, 42), supplied by the caller,
 *                    times the (p+1)-point Gauss-Legendre rule in zeta.
 * Each element follows Algorithm 2 of section 2 (quadrature points outermost), with the element
 * entry of eq. (sum_int) of section 5.1: the convection-diffusion-reaction form of fem_oracle.c or
 * the isotropic elastostatics of section 5.1.
 */
#include "fem_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PR_MAX_P 7
#define PR_MAX_T 36   /* triangle nodes at p = 7 */
#define PR_MAX_N 8    /* GLL nodes at p = 7 */
#define PR_MAX_NS (PR_MAX_T * PR_MAX_N)
#define PR_MAX_TQ 64

int oracle_prism_ns(int p) { return (p < 1 || p > PR_MAX_P) ? -1 : (p + 1) * (p + 1) * (p + 2) / 2; }

/* Monomial m <-> (m1, m2), m1 + m2 <= p, m2 outer; the lattice node t <-> (a, b) likewise. */
static void lattice_index(int p, int t, int *a, int *b)
{
    int k = 0;
    for (int bb = 0; bb <= p; ++bb)
        for (int aa = 0; aa + bb <= p; ++aa, ++k)
            if (k == t) {
                *a = aa;
                *b = bb;
                return;
            }
}

/* Coefficients of the triangle's Lagrange basis in the centred monomials u^m1 v^m2,
 * u = 3 xi1 - 1, v = 3 xi2 - 1 (centred on the triangle's centroid, so that the Vandermonde
 * matrix stays well conditioned up to p = 7): C[m][t] with phi_t = sum_m C[m][t] u^m1 v^m2,
 * i.e. C = V^{-1} for V[t][m] = (node t)^m, by Gauss-Jordan elimination with partial pivoting in
 * extended precision. Returns 0, or -1 for a singular matrix. */
static int triangle_coefficients(int p, long double C[PR_MAX_T][PR_MAX_T])
{
    const int nt = (p + 1) * (p + 2) / 2;
    long double M[PR_MAX_T][2 * PR_MAX_T];
    for (int t = 0; t < nt; ++t) {
        int a = 0, b = 0;
        lattice_index(p, t, &a, &b);
        const long double u = 3.0L * a / p - 1.0L, v = 3.0L * b / p - 1.0L;
        for (int m = 0; m < nt; ++m) {
            int m1 = 0, m2 = 0;
            lattice_index(p, m, &m1, &m2);
            M[t][m] = powl(u, m1) * powl(v, m2);
            M[t][nt + m] = (t == m) ? 1.0L : 0.0L;
        }
    }
    for (int col = 0; col < nt; ++col) {
        int piv = col;
        for (int r = col + 1; r < nt; ++r)
            if (fabsl(M[r][col]) > fabsl(M[piv][col]))
                piv = r;
        if (M[piv][col] == 0.0L)
            return -1;
        if (piv != col)
            for (int k = 0; k < 2 * nt; ++k) {
                long double tmp = M[col][k];
                M[col][k] = M[piv][k];
                M[piv][k] = tmp;
            }
        const long double d = M[col][col];
        for (int k = 0; k < 2 * nt; ++k)
            M[col][k] /= d;
        for (int r = 0; r < nt; ++r) {
            if (r == col || M[r][col] == 0.0L)
                continue;
            const long double f = M[r][col];
            for (int k = 0; k < 2 * nt; ++k)
                M[r][k] -= f * M[col][k];
        }
    }
    /* rows of M's right half hold V^{-1}[m][t] */
    for (int m = 0; m < nt; ++m)
        for (int t = 0; t < nt; ++t)
            C[m][t] = M[m][nt + t];
    return 0;
}

/* Values and first derivatives (d/dxi1, d/dxi2) of the triangle basis at (x, y), summed in
 * extended precision and rounded once. */
static void triangle_eval(int p, long double C[PR_MAX_T][PR_MAX_T], double x, double y,
                          double *val, double *dx, double *dy)
{
    const int nt = (p + 1) * (p + 2) / 2;
    long double sv[PR_MAX_T], sx[PR_MAX_T], sy[PR_MAX_T];
    for (int t = 0; t < nt; ++t)
        sv[t] = sx[t] = sy[t] = 0.0L;
    const long double u = 3.0L * x - 1.0L, v = 3.0L * y - 1.0L;
    for (int m = 0; m < nt; ++m) {
        int m1 = 0, m2 = 0;
        lattice_index(p, m, &m1, &m2);
        const long double mv = powl(u, m1) * powl(v, m2);
        const long double mx = m1 ? 3.0L * m1 * powl(u, m1 - 1) * powl(v, m2) : 0.0L;
        const long double my = m2 ? 3.0L * m2 * powl(u, m1) * powl(v, m2 - 1) : 0.0L;
        for (int t = 0; t < nt; ++t) {
            sv[t] += C[m][t] * mv;
            sx[t] += C[m][t] * mx;
            sy[t] += C[m][t] * my;
        }
    }
    for (int t = 0; t < nt; ++t) {
        val[t] = (double)sv[t];
        dx[t] = (double)sx[t];
        dy[t] = (double)sy[t];
    }
}

/* phi[i][0..3] = (phi_i, d/dxi1, d/dxi2, d/dzeta) of the prism basis at one point, given the
 * triangle basis coefficients and the GLL nodes. */
static void prism_shape(int p, long double C[PR_MAX_T][PR_MAX_T], const double *gll, double x, double y,
                        double z, double (*phi)[4])
{
    const int nt = (p + 1) * (p + 2) / 2, n = p + 1;
    double T[PR_MAX_T], Tx[PR_MAX_T], Ty[PR_MAX_T], L[PR_MAX_N], D[PR_MAX_N];
    triangle_eval(p, C, x, y, T, Tx, Ty);
    oracle_lagrange(n, gll, z, L, D);
    for (int c = 0; c < n; ++c)
        for (int t = 0; t < nt; ++t) {
            const int i = t + nt * c;
            phi[i][0] = T[t] * L[c];
            phi[i][1] = Tx[t] * L[c];
            phi[i][2] = Ty[t] * L[c];
            phi[i][3] = T[t] * D[c];
        }
}

int oracle_prism_shape(int p, double xi1, double xi2, double zeta, double *phi)
{
    if (p < 1 || p > PR_MAX_P || !phi)
        return -1;
    long double C[PR_MAX_T][PR_MAX_T];
    double gll[PR_MAX_N];
    if (triangle_coefficients(p, C) != 0)
        return -1;
    oracle_gll_nodes(p, gll);
    prism_shape(p, C, gll, xi1, xi2, zeta, (double (*)[4])phi);
    return 0;
}

/* The prism map at (xi1, xi2, zeta): position x, Jacobian J[a][b] = dx_a / dxi_b (xi_3 = zeta),
 * determinant and inverse (adjugate / det). X is the element's [6][3] vertex array. */
static void prism_jacobian(const double *X, double x1, double x2, double z, double *x,
                           double J[3][3], double *det, double Ji[3][3])
{
    const double lam[3] = {1.0 - x1 - x2, x1, x2};
    const double dl1[3] = {-1.0, 1.0, 0.0}, dl2[3] = {-1.0, 0.0, 1.0};
    for (int a = 0; a < 3; ++a) {
        x[a] = 0.0;
        for (int b = 0; b < 3; ++b)
            J[a][b] = 0.0;
    }
    for (int h = 0; h < 2; ++h) {
        const double s = h ? 1.0 : -1.0;
        const double fz = 0.5 * (1.0 + s * z);
        for (int t = 0; t < 3; ++t) {
            const int v = t + 3 * h;
            const double Nv = lam[t] * fz;
            const double dN[3] = {dl1[t] * fz, dl2[t] * fz, lam[t] * 0.5 * s};
            for (int a = 0; a < 3; ++a) {
                x[a] += X[v * 3 + a] * Nv;
                for (int b = 0; b < 3; ++b)
                    J[a][b] += X[v * 3 + a] * dN[b];
            }
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

/* Point coefficients of the scalar form (as in fem_oracle.c): K row-major, b, c, f. */
static void prism_point_coefficients(int mode, const double *rec, const double *field,
                                     const double *xq, double *K, double *bv, double *c, double *f)
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
    const double lam[3] = {pow(10.0, g[0]), pow(10.0, g[1]), pow(10.0, g[2])};
    for (int r = 0; r < 3; ++r)
        for (int s = 0; s < 3; ++s) {
            double acc = 0.0;
            for (int t = 0; t < 3; ++t)
                acc += rec[r * 3 + t] * lam[t] * rec[s * 3 + t];
            K[r * 3 + s] = acc;
        }
    bv[0] = g[3];
    bv[1] = g[4];
    bv[2] = g[5];
    *c = 0.5 * (1.0 + g[6]);
    *f = rec[9];
}

/* One prism (Algorithm 2): A and b of the scalar form, or the 3 x 3 block matrix
 * A[i][k][s][r] and b[i][s] of elastostatics (mode ORACLE_COEF_ELASTIC). Returns flag bits. */
static int prism_one(int p, const double *X, int mode, const double *rec, const double *field,
                     int ntq, const double *tri, double *A, double *bvec)
{
    const int n = p + 1, nt = (p + 1) * (p + 2) / 2, ns = nt * n;
    const int nblk = mode == ORACLE_COEF_ELASTIC ? 9 : 1, ncomp = mode == ORACLE_COEF_ELASTIC ? 3 : 1;
    long double C[PR_MAX_T][PR_MAX_T];
    double gll[PR_MAX_N], gx[PR_MAX_N], gw[PR_MAX_N];
    double phi[PR_MAX_NS][4], psi[PR_MAX_NS][4];
    int flags = 0;

    triangle_coefficients(p, C);
    oracle_gll_nodes(p, gll);
    oracle_gauss_legendre(n, gx, gw);
    for (int t = 0; t < 18; ++t)
        if (!isfinite(X[t]))
            flags |= ORACLE_FLAG_NONFINITE;

    double cel[3][3][3][3];
    if (mode == ORACLE_COEF_ELASTIC) {
        const double E = rec[0], nu = rec[1];
        const double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), mu = E / (2.0 * (1.0 + nu));
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                for (int k = 0; k < 3; ++k)
                    for (int l = 0; l < 3; ++l)
                        cel[i][j][k][l] = lam * (i == j) * (k == l) + mu * ((i == k) * (j == l) + (i == l) * (j == k));
    }

    memset(A, 0, sizeof(double) * nblk * (size_t)ns * ns);
    if (bvec)
        memset(bvec, 0, sizeof(double) * ncomp * (size_t)ns);

    for (int qz = 0; qz < n; ++qz)
        for (int qt = 0; qt < ntq; ++qt) {
            const double x1 = tri[3 * qt], x2 = tri[3 * qt + 1], z = gx[qz];
            const double wq = tri[3 * qt + 2] * gw[qz];

            /* reference values and derivatives phi^Q[i_Q] */
            prism_shape(p, C, gll, x1, x2, z, phi);

            /* Jacobian, determinant and inverse of the prism map */
            double J[3][3], Ji[3][3], det, xq[3];
            prism_jacobian(X, x1, x2, z, xq, J, &det, Ji);
            if (!(det > 0.0))
                flags |= ORACLE_FLAG_DETJ;

            /* physical derivatives psi^Q[i_Q]: d_k phi = sum_m (J^{-1})_{mk} d phi / d xi_m */
            for (int i = 0; i < ns; ++i) {
                psi[i][0] = phi[i][0];
                for (int k = 0; k < 3; ++k)
                    psi[i][1 + k] = Ji[0][k] * phi[i][1] + Ji[1][k] * phi[i][2] + Ji[2][k] * phi[i][3];
            }
            const double dw = det * wq;

            if (mode == ORACLE_COEF_ELASTIC) {
                for (int i = 0; i < 3; ++i)
                    for (int k = 0; k < 3; ++k) {
                        double *blk = A + (size_t)(3 * i + k) * ns * ns;
                        for (int s = 0; s < ns; ++s)
                            for (int r = 0; r < ns; ++r) {
                                double t = 0.0;
                                for (int j = 0; j < 3; ++j)
                                    for (int l = 0; l < 3; ++l)
                                        t += cel[i][j][k][l] * psi[r][1 + l] * psi[s][1 + j];
                                blk[(size_t)s * ns + r] += dw * t;
                            }
                    }
                if (bvec)
                    for (int i = 0; i < 3; ++i)
                        for (int s = 0; s < ns; ++s)
                            bvec[(size_t)i * ns + s] += dw * rec[2 + i] * psi[s][0];
                continue;
            }

            /* coefficients at the point, c^Q[i_Q], then every entry (i_DOF, j_DOF) */
            double K[9], bv[3], cc, ff;
            prism_point_coefficients(mode, rec, field, xq, K, bv, &cc, &ff);
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

    for (size_t t = 0; t < (size_t)nblk * ns * ns; ++t)
        if (!isfinite(A[t]))
            flags |= ORACLE_FLAG_NONFINITE;
    return flags;
}

int oracle_integrate_prism(int64_t nel, int p, const double *geom, int mode, const double *coef,
                           const double *field, int ntq, const double *tri, double *out_A,
                           double *out_b, int32_t *flags, int nthreads)
{
    if (nel < 0 || p < 1 || p > PR_MAX_P)
        return -1;
    if (mode != ORACLE_COEF_ELEMENT && mode != ORACLE_COEF_FIELD && mode != ORACLE_COEF_ELASTIC)
        return -1;
    if (ntq < 1 || ntq > PR_MAX_TQ || !tri)
        return -1;
    if (nel == 0)
        return 0;
    if (!geom || !coef || !out_A || (mode == ORACLE_COEF_FIELD && !field))
        return -1;
    {
        long double C[PR_MAX_T][PR_MAX_T];
        if (triangle_coefficients(p, C) != 0)
            return -1;
    }
    const int64_t ns = oracle_prism_ns(p);
    const int rec_len = mode == ORACLE_COEF_ELEMENT ? 14 : (mode == ORACLE_COEF_FIELD ? 10 : 5);
    const int64_t nblk = mode == ORACLE_COEF_ELASTIC ? 9 : 1, ncomp = mode == ORACLE_COEF_ELASTIC ? 3 : 1;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t e = 0; e < nel; ++e) {
        const int fl = prism_one(p, geom + e * 18, mode, coef + e * rec_len, field, ntq, tri,
                                 out_A + e * nblk * ns * ns, out_b ? out_b + e * ncomp * ns : NULL);
        if (flags)
            flags[e] = fl;
    }
    return 0;
}
