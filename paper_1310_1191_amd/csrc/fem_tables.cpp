// fem_tables.cpp -- FP64 reference-element tables of libfem (see fem_tables.h).
#include "fem_tables.h"

#include <algorithm>
#include <cmath>

namespace fem {

namespace {

// P_n(x), P_n'(x) and P_{n-1}(x) by the upward recurrence, differentiating the recurrence
// itself: (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1},
//         (k+1) P'_{k+1} = (2k+1) (P_k + x P'_k) - k P'_{k-1}.
void legendre_with_derivative(int n, double x, double &pn, double &dpn, double &pnm1)
{
    double p_prev = 0.0, p_cur = 1.0, d_prev = 0.0, d_cur = 0.0;
    for (int k = 0; k < n; ++k) {
        const double p_next = ((2 * k + 1) * x * p_cur - k * p_prev) / (k + 1);
        const double d_next = ((2 * k + 1) * (p_cur + x * d_cur) - k * d_prev) / (k + 1);
        p_prev = p_cur;
        p_cur = p_next;
        d_prev = d_cur;
        d_cur = d_next;
    }
    pn = p_cur;
    dpn = d_cur;
    pnm1 = p_prev;
}

}  // namespace

void gauss_legendre_rule(int n, double *x, double *w)
{
    // Newton from the Chebyshev nodes cos(pi (2k+1) / (2n)); weights 2 (1-x^2) / (n P_{n-1})^2.
    for (int k = 0; k < n; ++k) {
        double r = -std::cos(M_PI * (2.0 * k + 1.0) / (2.0 * n));
        for (int it = 0; it < 64; ++it) {
            double pn, dpn, pnm1;
            legendre_with_derivative(n, r, pn, dpn, pnm1);
            const double step = pn / dpn;
            r -= step;
            if (std::fabs(step) <= 1e-17)
                break;
        }
        double pn, dpn, pnm1;
        legendre_with_derivative(n, r, pn, dpn, pnm1);
        x[k] = r;
        w[k] = 2.0 * (1.0 - r * r) / (double(n) * n * pnm1 * pnm1);
    }
    if (n % 2 == 1)
        x[n / 2] = 0.0;
    std::sort(x, x + n);  // already ascending; keeps the contract explicit
}

void lobatto_nodes(int p, double *x)
{
    // Interior nodes: roots of P_p', i.e. of the Jacobi polynomial P^{(1,1)}_{p-1}. Newton on
    // P_p' with P_p'' from the Legendre equation (1-x^2) P'' = 2 x P' - p(p+1) P, started from
    // the interior Gauss points of order p (they interlace the roots of P_p').
    x[0] = -1.0;
    x[p] = 1.0;
    if (p < 2)
        return;
    std::vector<double> g(p), gw(p);
    gauss_legendre_rule(p, g.data(), gw.data());
    for (int k = 1; k < p; ++k) {
        double r = 0.5 * (g[k - 1] + g[k]);
        for (int it = 0; it < 64; ++it) {
            double pn, dpn, pnm1;
            legendre_with_derivative(p, r, pn, dpn, pnm1);
            const double d2 = (2.0 * r * dpn - p * (p + 1.0) * pn) / (1.0 - r * r);
            const double step = dpn / d2;
            r -= step;
            if (std::fabs(step) <= 1e-17)
                break;
        }
        x[k] = r;
    }
    if (p % 2 == 0)
        x[p / 2] = 0.0;
}

HostDegreeTables make_degree_tables(int p)
{
    HostDegreeTables t;
    t.p = p;
    t.n = p + 1;
    t.ns = t.n * t.n * t.n;
    const int n = t.n;
    t.xq.resize(n);
    t.wq.resize(n);
    gauss_legendre_rule(n, t.xq.data(), t.wq.data());
    std::vector<double> nodes(n);
    lobatto_nodes(p, nodes.data());
    // Barycentric weights beta_a = 1 / prod_{b != a} (x_a - x_b); then
    // l_a(x) = beta_a prod_{b != a} (x - x_b) and l_a'(x) = beta_a sum_{m != a} prod_{b != a, m} (x - x_b).
    // (A Gauss point can coincide with a Lobatto node -- x = 0 when both counts are odd -- so no
    // 1 / (x - x_b) form is used.)
    std::vector<double> beta(n, 1.0);
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b)
            if (b != a)
                beta[a] /= (nodes[a] - nodes[b]);
    t.L.assign(n * n, 0.0);
    t.D.assign(n * n, 0.0);
    for (int q = 0; q < n; ++q) {
        const double x = t.xq[q];
        for (int a = 0; a < n; ++a) {
            double prod = beta[a];
            for (int b = 0; b < n; ++b)
                if (b != a)
                    prod *= (x - nodes[b]);
            double der = 0.0;
            for (int m = 0; m < n; ++m) {
                if (m == a)
                    continue;
                double term = beta[a];
                for (int b = 0; b < n; ++b)
                    if (b != a && b != m)
                        term *= (x - nodes[b]);
                der += term;
            }
            t.L[q * n + a] = prod;
            t.D[q * n + a] = der;
        }
    }
    std::vector<double> B = reference_operand(t);
    double bmax = 0.0;
    for (int q = 0; q < t.ns; ++q)
        for (int i = 0; i < t.ns; ++i) {
            double s = 0.0;
            for (int r = 0; r < 4; ++r)
                s += std::fabs(B[(size_t(q) * 4 + r) * t.ns + i]);
            bmax = std::max(bmax, s);
        }
    t.bmax = bmax;
    return t;
}

std::vector<double> reference_operand(const HostDegreeTables &t)
{
    const int n = t.n, ns = t.ns;
    std::vector<double> B(size_t(ns) * 4 * ns);
    for (int q = 0; q < ns; ++q) {
        const int q1 = q % n, q2 = (q / n) % n, q3 = q / (n * n);
        for (int i = 0; i < ns; ++i) {
            const int a = i % n, b = (i / n) % n, c = i / (n * n);
            const double la = t.L[q1 * n + a], lb = t.L[q2 * n + b], lc = t.L[q3 * n + c];
            const double da = t.D[q1 * n + a], db = t.D[q2 * n + b], dc = t.D[q3 * n + c];
            double *row = &B[size_t(q) * 4 * ns];
            row[0 * ns + i] = la * lb * lc;
            row[1 * ns + i] = da * lb * lc;
            row[2 * ns + i] = la * db * lc;
            row[3 * ns + i] = la * lb * dc;
        }
    }
    return B;
}

}  // namespace fem
