// fem_prism_tables.cpp -- FP64 reference tables of the prism (the reference element of section 2
// of the paper, Tables 1-2), built once in fem_init (see fem_tables.h).
//
// Element: triangle T = {xi1, xi2 >= 0, xi1 + xi2 <= 1} times zeta in [-1, 1]. Shape function
// i = t + Nt c is the Lagrange polynomial of triangle-lattice node t = (a/p, b/p) (b outer, a
// inner) times the 1-D Lagrange polynomial of GLL node c. Quadrature point q = qt + NTQ qz: a fully
// symmetric degree-2p triangle rule with the point counts of Table 1 times the (p+1)-point
// Gauss-Legendre rule in zeta.
#include <algorithm>
#include <cmath>
#include <vector>

#include "fem_layout.h"
#include "fem_tables.h"

namespace fem {

namespace {

// Orbits of the symmetric triangle rules: kind 0 the centroid (weight w), kind 1 the three
// points with barycentrics (a, a, 1 - 2a), kind 2 the six with (a, b, 1 - a - b). The values start
// the refinement and pick which of the rules of that degree and size is meant.
struct Orbit {
    int kind;
    double w, a, b;
};
const std::vector<Orbit> &rule_seeds(int p)
{
    static const std::vector<Orbit> s[8] = {
        {},
        {{1, 0.16667, 0.16667, 0}},
        {{1, 0.1117, 0.4459, 0}, {1, 0.05498, 0.09158, 0}},
        {{1, 0.08567, 0.2194, 0}, {1, 0.04037, 0.4801, 0}, {2, 0.02032, 0.01937, 0.8390}},
        {{0, 0.07216, 0, 0}, {1, 0.01623, 0.05055, 0}, {1, 0.04755, 0.4593, 0},
         {1, 0.05161, 0.1706, 0}, {2, 0.01362, 0.008395, 0.7285}},
        {{0, 0.04087, 0, 0}, {1, 0.02298, 0.1422, 0}, {1, 0.006676, 0.03206, 0},
         {2, 0.01709, 0.02962, 0.6012}, {2, 0.01265, 0.1637, 0.02837}, {2, 0.03195, 0.3218, 0.1481}},
        {{1, 0.02185, 0.4397, 0}, {1, 0.03143, 0.2712, 0}, {1, 0.003083, 0.02132, 0},
         {1, 0.01287, 0.4882, 0}, {1, 0.0174, 0.1276, 0}, {2, 0.01118, 0.02284, 0.2813},
         {2, 0.02019, 0.1153, 0.2757}, {2, 0.008658, 0.02573, 0.1163}},
        {{1, 0.01094, 0.4890, 0}, {1, 0.002462, 0.01939, 0}, {1, 0.01639, 0.4176, 0},
         {1, 0.02108, 0.1772, 0}, {1, 0.007217, 0.0618, 0}, {1, 0.02589, 0.2735, 0},
         {2, 0.01929, 0.09292, 0.3369}, {2, 0.01233, 0.05712, 0.1723},
         {2, 0.002505, 0.001268, 0.119}, {2, 0.007218, 0.01465, 0.2984}},
    };
    return s[p];
}

int orbit_params(int kind) { return kind == 0 ? 1 : (kind == 1 ? 2 : 3); }

// Points (xi1, xi2) = (lambda1, lambda2) of the rule for parameters th (orbit by orbit:
// w, then a, then b) and d(xi1, xi2)/d(th) as dense rows.
void expand_rule(const std::vector<Orbit> &orb, const std::vector<double> &th, std::vector<double> &x,
                 std::vector<double> &y, std::vector<double> &w, std::vector<int> &owner,
                 std::vector<double> &dxa, std::vector<double> &dya, std::vector<double> &dxb,
                 std::vector<double> &dyb)
{
    x.clear(); y.clear(); w.clear(); owner.clear(); dxa.clear(); dya.clear(); dxb.clear(); dyb.clear();
    int k = 0;
    for (size_t o = 0; o < orb.size(); ++o) {
        const int kind = orb[o].kind;
        auto add = [&](double px, double py, double ax, double ay, double bx, double by) {
            x.push_back(px); y.push_back(py); w.push_back(th[k]); owner.push_back(k);
            dxa.push_back(ax); dya.push_back(ay); dxb.push_back(bx); dyb.push_back(by);
        };
        if (kind == 0) {
            add(1.0 / 3.0, 1.0 / 3.0, 0, 0, 0, 0);
        } else if (kind == 1) {
            const double a = th[k + 1], c = 1.0 - 2.0 * a;
            add(a, c, 1, -2, 0, 0);
            add(c, a, -2, 1, 0, 0);
            add(a, a, 1, 1, 0, 0);
        } else {
            const double a = th[k + 1], b = th[k + 2], c = 1.0 - a - b;
            // (lambda1, lambda2) over the six arrangements of (a, b, c); d/da and d/db of each
            const double v[3] = {a, b, c};
            const double da[3] = {1, 0, -1}, db[3] = {0, 1, -1};
            const int pr[6][2] = {{1, 2}, {2, 1}, {0, 2}, {2, 0}, {0, 1}, {1, 0}};
            for (int s = 0; s < 6; ++s)
                add(v[pr[s][0]], v[pr[s][1]], da[pr[s][0]], da[pr[s][1]], db[pr[s][0]], db[pr[s][1]]);
        }
        k += orbit_params(kind);
    }
}

// Jacobi polynomials P_n^{(al, 0)}(t), n = 0..N, and their derivatives, by the three-term
// recurrence (and its derivative).
void jacobi(int N, double al, double t, double *P, double *D)
{
    P[0] = 1.0;
    D[0] = 0.0;
    if (N == 0) return;
    P[1] = 0.5 * ((al + 2.0) * t + al);
    D[1] = 0.5 * (al + 2.0);
    for (int n = 2; n <= N; ++n) {
        const double a1 = 2.0 * n * (n + al) * (2.0 * n + al - 2.0);
        const double a2 = (2.0 * n + al - 1.0) * al * al;
        const double a3 = (2.0 * n + al - 2.0) * (2.0 * n + al - 1.0) * (2.0 * n + al);
        const double a4 = 2.0 * (n + al - 1.0) * (n - 1.0) * (2.0 * n + al);
        P[n] = ((a2 + a3 * t) * P[n - 1] - a4 * P[n - 2]) / a1;
        D[n] = (a3 * P[n - 1] + (a2 + a3 * t) * D[n - 1] - a4 * D[n - 2]) / a1;
    }
}

// The orthogonal (Proriol-Koornwinder-Dubiner) polynomials psi_mn, m + n <= d, on the triangle
// and their gradients at (x, y): psi_mn = q_m(u, v) P_n^{(2m+1, 0)}(2y - 1) with u = 2x - 1 + y,
// v = 1 - y and q_m(u, v) = v^m P_m(u / v) (q_0 = 1, q_1 = u, (m+1) q_{m+1} = (2m+1) u q_m -
// m v^2 q_{m-1}). They integrate to 1/2 (m = n = 0) and to 0 otherwise.
void orthogonal_basis(int d, double x, double y, std::vector<double> &f, std::vector<double> &fx,
                      std::vector<double> &fy)
{
    const double u = 2.0 * x - 1.0 + y, v = 1.0 - y;
    std::vector<double> q(d + 1), qx(d + 1), qy(d + 1);
    q[0] = 1.0; qx[0] = 0.0; qy[0] = 0.0;
    if (d >= 1) { q[1] = u; qx[1] = 2.0; qy[1] = 1.0; }
    for (int m = 1; m < d; ++m) {
        q[m + 1] = ((2 * m + 1) * u * q[m] - m * v * v * q[m - 1]) / (m + 1);
        qx[m + 1] = ((2 * m + 1) * (2.0 * q[m] + u * qx[m]) - m * v * v * qx[m - 1]) / (m + 1);
        qy[m + 1] = ((2 * m + 1) * (q[m] + u * qy[m]) - m * (-2.0 * v * q[m - 1] + v * v * qy[m - 1])) / (m + 1);
    }
    f.clear(); fx.clear(); fy.clear();
    std::vector<double> P(d + 1), D(d + 1);
    for (int m = 0; m <= d; ++m) {
        jacobi(d - m, 2.0 * m + 1.0, 2.0 * y - 1.0, P.data(), D.data());
        for (int n = 0; n + m <= d; ++n) {
            f.push_back(q[m] * P[n]);
            fx.push_back(qx[m] * P[n]);
            fy.push_back(qy[m] * P[n] + q[m] * 2.0 * D[n]);
        }
    }
}

// Solve the dense system M z = r (n x n, row-major) by Gaussian elimination with partial
// pivoting; false if singular.
bool solve_dense(int n, std::vector<double> M, std::vector<double> &r)
{
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int i = c + 1; i < n; ++i)
            if (std::fabs(M[i * n + c]) > std::fabs(M[piv * n + c])) piv = i;
        if (M[piv * n + c] == 0.0) return false;
        if (piv != c) {
            for (int k = 0; k < n; ++k) std::swap(M[c * n + k], M[piv * n + k]);
            std::swap(r[c], r[piv]);
        }
        for (int i = c + 1; i < n; ++i) {
            const double f = M[i * n + c] / M[c * n + c];
            if (f == 0.0) continue;
            for (int k = c; k < n; ++k) M[i * n + k] -= f * M[c * n + k];
            r[i] -= f * r[c];
        }
    }
    for (int c = n - 1; c >= 0; --c) {
        double s = r[c];
        for (int k = c + 1; k < n; ++k) s -= M[c * n + k] * r[k];
        r[c] = s / M[c * n + c];
    }
    return true;
}

// Silvester's factor R_m(l) = prod_{k < m} (p l - k) / (k + 1) and its derivative.
void silvester(int m, int p, double l, double &R, double &dR)
{
    R = 1.0;
    dR = 0.0;
    for (int k = 0; k < m; ++k) {
        const double f = (p * l - k) / (k + 1), df = double(p) / (k + 1);
        dR = dR * f + R * df;
        R *= f;
    }
}

}  // namespace

bool prism_triangle_rule(int p, std::vector<double> &x, std::vector<double> &y, std::vector<double> &w)
{
    if (p < 1 || p > 7) return false;
    const std::vector<Orbit> &orb = rule_seeds(p);
    std::vector<double> th;
    for (const Orbit &o : orb) {
        th.push_back(o.w);
        if (o.kind >= 1) th.push_back(o.a);
        if (o.kind == 2) th.push_back(o.b);
    }
    const int nth = int(th.size()), d = 2 * p;
    std::vector<int> owner;
    std::vector<double> dxa, dya, dxb, dyb, f, fx, fy;
    double resid = 1.0;
    for (int it = 0; it < 50; ++it) {
        expand_rule(orb, th, x, y, w, owner, dxa, dya, dxb, dyb);
        // residuals r_j = sum_k w_k psi_j(x_k) - int psi_j and the Jacobian d r_j / d th
        std::vector<double> r, J;
        for (size_t k = 0; k < x.size(); ++k) {
            orthogonal_basis(d, x[k], y[k], f, fx, fy);
            if (r.empty()) {
                r.assign(f.size(), 0.0);
                J.assign(f.size() * nth, 0.0);
            }
            const int o = owner[k];
            for (size_t j = 0; j < f.size(); ++j) {
                r[j] += w[k] * f[j];
                J[j * nth + o] += f[j];
                if (o + 1 < nth && (dxa[k] != 0.0 || dya[k] != 0.0))
                    J[j * nth + o + 1] += w[k] * (fx[j] * dxa[k] + fy[j] * dya[k]);
                if (o + 2 < nth && (dxb[k] != 0.0 || dyb[k] != 0.0))
                    J[j * nth + o + 2] += w[k] * (fx[j] * dxb[k] + fy[j] * dyb[k]);
            }
        }
        r[0] -= 0.5;
        resid = 0.0;
        for (double v : r) resid = std::max(resid, std::fabs(v));
        // Gauss-Newton step from the normal equations J^T J s = -J^T r
        std::vector<double> N(size_t(nth) * nth, 0.0), g(nth, 0.0);
        for (size_t j = 0; j < r.size(); ++j)
            for (int a = 0; a < nth; ++a) {
                g[a] -= J[j * nth + a] * r[j];
                for (int b = 0; b < nth; ++b) N[a * nth + b] += J[j * nth + a] * J[j * nth + b];
            }
        if (!solve_dense(nth, N, g)) return false;
        double smax = 0.0;
        for (int a = 0; a < nth; ++a) {
            th[a] += g[a];
            smax = std::max(smax, std::fabs(g[a]));
        }
        if (smax < 1e-16 && resid < 1e-14) break;
    }
    expand_rule(orb, th, x, y, w, owner, dxa, dya, dxb, dyb);
    if (int(x.size()) != prism_tri_points(p) || resid > 1e-13) return false;
    for (size_t k = 0; k < x.size(); ++k)
        if (!(w[k] > 0.0 && x[k] > 0.0 && y[k] > 0.0 && x[k] + y[k] < 1.0)) return false;
    return true;
}

bool make_prism_tables(int p, HostPrismTables &t)
{
    if (p < 1 || p > 7) return false;
    t.p = p;
    t.n = p + 1;
    t.nt = (p + 1) * (p + 2) / 2;
    t.ns = t.nt * t.n;
    t.ntq = prism_tri_points(p);
    t.nq = t.ntq * t.n;
    std::vector<double> tx, ty, tw;
    if (!prism_triangle_rule(p, tx, ty, tw)) return false;
    // vertical factors: Gauss-Legendre points and the GLL Lagrange values / derivatives there
    const HostDegreeTables line = make_degree_tables(p);
    // triangle factors at the triangle points: Silvester products over the barycentrics
    std::vector<double> T(size_t(t.ntq) * t.nt), T1(T.size()), T2(T.size());
    for (int qt = 0; qt < t.ntq; ++qt) {
        const double l1 = tx[qt], l2 = ty[qt], l0 = 1.0 - l1 - l2;
        int node = 0;
        for (int b = 0; b <= p; ++b)
            for (int a = 0; a + b <= p; ++a, ++node) {
                double Ra, dRa, Rb, dRb, Rc, dRc;
                silvester(a, p, l1, Ra, dRa);
                silvester(b, p, l2, Rb, dRb);
                silvester(p - a - b, p, l0, Rc, dRc);
                const size_t k = size_t(qt) * t.nt + node;
                T[k] = Ra * Rb * Rc;
                T1[k] = dRa * Rb * Rc - Ra * Rb * dRc;  // d lambda0 / d xi1 = -1
                T2[k] = Ra * dRb * Rc - Ra * Rb * dRc;
            }
    }
    t.pts.assign(size_t(t.nq) * 4, 0.0);
    t.B.assign(size_t(t.nq) * 4 * t.ns, 0.0);
    t.phi.assign(size_t(t.nq) * t.ns, 0.0);
    double bmax = 0.0;
    for (int qz = 0; qz < t.n; ++qz)
        for (int qt = 0; qt < t.ntq; ++qt) {
            const int q = qt + t.ntq * qz;
            t.pts[q * 4 + 0] = tx[qt];
            t.pts[q * 4 + 1] = ty[qt];
            t.pts[q * 4 + 2] = line.xq[qz];
            t.pts[q * 4 + 3] = tw[qt] * line.wq[qz];
            double *row = &t.B[size_t(q) * 4 * t.ns];
            for (int c = 0; c < t.n; ++c) {
                const double L = line.L[qz * t.n + c], D = line.D[qz * t.n + c];
                for (int tt = 0; tt < t.nt; ++tt) {
                    const int i = tt + t.nt * c;
                    const size_t k = size_t(qt) * t.nt + tt;
                    row[0 * t.ns + i] = T[k] * L;
                    row[1 * t.ns + i] = T1[k] * L;
                    row[2 * t.ns + i] = T2[k] * L;
                    row[3 * t.ns + i] = T[k] * D;
                    t.phi[size_t(q) * t.ns + i] = T[k] * L;
                    bmax = std::max(bmax, std::fabs(row[i]) + std::fabs(row[t.ns + i]) +
                                              std::fabs(row[2 * t.ns + i]) + std::fabs(row[3 * t.ns + i]));
                }
            }
        }
    t.bmax = bmax;
    return true;
}

}  // namespace fem
