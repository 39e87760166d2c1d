// fem_trilinear.h -- trilinear hexahedra (p = 1) on the vector ALU.
//
// At p = 1 an element has 8 shape functions and 8 Gauss points, so the contraction of section 2
// (A = B^T blockdiag(Dh_q) B) is only 8 x 8 x 32 per element: far too small to feed the matrix
// cores, while the element's memory traffic (a 304-byte input record, 64 + 8 output values) is
// what bounds the launch. Here eight lanes own one element and a wave owns eight elements:
//
//   1. the element's 8 lanes read its vertex coordinates and coefficient record side by side
//      (one contiguous 192-byte and one 112-byte record per element);
//   2. lane k forms the subset-k coefficients of the trilinear form and then, at Gauss point
//      k = k1 + 2 k2 + 4 k3, the Jacobian terms and the folded point matrix
//      Dh_k = w_k detJ_k G^T D G (FP64, the same functions and formulas as the tile kernels),
//      and w_k detJ_k f;
//      Still as point k it forms, for every row i, u_s(k, i) = sum_r B[(k, r)][i] Dh_k[r][s]
//      and hands the 4-vectors over through the wave's LDS;
//   3. lane k, now the owner of row k of A (owner computes, section 4.1), sums the 8 points:
//      A_kj = sum_q sum_s u_s(q, k) B[(q, s)][j], and b_k = sum_q (w detJ f)_q phi_k(xi_q) in
//      FP64, both sum-factorised over the three directions (B is a tensor product);
//   4. lane k stores row k (eight contiguous values: a wave writes its eight matrices as one
//      contiguous run) and b_k.
// A persistent wave walks over groups of eight elements and loads the next group's inputs into
// registers while it works on the current group.
//
// The reference values are those of Table 1's p = 1 element: nodes -1, +1 per direction
// (Gauss-Lobatto), Lagrange factors L_0 = (1 - xi)/2, L_1 = (1 + xi)/2, derivatives -1/2, +1/2,
// and the 2-point Gauss-Legendre rule (points -1/sqrt(3), +1/sqrt(3), weights 1). They are
// compile-time constants here; a lane selects its factors from two constants by its own bits.
//
// Only the lanes of one wave exchange data (through the wave's own LDS area), so the kernel has
// no workgroup barrier. DT is the arithmetic and output type of A: double for the FP64
// precision, float for the FP32-output precisions (FP32 products, FP32 sums). ELEMENT
// coefficients only; the Jacobian terms are computed (SUP false) or supplied (SUP true, the
// NOJAC form of section 4).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fem_geometry.h"
#include "fem_kernel.h"

namespace fem {

constexpr int TRI_WAVES = 4;            // waves per workgroup
constexpr int TRI_NT = 64 * TRI_WAVES;  // threads per workgroup
constexpr int TRI_EPW = 8;              // elements per wave

// 1/sqrt(3), the positive point of the 2-point Gauss-Legendre rule
constexpr double TRI_G = 0.57735026918962576450914878050195746;
// L_a(x_q): TRI_LA where node a and point q lie on the same side, TRI_LB otherwise
constexpr double TRI_LA = 0.5 * (1.0 + TRI_G), TRI_LB = 0.5 * (1.0 - TRI_G);
template <class DT>
struct TriWaveLds {
    union {
        struct {
            double X[TRI_EPW][8][3];  // vertex coordinates
            double rec[TRI_EPW][14];  // coefficient records
            double tc[TRI_EPW][24];   // trilinear forms
        } in;
        DT U[TRI_EPW][8][8][4];       // u_s(q, i) per element, point q and row i
    };
    double wf[TRI_EPW][8];            // w detJ f per point
};

__device__ inline void tri_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// waves per SIMD the register budget must allow, and the persistent workgroups per CU (the LDS
// of a workgroup is 34 KB with FP32 and 66 KB with FP64 u-vectors)
template <class DT> constexpr int tri_occ() { return sizeof(DT) == 4 ? 3 : 2; }

// One lane's share of an element's input: vertex k, coefficients 2k and 2k + 1, and (supplied
// terms) the 10 Jacobian terms of point k.
template <bool SUP>
struct TriIn {
    double x[3], r[2];
    double jt[SUP ? 10 : 1];
};

template <bool SUP>
__device__ inline void tri_fetch(const KArgs &a, int64_t e, bool valid, int k, TriIn<SUP> &in)
{
    if (!valid) return;
    if constexpr (SUP) {
        const double *jt = a.jac + ((a.b_off ? a.b_off[e] : e * 8) + k) * 10;
#pragma unroll
        for (int t = 0; t < 10; ++t) in.jt[t] = jt[t];
    } else {
        const double *g = a.geom + e * 24 + 3 * k;
        in.x[0] = g[0];
        in.x[1] = g[1];
        in.x[2] = g[2];
    }
    if (k < 7) {
        const double *r = a.elem + e * 14 + 2 * k;
        in.r[0] = r[0];
        in.r[1] = r[1];
    }
}

template <class DT, bool SUP>
__device__ inline void tri_group(const KArgs &a, TriWaveLds<DT> &L, int el, int k, int64_t e, bool valid,
                                 const TriIn<SUP> &in)
{
    // 1. the element's vertices and coefficient record into the wave's LDS
    if (valid) {
        if constexpr (!SUP) {
            L.in.X[el][k][0] = in.x[0];
            L.in.X[el][k][1] = in.x[1];
            L.in.X[el][k][2] = in.x[2];
        }
        if (k < 7) {
            L.in.rec[el][2 * k] = in.r[0];
            L.in.rec[el][2 * k + 1] = in.r[1];
        }
    }
    tri_wave_sync();

    // 2. Jacobian terms and the point matrix at Gauss point k
    constexpr double G = TRI_G;
    const double x1 = (k & 1) ? G : -G, x2 = (k & 2) ? G : -G, x3 = (k & 4) ? G : -G;
    const double w = 1.0;
    double Ji[3][3], det;
    if constexpr (SUP) {
        det = in.jt[0];
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
            for (int n = 0; n < 3; ++n) Ji[m][n] = in.jt[1 + 3 * m + n];
    } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) L.in.tc[el][c * 8 + k] = trilinear_coeff(&L.in.X[el][0][0], c, k);
        tri_wave_sync();
        det = jacobian_terms(L.in.tc[el], x1, x2, x3, Ji);
    }
    const double *rec = L.in.rec[el];
    double K[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int s = 0; s < 3; ++s) K[r][s] = rec[r * 3 + s];
    const double bv[3] = {rec[9], rec[10], rec[11]};
    const double cc = rec[12], ff = rec[13];
    const double wd = w * det;
    bool finite = isfinite(wd * ff);
    double dh[13];
    // row 0: Dh[0][0] = wd c, Dh[0][1+n] = wd (J^{-1} b)_n; rows 1..3: wd (J^{-1} K J^{-T})
    dh[0] = wd * cc;
#pragma unroll
    for (int n = 0; n < 3; ++n) dh[1 + n] = wd * (Ji[n][0] * bv[0] + Ji[n][1] * bv[1] + Ji[n][2] * bv[2]);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const double T0 = Ji[m][0] * K[0][0] + Ji[m][1] * K[1][0] + Ji[m][2] * K[2][0];
        const double T1 = Ji[m][0] * K[0][1] + Ji[m][1] * K[1][1] + Ji[m][2] * K[2][1];
        const double T2 = Ji[m][0] * K[0][2] + Ji[m][1] * K[1][2] + Ji[m][2] * K[2][2];
#pragma unroll
        for (int n = 0; n < 3; ++n) dh[4 + 3 * m + n] = wd * (T0 * Ji[n][0] + T1 * Ji[n][1] + T2 * Ji[n][2]);
    }
    DT d[13];
#pragma unroll
    for (int u = 0; u < 13; ++u) {
        finite = finite && isfinite(dh[u]);
        d[u] = DT(dh[u]);
    }
    // per-element flags: detJ <= 0 (or NaN) and non-finite terms at any of its points
    const uint64_t bad_det = __ballot(valid && !(det > 0.0));
    const uint64_t bad_val = __ballot(valid && !finite);
    constexpr double LA = TRI_LA, LB = TRI_LB;
    tri_wave_sync();  // every lane is done with the coordinates and records (U overlays them)
    L.wf[el][k] = wd * ff;
    // u_s(k, i) = sum_r B[(k, r)][i] Dh_k[r][s], every row i, by the tensor-product structure:
    // B[(k, 0)][i] = l_1(i_1) l_2(i_2) l_3(i_3) with l_d(a) = LA where node side a and point
    // side k_d agree, LB otherwise; B[(k, d)][i] has sg(i_d) = -+1/2 in place of l_d(i_d). So
    // u_0(i) = Dh[0][0] P(i) and u_s(i) = Dh[0][s] P(i) + sum_d sg(i_d) Dh[d][s] Q_d(i without
    // i_d), P = l_1 l_2 l_3 and Q_d the product of the other two factors.
    typedef DT dt4 __attribute__((ext_vector_type(4)));
    dt4 uo[8];  // u(k, i), i = 0..7
    {
        DT l[3][2];
#pragma unroll
        for (int dd = 0; dd < 3; ++dd) {
            const bool kd = (k >> dd) & 1;
            l[dd][0] = DT(kd ? LB : LA);
            l[dd][1] = DT(kd ? LA : LB);
        }
        DT Q1[2][2], Q2[2][2], Q3[2][2];  // Q1[i2][i3], Q2[i1][i3], Q3[i1][i2]
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                Q1[x][y] = l[1][x] * l[2][y];
                Q2[x][y] = l[0][x] * l[2][y];
                Q3[x][y] = l[0][x] * l[1][y];
            }
        // half of Dh[d][s] (d, s = 1..3): the +-1/2 of B[(k, d)] becomes the sign of the term
        DT h[3][3];
#pragma unroll
        for (int dd = 0; dd < 3; ++dd)
#pragma unroll
            for (int n = 0; n < 3; ++n) h[dd][n] = DT(0.5) * d[4 + 3 * dd + n];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int i1 = i & 1, i2 = (i >> 1) & 1, i3 = i >> 2;
            const DT P = l[0][i1] * Q1[i2][i3];
            dt4 &u = uo[i];
            u[0] = d[0] * P;
#pragma unroll
            for (int n = 0; n < 3; ++n) {
                DT v = d[1 + n] * P;
                v += (i1 ? h[0][n] : -h[0][n]) * Q1[i2][i3];
                v += (i2 ? h[1][n] : -h[1][n]) * Q2[i1][i3];
                v += (i3 ? h[2][n] : -h[2][n]) * Q3[i1][i2];
                u[1 + n] = v;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) *reinterpret_cast<dt4 *>(L.U[el][k][i]) = uo[i];
    tri_wave_sync();
    // row k gathers u(q, k) of the 8 points
    dt4 u[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) u[q] = *reinterpret_cast<const dt4 *>(L.U[el][q][k]);

    // 3. row k: A_kj = sum_q sum_s u_s(q, k) B[(q, s)][j], sum-factorised over the three
    // directions (L(a, x) = LA where node side a and point side x agree, LB otherwise):
    //   s = 0: three passes, each replacing a point index by a node index;
    //   s = d: the sum over q_d first (B[(q, d)][j] carries sg(j_d), not a factor of q_d), two
    //   passes over the other directions, then acc[j] += sg(j_d) W.
    // b_k = sum_q (w detJ f)_q phi_k(xi_q) in FP64, sum-factorised the same way.
    DT acc[8];
    double bk;
    {
        const DT A_ = DT(LA), B_ = DT(LB);
        auto Lf = [&](int a, int x) { return a == x ? A_ : B_; };
        // s = 0: u[q1 + 2 q2 + 4 q3][0]
        DT t1[2][2][2], t2[2][2][2];  // t1[j1][q2][q3], t2[j1][j2][q3]
#pragma unroll
        for (int j1 = 0; j1 < 2; ++j1)
#pragma unroll
            for (int q2 = 0; q2 < 2; ++q2)
#pragma unroll
                for (int q3 = 0; q3 < 2; ++q3)
                    t1[j1][q2][q3] = Lf(j1, 0) * u[2 * q2 + 4 * q3][0] + Lf(j1, 1) * u[1 + 2 * q2 + 4 * q3][0];
#pragma unroll
        for (int j1 = 0; j1 < 2; ++j1)
#pragma unroll
            for (int j2 = 0; j2 < 2; ++j2)
#pragma unroll
                for (int q3 = 0; q3 < 2; ++q3)
                    t2[j1][j2][q3] = Lf(j2, 0) * t1[j1][0][q3] + Lf(j2, 1) * t1[j1][1][q3];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int j1 = j & 1, j2 = (j >> 1) & 1, j3 = j >> 2;
            acc[j] = Lf(j3, 0) * t2[j1][j2][0] + Lf(j3, 1) * t2[j1][j2][1];
        }
        // s = d + 1: V over the two other directions (e, f) of the sum over q_d, then two passes
#pragma unroll
        for (int dd = 0; dd < 3; ++dd) {
            const int e = dd == 0 ? 1 : 0, f = dd == 2 ? 1 : 2;  // the other directions, e < f
            DT V[2][2], W1[2][2], W[2][2];                      // [x_e][x_f]
#pragma unroll
            for (int xe = 0; xe < 2; ++xe)
#pragma unroll
                for (int xf = 0; xf < 2; ++xf) {
                    const int q0 = (xe << e) | (xf << f);
                    V[xe][xf] = u[q0][1 + dd] + u[q0 | (1 << dd)][1 + dd];
                }
#pragma unroll
            for (int je = 0; je < 2; ++je)
#pragma unroll
                for (int xf = 0; xf < 2; ++xf) W1[je][xf] = Lf(je, 0) * V[0][xf] + Lf(je, 1) * V[1][xf];
#pragma unroll
            for (int je = 0; je < 2; ++je)
#pragma unroll
                for (int jf = 0; jf < 2; ++jf) W[je][jf] = Lf(jf, 0) * W1[je][0] + Lf(jf, 1) * W1[je][1];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int jd = (j >> dd) & 1, je = (j >> e) & 1, jf = (j >> f) & 1;
                acc[j] += DT(jd ? 0.5 : -0.5) * W[je][jf];
            }
        }
        // b_k: the lane's node sides k_d pick L(k_d, .) per direction
        double lk[3][2];
#pragma unroll
        for (int dd = 0; dd < 3; ++dd) {
            const bool kd = (k >> dd) & 1;
            lk[dd][0] = kd ? LB : LA;
            lk[dd][1] = kd ? LA : LB;
        }
        const double *wf = L.wf[el];
        double c1[4];  // [q2 + 2 q3]
#pragma unroll
        for (int r = 0; r < 4; ++r) c1[r] = lk[0][0] * wf[2 * r] + lk[0][1] * wf[2 * r + 1];
        const double c2a = lk[1][0] * c1[0] + lk[1][1] * c1[1], c2b = lk[1][0] * c1[2] + lk[1][1] * c1[3];
        bk = lk[2][0] * c2a + lk[2][1] * c2b;
    }

    // 4. row k of A and b_k
    if (valid) {
        DT *outA = reinterpret_cast<DT *>(a.out_A) + (a.a_off ? a.a_off[e] : a.a_base + e * a.a_stride) + k * 8;
        if ((reinterpret_cast<uintptr_t>(outA) & 15) == 0) {
            typedef DT dt4 __attribute__((ext_vector_type(4)));
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const dt4 v = {acc[4 * h], acc[4 * h + 1], acc[4 * h + 2], acc[4 * h + 3]};
                *reinterpret_cast<dt4 *>(outA + 4 * h) = v;
            }
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) outA[j] = acc[j];
        }
        if (a.out_b) {
            DT *outb = reinterpret_cast<DT *>(a.out_b) + (a.b_off ? a.b_off[e] : a.b_base + e * a.b_stride);
            outb[k] = DT(bk);
        }
        if (a.status && k == 0) {
            if ((bad_det >> (8 * el)) & 0xffu) atomicAdd(&a.status[0], 1);
            if ((bad_val >> (8 * el)) & 0xffu) atomicAdd(&a.status[1], 1);
        }
    }
    tri_wave_sync();  // the next group rewrites the wave's LDS
}

// Persistent grid: wave w of the grid takes the element groups (of 8) w, w + W, w + 2W, ...;
// the inputs of its next group are loaded while it works on the current one.
template <class DT, bool SUP>
__global__ void __launch_bounds__(TRI_NT) __attribute__((amdgpu_waves_per_eu(tri_occ<DT>(), 8)))
k_trilinear(KArgs a)
{
    __shared__ TriWaveLds<DT> lds[TRI_WAVES];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int el = lane >> 3, k = lane & 7;
    int64_t nel = a.nel;
    const int32_t *elist = a.elist;
    if (a.seg) {
        elist = a.elist + a.seg[0];
        nel = a.seg[1];
    }
    const int64_t ngroups = (nel + TRI_EPW - 1) / TRI_EPW;
    const int64_t gstride = int64_t(gridDim.x) * TRI_WAVES;
    int64_t grp = int64_t(blockIdx.x) * TRI_WAVES + wv;
    if (grp >= ngroups) return;  // the whole wave has no group
    auto locate = [&](int64_t g, int64_t &e) {
        const int64_t idx = g * TRI_EPW + el;
        const bool v = idx < nel;
        e = v ? element_id(elist, idx) : 0;
        return v;
    };
    TriIn<SUP> cur{}, nxt{};
    int64_t e, en = 0;
    bool valid = locate(grp, e), vn = false;
    tri_fetch<SUP>(a, e, valid, k, cur);
    for (;;) {
        const int64_t gn = grp + gstride;
        const bool more = gn < ngroups;
        if (more) {
            vn = locate(gn, en);
            tri_fetch<SUP>(a, en, vn, k, nxt);
        }
        tri_group<DT, SUP>(a, lds[wv], el, k, e, valid, cur);
        if (!more) break;
        grp = gn;
        e = en;
        valid = vn;
        cur = nxt;
    }
}

// Launch over a.nel elements (exact, or an upper bound when a.seg supplies the count): at most
// the workgroups the device holds at once (tri_occ per CU).
template <class DT>
hipError_t launch_trilinear(const KArgs &a, hipStream_t s, int cus)
{
    if (a.mode != 0) return hipErrorInvalidValue;
    const int64_t per = int64_t(TRI_WAVES) * TRI_EPW;
    const int64_t need = (a.nel + per - 1) / per, cap = int64_t(cus) * tri_occ<DT>();
    const int64_t grid = need < cap ? need : cap;
    if (grid <= 0) return hipSuccess;
    if (a.jac)
        hipLaunchKernelGGL((k_trilinear<DT, true>), dim3((unsigned)grid), dim3(TRI_NT), 0, s, a);
    else
        hipLaunchKernelGGL((k_trilinear<DT, false>), dim3((unsigned)grid), dim3(TRI_NT), 0, s, a);
    return hipGetLastError();
}

}  // namespace fem
