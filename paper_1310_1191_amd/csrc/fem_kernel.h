// fem_kernel.h -- the element-integration kernel of libfem for CDNA4 (gfx950).
//
// One launch integrates many elements of one degree p (section 4.1 of the paper: a single
// launch for a large set of elements; elements are spread over workgroups and the entries of
// A^e over threads, "owner computes", no atomics on A). Per element it evaluates Algorithm 2 of
// section 2 in the following arrangement:
//
//   prologue (FP64): trilinear Jacobian J, detJ and J^{-1} at every quadrature point, the point
//     coefficients (constant, or from the coefficient fields at x_q) and the folded 4x4 point
//     matrix  Dh_q = w_q detJ_q G^T D G,  G = blockdiag(1, J^{-T}),  D = [[c, b^T], [0, K]]
//     (rows: test value / derivatives, columns: trial); psi^Q = G phi^Q of section 2 is never
//     formed. Dh_q and w_q detJ_q f go to LDS.
//   contraction: A = B^T C with C[(q, r)][j] = sum_s Dh_q[r][s] B[(q, s)][j], a GEMM of depth
//     4 N_Q on the matrix cores. B^T comes from a constant fragment table; C is produced per
//     lane in registers from the 1-D Lagrange values L[q][a], D[q][a] (tensor-product structure
//     of B), in the slot order of fem_layout.h.
//   load vector: b_i = sum_q w_q detJ_q f phi_i(xi_q), FP64 accumulation.
//   epilogue: accumulators are scaled back (split paths) and stored unpadded, row-major.
//
// A workgroup owns one work item = (group of EG elements, row tile, column tile). The columns
// of a work item are the EG elements' trial functions side by side, NSP apart, so small
// elements (p = 1, NSP = 8) share one MFMA column block.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "fem_layout.h"

namespace fem {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// Kernel arguments (device pointers). Tables are those of the launch's degree.
struct KArgs {
    int64_t nel;             // elements in this launch
    const double *geom;      // [*][8][3]
    const double *elem;      // [*][14] (ELEMENT) or [*][10] (FIELD)
    const double *field;     // [175] (FIELD)
    const int32_t *elist;    // element ids of this launch, or null for 0..nel-1
    const int64_t *seg;      // device {start, count}: use elist + start and nel = count, or null
    const int64_t *a_off;    // [*] element offsets into out_A, or null for e * Ns^2
    const int64_t *b_off;    // [*] element offsets into out_b, or null for e * Ns
    void *out_A;
    void *out_b;             // may be null
    int32_t *status;         // [2] or null
    int32_t mode;            // 0 ELEMENT, 1 FIELD
    const double *xq, *wq;   // [n] Gauss points and weights
    const double *LD64;      // [n][n][2]: (L, D)[gauss point][node]
    const float *LD32;       // the same, rounded to FP32
    const void *row_hi;      // row-operand fragment table (fem_layout.h)
    const void *row_lo;      // second table of the split paths, else null
    float c_bound;           // split paths: 2^15 / max_{q,j} sum_r |B[(q,r)][j]|
    float row_scale_inv;     // 1 / (power-of-two scale of the row table)
};

template <int EG_, int WGM_, int WGN_, int WM_, int WN_, int OCC_ = 1>
struct Cfg {
    static constexpr int OCC = OCC_;  // waves per SIMD the register budget must allow
    static constexpr int EG = EG_;    // elements per work item
    static constexpr int WGM = WGM_;  // waves along rows
    static constexpr int WGN = WGN_;  // waves along columns
    static constexpr int WM = WM_;    // row blocks per wave
    static constexpr int WN = WN_;    // column blocks per wave
    static constexpr int NW = WGM_ * WGN_;
};

// ------------------------------------------------------------------------------------------
// compile-time shape of a (degree, precision, config) instance
// ------------------------------------------------------------------------------------------
template <int P, int PREC, class C>
struct Shape {
    static constexpr int FAM = family_of(PREC);
    static constexpr int N = P + 1, NS = N * N * N, NQ = NS;
    static constexpr int TM = fam_tm(FAM), KGP = fam_kgp(FAM), PPL = fam_ppl(FAM);
    static constexpr int SLOTS = fam_slots(FAM);
    static constexpr int NG = groups_of(P, FAM), NQP = NG * KGP;
    static constexpr int NRB = rblocks_of(P, FAM);
    static constexpr int NSP = (2 * NS <= TM) ? NS : NRB * TM;  // column pitch per element
    static constexpr int EG = C::EG;
    static_assert((EG * NSP) % TM == 0, "element group must fill whole column blocks");
    static constexpr int NCB = EG * NSP / TM;
    static constexpr int TRB = C::WGM * C::WM, TCB = C::WGN * C::WN;
    static constexpr int RT = (NRB + TRB - 1) / TRB, CT = (NCB + TCB - 1) / TCB;
    static constexpr int NT = C::NW * 64;
    static constexpr bool SPLIT = (PREC == PREC_SPLIT_BF16 || PREC == PREC_SPLIT_F16);
    using DT = typename std::conditional<PREC == PREC_F64, double, float>::type;
    static constexpr int DSTR = 16;  // LDS stride of one point matrix (13 used)

    // dynamic LDS layout (bytes)
    static constexpr size_t off_geo = 0;                                  // EG*24 double
    static constexpr size_t off_rec = off_geo + EG * 24 * 8;              // EG*14 double
    static constexpr size_t off_tc = off_rec + EG * 14 * 8;               // EG*24 double
    static constexpr size_t off_fld = off_tc + EG * 24 * 8;               // 176 double
    static constexpr size_t off_ld64 = off_fld + 176 * 8;                 // N*N*2 double
    static constexpr size_t off_ld32 = off_ld64 + N * N * 2 * 8;          // N*N*2 float (pad 2)
    static constexpr size_t off_qw = off_ld32 + ((N * N * 2 * 4 + 15) / 16) * 16;  // 2N double
    static constexpr size_t off_wf = off_qw + ((2 * N * 8 + 15) / 16) * 16;       // EG*NQP double
    static constexpr size_t off_D = off_wf + EG * NQP * 8;                         // EG*NQP*16 DT
    static constexpr size_t off_misc = off_D + size_t(EG) * NQP * DSTR * sizeof(DT);
    static constexpr size_t lds_bytes = off_misc + EG * 16;  // dmax(u32), flag(i32), sc(f32), unsc(f32)
    static constexpr int grid_per_group = RT * CT;
};

// ------------------------------------------------------------------------------------------
// helpers
// ------------------------------------------------------------------------------------------
__device__ inline int64_t element_id(const int32_t *elist, int64_t idx)
{
    return elist ? (int64_t)elist[idx] : idx;
}

// The 7 coefficient fields at x (descriptor in LDS): g_s = sum_m a sin(2 pi k.x + theta).
__device__ inline void eval_fields(const double *fld, const double x[3], double g[7])
{
#pragma unroll 1
    for (int s = 0; s < 7; ++s) {
        double acc = 0.0;
#pragma unroll 1
        for (int m = 0; m < 5; ++m) {
            const double *md = fld + (s * 5 + m) * 5;
            const double arg = 2.0 * M_PI * (md[1] * x[0] + md[2] * x[1] + md[3] * x[2]) + md[4];
            acc += md[0] * sin(arg);
        }
        g[s] = acc;
    }
}

// C values (r = 0..3) of one (point, trial function) from the folded point matrix Dh (13
// entries: row 0 = Dh[0][0..3], rows 1..3 = Dh[r][1..3]) and the 1-D factors.
template <typename T>
__device__ inline void column_values(const T *Dh, T la, T da, T lb, T db, T lc, T dc, T out[4])
{
    const T lbc = lb * lc;
    const T phi = la * lbc;
    const T d1 = da * lbc;
    const T d2 = la * db * lc;
    const T d3 = la * lb * dc;
    out[0] = Dh[0] * phi + Dh[1] * d1 + Dh[2] * d2 + Dh[3] * d3;
    out[1] = Dh[4] * d1 + Dh[5] * d2 + Dh[6] * d3;
    out[2] = Dh[7] * d1 + Dh[8] * d2 + Dh[9] * d3;
    out[3] = Dh[10] * d1 + Dh[11] * d2 + Dh[12] * d3;
}

// Fragments per precision.
template <int PREC> struct Frag;
template <> struct Frag<PREC_F64> {
    using row = f64x4; using col = f64x4; using acc = f64x4;
    static constexpr int ACC_N = 4;
};
template <> struct Frag<PREC_F32> {
    using row = f32x4; using col = f32x4; using acc = f32x16;
    static constexpr int ACC_N = 16;
};
template <> struct Frag<PREC_BF16> {
    using row = bf16x8; using col = bf16x8; using acc = f32x16;
    static constexpr int ACC_N = 16;
};
struct SplitBF { bf16x8 hi, lo; };
struct SplitH { f16x8 hi, lo; };
template <> struct Frag<PREC_SPLIT_BF16> {
    using row = SplitBF; using col = SplitBF; using acc = f32x16;
    static constexpr int ACC_N = 16;
};
template <> struct Frag<PREC_SPLIT_F16> {
    using row = SplitH; using col = SplitH; using acc = f32x16;
    static constexpr int ACC_N = 16;
};

template <int PREC>
__device__ inline typename Frag<PREC>::row load_row(const KArgs &a, size_t frag, int lane)
{
    if constexpr (PREC == PREC_F64) {
        return reinterpret_cast<const f64x4 *>(a.row_hi)[frag * 64 + lane];
    } else if constexpr (PREC == PREC_F32) {
        return reinterpret_cast<const f32x4 *>(a.row_hi)[frag * 64 + lane];
    } else if constexpr (PREC == PREC_BF16) {
        return reinterpret_cast<const bf16x8 *>(a.row_hi)[frag * 64 + lane];
    } else if constexpr (PREC == PREC_SPLIT_BF16) {
        SplitBF r;
        r.hi = reinterpret_cast<const bf16x8 *>(a.row_hi)[frag * 64 + lane];
        r.lo = reinterpret_cast<const bf16x8 *>(a.row_lo)[frag * 64 + lane];
        return r;
    } else {
        SplitH r;
        r.hi = reinterpret_cast<const f16x8 *>(a.row_hi)[frag * 64 + lane];
        r.lo = reinterpret_cast<const f16x8 *>(a.row_lo)[frag * 64 + lane];
        return r;
    }
}

// Pack the lane's slot values into the column fragment (split: x = hi + lo, both rounded to
// nearest; lo carries the rounding error of hi).
template <int PREC, typename T>
__device__ inline typename Frag<PREC>::col pack_col(const T v[])
{
    if constexpr (PREC == PREC_F64) {
        f64x4 r = {v[0], v[1], v[2], v[3]};
        return r;
    } else if constexpr (PREC == PREC_F32) {
        f32x4 r = {v[0], v[1], v[2], v[3]};
        return r;
    } else if constexpr (PREC == PREC_BF16) {
        bf16x8 r;
        for (int t = 0; t < 8; ++t) r[t] = (__bf16)v[t];
        return r;
    } else if constexpr (PREC == PREC_SPLIT_BF16) {
        SplitBF r;
        for (int t = 0; t < 8; ++t) {
            const __bf16 h = (__bf16)v[t];
            r.hi[t] = h;
            r.lo[t] = (__bf16)(v[t] - (float)h);
        }
        return r;
    } else {
        SplitH r;
        for (int t = 0; t < 8; ++t) {
            const _Float16 h = (_Float16)v[t];
            r.hi[t] = h;
            r.lo[t] = (_Float16)(v[t] - (float)h);
        }
        return r;
    }
}

template <int PREC>
__device__ inline void mma(typename Frag<PREC>::acc &c, const typename Frag<PREC>::row &a,
                           const typename Frag<PREC>::col &b)
{
    if constexpr (PREC == PREC_F64) {
#pragma unroll
        for (int s = 0; s < 4; ++s) c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b[s], c, 0, 0, 0);
    } else if constexpr (PREC == PREC_F32) {
#pragma unroll
        for (int s = 0; s < 4; ++s) c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s], b[s], c, 0, 0, 0);
    } else if constexpr (PREC == PREC_BF16) {
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    } else if constexpr (PREC == PREC_SPLIT_BF16) {
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.lo, b.hi, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.hi, b.lo, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.hi, b.hi, c, 0, 0, 0);
    } else {
        c = __builtin_amdgcn_mfma_f32_32x32x16_f16(a.lo, b.hi, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_f16(a.hi, b.lo, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_f16(a.hi, b.hi, c, 0, 0, 0);
    }
}

// Row of accumulator entry v held by `lane` (column is lane % TM). The FP64 16x16 result holds
// row lane/16 + 4v; the 32x32 FP32-accumulator results hold row 8(v/4) + 4(lane/32) + v%4.
template <int FAM>
__device__ inline int acc_row(int lane, int v)
{
    if constexpr (FAM == MF_F64) return (lane >> 4) + 4 * v;
    else return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
}

// ------------------------------------------------------------------------------------------
// the kernel
// ------------------------------------------------------------------------------------------
template <int P, int PREC, class C>
__device__ inline void integrate_item(const KArgs &a, int64_t wi, const int64_t nel,
                                      const int32_t *elist, unsigned char *smem)
{
    using S = Shape<P, PREC, C>;
    using DT = typename S::DT;
    using F = Frag<PREC>;
    constexpr int N = S::N, NS = S::NS, NQ = S::NQ, NQP = S::NQP, EG = S::EG, NT = S::NT;
    constexpr int TM = S::TM, FAM = S::FAM;

    double *s_geo = reinterpret_cast<double *>(smem + S::off_geo);
    double *s_rec = reinterpret_cast<double *>(smem + S::off_rec);
    double *s_tc = reinterpret_cast<double *>(smem + S::off_tc);
    double *s_fld = reinterpret_cast<double *>(smem + S::off_fld);
    double *s_ld64 = reinterpret_cast<double *>(smem + S::off_ld64);
    float *s_ld32 = reinterpret_cast<float *>(smem + S::off_ld32);
    double *s_qw = reinterpret_cast<double *>(smem + S::off_qw);
    double *s_wf = reinterpret_cast<double *>(smem + S::off_wf);
    DT *s_D = reinterpret_cast<DT *>(smem + S::off_D);
    unsigned *s_dmax = reinterpret_cast<unsigned *>(smem + S::off_misc);
    int *s_flag = reinterpret_cast<int *>(smem + S::off_misc + EG * 4);
    float *s_sc = reinterpret_cast<float *>(smem + S::off_misc + EG * 8);
    float *s_unsc = reinterpret_cast<float *>(smem + S::off_misc + EG * 12);

    const int tid = threadIdx.x;
    const int ct = (int)(wi % S::CT);
    wi /= S::CT;
    const int rt = (int)(wi % S::RT);
    const int64_t grp = wi / S::RT;
    const int64_t e0 = grp * EG;
    const int neg = (int)((nel - e0) < EG ? (nel - e0) : EG);
    const int reclen = a.mode == 0 ? 14 : 10;

    // ---- element data, tables and field descriptor into LDS ----
    for (int t = tid; t < EG * 24; t += NT) {
        const int el = t / 24, c = t % 24;
        s_geo[t] = el < neg ? a.geom[element_id(elist, e0 + el) * 24 + c] : 0.0;
    }
    for (int t = tid; t < EG * 14; t += NT) {
        const int el = t / 14, c = t % 14;
        s_rec[t] = (el < neg && c < reclen) ? a.elem[element_id(elist, e0 + el) * reclen + c] : 0.0;
    }
    if (a.mode == 1)
        for (int t = tid; t < 175; t += NT) s_fld[t] = a.field[t];
    for (int t = tid; t < N * N * 2; t += NT) {
        s_ld64[t] = a.LD64[t];
        s_ld32[t] = a.LD32[t];
    }
    for (int t = tid; t < N; t += NT) {
        s_qw[t] = a.xq[t];
        s_qw[N + t] = a.wq[t];
    }
    if (tid < EG) {
        s_dmax[tid] = 0u;
        s_flag[tid] = 0;
    }
    __syncthreads();

    // ---- trilinear form x(xi) = sum_S c_S prod_{d in S} xi_d, c_S = 1/8 sum_v X_v prod s_vd ----
    for (int t = tid; t < EG * 24; t += NT) {
        const int el = t / 24, coord = (t % 24) / 8, sub = t % 8;
        double acc = 0.0;
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const int neg_bits = __popc(sub & ~v);
            const double x = s_geo[el * 24 + v * 3 + coord];
            acc += (neg_bits & 1) ? -x : x;
        }
        s_tc[t] = 0.125 * acc;
    }
    __syncthreads();

    // ---- FIELD mode, pass 1: the 7 coefficient fields at x_q, staged in the point's Dh slot ----
    if (a.mode == 1) {
#pragma unroll 1
        for (int t = tid; t < EG * NQP; t += NT) {
            const int el = t / NQP, q = t % NQP;
            if (el >= neg || q >= NQ) continue;
            const int q1 = q % N, q2 = (q / N) % N, q3 = q / (N * N);
            const double x1 = s_qw[q1], x2 = s_qw[q2], x3 = s_qw[q3];
            const double *tc = s_tc + el * 24;
            double xq[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double *k = tc + c * 8;
                xq[c] = k[0] + k[1] * x1 + k[2] * x2 + k[4] * x3 + x1 * (k[3] * x2 + k[5] * x3) +
                        x2 * x3 * (k[6] + k[7] * x1);
            }
            double g[7];
            eval_fields(s_fld, xq, g);
            double *stage = reinterpret_cast<double *>(s_D + (size_t)t * S::DSTR);
#pragma unroll
            for (int u = 0; u < 7; ++u) stage[u] = g[u];
        }
        __syncthreads();
    }

    // ---- pass 2, per quadrature point: J, detJ, J^{-1}, coefficients, folded point matrix ----
#pragma unroll 1
    for (int t = tid; t < EG * NQP; t += NT) {
        const int el = t / NQP, q = t % NQP;
        DT *Dr = s_D + (size_t)t * S::DSTR;
        if (el >= neg || q >= NQ) {
#pragma unroll
            for (int u = 0; u < S::DSTR; ++u) Dr[u] = DT(0);
            s_wf[t] = 0.0;
            continue;
        }
        const int q1 = q % N, q2 = (q / N) % N, q3 = q / (N * N);
        const double x1 = s_qw[q1], x2 = s_qw[q2], x3 = s_qw[q3];
        const double w = s_qw[N + q1] * s_qw[N + q2] * s_qw[N + q3];
        const double *tc = s_tc + el * 24;
        double J[3][3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double *k = tc + c * 8;
            J[c][0] = k[1] + k[3] * x2 + k[5] * x3 + k[7] * x2 * x3;
            J[c][1] = k[2] + k[3] * x1 + k[6] * x3 + k[7] * x1 * x3;
            J[c][2] = k[4] + k[5] * x1 + k[6] * x2 + k[7] * x1 * x2;
        }
        // J^{-1} = adj(J) / detJ
        double Ji[3][3];
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

        const double *rec = s_rec + el * 14;
        double K[3][3], bv[3], cc, ff;
        if (a.mode == 0) {
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int s = 0; s < 3; ++s) K[r][s] = rec[r * 3 + s];
            bv[0] = rec[9];
            bv[1] = rec[10];
            bv[2] = rec[11];
            cc = rec[12];
            ff = rec[13];
        } else {
            const double *g = reinterpret_cast<const double *>(Dr);
            const double lam0 = exp10(g[0]), lam1 = exp10(g[1]), lam2 = exp10(g[2]);
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int s = 0; s < 3; ++s)
                    K[r][s] = rec[r * 3 + 0] * lam0 * rec[s * 3 + 0] +
                              rec[r * 3 + 1] * lam1 * rec[s * 3 + 1] +
                              rec[r * 3 + 2] * lam2 * rec[s * 3 + 2];
            bv[0] = g[3];
            bv[1] = g[4];
            bv[2] = g[5];
            cc = 0.5 * (1.0 + g[6]);
            ff = rec[9];
        }
        const double wd = w * det;
        int fl = (det > 0.0) ? 0 : 1;
        bool finite = isfinite(wd * ff);
        double mx = 0.0;
        // row 0: Dh[0][0] = wd c, Dh[0][1+n] = wd (J^{-1} b)_n
        {
            const double d0 = wd * cc;
            finite = finite && isfinite(d0);
            mx = fmax(mx, fabs(d0));
            Dr[0] = DT(d0);
#pragma unroll
            for (int n = 0; n < 3; ++n) {
                const double v = wd * (Ji[n][0] * bv[0] + Ji[n][1] * bv[1] + Ji[n][2] * bv[2]);
                finite = finite && isfinite(v);
                mx = fmax(mx, fabs(v));
                Dr[1 + n] = DT(v);
            }
        }
        // rows 1..3: Dh[1+m][1+n] = wd (J^{-1} K J^{-T})[m][n]
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            double T0 = Ji[m][0] * K[0][0] + Ji[m][1] * K[1][0] + Ji[m][2] * K[2][0];
            double T1 = Ji[m][0] * K[0][1] + Ji[m][1] * K[1][1] + Ji[m][2] * K[2][1];
            double T2 = Ji[m][0] * K[0][2] + Ji[m][1] * K[1][2] + Ji[m][2] * K[2][2];
#pragma unroll
            for (int n = 0; n < 3; ++n) {
                const double v = wd * (T0 * Ji[n][0] + T1 * Ji[n][1] + T2 * Ji[n][2]);
                finite = finite && isfinite(v);
                mx = fmax(mx, fabs(v));
                Dr[4 + 3 * m + n] = DT(v);
            }
        }
        Dr[13] = DT(0);
        Dr[14] = DT(0);
        Dr[15] = DT(0);
        if (!finite) fl |= 2;
        s_wf[t] = wd * ff;
        if (S::SPLIT) atomicMax(&s_dmax[el], __float_as_uint(finite ? (float)mx : 0.0f));
        if (fl) atomicOr(&s_flag[el], fl);
    }
    __syncthreads();

    if (tid < EG) {
        float sc = 1.0f;
        if (S::SPLIT) {
            // largest power of two sc with sc * max|Dh| * bmax <= 2^15, i.e. sc <= c_bound / max|Dh|
            const float dm = __uint_as_float(s_dmax[tid]);
            if (dm > 0.0f) {
                float ratio = a.c_bound / dm;
                ratio = ratio < 1e30f ? ratio : 1e30f;
                int ex;
                frexpf(ratio, &ex);  // 2^(ex-1) <= ratio < 2^ex
                int e2 = ex - 1;
                e2 = e2 > 120 ? 120 : (e2 < -120 ? -120 : e2);
                sc = ldexpf(1.0f, e2);
            }
        }
        s_sc[tid] = sc;
        s_unsc[tid] = a.row_scale_inv / sc;
        if (rt == 0 && ct == 0 && a.status && tid < neg) {
            const int fl = s_flag[tid];
            if (fl & 1) atomicAdd(&a.status[0], 1);
            if (fl & 2) atomicAdd(&a.status[1], 1);
        }
    }
    __syncthreads();
    if (S::SPLIT) {
        for (int t = tid; t < EG * NQP * S::DSTR; t += NT) s_D[t] *= s_sc[t / (NQP * S::DSTR)];
        __syncthreads();
    }

    // ---- contraction on the matrix cores ----
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / C::WGN, wn = wave % C::WGN;
    const int rb0 = rt * S::TRB + wm * C::WM;
    const int cb0 = ct * S::TCB + wn * C::WN;
    const DT *ld = nullptr;
    if constexpr (PREC == PREC_F64) ld = s_ld64; else ld = s_ld32;

    int col_el[C::WN], col_a[C::WN], col_b[C::WN], col_c[C::WN];
    bool col_ok[C::WN];
#pragma unroll
    for (int j = 0; j < C::WN; ++j) {
        const int cb = cb0 + j;
        const int col = cb * TM + (lane % TM);
        const int el = col / S::NSP, jj = col % S::NSP;
        col_ok[j] = (cb < S::NCB) && (jj < NS) && (el < neg);
        const int jc = col_ok[j] ? jj : 0;
        col_el[j] = (cb < S::NCB) ? el : 0;
        col_a[j] = jc % N;
        col_b[j] = (jc / N) % N;
        col_c[j] = jc / (N * N);
    }
    bool row_ok[C::WM];
#pragma unroll
    for (int i = 0; i < C::WM; ++i) row_ok[i] = (rb0 + i) < S::NRB;

    typename F::acc acc[C::WM][C::WN];
#pragma unroll
    for (int i = 0; i < C::WM; ++i)
#pragma unroll
        for (int j = 0; j < C::WN; ++j)
#pragma unroll
            for (int v = 0; v < F::ACC_N; ++v) acc[i][j][v] = 0;

    const int half = lane / TM;
#pragma unroll 1
    for (int g = 0; g < S::NG; ++g) {
        typename F::row ra[C::WM];
#pragma unroll
        for (int i = 0; i < C::WM; ++i)
            if (row_ok[i]) ra[i] = load_row<PREC>(a, (size_t)g * S::NRB + rb0 + i, lane);
#pragma unroll
        for (int j = 0; j < C::WN; ++j) {
            if (cb0 + j >= S::NCB) continue;
            DT vals[S::SLOTS];
#pragma unroll
            for (int pp = 0; pp < S::PPL; ++pp) {
                const int q = g * S::KGP + half * S::PPL + pp;
                const int qc = q < NQ ? q : 0;
                const int q1 = qc % N, q2 = (qc / N) % N, q3 = qc / (N * N);
                const DT *Dh = s_D + ((size_t)col_el[j] * NQP + q) * S::DSTR;
                DT dloc[13];
#pragma unroll
                for (int u = 0; u < 13; ++u) dloc[u] = Dh[u];
                const DT la = ld[(q1 * N + col_a[j]) * 2], da = ld[(q1 * N + col_a[j]) * 2 + 1];
                const DT lb = ld[(q2 * N + col_b[j]) * 2], db = ld[(q2 * N + col_b[j]) * 2 + 1];
                const DT lc = ld[(q3 * N + col_c[j]) * 2], dc = ld[(q3 * N + col_c[j]) * 2 + 1];
                DT out[4];
                column_values<DT>(dloc, la, da, lb, db, lc, dc, out);
#pragma unroll
                for (int r = 0; r < 4; ++r) vals[pp * 4 + r] = col_ok[j] ? out[r] : DT(0);
            }
            const typename F::col cf = pack_col<PREC, DT>(vals);
#pragma unroll
            for (int i = 0; i < C::WM; ++i)
                if (row_ok[i]) mma<PREC>(acc[i][j], ra[i], cf);
        }
    }

    // ---- epilogue: unpadded row-major store ----
    using OT = typename std::conditional<PREC == PREC_F64, double, float>::type;
    OT *outA = reinterpret_cast<OT *>(a.out_A);
#pragma unroll
    for (int j = 0; j < C::WN; ++j) {
        if (!col_ok[j]) continue;
        const int col = (cb0 + j) * TM + (lane % TM);
        const int el = col / S::NSP, jj = col % S::NSP;
        const int64_t e = element_id(elist, e0 + el);
        const int64_t base = a.a_off ? a.a_off[e] : e * (int64_t)NS * NS;
        const float us = s_unsc[el];
#pragma unroll
        for (int i = 0; i < C::WM; ++i) {
            if (!row_ok[i]) continue;
#pragma unroll
            for (int v = 0; v < F::ACC_N; ++v) {
                const int row = (rb0 + i) * TM + acc_row<FAM>(lane, v);
                if (row < NS) {
                    if constexpr (PREC == PREC_F64) outA[base + (int64_t)row * NS + jj] = acc[i][j][v];
                    else outA[base + (int64_t)row * NS + jj] = acc[i][j][v] * us;
                }
            }
        }
    }

    // ---- load vector (FP64), by the column-tile-0 workgroup of each row tile ----
    if (ct == 0 && a.out_b) {
        const int r0 = rt * S::TRB * TM;
        const int r1 = (r0 + S::TRB * TM) < NS ? (r0 + S::TRB * TM) : NS;
        const int rows = r1 - r0;
        OT *outb = reinterpret_cast<OT *>(a.out_b);
#pragma unroll 1
        for (int t = tid; t < EG * rows; t += NT) {
            const int el = t / rows, r = r0 + t % rows;
            if (el >= neg) continue;
            const int ra_ = r % N, rb_ = (r / N) % N, rc_ = r / (N * N);
            const double *wf = s_wf + (size_t)el * NQP;
            double sum = 0.0;
#pragma unroll 1
            for (int q3 = 0; q3 < N; ++q3) {
                const double l3 = s_ld64[(q3 * N + rc_) * 2];
#pragma unroll 1
                for (int q2 = 0; q2 < N; ++q2) {
                    const double l23 = l3 * s_ld64[(q2 * N + rb_) * 2];
#pragma unroll
                    for (int q1 = 0; q1 < N; ++q1)
                        sum += wf[q1 + N * (q2 + N * q3)] * s_ld64[(q1 * N + ra_) * 2] * l23;
                }
            }
            const int64_t e = element_id(elist, e0 + el);
            const int64_t base = a.b_off ? a.b_off[e] : e * (int64_t)NS;
            outb[base + r] = (OT)sum;
        }
    }
}

// Grid-stride loop over work items; the element count comes from the host (nel) or, for the
// buckets of a mixed-degree call, from device memory (seg), so no host synchronisation is
// needed between bucketing and integration.
template <int P, int PREC, class C>
__global__ void __launch_bounds__(C::NW * 64) __attribute__((amdgpu_waves_per_eu(C::OCC, 8)))
k_integrate(const KArgs a)
{
    using S = Shape<P, PREC, C>;
    extern __shared__ __align__(16) unsigned char smem[];
    int64_t nel = a.nel;
    const int32_t *elist = a.elist;
    if (a.seg) {
        elist = a.elist + a.seg[0];
        nel = a.seg[1];
    }
    const int64_t total = ((nel + S::EG - 1) / S::EG) * S::RT * S::CT;
    for (int64_t wi = blockIdx.x; wi < total; wi += gridDim.x) {
        integrate_item<P, PREC, C>(a, wi, nel, elist, smem);
        __syncthreads();
    }
}

}  // namespace fem
