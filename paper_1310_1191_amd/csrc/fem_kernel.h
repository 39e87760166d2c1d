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
//     4 N_Q on the matrix cores. B^T (test functions) is a constant fragment table, staged
//     through LDS chunk by chunk, kept resident in LDS, or streamed by each wave straight from
//     the L2-resident table into registers one k-group ahead (RES). C (trial functions) is produced
//     from the 1-D Lagrange values (tensor-product structure of B) either cooperatively into a
//     double-buffered LDS area while the waves multiply the previous chunk (PROD 0), or by each
//     wave for its own column blocks, in registers, right before its MFMAs (PROD 1).
//   load vector: b_i = sum_q w_q detJ_q f phi_i(xi_q), FP64, sum-factorised over the tensor
//     product.
//   epilogue: accumulators are scaled back (split paths) and stored unpadded, row-major; when a
//     workgroup owns whole elements the tile is staged in LDS and written with aligned 16-byte
//     stores.
//
// A workgroup owns work items = (group of EG elements, row tile, column tile) in a persistent
// grid-stride loop; the next item's element data is fetched while the current one is multiplied.
// The columns of a work item are the EG elements' trial functions side by side, NSP apart, so
// small elements (p = 1, NSP = 8) share one MFMA column block. k_integrate runs one degree per
// launch; k_integrate_mixed runs the buckets of every degree in one persistent launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstddef>

#include <type_traits>

#include "fem_geometry.h"
#include "fem_layout.h"

namespace fem {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// Kernel arguments (device pointers). Tables are those of the launch's degree.
struct KArgs {
    int64_t nel;             // elements in this launch
    const double *geom;      // [*][8][3]
    const double *elem;      // [*][14] (ELEMENT) or [*][10] (FIELD)
    const double *field;     // [175] (FIELD)
    const double *jac;       // supplied Jacobian terms [*][Nq][10] = detJ, J^{-1} row-major (element e
                             // at 10 (b_off ? b_off[e] : e Nq)), or null to compute them from geom
    const int32_t *elist;    // element ids of this launch, or null for 0..nel-1
    const int64_t *seg;      // device {start, count}: use elist + start and nel = count, or null
    const int64_t *a_off;    // [*] element offsets into out_A, or null for e * Ns^2
    const int64_t *b_off;    // [*] element offsets into out_b, or null for e * Ns
    void *out_A;
    void *out_b;             // may be null
    int32_t *status;         // [2] or null
    int32_t mode;            // 0 ELEMENT, 1 FIELD, 2 ELASTIC (block comp_i, comp_k)
    int32_t comp_i, comp_k;  // ELASTIC: test and trial component of this launch's block
    int64_t at_base;         // ELASTIC, > 0: the block is also written transposed, element e's
                             // copy at at_base + e a_stride (block (k, i) = block (i, k)^T), by
                             // the tiles with TRANS_EPI only; 0: no copy
    int64_t a_base, a_stride;  // without a_off: element e's matrix starts at a_base + e a_stride
    int64_t b_base, b_stride;  // without b_off: element e's vector starts at b_base + e b_stride
    const double *xq, *wq;   // [n] Gauss points and weights
    const double *LD64;      // [n][n][2]: (L, D)[gauss point][node]
    const float *LD32;       // the same, rounded to FP32
    const double *phi64;     // prisms: [Nq][Ns] shape-function values at the points (load vector)
    const void *row_hi;      // row-operand fragment table (fem_layout.h)
    const void *row_lo;      // second table of the split paths, else null
    const void *bcol;        // B[(q, s)][j] in the column-operand fragment layout (FP32; FP64 path FP64)
    float c_bound;           // split paths: 2^15 / max_{q,j} sum_r |B[(q,r)][j]|
    float row_scale_inv;     // 1 / (power-of-two scale of the row table)
};

template <int EG_, int WGM_, int WGN_, int WM_, int WN_, int OCC_, int KC_, int RES_, int PROD_ = 0,
          int BT_ = 0, int TE_ = 0, int OPQ_ = 0>
struct Cfg {
    static constexpr int PROD = PROD_;  // 0: C chunks produced by the whole workgroup into LDS;
                                        // 1: each wave produces its own C fragments in registers
    static constexpr int EG = EG_;    // elements per work item
    static constexpr int WGM = WGM_;  // waves along rows
    static constexpr int WGN = WGN_;  // waves along columns
    static constexpr int WM = WM_;    // row blocks per wave
    static constexpr int WN = WN_;    // column blocks per wave
    static constexpr int OCC = OCC_;  // waves per SIMD the register budget must allow
    static constexpr int KC = KC_;    // k-groups per LDS chunk of the column operand
    static constexpr int RES = RES_;  // row operand: 0 staged through LDS per chunk, 1 the whole
                                      // table resident in LDS, 2 streamed from the table
                                      // (L2) into registers one k-group ahead, 3 the wave's
                                      // whole share of the table held in registers (loaded
                                      // once per item, k loop unrolled; small tables only)
    static constexpr int BT = BT_;    // PROD 1 only: 1 reads the B factors of the column operand
                                      // from a precomputed table instead of forming them from the
                                      // 1-D Lagrange tables
    static constexpr int TE = TE_;    // 1: the epilogue can also write the block transposed
                                      // (elasticity's lower blocks, KArgs::at_base)
    static constexpr int OPQ = OPQ_;  // 1: the per-thread addresses are formed again in every
                                      // item instead of being kept across the item loop
    static constexpr int NW = WGM_ * WGN_;
};

// ------------------------------------------------------------------------------------------
// compile-time shape of a (degree, precision, config) instance
// ------------------------------------------------------------------------------------------
template <int P, int PREC, class C>
struct Shape {
    static constexpr int FAM = family_of(PREC);
    // prisms: N counts the vertical (Gauss-Legendre / GLL) points and nodes; the 1-D tables,
    // the trilinear map and the sum factorisation belong to the hexahedron
    static constexpr bool PRISM = is_prism(P);
    static constexpr int N = deg_of(P) + 1, NS = ns_of(P), NQ = nq_of(P);
    static constexpr int GEO = PRISM ? 18 : 24;  // vertex coordinates per element
    static_assert(!PRISM || (C::PROD == 1 && C::BT == 1),
                  "prisms produce the column operand per wave from the B-factor table");
    static constexpr int TM = fam_tm(FAM), KGP = fam_kgp(FAM), PPL = fam_ppl(FAM);
    static constexpr int SLOTS = fam_slots(FAM);
    static constexpr int NG = groups_of(P, FAM);
    static constexpr int KC = C::KC < NG ? C::KC : NG;
    static_assert(KC == NG || (8 % KC == 0), "chunks of 1, 2, 4 or 8 k-groups, or one chunk");
    static constexpr int NGP = (NG + KC - 1) / KC * KC;   // <= the table's padded group count
    static constexpr int NCH = NGP / KC;
    static constexpr int NQP = NGP * KGP;
    static constexpr int NRB = rblocks_of(P, FAM);
    static constexpr int NSP = col_pitch(P, FAM);  // column pitch per element
    static constexpr int EG = C::EG;
    static_assert((EG * NSP) % TM == 0, "element group must fill whole column blocks");
    static constexpr int NCB = EG * NSP / TM;
    static constexpr int TRB = C::WGM * C::WM, TCB = C::WGN * C::WN;
    static constexpr int RT = (NRB + TRB - 1) / TRB, CT = (NCB + TCB - 1) / TCB;
    static constexpr int NT = C::NW * 64;
    static constexpr bool SPLIT = (PREC == PREC_SPLIT_BF16 || PREC == PREC_SPLIT_F16);
    using DT = typename std::conditional<PREC == PREC_F64, double, float>::type;
    static constexpr int DSTR = 16;  // LDS stride of one point matrix (13 used)
    // column operand chunk: [k-group][column block][part][lane] x FRAGB bytes
    static constexpr int NCOL = TCB * TM;
    static_assert(C::PROD == 1 || NT % NCOL == 0, "the producers cover the tile's columns");
    // PROD 1: every column block of a wave belongs to one element (the point matrices of a
    // point are read once for all of the wave's column blocks)
    static constexpr bool WAVE_ONE_EL = (C::EG == 1) || (NSP % (C::WN * TM)) == 0;
    static constexpr int PCH = KC * KGP;                  // points per chunk
    static constexpr int NPART = SPLIT ? 2 : 1;
    static constexpr int FRAGB = (PREC == PREC_F64) ? 32 : 16;
    static constexpr size_t CBUF = C::PROD ? 0 : size_t(KC) * TCB * NPART * 64 * FRAGB;
    // row operand fragment bytes per lane (both parts)
    static constexpr int ROWB = (PREC == PREC_F64) ? 32 : (SPLIT ? 32 : 16);
    static constexpr size_t ROWTAB = C::RES == 1 ? size_t(NGP) * NRB * 64 * ROWB : 0;
    static_assert(C::RES != 3 || NGP * C::WM * ROWB / 4 <= 64, "register-resident rows: at most 64 VGPRs");
    static_assert(C::RES < 2 || C::PROD == 1, "rows held in registers need per-wave production");
    // element data prefetched per thread: 24 coordinates and up to 14 coefficients per element
    static constexpr int EREC = 38;
    static constexpr int PFN = (EG * EREC + NT - 1) / NT;

    // dynamic LDS layout (bytes); the point matrices and the column chunks come last so that
    // the output staging area of the epilogue can overlay them
    static constexpr size_t al16(size_t x) { return (x + 15) / 16 * 16; }
    static constexpr size_t off_geo = 0;                                  // EG*24 double
    static constexpr size_t off_rec = off_geo + EG * 24 * 8;              // EG*14 double
    static constexpr size_t off_tc = off_rec + EG * 14 * 8;               // EG*24 double
    static constexpr size_t off_fld = off_tc + EG * 24 * 8;               // 176 double
    // 1-D tables, each followed by an all-zero copy of itself (padding columns read zeros)
    static constexpr size_t off_ld64 = off_fld + 176 * 8;                 // 2 x N*N*2 double
    static constexpr size_t off_ld32 = off_ld64 + 2 * N * N * 2 * 8;      // 2 x N*N*2 float
    // hexahedra: 2N double (1-D points, weights); prisms: NQP x (xi1, xi2, zeta, w) double
    static constexpr size_t QW = PRISM ? 4 * size_t(NQP) : 2 * size_t(N);
    static constexpr size_t off_qw = off_ld32 + al16(2 * N * N * 2 * 4);
    static constexpr size_t off_wf = off_qw + al16(QW * 8);               // EG*NQP double
    static constexpr size_t off_misc = off_wf + EG * NQP * 8;             // dmax (u32), flag (i32)
    static constexpr size_t off_pt = off_misc + al16(EG * 8);             // 3 x NQP int
    static constexpr size_t off_row = off_pt + al16(3 * NQP * 4);         // resident row table
    static constexpr size_t off_D = off_row + ROWTAB;                     // EG*NQP*16 DT
    static constexpr size_t d_bytes = size_t(EG) * NQP * DSTR * sizeof(DT);
    static constexpr size_t off_cb = off_D + d_bytes;                     // 2 column chunks
    // Output staging: used when one workgroup owns whole elements (one row and one column
    // tile) and the tile, [NS rows][EG*NSP + 1 columns] of the output type, fits in 64 KiB;
    // otherwise the accumulators are stored directly.
    using OT = DT;
    // Staged images hold the output exactly as it lies in memory (row-major, pitch NS), shifted
    // by the destination's misalignment so that 16-byte global vectors are 16-byte LDS vectors.
    static constexpr int VW = 16 / sizeof(OT);
    static constexpr int IMG = (NS * NS + 2 * VW - 1) / VW * VW;      // one element
    // When every wave owns whole elements (all rows and exactly one element's columns), each
    // wave can stage one row block of its element at a time and write it as one contiguous range
    // of 16-byte vectors (whole cache lines, no partial-line writes to HBM). Single-wave
    // workgroups always do so (it needs the least LDS); otherwise the whole tile is staged when
    // it fits in 64 KiB.
    static constexpr bool WAVE_OWNS_EL = C::PROD == 1 && RT == 1 && CT == 1 && C::WN * TM == NSP &&
                                         C::WM * TM >= NS && C::WGM == 1;
    static constexpr bool STAGE_OUT = (RT == 1 && CT == 1) && size_t(EG) * IMG * sizeof(OT) <= 65536 &&
                                      !(WAVE_OWNS_EL && C::NW == 1);
    static constexpr bool STAGE_WAVE = !STAGE_OUT && WAVE_OWNS_EL;
    // Tiles with TE can also write the transposed block (elasticity's lower blocks): with an odd
    // Ns from a per-wave or whole-element staged image (its column reads then free of bank
    // conflicts), otherwise straight from the accumulators (32-wide families: four consecutive
    // rows per lane, one run of a transposed row, 16-byte stores where Ns is a multiple of 4;
    // FP64: one value per row and four lanes per run). (Separate tiles, so the other instances
    // carry none of this code.)
    static constexpr bool TRANS_EPI = C::TE && (STAGE_WAVE || STAGE_OUT) && (NS % 2 == 1);
    static constexpr int WIMG = (TM * NS + 2 * VW - 1) / VW * VW;     // one row block
    // Otherwise a workgroup that owns whole elements with one row of waves stages one row block
    // of all its elements at a time.
    static constexpr bool STAGE_RB = !STAGE_OUT && !STAGE_WAVE && RT == 1 && CT == 1 && C::WGM == 1 &&
                                     size_t(EG) * WIMG * sizeof(OT) <= 65536;
    static constexpr bool TRANS_REG = C::TE && !TRANS_EPI;
    static constexpr size_t out_bytes = STAGE_OUT ? size_t(EG) * IMG * sizeof(OT)
                                      : STAGE_WAVE ? size_t(C::NW) * WIMG * sizeof(OT)
                                      : STAGE_RB ? size_t(EG) * WIMG * sizeof(OT) : 0;
    static constexpr int NBUF = NCH > 1 ? 2 : 1;
    // row operand staged per chunk (tables not resident): [k-group][row block][16-B piece][lane]
    static constexpr int RPART = ROWB / 16;                                 // 16-B pieces per lane
    static constexpr int RPIECES = C::RES ? 0 : KC * TRB * RPART * 64;
    static constexpr int RPT = C::RES ? 0 : (RPIECES + NT - 1) / NT;       // pieces per thread
    static constexpr size_t RBUF = size_t(RPIECES) * 16;
    static constexpr size_t main_bytes0 = d_bytes + NBUF * (CBUF + RBUF);
    // the load vector's two EG*NS double temporaries overlay the chunk buffers after the loop
    static constexpr size_t off_t1 = off_cb, off_t2 = off_cb + EG * NS * 8;
    static constexpr size_t tmp_bytes = 2 * EG * NS * 8;
    // the load-vector temporaries live at off_cb after the loop
    static constexpr size_t main_bytes = main_bytes0 > d_bytes + tmp_bytes ? main_bytes0 : d_bytes + tmp_bytes;
    static constexpr size_t lds_bytes = off_D + (main_bytes > out_bytes ? main_bytes : out_bytes);
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

// The same with a 32-bit fragment index: the address is a uniform table base plus a 32-bit
// per-lane byte offset, which the hardware's scalar-base addressing takes directly.
template <int PREC>
__device__ inline typename Frag<PREC>::row load_row_off(const KArgs &a, unsigned frag, int lane)
{
    constexpr unsigned FB = (PREC == PREC_F64) ? 32u : 16u;
    const unsigned off = (frag * 64u + (unsigned)lane) * FB;
    const char *hi = reinterpret_cast<const char *>(a.row_hi);
    if constexpr (PREC == PREC_F64) {
        return *reinterpret_cast<const f64x4 *>(hi + off);
    } else if constexpr (PREC == PREC_F32) {
        return *reinterpret_cast<const f32x4 *>(hi + off);
    } else if constexpr (PREC == PREC_BF16) {
        return *reinterpret_cast<const bf16x8 *>(hi + off);
    } else if constexpr (PREC == PREC_SPLIT_BF16) {
        const char *lo = reinterpret_cast<const char *>(a.row_lo);
        SplitBF r;
        r.hi = *reinterpret_cast<const bf16x8 *>(hi + off);
        r.lo = *reinterpret_cast<const bf16x8 *>(lo + off);
        return r;
    } else {
        const char *lo = reinterpret_cast<const char *>(a.row_lo);
        SplitH r;
        r.hi = *reinterpret_cast<const f16x8 *>(hi + off);
        r.lo = *reinterpret_cast<const f16x8 *>(lo + off);
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
#pragma unroll
        for (int t = 0; t < 8; t += 2) {
            const f32x2 x = {v[t], v[t + 1]};
            const bf16x2 h = __builtin_convertvector(x, bf16x2);
            const f32x2 hf = __builtin_convertvector(h, f32x2);
            const bf16x2 l = __builtin_convertvector(x - hf, bf16x2);
            r.hi[t] = h[0];
            r.hi[t + 1] = h[1];
            r.lo[t] = l[0];
            r.lo[t + 1] = l[1];
        }
        return r;
    } else {
        // hi = fp16(x) (round to nearest even); lo = fp16(x - hi), the difference formed exactly in
        // FP32 by a mixed-precision FMA that reads hi in FP16 and writes one half of the lo pair
        SplitH r;
#pragma unroll
        for (int t = 0; t < 8; t += 2) {
            const f32x2 x = {v[t], v[t + 1]};
            const f16x2 h = __builtin_convertvector(x, f16x2);
            f16x2 l;
            asm("v_fma_mixlo_f16 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(l) : "v"(h), "v"(v[t]));
            asm("v_fma_mixhi_f16 %0, -%1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]"
                : "+v"(l) : "v"(h), "v"(v[t + 1]));
            r.hi[t] = h[0];
            r.hi[t + 1] = h[1];
            r.lo[t] = l[0];
            r.lo[t + 1] = l[1];
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

// One of the products of the split paths (stage 0: lo*hi, 1: hi*lo, 2: hi*hi); the unsplit
// paths do all their work in stage 0. Issuing a stage for every accumulator before the next
// stage keeps independent MFMAs back to back.
template <int PREC, int STAGE>
__device__ inline void mma_stage(typename Frag<PREC>::acc &c, const typename Frag<PREC>::row &a,
                                 const typename Frag<PREC>::col &b)
{
    if constexpr (PREC == PREC_SPLIT_BF16) {
        if constexpr (STAGE == 0) c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.lo, b.hi, c, 0, 0, 0);
        if constexpr (STAGE == 1) c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.hi, b.lo, c, 0, 0, 0);
        if constexpr (STAGE == 2) c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.hi, b.hi, c, 0, 0, 0);
    } else if constexpr (PREC == PREC_SPLIT_F16) {
        if constexpr (STAGE == 0) c = __builtin_amdgcn_mfma_f32_32x32x16_f16(a.lo, b.hi, c, 0, 0, 0);
        if constexpr (STAGE == 1) c = __builtin_amdgcn_mfma_f32_32x32x16_f16(a.hi, b.lo, c, 0, 0, 0);
        if constexpr (STAGE == 2) c = __builtin_amdgcn_mfma_f32_32x32x16_f16(a.hi, b.hi, c, 0, 0, 0);
    } else if constexpr (STAGE == 0) {
        mma<PREC>(c, a, b);
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
// column-operand chunk access
// ------------------------------------------------------------------------------------------
// Largest power of two sc with sc * max|Dh| * bmax <= 2^15 (max|C| then fits FP16), i.e.
// sc <= c_bound / max|Dh|. Every thread that needs it recomputes it from the element maximum.
__device__ inline float split_scale(unsigned dmax_bits, float c_bound)
{
    const float dm = __uint_as_float(dmax_bits);
    if (!(dm > 0.0f)) return 1.0f;
    float ratio = c_bound / dm;
    ratio = ratio < 1e30f ? ratio : 1e30f;
    int ex;
    frexpf(ratio, &ex);  // 2^(ex-1) <= ratio < 2^ex
    int e2 = ex - 1;
    e2 = e2 > 120 ? 120 : (e2 < -120 ? -120 : e2);
    return ldexpf(1.0f, e2);
}

// Store the 4 values (r = 0..3) of one (point, column) pair into a column chunk. `kgl` is the
// k-group within the chunk, `w` the point within the k-group, `c` the column within the tile.
template <int PREC, class S, typename T>
__device__ inline void put_col(unsigned char *buf, int kgl, int w, int c, const T v[4])
{
    constexpr int TM = S::TM;
    const int h = w / S::PPL, sub = w % S::PPL;
    const int lane = (c % TM) + TM * h;
    const int cbt = c / TM;
    const size_t frag = (size_t)(kgl * S::TCB + cbt) * S::NPART;
    if constexpr (PREC == PREC_F64) {
        f64x2 *d = reinterpret_cast<f64x2 *>(buf + (frag * 64 + lane) * 32);
        d[0] = f64x2{v[0], v[1]};
        d[1] = f64x2{v[2], v[3]};
    } else if constexpr (PREC == PREC_F32) {
        *reinterpret_cast<f32x4 *>(buf + (frag * 64 + lane) * 16) = f32x4{v[0], v[1], v[2], v[3]};
    } else {
        typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));
        const f32x2 x01 = {v[0], v[1]}, x23 = {v[2], v[3]};
        unsigned char *p = buf + (frag * 64 + lane) * 16 + sub * 8;
        if constexpr (PREC == PREC_BF16) {
            const bf16x2 h01 = __builtin_convertvector(x01, bf16x2);
            const bf16x2 h23 = __builtin_convertvector(x23, bf16x2);
            typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
            *reinterpret_cast<bf16x4 *>(p) = bf16x4{h01[0], h01[1], h23[0], h23[1]};
        } else if constexpr (PREC == PREC_SPLIT_BF16) {
            const bf16x2 h01 = __builtin_convertvector(x01, bf16x2);
            const bf16x2 h23 = __builtin_convertvector(x23, bf16x2);
            const bf16x2 l01 = __builtin_convertvector(x01 - __builtin_convertvector(h01, f32x2), bf16x2);
            const bf16x2 l23 = __builtin_convertvector(x23 - __builtin_convertvector(h23, f32x2), bf16x2);
            typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
            *reinterpret_cast<bf16x4 *>(p) = bf16x4{h01[0], h01[1], h23[0], h23[1]};
            *reinterpret_cast<bf16x4 *>(p + 64 * 16) = bf16x4{l01[0], l01[1], l23[0], l23[1]};
        } else {
            const f16x2 h01 = __builtin_convertvector(x01, f16x2);
            const f16x2 h23 = __builtin_convertvector(x23, f16x2);
            const f16x2 l01 = __builtin_convertvector(x01 - __builtin_convertvector(h01, f32x2), f16x2);
            const f16x2 l23 = __builtin_convertvector(x23 - __builtin_convertvector(h23, f32x2), f16x2);
            typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
            *reinterpret_cast<f16x4 *>(p) = f16x4{h01[0], h01[1], h23[0], h23[1]};
            *reinterpret_cast<f16x4 *>(p + 64 * 16) = f16x4{l01[0], l01[1], l23[0], l23[1]};
        }
    }
}

// A wave's column fragment of column block cbt (within the tile) and k-group kgl of a chunk.
template <int PREC, class S>
__device__ inline typename Frag<PREC>::col get_col(const unsigned char *buf, int kgl, int cbt, int lane)
{
    const size_t frag = (size_t)(kgl * S::TCB + cbt) * S::NPART;
    if constexpr (PREC == PREC_F64) {
        return *reinterpret_cast<const f64x4 *>(buf + (frag * 64 + lane) * 32);
    } else if constexpr (PREC == PREC_F32) {
        return *reinterpret_cast<const f32x4 *>(buf + (frag * 64 + lane) * 16);
    } else if constexpr (PREC == PREC_BF16) {
        return *reinterpret_cast<const bf16x8 *>(buf + (frag * 64 + lane) * 16);
    } else if constexpr (PREC == PREC_SPLIT_BF16) {
        SplitBF r;
        r.hi = *reinterpret_cast<const bf16x8 *>(buf + (frag * 64 + lane) * 16);
        r.lo = *reinterpret_cast<const bf16x8 *>(buf + ((frag + 1) * 64 + lane) * 16);
        return r;
    } else {
        SplitH r;
        r.hi = *reinterpret_cast<const f16x8 *>(buf + (frag * 64 + lane) * 16);
        r.lo = *reinterpret_cast<const f16x8 *>(buf + ((frag + 1) * 64 + lane) * 16);
        return r;
    }
}

// Row fragment from the LDS-resident copy of the table (layout [frag][part][lane] x 16 B, or
// [frag][lane] x 32 B for FP64).
template <int PREC>
__device__ inline typename Frag<PREC>::row lds_row(const unsigned char *tab, size_t frag, int lane)
{
    if constexpr (PREC == PREC_F64) {
        return *reinterpret_cast<const f64x4 *>(tab + (frag * 64 + lane) * 32);
    } else if constexpr (PREC == PREC_F32) {
        return *reinterpret_cast<const f32x4 *>(tab + (frag * 64 + lane) * 16);
    } else if constexpr (PREC == PREC_BF16) {
        return *reinterpret_cast<const bf16x8 *>(tab + (frag * 64 + lane) * 16);
    } else if constexpr (PREC == PREC_SPLIT_BF16) {
        SplitBF r;
        r.hi = *reinterpret_cast<const bf16x8 *>(tab + (frag * 128 + lane) * 16);
        r.lo = *reinterpret_cast<const bf16x8 *>(tab + (frag * 128 + 64 + lane) * 16);
        return r;
    } else {
        SplitH r;
        r.hi = *reinterpret_cast<const f16x8 *>(tab + (frag * 128 + lane) * 16);
        r.lo = *reinterpret_cast<const f16x8 *>(tab + (frag * 128 + 64 + lane) * 16);
        return r;
    }
}

// ------------------------------------------------------------------------------------------
// one work item
// ------------------------------------------------------------------------------------------
struct Item {
    int64_t e0;  // first element index (into elist, or the element id itself)
    int neg;     // elements present (<= EG)
    int rt, ct;  // row and column tile
};

template <class S>
__device__ inline Item decode_item(int64_t wi, int64_t nel)
{
    Item it;
    it.ct = (int)(wi % S::CT);
    wi /= S::CT;
    it.rt = (int)(wi % S::RT);
    it.e0 = (wi / S::RT) * S::EG;
    it.neg = (int)((nel - it.e0) < S::EG ? (nel - it.e0) : S::EG);
    return it;
}

// Fetch the element data of an item into registers (24 coordinates then the coefficient record
// of each element; entries past the record length or the element count are 0). With supplied
// Jacobian terms (SUP) the vertices may be absent and then read as 0.
template <class S, bool SUP>
__device__ inline void fetch_elements(const KArgs &a, const int32_t *elist, const Item &it,
                                      int reclen, double (&pf)[S::PFN])
{
#pragma unroll
    for (int k = 0; k < S::PFN; ++k) {
        const int f = threadIdx.x + k * S::NT;
        const int el = f / S::EREC, comp = f % S::EREC;
        double v = 0.0;
        if (el < it.neg) {
            const int64_t e = element_id(elist, it.e0 + el);
            if (comp < S::GEO) {
                if constexpr (SUP) v = a.geom ? a.geom[e * S::GEO + comp] : 0.0;
                else v = a.geom[e * S::GEO + comp];
            }
            else if (comp >= 24 && comp - 24 < reclen) v = a.elem[e * reclen + (comp - 24)];
        }
        pf[k] = v;
    }
}

template <int P, int PREC, class C, bool SUP>
__device__ inline void integrate_item(const KArgs &a, const Item &it, const int32_t *elist,
                                      int reclen, unsigned char *smem, const double (&pf)[Shape<P, PREC, C>::PFN],
                                      double (&pf_next)[Shape<P, PREC, C>::PFN], bool has_next,
                                      const Item &it_next)
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
    double *s_qw = reinterpret_cast<double *>(smem + S::off_qw);
    double *s_wf = reinterpret_cast<double *>(smem + S::off_wf);
    double *s_t1 = reinterpret_cast<double *>(smem + S::off_t1);
    double *s_t2 = reinterpret_cast<double *>(smem + S::off_t2);
    unsigned *s_dmax = reinterpret_cast<unsigned *>(smem + S::off_misc);
    int *s_flag = reinterpret_cast<int *>(smem + S::off_misc + EG * 4);
    int *s_pt = reinterpret_cast<int *>(smem + S::off_pt);
    const unsigned char *s_row = smem + S::off_row;
    DT *s_D = reinterpret_cast<DT *>(smem + S::off_D);
    unsigned char *s_cb0 = smem + S::off_cb;
    unsigned char *s_cb1 = smem + S::off_cb + S::CBUF;
    unsigned char *s_rb0 = smem + S::off_cb + S::NBUF * S::CBUF;
    unsigned char *s_rb1 = s_rb0 + S::RBUF;

    // OPQ tiles pass the thread index through an empty asm statement once per item, so the
    // per-thread addresses derived from it are formed again in each item instead of being kept
    // across the item loop: where that loop spilled them, their reloads at the top of the next
    // item waited, in the in-order vector-memory counter, for all of this item's output stores.
    int tid = threadIdx.x;
    if constexpr (C::OPQ) asm volatile("" : "+v"(tid));
    const int neg = it.neg, rt = it.rt, ct = it.ct;
    const int64_t e0 = it.e0;

    // ---- element data (fetched earlier) into LDS ----
    if constexpr (C::OCC > 1) __builtin_amdgcn_s_setprio(0);  // prologue: lowest
    // The item's first phases take the thread index through an empty asm statement: their
    // addresses are formed again here instead of being held across the item loop, where the
    // compiler spilled them and the reloads at the top of the item waited for the previous
    // item's stores (the vector-memory counter is in order).
    int tid_top = threadIdx.x;
    asm volatile("" : "+v"(tid_top));
#pragma unroll
    for (int k = 0; k < S::PFN; ++k) {
        const int f = tid_top + k * NT;
        const int el = f / S::EREC, comp = f % S::EREC;
        if (el < EG) {
            if (comp < 24) s_geo[el * 24 + comp] = pf[k];
            else s_rec[el * 14 + (comp - 24)] = pf[k];
        }
    }
    if (tid_top < EG) {
        s_dmax[tid_top] = 0u;
        s_flag[tid_top] = 0;
    }
    __syncthreads();

    // ---- trilinear form x(xi) = sum_S c_S prod_{d in S} xi_d, c_S = 1/8 sum_v X_v prod s_vd ----
    if constexpr (!S::PRISM) {
        for (int t = tid_top; t < EG * 24; t += NT) {
            const int el = t / 24, coord = (t % 24) / 8, sub = t % 8;
            s_tc[t] = trilinear_coeff(s_geo + el * 24, coord, sub);
        }
        __syncthreads();
    }

    // ---- FIELD mode, pass 1: the 7 coefficient fields at x_q, staged in the point's Dh slot ----
    if (a.mode == 1) {
#pragma unroll 1
        for (int t = tid; t < EG * NQP; t += NT) {
            const int el = t / NQP, q = t % NQP;
            if (el >= neg || q >= NQ) continue;
            double xq[3];
            if constexpr (S::PRISM) {
                prism_point(s_geo + el * 24, s_qw[4 * q], s_qw[4 * q + 1], s_qw[4 * q + 2], xq);
            } else {
                const int q1 = q % N, q2 = (q / N) % N, q3 = q / (N * N);
                trilinear_point(s_tc + el * 24, s_qw[q1], s_qw[q2], s_qw[q3], xq);
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
        double x1, x2, x3, w;
        if constexpr (S::PRISM) {
            x1 = s_qw[4 * q];
            x2 = s_qw[4 * q + 1];
            x3 = s_qw[4 * q + 2];
            w = s_qw[4 * q + 3];
        } else {
            const int q1 = q % N, q2 = (q / N) % N, q3 = q / (N * N);
            x1 = s_qw[q1];
            x2 = s_qw[q2];
            x3 = s_qw[q3];
            w = s_qw[N + q1] * s_qw[N + q2] * s_qw[N + q3];
        }
        double Ji[3][3], det;
        if constexpr (SUP) {
            // supplied terms (the NOJAC variant of section 4): detJ, then J^{-1} row-major
            const int64_t e = element_id(elist, e0 + el);
            const double *jt = a.jac + ((a.b_off ? a.b_off[e] : e * NQ) + q) * 10;
            det = jt[0];
#pragma unroll
            for (int m = 0; m < 3; ++m)
#pragma unroll
                for (int n = 0; n < 3; ++n) Ji[m][n] = jt[1 + 3 * m + n];
        } else if constexpr (S::PRISM) {
            det = prism_jacobian_terms(s_geo + el * 24, x1, x2, x3, Ji);
        } else {
            det = jacobian_terms(s_tc + el * 24, x1, x2, x3, Ji);
        }

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
        } else if (a.mode == 2) {
            // isotropic elasticity, block (comp_i, comp_k): K_jl = c_{i j k l} with
            // c_ijkl = lambda d_ij d_kl + mu (d_ik d_jl + d_il d_jk) (section 5.1)
            const double E = rec[0], nu = rec[1];
            const double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), mu = E / (2.0 * (1.0 + nu));
            const int ci = a.comp_i, ck = a.comp_k;
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int s = 0; s < 3; ++s)
                    K[r][s] = lam * (r == ci && s == ck) + mu * ((ci == ck && r == s) + (r == ck && s == ci));
            bv[0] = bv[1] = bv[2] = 0.0;
            cc = 0.0;
            ff = rec[2 + ci];
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

    if (tid < neg && rt == 0 && ct == 0 && a.status) {
        const int fl = s_flag[tid];
        if (fl & 1) atomicAdd(&a.status[0], 1);
        if (fl & 2) atomicAdd(&a.status[1], 1);
    }
    if constexpr (S::SPLIT) {
        // exact power-of-two scaling of each element's point matrices (FP16 range)
#pragma unroll 1
        for (int t = tid; t < EG * NQP; t += NT) {
            const DT sc = DT(split_scale(s_dmax[t / NQP], a.c_bound));
            DT *Dr = s_D + (size_t)t * S::DSTR;
#pragma unroll
            for (int u = 0; u < 13; ++u) Dr[u] *= sc;
        }
        __syncthreads();
    }

    // the element data of the next item travels while this one is multiplied
    if (has_next) fetch_elements<S, SUP>(a, elist, it_next, reclen, pf_next);

    // ---- producer setup: this thread's column of the tile ----
    using DT2 = typename std::conditional<PREC == PREC_F64, f64x2, f32x2>::type;
    const DT2 *ld2 = nullptr;
    if constexpr (PREC == PREC_F64) ld2 = reinterpret_cast<const DT2 *>(s_ld64);
    else ld2 = reinterpret_cast<const DT2 *>(smem + S::off_ld32);
    const int pc = tid % S::NCOL;
    const int pp0 = tid / S::NCOL;
    int p_el, p_a, p_b, p_c;
    bool p_ok;
    {
        const int cbg = ct * S::TCB + pc / TM;
        const int col = cbg * TM + pc % TM;
        const int el = col / S::NSP, jj = col % S::NSP;
        p_ok = cbg < S::NCB && jj < NS && el < neg;
        const int jc = (p_ok ? jj : 0);
        p_el = (cbg < S::NCB) ? el : 0;
        p_a = jc % N;
        p_b = (jc / N) % N;
        p_c = jc / (N * N);
    }

    // A production unit owns one lane slot of a column fragment: column c of the tile and the
    // PPL points of lane group h in k-group kgl, written as whole 16-byte pieces.
    constexpr int HPG = S::KGP / S::PPL;
    constexpr int UNITS = S::KC * HPG * S::NCOL;
    static_assert(C::PROD == 1 || NT % S::NCOL == 0, "producer columns are fixed per thread");
    const unsigned char *ldb = reinterpret_cast<const unsigned char *>(ld2);
    // padding columns read the first-direction factor from the zero copy of the table
    const int p_ab = (p_a + (p_ok ? 0 : N * N)) * (int)sizeof(DT2);
    const int p_bb = p_b * (int)sizeof(DT2), p_cb = p_c * (int)sizeof(DT2);
    const DT *Dbase = s_D + (size_t)p_el * NQP * S::DSTR;
    auto produce_chunk = [&](int ch, unsigned char *buf) {
#pragma unroll
        for (int u = tid; u < UNITS; u += NT) {
            const int h = (u / S::NCOL) % HPG, kgl = u / (S::NCOL * HPG);
            DT vals[S::SLOTS];
#pragma unroll
            for (int sub = 0; sub < S::PPL; ++sub) {
                const int q = (ch * S::KC + kgl) * S::KGP + h * S::PPL + sub;
                const DT *Dh = Dbase + q * S::DSTR;
                DT dloc[13];
#pragma unroll
                for (int uu = 0; uu < 13; ++uu) dloc[uu] = Dh[uu];
                const DT2 fa = *reinterpret_cast<const DT2 *>(ldb + s_pt[q] + p_ab);
                const DT2 fb = *reinterpret_cast<const DT2 *>(ldb + s_pt[NQP + q] + p_bb);
                const DT2 fc = *reinterpret_cast<const DT2 *>(ldb + s_pt[2 * NQP + q] + p_cb);
                DT out[4];
                column_values<DT>(dloc, fa[0], fa[1], fb[0], fb[1], fc[0], fc[1], out);
#pragma unroll
                for (int r = 0; r < 4; ++r) vals[sub * 4 + r] = out[r];
            }
            const int lane_s = (pc % TM) + TM * h;
            const size_t frag = (size_t)(kgl * S::TCB + pc / TM) * S::NPART;
            const typename F::col cf = pack_col<PREC, DT>(vals);
            if constexpr (PREC == PREC_F64) {
                *reinterpret_cast<f64x4 *>(buf + (frag * 64 + lane_s) * 32) = cf;
            } else if constexpr (PREC == PREC_F32 || PREC == PREC_BF16) {
                *reinterpret_cast<typename F::col *>(buf + (frag * 64 + lane_s) * 16) = cf;
            } else {
                *reinterpret_cast<decltype(cf.hi) *>(buf + (frag * 64 + lane_s) * 16) = cf.hi;
                *reinterpret_cast<decltype(cf.lo) *>(buf + ((frag + 1) * 64 + lane_s) * 16) = cf.lo;
            }
        }
    };

    // ---- consumer setup ----
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = C::WGM == 1 ? 0 : wave / C::WGN, wn = C::WGN == 1 ? 0 : wave % C::WGN;
    const int rb0 = (S::RT == 1 ? 0 : rt * S::TRB) + wm * C::WM;
    const int cbt0 = wn * C::WN;    // first column block of the wave within the tile
    // Row blocks past the element's last block (ragged tiles) recompute the last valid block;
    // their results are never stored.
    int rbl[C::WM];
#pragma unroll
    for (int i = 0; i < C::WM; ++i) rbl[i] = (rb0 + i) < S::NRB ? (rb0 + i) : (S::NRB - 1);

    typename F::acc acc[C::WM][C::WN];
#pragma unroll
    for (int i = 0; i < C::WM; ++i)
#pragma unroll
        for (int j = 0; j < C::WN; ++j)
#pragma unroll
            for (int v = 0; v < F::ACC_N; ++v) acc[i][j][v] = 0;

    // row operand of chunk ch: fetched from the global table into registers a chunk ahead, then
    // written to an LDS buffer; the resident variant reads the whole table from LDS
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    u32x4 rstage[S::RPT > 0 ? S::RPT : 1];
    const int rbT0 = S::RT == 1 ? 0 : rt * S::TRB;
    auto fetch_rows = [&](int ch) {
        if constexpr (!C::RES) {
            const u32x4 *hi = reinterpret_cast<const u32x4 *>(a.row_hi);
            const u32x4 *lo = reinterpret_cast<const u32x4 *>(a.row_lo);
#pragma unroll
            for (int k = 0; k < S::RPT; ++k) {
                const int piece = tid + k * NT;
                if (S::RPIECES % NT == 0 || piece < S::RPIECES) {
                    const int l = piece % 64, part = (piece / 64) % S::RPART;
                    const int rbt = (piece / (64 * S::RPART)) % S::TRB, kgl = piece / (64 * S::RPART * S::TRB);
                    const int rb = (rbT0 + rbt) < S::NRB ? (rbT0 + rbt) : (S::NRB - 1);
                    const unsigned frag = (unsigned)((ch * S::KC + kgl) * S::NRB + rb);
                    if constexpr (S::SPLIT) rstage[k] = (part ? lo : hi)[frag * 64u + l];
                    else rstage[k] = hi[(frag * 64u + l) * S::RPART + part];
                }
            }
        }
    };
    auto store_rows = [&](unsigned char *rbuf) {
        if constexpr (!C::RES) {
#pragma unroll
            for (int k = 0; k < S::RPT; ++k) {
                const int piece = tid + k * NT;
                if (S::RPIECES % NT == 0 || piece < S::RPIECES) {
                    const int l = piece % 64, part = (piece / 64) % S::RPART;
                    const int frag = piece / (64 * S::RPART);
                    // LDS piece layout: [frag][lane][part] so that one lane's pieces are adjacent
                    reinterpret_cast<u32x4 *>(rbuf)[(frag * 64 + l) * S::RPART + part] = rstage[k];
                }
            }
        }
    };
    auto get_row = [&](const unsigned char *rbuf, int kgl, int i, int g) -> typename F::row {
        if constexpr (C::RES == 1) {
            return lds_row<PREC>(s_row, (size_t)g * S::NRB + rbl[i], lane);
        } else {
            const int frag = kgl * S::TRB + wm * C::WM + i;
            const unsigned char *p = rbuf + (size_t)(frag * 64 + lane) * S::RPART * 16;
            if constexpr (PREC == PREC_F64) return *reinterpret_cast<const f64x4 *>(p);
            else if constexpr (PREC == PREC_F32) return *reinterpret_cast<const f32x4 *>(p);
            else if constexpr (PREC == PREC_BF16) return *reinterpret_cast<const bf16x8 *>(p);
            else if constexpr (PREC == PREC_SPLIT_BF16) {
                SplitBF r;
                r.hi = *reinterpret_cast<const bf16x8 *>(p);
                r.lo = *reinterpret_cast<const bf16x8 *>(p + 16);
                return r;
            } else {
                SplitH r;
                r.hi = *reinterpret_cast<const f16x8 *>(p);
                r.lo = *reinterpret_cast<const f16x8 *>(p + 16);
                return r;
            }
        }
    };
    auto multiply = [&](const typename F::row (&r)[C::WM], const unsigned char *buf, int kgl) {
        typename F::col cf[C::WN];
#pragma unroll
        for (int j = 0; j < C::WN; ++j) cf[j] = get_col<PREC, S>(buf, kgl, cbt0 + j, lane);
#pragma unroll
        for (int i = 0; i < C::WM; ++i)
#pragma unroll
            for (int j = 0; j < C::WN; ++j) mma_stage<PREC, 0>(acc[i][j], r[i], cf[j]);
        if constexpr (S::SPLIT) {
#pragma unroll
            for (int i = 0; i < C::WM; ++i)
#pragma unroll
                for (int j = 0; j < C::WN; ++j) mma_stage<PREC, 1>(acc[i][j], r[i], cf[j]);
#pragma unroll
            for (int i = 0; i < C::WM; ++i)
#pragma unroll
                for (int j = 0; j < C::WN; ++j) mma_stage<PREC, 2>(acc[i][j], r[i], cf[j]);
        }
    };
    // per-wave production (PROD 1): lane's column of each of the wave's column blocks
    int w_ab[C::WN], w_bb[C::WN], w_cb[C::WN], w_el[C::WN];
#pragma unroll
    for (int j = 0; j < C::WN; ++j) {
        const int cbg = ct * S::TCB + cbt0 + j;
        const int cbc = cbg < S::NCB ? cbg : S::NCB - 1;
        const int col = cbc * TM + lane % TM;
        const int el = col / S::NSP, jj = col % S::NSP;
        const bool ok = cbg < S::NCB && jj < NS && el < neg;
        const int jc = ok ? jj : 0;
        w_el[j] = el;
        w_ab[j] = (jc % N + (ok ? 0 : N * N)) * (int)sizeof(DT2);
        w_bb[j] = ((jc / N) % N) * (int)sizeof(DT2);
        w_cb[j] = (jc / (N * N)) * (int)sizeof(DT2);
    }
    const int w_q0 = (lane / TM) * S::PPL;
    // PROD 1: point data of k-group g for one element (the PPL points of this lane's half-wave)
    // BT: byte offset of the lane's slots in the B table per column block, and the group stride
    constexpr bool PACKED = packed_columns(P, FAM);  // several elements share a column block
    constexpr int TBN = PACKED ? 1 : S::NRB;
    constexpr size_t BGSTRIDE = size_t(TBN) * 64 * S::SLOTS * sizeof(DT);
    int w_bt[C::WN];
#pragma unroll
    for (int j = 0; j < C::WN; ++j) {
        const int cbg = ct * S::TCB + cbt0 + j;
        const int cbc = cbg < S::NCB ? cbg : S::NCB - 1;
        const int jj = (cbc * TM + lane % TM) % S::NSP;
        w_bt[j] = ((PACKED ? 0 : jj / TM) * 64 + lane) * S::SLOTS * (int)sizeof(DT);
    }
    struct Pts {
        DT d[S::PPL][13];
        int oa[S::PPL], ob[S::PPL], oc[S::PPL];
        DT b[C::WN][S::SLOTS];
    };
    auto load_pts = [&](int g, int el, Pts &pt) {
#pragma unroll
        for (int sub = 0; sub < S::PPL; ++sub) {
            const int q = g * S::KGP + w_q0 + sub;
            const DT *Dh = s_D + ((size_t)el * NQP + q) * S::DSTR;
#pragma unroll
            for (int uu = 0; uu < 13; ++uu) pt.d[sub][uu] = Dh[uu];
            if constexpr (!C::BT) {
                pt.oa[sub] = s_pt[q];
                pt.ob[sub] = s_pt[NQP + q];
                pt.oc[sub] = s_pt[2 * NQP + q];
            }
        }
    };
    // BT: the lane's B factors of column block j at k-group g (L2-resident table)
    auto load_btab = [&](int g, int j, Pts &pt) {
        if constexpr (C::BT) {
            const char *src = reinterpret_cast<const char *>(a.bcol) + (size_t)g * BGSTRIDE + w_bt[j];
            typedef DT dt4 __attribute__((ext_vector_type(4)));
#pragma unroll
            for (int h = 0; h < S::SLOTS / 4; ++h) {
                const dt4 x = *reinterpret_cast<const dt4 *>(src + h * 4 * sizeof(DT));
#pragma unroll
                for (int u = 0; u < 4; ++u) pt.b[j][h * 4 + u] = x[u];
            }
        }
    };
    // column block j of the wave from the point data
    auto col_from = [&](const Pts &pt, int j) -> typename F::col {
        DT vals[S::SLOTS];
#pragma unroll
        for (int sub = 0; sub < S::PPL; ++sub) {
            DT out[4];
            if constexpr (C::BT) {
                const DT *bq = pt.b[j] + sub * 4;
                const DT *d = pt.d[sub];
                out[0] = d[0] * bq[0] + d[1] * bq[1] + d[2] * bq[2] + d[3] * bq[3];
                out[1] = d[4] * bq[1] + d[5] * bq[2] + d[6] * bq[3];
                out[2] = d[7] * bq[1] + d[8] * bq[2] + d[9] * bq[3];
                out[3] = d[10] * bq[1] + d[11] * bq[2] + d[12] * bq[3];
            } else {
                const DT2 fa = *reinterpret_cast<const DT2 *>(ldb + pt.oa[sub] + w_ab[j]);
                const DT2 fb = *reinterpret_cast<const DT2 *>(ldb + pt.ob[sub] + w_bb[j]);
                const DT2 fc = *reinterpret_cast<const DT2 *>(ldb + pt.oc[sub] + w_cb[j]);
                column_values<DT>(pt.d[sub], fa[0], fa[1], fb[0], fb[1], fc[0], fc[1], out);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) vals[sub * 4 + r] = out[r];
        }
        return pack_col<PREC, DT>(vals);
    };
    // the wave's column operand of the current k-group; column block j of k-group g + 1 is
    // produced right after the MFMAs that read block j of k-group g are issued, so the
    // production overlaps the matrix cores
    typename F::col cfw[C::WN];
    auto produce_first = [&]() {
        Pts pt;
        if constexpr (S::WAVE_ONE_EL) load_pts(0, w_el[0], pt);
#pragma unroll
        for (int j = 0; j < C::WN; ++j) {
            if constexpr (!S::WAVE_ONE_EL) load_pts(0, w_el[j], pt);
            load_btab(0, j, pt);
            cfw[j] = col_from(pt, j);
        }
    };
    // gn: the k-group produced for the next step (g + 1), or -1 for none; after_mma() runs as
    // soon as the last MFMA that reads r is issued (the streamed-row loop reloads r there)
    auto step_regs = [&](const typename F::row (&r)[C::WM], int g, int gn, auto &&after_mma) {
        const bool more = gn >= 0;
        Pts pt;
        if constexpr (S::WAVE_ONE_EL) {
            if (more) {
                load_pts(gn, w_el[0], pt);
#pragma unroll
                for (int j = 0; j < C::WN; ++j) load_btab(gn, j, pt);
            }
        }
#pragma unroll
        for (int j = 0; j < C::WN; ++j) {
#pragma unroll
            for (int i = 0; i < C::WM; ++i) mma_stage<PREC, 0>(acc[i][j], r[i], cfw[j]);
            if constexpr (S::SPLIT) {
#pragma unroll
                for (int i = 0; i < C::WM; ++i) mma_stage<PREC, 1>(acc[i][j], r[i], cfw[j]);
#pragma unroll
                for (int i = 0; i < C::WM; ++i) mma_stage<PREC, 2>(acc[i][j], r[i], cfw[j]);
            }
            if (j == C::WN - 1) after_mma();
            if (more) {
                if constexpr (!S::WAVE_ONE_EL) {
                    load_pts(gn, w_el[j], pt);
                    load_btab(gn, j, pt);
                }
                cfw[j] = col_from(pt, j);
            }
        }
    };

    auto consume_chunk = [&](int ch, const unsigned char *cbuf, const unsigned char *rbuf) {
        if constexpr (C::PROD == 0) {
#pragma unroll
            for (int kgl = 0; kgl < S::KC; ++kgl) {
                typename F::row rr[C::WM];
#pragma unroll
                for (int i = 0; i < C::WM; ++i) rr[i] = get_row(rbuf, kgl, i, ch * S::KC + kgl);
                multiply(rr, cbuf, kgl);
            }
        } else {
#pragma unroll
            for (int kgl = 0; kgl < S::KC; ++kgl) {
                const int g = ch * S::KC + kgl;
                typename F::row rr[C::WM];
#pragma unroll
                for (int i = 0; i < C::WM; ++i) rr[i] = get_row(rbuf, kgl, i, g);
                step_regs(rr, g, g + 1 < S::NGP ? g + 1 : -1, [] {});
            }
        }
    };

    // Tiles with two or more waves per SIMD order their waves' issue by phase: the main loop
    // (matrix-core work) first, then the load vector and the stores, then the prologue, so
    // that the waves on one SIMD overlap one another's phases instead of contending.
    if constexpr (C::OCC > 1) __builtin_amdgcn_s_setprio(2);
    if constexpr (C::RES == 3) {
        // ---- main loop, rows held in registers: the wave's row fragments of every k-group are
        // loaded at once (one L2 round trip per item), the k loop is unrolled, no barrier.
        typename F::row rres[S::NGP][C::WM];
#pragma unroll
        for (int g = 0; g < S::NGP; ++g)
#pragma unroll
            for (int i = 0; i < C::WM; ++i)
                rres[g][i] = load_row_off<PREC>(a, (unsigned)(g * S::NRB + rbl[i]), lane);
        produce_first();
#pragma unroll
        for (int g = 0; g < S::NGP; ++g) step_regs(rres[g], g, g + 1 < S::NGP ? g + 1 : -1, [] {});
    } else if constexpr (C::RES == 2) {
        // ---- main loop, rows streamed: each wave loads its row fragments of k-group g + 1 from
        // the table (L2-resident) while it multiplies k-group g; no workgroup barrier. The last
        // iteration reloads and reproduces k-group NGP - 1, so the loop body has no branch.
        typename F::row rr[C::WM];
#pragma unroll
        for (int i = 0; i < C::WM; ++i) rr[i] = load_row_off<PREC>(a, (unsigned)rbl[i], lane);
        produce_first();
#pragma unroll 1
        for (int g = 0; g < S::NGP; ++g) {
            const int gn = g + 1 < S::NGP ? g + 1 : g;
            // the next rows are loaded into the same registers once the last MFMA reading them
            // is issued; their latency hides behind the production of the last column block
            step_regs(rr, g, gn, [&] {
#pragma unroll
                for (int i = 0; i < C::WM; ++i)
                    rr[i] = load_row_off<PREC>(a, (unsigned)(gn * S::NRB + rbl[i]), lane);
            });
        }
    } else {
        // ---- main loop: produce chunk c+1 and fetch its rows while multiplying chunk c ----
        fetch_rows(0);
        store_rows(s_rb0);
        if constexpr (C::PROD == 0) produce_chunk(0, s_cb0);
        else produce_first();
        __syncthreads();
#pragma unroll 1
        for (int ch = 0; ch + 1 < S::NCH; ++ch) {
            const bool odd = ch & 1;
            fetch_rows(ch + 1);
            // reads of the current chunk are issued before the writes of the next one, so the
            // MFMAs do not wait behind the producer's LDS stores and the two interleave
            consume_chunk(ch, odd ? s_cb1 : s_cb0, odd ? s_rb1 : s_rb0);
            if constexpr (C::PROD == 0) produce_chunk(ch + 1, odd ? s_cb0 : s_cb1);
            store_rows(odd ? s_rb0 : s_rb1);
            if constexpr (C::PROD == 0 || !C::RES) __syncthreads();  // chunk buffers change hands
        }
        consume_chunk(S::NCH - 1, ((S::NCH - 1) & 1) ? s_cb1 : s_cb0, ((S::NCH - 1) & 1) ? s_rb1 : s_rb0);
    }

    if constexpr (C::OCC > 1) __builtin_amdgcn_s_setprio(1);
    using OT = typename S::OT;
    __syncthreads();  // every wave is done with the point matrices and the chunks

    // ---- load vector b_i = sum_q w_q detJ_q f phi_i(xi_q), FP64, by one workgroup per element.
    // The sum runs over q1, q2, q3 in turn (phi_i is a product of 1-D factors); same terms, the
    // additions grouped by direction.
    if (S::PRISM && rt == 0 && ct == 0 && a.out_b) {
        // prisms: b_i = sum_q (w detJ f)_q phi_i(xi_q), the values read from the FP64 table
        OT *outb = reinterpret_cast<OT *>(a.out_b);
        for (int t = tid; t < EG * NS; t += NT) {
            const int el = t / NS, r = t % NS;
            if (el >= neg) continue;
            const double *wf = s_wf + (size_t)el * NQP;
            double sum = 0.0;
#pragma unroll 4
            for (int q = 0; q < NQ; ++q) sum += wf[q] * a.phi64[(size_t)q * NS + r];
            const int64_t e = element_id(elist, e0 + el);
            const int64_t base = a.b_off ? a.b_off[e] : a.b_base + e * a.b_stride;
            outb[base + r] = (OT)sum;
        }
    }
    if (!S::PRISM && rt == 0 && ct == 0 && a.out_b) {
        const int tot = EG * NS;
        // t1[el][q3][q2][a] = sum_q1 L[q1][a] wf[el][q1 + N q2 + N^2 q3]
        for (int t = tid; t < tot; t += NT) {
            const int el = t / NS, r = t % NS;
            const int a_ = r % N, q2 = (r / N) % N, q3 = r / (N * N);
            const double *wf = s_wf + (size_t)el * NQP + N * (q2 + N * q3);
            double sum = 0.0;
#pragma unroll
            for (int q1 = 0; q1 < N; ++q1) sum += s_ld64[(q1 * N + a_) * 2] * wf[q1];
            s_t1[t] = sum;
        }
        __syncthreads();
        // t2[el][q3][b][a] = sum_q2 L[q2][b] t1[el][q3][q2][a]
        for (int t = tid; t < tot; t += NT) {
            const int el = t / NS, r = t % NS;
            const int a_ = r % N, b_ = (r / N) % N, q3 = r / (N * N);
            const double *t1 = s_t1 + (size_t)el * NS + N * N * q3 + a_;
            double sum = 0.0;
#pragma unroll
            for (int q2 = 0; q2 < N; ++q2) sum += s_ld64[(q2 * N + b_) * 2] * t1[N * q2];
            s_t2[t] = sum;
        }
        __syncthreads();
        // b[el][c][b][a] = sum_q3 L[q3][c] t2[el][q3][b][a]
        OT *outb = reinterpret_cast<OT *>(a.out_b);
        for (int t = tid; t < tot; t += NT) {
            const int el = t / NS, r = t % NS;
            if (el >= neg) continue;
            const int ab = r % (N * N), c_ = r / (N * N);
            const double *t2 = s_t2 + (size_t)el * NS + ab;
            double sum = 0.0;
#pragma unroll
            for (int q3 = 0; q3 < N; ++q3) sum += s_ld64[(q3 * N + c_) * 2] * t2[N * N * q3];
            const int64_t e = element_id(elist, e0 + el);
            const int64_t base = a.b_off ? a.b_off[e] : a.b_base + e * a.b_stride;
            outb[base + r] = (OT)sum;
        }
        __syncthreads();  // the temporaries overlay the staging area below
    }

    // ---- epilogue: unpadded row-major store ----
    OT *outA = reinterpret_cast<OT *>(a.out_A);
    static_assert(S::off_D % 16 == 0, "staged images start 16-byte aligned");
    constexpr int VW = S::VW;
    typedef OT vec_t __attribute__((ext_vector_type(VW)));
    // Write n values from a staged image to dst (img[x] belongs at dst[x]; img is 16-byte aligned
    // where dst is) with whole 16-byte vectors between a scalar head and tail. Threads t of NTH.
    auto copy_out = [&](OT *dst, const OT *img, int n, int t, int nth) {
        const int mis = (int)((reinterpret_cast<uintptr_t>(dst) & 15) / sizeof(OT));
        const int head = mis ? (VW - mis < n ? VW - mis : n) : 0;
        const int nvec = (n - head) / VW;
        const int tail0 = head + nvec * VW;
        if (t < head) dst[t] = img[t];
        for (int k = t; k < nvec; k += nth) {
            const int idx = head + k * VW;
            *reinterpret_cast<vec_t *>(dst + idx) = *reinterpret_cast<const vec_t *>(img + idx);
        }
        for (int x = tail0 + t; x < n; x += nth) dst[x] = img[x];
    };
    // offset of an image so that image index x sits at the same position within 16 bytes as dst[x]
    auto img_shift = [](const OT *dst) { return (int)((reinterpret_cast<uintptr_t>(dst) & 15) / sizeof(OT)); };
    // The transposed copy (elastic blocks, a.at_base > 0; per-wave staging, TRANS_EPI) of staged
    // rows r0 .. r0 + nrow - 1, img[rl * NS + c]: destination row c receives them as one
    // contiguous run at column r0.
    const bool trans = a.at_base > 0;
    auto copy_out_t = [&](OT *dT, const OT *img, int nrow, int r0, int t, int nth) {
#pragma unroll 1
        for (int x = t; x < NS * TM; x += nth) {
            const int c = x / TM, rl = x % TM;
            if (rl < nrow) dT[(int64_t)c * NS + r0 + rl] = img[rl * NS + c];
        }
    };
    // The transposed copy straight from one accumulator block (TRANS_REG): this lane's column jj
    // of the block starting at row r0 becomes row jj of the transposed block; its accumulator
    // entries 4g .. 4g + 3 are four consecutive rows, so one 16-byte store each where the
    // destination is 16-byte aligned and all four rows exist, else scalar stores.
    auto write_t = [&](OT *dT, const typename F::acc &ac, int r0, int jj, float us) {
        if constexpr (S::TRANS_REG && FAM == MF_F64) {
            if (jj >= NS) return;
            OT *rowp = dT + (int64_t)jj * NS;
#pragma unroll
            for (int v = 0; v < F::ACC_N; ++v) {
                const int row = r0 + acc_row<FAM>(lane, v);
                if (row < NS) rowp[row] = ac[v];
            }
        } else if constexpr (S::TRANS_REG) {
            static_assert(std::is_same<OT, float>::value, "the 32-wide families write FP32");
            if (jj >= NS) return;
            OT *rowp = dT + (int64_t)jj * NS;
            const bool vec = (reinterpret_cast<uintptr_t>(rowp) & 15) == 0;
#pragma unroll
            for (int g = 0; g < F::ACC_N / 4; ++g) {
                const int row = r0 + acc_row<FAM>(lane, 4 * g);
                if (row >= NS) continue;
                const float v0 = ac[4 * g] * us, v1 = ac[4 * g + 1] * us, v2 = ac[4 * g + 2] * us,
                            v3 = ac[4 * g + 3] * us;
                if (NS % 4 == 0 && vec) {  // Ns % 4 == 0: all four rows are in range
                    f32x4 q = {v0, v1, v2, v3};
                    *reinterpret_cast<f32x4 *>(rowp + row) = q;
                } else {
                    rowp[row] = v0;
                    if (row + 1 < NS) rowp[row + 1] = v1;
                    if (row + 2 < NS) rowp[row + 2] = v2;
                    if (row + 3 < NS) rowp[row + 3] = v3;
                }
            }
        }
    };
    if constexpr (S::STAGE_WAVE) {
        // This wave's element: column blocks cbt0 .. cbt0 + WN - 1 of the tile are its columns.
        const int el = (cbt0 * TM) / S::NSP;
        OT *stage = reinterpret_cast<OT *>(smem + S::off_D) + (size_t)wave * S::WIMG;
        if (el < neg) {
            const int64_t e = element_id(elist, e0 + el);
            OT *dst0 = outA + (a.a_off ? a.a_off[e] : a.a_base + e * a.a_stride);
            const float us = S::SPLIT ? a.row_scale_inv / split_scale(s_dmax[el], a.c_bound)
                                      : a.row_scale_inv;
#pragma unroll
            for (int i = 0; i < C::WM; ++i) {
                const int r0 = i * TM;
                if (r0 >= NS) break;
                const int nrow = NS - r0 < TM ? NS - r0 : TM;
                OT *dst = dst0 + (int64_t)r0 * NS;
                OT *img = stage + img_shift(dst);
#pragma unroll
                for (int j = 0; j < C::WN; ++j) {
                    const int jj = j * TM + (lane % TM);
#pragma unroll
                    for (int v = 0; v < F::ACC_N; ++v) {
                        const int rl = acc_row<FAM>(lane, v);
                        if (jj < NS && rl < nrow)
                            img[rl * NS + jj] = (PREC == PREC_F64) ? OT(acc[i][j][v]) : OT(acc[i][j][v] * us);
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                // rows r0 .. r0 + nrow - 1 are one contiguous range of the element's matrix
                copy_out(dst, img, nrow * NS, lane, 64);
                if constexpr (S::TRANS_EPI)
                    if (trans) copy_out_t(outA + a.at_base + e * a.a_stride, img, nrow, r0, lane, 64);
                if constexpr (S::TRANS_REG)
                    if (trans) {
#pragma unroll
                        for (int j = 0; j < C::WN; ++j)
                            write_t(outA + a.at_base + e * a.a_stride, acc[i][j], r0, j * TM + (lane % TM), us);
                    }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
    } else if constexpr (S::STAGE_RB) {
        // One row block of every element at a time (all waves hold the same row blocks).
        OT *s_img = reinterpret_cast<OT *>(smem + S::off_D);
#pragma unroll
        for (int i = 0; i < C::WM; ++i) {
            const int r0 = i * TM;
            if (r0 >= NS) break;
            const int nrow = NS - r0 < TM ? NS - r0 : TM;
#pragma unroll
            for (int j = 0; j < C::WN; ++j) {
                const int cb = cbt0 + j;
                const int col = cb * TM + (lane % TM);
                const int el = col / S::NSP, jj = col % S::NSP;
                if (jj >= NS || el >= neg) continue;
                const int64_t e = element_id(elist, e0 + el);
                OT *dst = outA + (a.a_off ? a.a_off[e] : a.a_base + e * a.a_stride) + (int64_t)r0 * NS;
                OT *img = s_img + el * S::WIMG + img_shift(dst);
                const float us = S::SPLIT ? a.row_scale_inv / split_scale(s_dmax[el], a.c_bound)
                                          : a.row_scale_inv;
#pragma unroll
                for (int v = 0; v < F::ACC_N; ++v) {
                    const int rl = acc_row<FAM>(lane, v);
                    if (rl < nrow)
                        img[rl * NS + jj] = (PREC == PREC_F64) ? OT(acc[i][j][v]) : OT(acc[i][j][v] * us);
                }
                if constexpr (S::TRANS_REG)
                    if (trans) write_t(outA + a.at_base + e * a.a_stride, acc[i][j], r0, jj, us);
            }
            __syncthreads();
            for (int el = 0; el < neg; ++el) {
                const int64_t e = element_id(elist, e0 + el);
                OT *dst = outA + (a.a_off ? a.a_off[e] : a.a_base + e * a.a_stride) + (int64_t)r0 * NS;
                copy_out(dst, s_img + el * S::WIMG + img_shift(dst), nrow * NS, tid, NT);
            }
            __syncthreads();
        }
    } else if constexpr (S::STAGE_OUT) {
        // The workgroup owns whole elements: stage each element's matrix as it lies in memory,
        // then write each element's contiguous Ns x Ns block with aligned 16-byte stores.
        OT *s_out = reinterpret_cast<OT *>(smem + S::off_D);
#pragma unroll
        for (int j = 0; j < C::WN; ++j) {
            const int cb = ct * S::TCB + cbt0 + j;
            if (cb >= S::NCB) continue;
            const int col = cb * TM + (lane % TM);
            const int el = col / S::NSP, jj = col % S::NSP;
            if (jj >= NS || el >= neg) continue;
            const int64_t e = element_id(elist, e0 + el);
            OT *img = s_out + el * S::IMG + img_shift(outA + (a.a_off ? a.a_off[e] : a.a_base + e * a.a_stride));
            const float us = S::SPLIT ? a.row_scale_inv / split_scale(s_dmax[el], a.c_bound)
                                      : a.row_scale_inv;
#pragma unroll
            for (int i = 0; i < C::WM; ++i) {
                if (rb0 + i >= S::NRB) continue;
#pragma unroll
                for (int v = 0; v < F::ACC_N; ++v) {
                    const int row = (rb0 + i) * TM + acc_row<FAM>(lane, v);
                    if (row < NS) {
                        if constexpr (PREC == PREC_F64) img[row * NS + jj] = acc[i][j][v];
                        else img[row * NS + jj] = acc[i][j][v] * us;
                    }
                }
                if constexpr (S::TRANS_REG)
                    if (trans) write_t(outA + a.at_base + e * a.a_stride, acc[i][j], (rb0 + i) * TM, jj, us);
            }
        }
        __syncthreads();
        for (int el = 0; el < neg; ++el) {
            const int64_t e = element_id(elist, e0 + el);
            OT *dst = outA + (a.a_off ? a.a_off[e] : a.a_base + e * a.a_stride);
            const OT *img = s_out + el * S::IMG + img_shift(dst);
            copy_out(dst, img, NS * NS, tid, NT);
            if constexpr (S::TRANS_EPI) {
                // the transposed block (elastic lower block): entry x = c Ns + r of the copy is
                // img[r Ns + c]; consecutive threads read LDS at the odd stride Ns
                if (trans) {
                    OT *dT = outA + a.at_base + e * a.a_stride;
                    for (int x = tid; x < NS * NS; x += NT) {
                        const int c = x / NS, r = x - c * NS;
                        dT[x] = img[r * NS + c];
                    }
                }
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < C::WN; ++j) {
            const int cb = ct * S::TCB + cbt0 + j;
            if (cb >= S::NCB) continue;
            const int col = cb * TM + (lane % TM);
            const int el = col / S::NSP, jj = col % S::NSP;
            if (jj >= NS || el >= neg) continue;
            const int64_t e = element_id(elist, e0 + el);
            const int64_t base = a.a_off ? a.a_off[e] : a.a_base + e * a.a_stride;
            const float us = S::SPLIT ? a.row_scale_inv / split_scale(s_dmax[el], a.c_bound)
                                      : a.row_scale_inv;
#pragma unroll
            for (int i = 0; i < C::WM; ++i) {
                if (rb0 + i >= S::NRB) continue;
#pragma unroll
                for (int v = 0; v < F::ACC_N; ++v) {
                    const int row = (rb0 + i) * TM + acc_row<FAM>(lane, v);
                    if (row < NS) {
                        if constexpr (PREC == PREC_F64) outA[base + (int64_t)row * NS + jj] = acc[i][j][v];
                        else outA[base + (int64_t)row * NS + jj] = acc[i][j][v] * us;
                    }
                }
                if constexpr (S::TRANS_REG)
                    if (trans) write_t(outA + a.at_base + e * a.a_stride, acc[i][j], (rb0 + i) * TM, jj, us);
            }
        }
    }

    __syncthreads();  // LDS is rewritten by the next item
}

// The work items wi, wi + stride, wi + 2 stride, ... of one degree, processed by one workgroup
// (a persistent loop); per-workgroup constants are loaded once. The element count comes from
// the host (nel) or, for the buckets of a mixed-degree call, from device memory (seg), so no
// host synchronisation is needed between bucketing and integration. Returns at once if wi is
// past the last item. Every thread of the workgroup must call it with the same arguments.
template <int P, int PREC, class C, bool SUP>
__device__ inline void run_items(const KArgs &a, int64_t wi, const int64_t stride, unsigned char *smem)
{
    using S = Shape<P, PREC, C>;
    constexpr int N = S::N, NT = S::NT;
    int64_t nel = a.nel;
    const int32_t *elist = a.elist;
    if (a.seg) {
        elist = a.elist + a.seg[0];
        nel = a.seg[1];
    }
    const int64_t total = ((nel + S::EG - 1) / S::EG) * S::RT * S::CT;
    if (wi >= total) return;
    const int tid = threadIdx.x;
    const int reclen = a.mode == 0 ? 14 : (a.mode == 1 ? 10 : 5);

    // ---- per-workgroup constants: tables, field descriptor, point rows, resident row table ----
    double *s_fld = reinterpret_cast<double *>(smem + S::off_fld);
    double *s_ld64 = reinterpret_cast<double *>(smem + S::off_ld64);
    float *s_ld32 = reinterpret_cast<float *>(smem + S::off_ld32);
    double *s_qw = reinterpret_cast<double *>(smem + S::off_qw);
    int *s_pt = reinterpret_cast<int *>(smem + S::off_pt);
    if (a.mode == 1)
        for (int t = tid; t < 175; t += NT) s_fld[t] = a.field[t];
    if constexpr (S::PRISM) {
        // points (xi1, xi2, zeta) and weights; padded points are zero
        for (int t = tid; t < 4 * S::NQP; t += NT) s_qw[t] = t < 4 * S::NQ ? a.xq[t] : 0.0;
    }
    if constexpr (!S::PRISM) {
    for (int t = tid; t < N * N * 2; t += NT) {
        s_ld64[t] = a.LD64[t];
        s_ld32[t] = a.LD32[t];
        s_ld64[N * N * 2 + t] = 0.0;
        s_ld32[N * N * 2 + t] = 0.0f;
    }
    for (int t = tid; t < N; t += NT) {
        s_qw[t] = a.xq[t];
        s_qw[N + t] = a.wq[t];
    }
    // per point: byte offsets of the 1-D table rows it reads (q1, q2, q3), three arrays
    {
        constexpr int ROWBYTES = N * 2 * sizeof(typename S::DT);
        for (int q = tid; q < S::NQP; q += NT) {
            const bool ok = q < S::NQ;
            s_pt[q] = ok ? (q % N) * ROWBYTES : 0;
            s_pt[S::NQP + q] = ok ? ((q / N) % N) * ROWBYTES : 0;
            s_pt[2 * S::NQP + q] = ok ? (q / (N * N)) * ROWBYTES : 0;
        }
    }
    }  // hexahedra
    if constexpr (C::RES == 1) {
        // [frag][part][lane] x 16 B (split), [frag][lane] x 16 B or 32 B otherwise
        typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
        u32x4 *dst = reinterpret_cast<u32x4 *>(smem + S::off_row);
        const u32x4 *hi = reinterpret_cast<const u32x4 *>(a.row_hi);
        const u32x4 *lo = reinterpret_cast<const u32x4 *>(a.row_lo);
        constexpr size_t nfrag = size_t(S::NGP) * S::NRB;
        if constexpr (S::SPLIT) {
            for (size_t t = tid; t < nfrag * 128; t += NT) {
                const size_t frag = t / 128, part = (t / 64) % 2, l = t % 64;
                dst[t] = part ? lo[frag * 64 + l] : hi[frag * 64 + l];
            }
        } else {
            constexpr int per = S::ROWB / 16;
            for (size_t t = tid; t < nfrag * 64 * per; t += NT) dst[t] = hi[t];
        }
    }

    Item it = decode_item<S>(wi, nel);
    double pf[S::PFN], pf_next[S::PFN];
    fetch_elements<S, SUP>(a, elist, it, reclen, pf);
    __syncthreads();
    for (;;) {
        const int64_t wn = wi + stride;
        const bool has_next = wn < total;
        const Item itn = has_next ? decode_item<S>(wn, nel) : it;
        integrate_item<P, PREC, C, SUP>(a, it, elist, reclen, smem, pf, pf_next, has_next, itn);
        if (!has_next) break;
        wi = wn;
        it = itn;
#pragma unroll
        for (int k = 0; k < S::PFN; ++k) pf[k] = pf_next[k];
    }
}

// One degree per launch: a persistent grid over that degree's work items. SUP: the Jacobian
// terms are read from a.jac (a separate instance, so the computing one carries none of it).
template <int P, int PREC, class C, bool SUP>
__global__ void __launch_bounds__(C::NW * 64) __attribute__((amdgpu_waves_per_eu(C::OCC, 8)))
k_integrate(const KArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    run_items<P, PREC, C, SUP>(a, blockIdx.x, gridDim.x, smem);
}

// Every degree in one launch. The work items of the degrees, heaviest degree first, form one
// index space that the persistent grid strides through; a workgroup handles its items of one
// degree as a run (constants loaded once per run), then moves on to the next degree.
struct MixedKArgs {
    KArgs deg[7];     // deg[p - 1]: the bucket of degree p (seg = its {start, count})
    int32_t tile[8];  // tile[p - 1]: the tile alternative (0, 1) degree p runs with
};
// mixed_args reads deg[d] from the kernel-argument segment, where the launch's only argument
// starts at offset 0: a plain copyable struct whose first member is deg
static_assert(std::is_trivially_copyable<MixedKArgs>::value && std::is_standard_layout<MixedKArgs>::value &&
                  offsetof(MixedKArgs, deg) == 0,
              "MixedKArgs is read through the argument segment");

// The arguments of degree d + 1, read from the kernel-argument segment (the launch's only
// argument, a MixedKArgs, starts at its offset 0) through a pointer the compiler cannot see
// through: a degree's arguments are then loaded where its segment uses them, instead of all
// seven degrees' arguments being loaded at kernel entry and held in scalar registers (which
// spills) for the whole launch.
__device__ inline const KArgs &mixed_args(int d)
{
    typedef const __attribute__((address_space(4))) MixedKArgs *kptr;
    kptr p = (kptr)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(p));
    return *(const KArgs *)(&p->deg[d]);
}

template <int P, int PREC, class C, bool SUP>
__device__ inline void mixed_segment(const KArgs &a, int64_t &base, unsigned char *smem)
{
    using S = Shape<P, PREC, C>;
    static_assert(C::NW * 64 == 256, "the mixed-degree kernel runs 256-thread workgroups");
    const int64_t count = a.seg[1];
    const int64_t total = ((count + S::EG - 1) / S::EG) * S::RT * S::CT;
    if (total > 0) {
        const int64_t g = gridDim.x;
        // first index >= base of the form blockIdx.x + k g, relative to base
        const int64_t wi = (((int64_t)blockIdx.x - base) % g + g) % g;
        if (wi < total) {
            run_items<P, PREC, C, SUP>(a, wi, g, smem);
            __syncthreads();  // the next degree's constants reuse the LDS
        }
    }
    base += total;
}

// Degree P's segment with the tile alternative the launch chose for it (uniform over the grid).
template <int P, int PREC, class MT, bool SUP>
__device__ inline void mixed_degree(const MixedKArgs &m, int64_t &base, unsigned char *smem)
{
    if constexpr (MT::template has_alt<P>()) {
        if (m.tile[P - 1] != 0) {
            mixed_segment<P, PREC, typename MT::template C<P, 1>, SUP>(mixed_args(P - 1), base, smem);
            return;
        }
    }
    mixed_segment<P, PREC, typename MT::template C<P, 0>, SUP>(mixed_args(P - 1), base, smem);
}

// MT: the tile set (MT::C<P, t>: alternative t of degree P; MT::has_alt<P>(): two alternatives).
template <int PREC, bool SUP, class MT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 8)))
k_integrate_mixed(const MixedKArgs m)
{
    extern __shared__ __align__(16) unsigned char smem[];
    int64_t base = 0;
    mixed_degree<7, PREC, MT, SUP>(m, base, smem);
    mixed_degree<6, PREC, MT, SUP>(m, base, smem);
    mixed_degree<5, PREC, MT, SUP>(m, base, smem);
    mixed_degree<4, PREC, MT, SUP>(m, base, smem);
    mixed_degree<3, PREC, MT, SUP>(m, base, smem);
    mixed_degree<2, PREC, MT, SUP>(m, base, smem);
    mixed_degree<1, PREC, MT, SUP>(m, base, smem);
}

}  // namespace fem
