// fem_layout.h -- the order in which the contraction A = B^T blockdiag(D_q) B is fed to the
// CDNA4 matrix cores, shared by the host table builder and the kernels.
//
// The contraction runs over k = (q, r): quadrature point q and r = 0 (value) or 1..3 (reference
// derivative), depth 4 N_Q. Each k-group holds KGP consecutive quadrature points. Within a
// group, lane l of a wave and per-lane slot v address
//     point = g*KGP + (l / TM) * PPL + v / 4,   r = v % 4,
// on both operands: the row operand B^T (test function i = rb*TM + l % TM, from a constant
// table) and the column operand C = D_q B (trial function j, produced per element in registers).
//
//   family  instruction (gfx950)          TM  KGP PPL  slots/lane  MFMA per group
//   MF_K16  v_mfma_f32_32x32x16_{bf16,f16} 32   4   2   8           1 (x3 when split)
//   MF_F32  v_mfma_f32_32x32x2_f32         32   2   1   4           4 (slot v = step)
//   MF_F64  v_mfma_f64_16x16x4_f64         16   4   1   4           4 (slot v = step)
//
// Row-operand tables are stored [g][rb][lane][slot], one 64-lane fragment per (g, rb), so a
// wave loads a fragment with one contiguous, fully coalesced access. Padded rows (i >= Ns) and
// padded points (q >= N_Q) hold zeros.
#pragma once

#ifdef __HIPCC__
#define FEM_HD __host__ __device__
#else
#define FEM_HD
#endif

namespace fem {

enum Precision : int { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16 = 2, PREC_SPLIT_BF16 = 3, PREC_SPLIT_F16 = 4 };
enum Family : int { MF_K16 = 0, MF_F32 = 1, MF_F64 = 2 };

FEM_HD constexpr int family_of(int prec)
{
    return prec == PREC_F64 ? MF_F64 : (prec == PREC_F32 ? MF_F32 : MF_K16);
}
FEM_HD constexpr int fam_tm(int fam) { return fam == MF_F64 ? 16 : 32; }
FEM_HD constexpr int fam_kgp(int fam) { return fam == MF_F32 ? 2 : 4; }
FEM_HD constexpr int fam_ppl(int fam) { return fam == MF_K16 ? 2 : 1; }
FEM_HD constexpr int fam_slots(int fam) { return fam == MF_K16 ? 8 : 4; }

// Element kinds share the kernels: the degree argument P of the tables and kernel templates is
// p for the hexahedron of degree p and PRISM_BASE + p for the prism of degree p (the reference
// element of section 2, Tables 1-2: the complete degree-p polynomials on the triangle times the
// 1-D degree-p polynomials in the vertical direction).
constexpr int PRISM_BASE = 10;
FEM_HD constexpr bool is_prism(int P) { return P > PRISM_BASE; }
FEM_HD constexpr int deg_of(int P) { return is_prism(P) ? P - PRISM_BASE : P; }
// Triangle points of the prism's quadrature (Table 1: N_Q / (p+1)).
FEM_HD constexpr int prism_tri_points(int p)
{
    return p == 1 ? 3 : p == 2 ? 6 : p == 3 ? 12 : p == 4 ? 16 : p == 5 ? 25 : p == 6 ? 33 : 42;
}
// Shape functions and quadrature points per element: (p+1)^3 and (p+1)^3 for the hexahedron,
// (p+1)^2 (p+2)/2 and prism_tri_points(p) (p+1) for the prism.
FEM_HD constexpr int ns_of(int P)
{
    return is_prism(P) ? (deg_of(P) + 1) * (deg_of(P) + 1) * (deg_of(P) + 2) / 2
                       : (P + 1) * (P + 1) * (P + 1);
}
FEM_HD constexpr int nq_of(int P)
{
    return is_prism(P) ? prism_tri_points(deg_of(P)) * (deg_of(P) + 1) : ns_of(P);
}
FEM_HD constexpr int groups_of(int p, int fam) { return (nq_of(p) + fam_kgp(fam) - 1) / fam_kgp(fam); }
// Row-operand tables hold this many k-groups (a multiple of 8, so that every chunk size of the
// kernels divides it); groups past groups_of() are zero.
FEM_HD constexpr int groups_padded(int p, int fam) { return (groups_of(p, fam) + 7) / 8 * 8; }
FEM_HD constexpr int rblocks_of(int p, int fam) { return (ns_of(p) + fam_tm(fam) - 1) / fam_tm(fam); }
// Column pitch of an element in the column operand: elements with at most half a block of trial
// functions share blocks at the smallest power-of-two pitch >= Ns (it divides the block width, so
// every block holds whole elements); larger elements start at a block boundary.
FEM_HD constexpr bool packed_columns(int p, int fam) { return 2 * ns_of(p) <= fam_tm(fam); }
FEM_HD constexpr int packed_pitch(int p)
{
    return ns_of(p) <= 1 ? 1 : ns_of(p) <= 2 ? 2 : ns_of(p) <= 4 ? 4 : ns_of(p) <= 8 ? 8 : 16;
}
FEM_HD constexpr int col_pitch(int p, int fam)
{
    return packed_columns(p, fam) ? packed_pitch(p) : rblocks_of(p, fam) * fam_tm(fam);
}

// Point and component addressed by (group g, lane l, slot v).
FEM_HD constexpr int slot_point(int fam, int g, int lane, int v)
{
    return g * fam_kgp(fam) + (lane / fam_tm(fam)) * fam_ppl(fam) + v / 4;
}
FEM_HD constexpr int slot_comp(int v) { return v % 4; }

// Power-of-two scale of the FP16 row-operand table (keeps small entries of B^T out of the FP16
// subnormal range; every |B| entry stays far below the FP16 maximum for p <= 7).
constexpr float F16_TABLE_SCALE = 256.0f;
// The per-element FP16 scale makes max |C| <= 2^15.
constexpr float F16_C_TARGET = 32768.0f;

}  // namespace fem
