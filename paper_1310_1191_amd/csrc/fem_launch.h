// fem_launch.h -- the compiled tile configurations ("variants") per (degree, precision family)
// and their launch. Variant 0 is the default; fem_autotune times all variants of a
// (degree, precision) and records the fastest.
#pragma once
#include "fem_kernel.h"
#include "fem_trilinear.h"

namespace fem {

constexpr int MAX_VARIANTS = 7;

// Cfg<EG, WGM, WGN, WM, WN, OCC, KC, RES, PROD, BT, TE, OPQ> (see fem_kernel.h). For the 32-wide families
// (FP32, BF16, split): p = 1 packs 16 elements of 8 trial functions into 4 column blocks
// (variants 3, 4: the two k-groups of row fragments held in registers; variant 5 the
// vector-ALU kernel of fem_trilinear.h, ELEMENT mode only);
// p = 2, 3 put 4 (8) and 2 (4) elements side by side; p = 4 gives one element to a workgroup
// (variant 3: one element to each wave, 4 x 4 blocks in registers); p >= 5 tile one element
// into row x column tiles (variant 2: 4 x 4 blocks per wave). FP64 uses 16-wide blocks. The
// elasticity defaults p = 2, 3, 6 variant 6, p = 4 variant 4 (FP32: 6) and p = 5, 7 variant 5
// are the tiles (2, 1, 4, 3 (5), 4, 4) whose epilogue also writes the transposed (lower) blocks;
// the last FP64 variant of p >= 2 (and variant 1 of the FP64 prisms) is the same twin of the
// FP64 default.
template <int P, int FAM, int V> struct VariantCfg { using type = void; };
// The vector-ALU kernel of trilinear hexahedra (fem_trilinear.h; ELEMENT mode only).
struct TrilinearCfg {};

// -- 32-wide families --
template <> struct VariantCfg<1, MF_K16, 0> { using type = Cfg<16, 1, 4, 1, 1, 2, 2, 1, 0>; };
template <> struct VariantCfg<1, MF_K16, 1> { using type = Cfg<16, 1, 4, 1, 1, 3, 2, 1, 1>; };
template <> struct VariantCfg<1, MF_K16, 2> { using type = Cfg<4, 1, 1, 1, 1, 3, 2, 2, 1, 1>; };
template <> struct VariantCfg<1, MF_K16, 3> { using type = Cfg<4, 1, 1, 1, 1, 3, 2, 3, 1, 1>; };
template <> struct VariantCfg<1, MF_K16, 4> { using type = Cfg<8, 1, 1, 1, 2, 3, 2, 3, 1, 1>; };
template <> struct VariantCfg<1, MF_K16, 5> { using type = TrilinearCfg; };
template <> struct VariantCfg<2, MF_K16, 0> { using type = Cfg<4, 1, 4, 1, 1, 3, 2, 1, 1>; };
template <> struct VariantCfg<2, MF_K16, 1> { using type = Cfg<8, 1, 4, 1, 2, 2, 2, 1, 1>; };
template <> struct VariantCfg<2, MF_K16, 2> { using type = Cfg<4, 1, 1, 1, 4, 2, 1, 2, 1, 1>; };
template <> struct VariantCfg<2, MF_K16, 3> { using type = Cfg<4, 1, 4, 1, 1, 3, 1, 2, 1, 1>; };
template <> struct VariantCfg<2, MF_K16, 4> { using type = Cfg<1, 1, 1, 1, 1, 3, 1, 2, 1, 1>; };
template <> struct VariantCfg<2, MF_K16, 5> { using type = Cfg<2, 1, 1, 1, 2, 3, 1, 2, 1, 1>; };
template <> struct VariantCfg<2, MF_K16, 6> { using type = Cfg<4, 1, 1, 1, 4, 2, 1, 2, 1, 1, 1>; };
template <> struct VariantCfg<3, MF_K16, 0> { using type = Cfg<4, 1, 4, 2, 2, 3, 1, 2, 1, 1>; };
template <> struct VariantCfg<3, MF_K16, 1> { using type = Cfg<8, 1, 8, 2, 2, 2, 1, 1, 1, 1>; };
template <> struct VariantCfg<3, MF_K16, 2> { using type = Cfg<4, 1, 4, 2, 2, 2, 1, 2, 1>; };
template <> struct VariantCfg<3, MF_K16, 3> { using type = Cfg<4, 1, 4, 2, 2, 2, 2, 0, 1>; };
template <> struct VariantCfg<3, MF_K16, 4> { using type = Cfg<4, 1, 4, 2, 2, 2, 1, 2, 1, 1>; };
template <> struct VariantCfg<3, MF_K16, 5> { using type = Cfg<1, 1, 1, 2, 2, 2, 1, 2, 1, 1>; };
template <> struct VariantCfg<3, MF_K16, 6> { using type = Cfg<8, 1, 8, 2, 2, 2, 1, 1, 1, 1, 1>; };
template <> struct VariantCfg<4, MF_K16, 0> { using type = Cfg<1, 1, 1, 4, 4, 1, 1, 0, 1, 0>; };
template <> struct VariantCfg<4, MF_K16, 1> { using type = Cfg<2, 1, 4, 4, 2, 1, 1, 0, 1>; };
template <> struct VariantCfg<4, MF_K16, 2> { using type = Cfg<2, 1, 4, 4, 2, 2, 1, 0, 1>; };
template <> struct VariantCfg<4, MF_K16, 3> { using type = Cfg<4, 1, 4, 4, 4, 1, 1, 0, 1>; };
template <> struct VariantCfg<4, MF_K16, 4> { using type = Cfg<4, 1, 4, 4, 4, 1, 1, 0, 1, 0, 1>; };
template <> struct VariantCfg<4, MF_K16, 5> { using type = Cfg<2, 1, 4, 4, 2, 2, 1, 0, 1, 1>; };
template <> struct VariantCfg<4, MF_K16, 6> { using type = Cfg<2, 1, 4, 4, 2, 2, 1, 0, 1, 1, 1>; };
template <> struct VariantCfg<5, MF_K16, 0> { using type = Cfg<1, 1, 4, 4, 1, 1, 2, 0, 0>; };
template <> struct VariantCfg<5, MF_K16, 1> { using type = Cfg<1, 1, 4, 4, 1, 1, 2, 0, 1>; };
template <> struct VariantCfg<5, MF_K16, 2> { using type = Cfg<1, 2, 2, 4, 4, 1, 1, 0, 1>; };
template <> struct VariantCfg<5, MF_K16, 3> { using type = Cfg<1, 2, 2, 4, 4, 1, 1, 0, 1, 1>; };
template <> struct VariantCfg<5, MF_K16, 4> { using type = Cfg<1, 1, 4, 7, 2, 1, 1, 0, 1, 0, 0, 1>; };
template <> struct VariantCfg<5, MF_K16, 5> { using type = Cfg<1, 1, 4, 7, 2, 1, 1, 0, 1, 0, 1, 1>; };
template <> struct VariantCfg<6, MF_K16, 0> { using type = Cfg<1, 1, 4, 6, 1, 1, 2, 0, 0>; };
template <> struct VariantCfg<6, MF_K16, 1> { using type = Cfg<1, 1, 4, 6, 1, 1, 2, 0, 1>; };
template <> struct VariantCfg<6, MF_K16, 2> { using type = Cfg<1, 3, 1, 4, 4, 1, 1, 0, 1>; };
template <> struct VariantCfg<6, MF_K16, 3> { using type = Cfg<1, 3, 1, 4, 4, 1, 1, 0, 1, 1>; };
template <> struct VariantCfg<6, MF_K16, 4> { using type = Cfg<1, 1, 4, 11, 1, 1, 1, 0, 1>; };
template <> struct VariantCfg<6, MF_K16, 5> { using type = Cfg<1, 4, 1, 3, 4, 1, 1, 0, 1>; };
template <> struct VariantCfg<6, MF_K16, 6> { using type = Cfg<1, 1, 4, 11, 1, 1, 1, 0, 1, 0, 1>; };
template <> struct VariantCfg<7, MF_K16, 0> { using type = Cfg<1, 1, 4, 8, 1, 1, 2, 0, 0>; };
template <> struct VariantCfg<7, MF_K16, 1> { using type = Cfg<1, 1, 4, 8, 1, 1, 2, 0, 1>; };
template <> struct VariantCfg<7, MF_K16, 2> { using type = Cfg<1, 2, 2, 4, 4, 1, 1, 0, 1>; };
template <> struct VariantCfg<7, MF_K16, 3> { using type = Cfg<1, 2, 2, 4, 4, 1, 1, 0, 1, 1>; };
template <> struct VariantCfg<7, MF_K16, 4> { using type = Cfg<1, 1, 4, 8, 2, 1, 1, 0, 1, 0, 0, 1>; };
template <> struct VariantCfg<7, MF_K16, 5> { using type = Cfg<1, 1, 4, 8, 2, 1, 1, 0, 1, 0, 1, 1>; };
// -- prisms (P = PRISM_BASE + p; Ns = 6, 18, 40, 75, 126, 196, 288): every variant produces the
// column operand per wave from the B-factor table (PROD 1, BT 1). p = 1 packs 16 elements at a
// pitch of 8 columns; p = 2, 3, 4 give one element to each wave (1 x 1, 2 x 2, 3 x 3 blocks);
// p = 5 as the hexahedron of p = 4; p = 6 one element per workgroup in four 7 x 2 wave tiles;
// p = 7 four tall 9 x 1 wave tiles (three column tiles) or three 9 x 1 waves. Variant 2 of
// p >= 2 is variant 0 whose epilogue also writes the transposed elasticity blocks.
template <> struct VariantCfg<11, MF_K16, 0> { using type = Cfg<16, 1, 1, 1, 4, 3, 1, 2, 1, 1>; };
template <> struct VariantCfg<11, MF_K16, 1> { using type = Cfg<16, 1, 4, 1, 1, 3, 1, 2, 1, 1>; };
template <> struct VariantCfg<12, MF_K16, 0> { using type = Cfg<4, 1, 1, 1, 4, 2, 1, 2, 1, 1>; };
template <> struct VariantCfg<12, MF_K16, 1> { using type = Cfg<4, 1, 4, 1, 1, 3, 1, 2, 1, 1>; };
template <> struct VariantCfg<12, MF_K16, 2> { using type = Cfg<4, 1, 1, 1, 4, 2, 1, 2, 1, 1, 1>; };
template <> struct VariantCfg<13, MF_K16, 0> { using type = Cfg<4, 1, 4, 2, 2, 2, 1, 2, 1, 1>; };
template <> struct VariantCfg<13, MF_K16, 1> { using type = Cfg<8, 1, 8, 2, 2, 2, 1, 1, 1, 1>; };
template <> struct VariantCfg<13, MF_K16, 2> { using type = Cfg<4, 1, 4, 2, 2, 2, 1, 2, 1, 1, 1>; };
template <> struct VariantCfg<14, MF_K16, 0> { using type = Cfg<4, 1, 4, 3, 3, 1, 1, 2, 1, 1>; };
template <> struct VariantCfg<14, MF_K16, 1> { using type = Cfg<4, 1, 4, 3, 3, 1, 1, 0, 1, 1>; };
template <> struct VariantCfg<14, MF_K16, 2> { using type = Cfg<4, 1, 4, 3, 3, 1, 1, 2, 1, 1, 1>; };
template <> struct VariantCfg<15, MF_K16, 0> { using type = Cfg<4, 1, 4, 4, 4, 1, 1, 0, 1, 1>; };
template <> struct VariantCfg<15, MF_K16, 1> { using type = Cfg<1, 1, 4, 4, 1, 1, 1, 0, 1, 1>; };
template <> struct VariantCfg<15, MF_K16, 2> { using type = Cfg<4, 1, 4, 4, 4, 1, 1, 0, 1, 1, 1>; };
template <> struct VariantCfg<16, MF_K16, 0> { using type = Cfg<1, 1, 4, 7, 2, 1, 1, 0, 1, 1>; };
template <> struct VariantCfg<16, MF_K16, 1> { using type = Cfg<1, 1, 4, 7, 1, 1, 1, 0, 1, 1>; };
template <> struct VariantCfg<16, MF_K16, 2> { using type = Cfg<1, 1, 4, 7, 2, 1, 1, 0, 1, 1, 1>; };
template <> struct VariantCfg<17, MF_K16, 0> { using type = Cfg<1, 1, 4, 9, 1, 1, 1, 0, 1, 1>; };
template <> struct VariantCfg<17, MF_K16, 1> { using type = Cfg<1, 1, 3, 9, 1, 1, 1, 0, 1, 1>; };
template <> struct VariantCfg<17, MF_K16, 2> { using type = Cfg<1, 1, 4, 9, 1, 1, 1, 0, 1, 1, 1>; };
template <int P, int V> struct VariantCfg<P, MF_F32, V> { using type = typename VariantCfg<P, MF_K16, V>::type; };
// -- FP64 (16-wide blocks) --
template <> struct VariantCfg<1, MF_F64, 0> { using type = Cfg<8, 1, 4, 1, 1, 2, 2, 1, 0>; };
template <> struct VariantCfg<1, MF_F64, 1> { using type = TrilinearCfg; };
template <> struct VariantCfg<2, MF_F64, 0> { using type = Cfg<2, 1, 4, 2, 1, 2, 2, 0, 0>; };
template <> struct VariantCfg<2, MF_F64, 1> { using type = Cfg<4, 1, 4, 2, 2, 2, 1, 2, 1, 1>; };
template <> struct VariantCfg<2, MF_F64, 2> { using type = Cfg<4, 1, 1, 2, 8, 2, 1, 2, 1, 1>; };
template <> struct VariantCfg<2, MF_F64, 3> { using type = Cfg<4, 1, 4, 2, 2, 2, 1, 2, 1, 1, 1>; };
template <> struct VariantCfg<3, MF_F64, 0> { using type = Cfg<1, 1, 4, 4, 1, 2, 2, 0, 0>; };
template <> struct VariantCfg<3, MF_F64, 1> { using type = Cfg<2, 1, 4, 4, 2, 2, 1, 2, 1, 1>; };
template <> struct VariantCfg<3, MF_F64, 2> { using type = Cfg<1, 1, 4, 4, 1, 2, 1, 2, 1, 1>; };
template <> struct VariantCfg<3, MF_F64, 3> { using type = Cfg<2, 1, 4, 4, 2, 2, 1, 2, 1, 1, 1>; };
template <> struct VariantCfg<4, MF_F64, 0> { using type = Cfg<1, 1, 4, 8, 1, 1, 1, 0, 0>; };
template <> struct VariantCfg<4, MF_F64, 1> { using type = Cfg<1, 1, 4, 8, 2, 1, 1, 0, 1>; };
template <> struct VariantCfg<4, MF_F64, 2> { using type = Cfg<1, 1, 4, 8, 2, 1, 1, 0, 1, 1>; };
template <> struct VariantCfg<4, MF_F64, 3> { using type = Cfg<1, 1, 4, 8, 2, 1, 1, 0, 1, 0, 1>; };
template <> struct VariantCfg<5, MF_F64, 0> { using type = Cfg<1, 1, 4, 7, 1, 1, 1, 0, 0>; };
template <> struct VariantCfg<5, MF_F64, 1> { using type = Cfg<1, 1, 4, 14, 1, 1, 1, 0, 0>; };
template <> struct VariantCfg<5, MF_F64, 2> { using type = Cfg<1, 1, 4, 14, 1, 1, 1, 0, 0, 0, 1>; };
template <> struct VariantCfg<6, MF_F64, 0> { using type = Cfg<1, 1, 4, 8, 1, 1, 1, 0, 0>; };
template <> struct VariantCfg<6, MF_F64, 1> { using type = Cfg<1, 1, 4, 11, 1, 1, 1, 0, 0>; };
template <> struct VariantCfg<6, MF_F64, 2> { using type = Cfg<1, 1, 4, 11, 1, 1, 1, 0, 0, 0, 1>; };
template <> struct VariantCfg<7, MF_F64, 0> { using type = Cfg<1, 1, 4, 8, 1, 1, 1, 0, 0>; };
template <> struct VariantCfg<7, MF_F64, 1> { using type = Cfg<1, 1, 4, 16, 1, 1, 1, 0, 0>; };
template <> struct VariantCfg<7, MF_F64, 2> { using type = Cfg<1, 1, 4, 16, 1, 1, 1, 0, 0, 0, 1>; };
// prisms, 16-wide blocks: p = 1 packs 8 elements per wave; p = 2, 3 one element per wave; p >= 4
// one element per workgroup in tall wave tiles holding every row block
template <> struct VariantCfg<11, MF_F64, 0> { using type = Cfg<8, 1, 1, 1, 4, 2, 1, 2, 1, 1>; };
template <> struct VariantCfg<12, MF_F64, 0> { using type = Cfg<4, 1, 4, 2, 2, 2, 1, 2, 1, 1>; };
template <> struct VariantCfg<12, MF_F64, 1> { using type = Cfg<4, 1, 4, 2, 2, 2, 1, 2, 1, 1, 1>; };
template <> struct VariantCfg<13, MF_F64, 0> { using type = Cfg<4, 1, 4, 3, 3, 1, 1, 2, 1, 1>; };
template <> struct VariantCfg<13, MF_F64, 1> { using type = Cfg<4, 1, 4, 3, 3, 1, 1, 2, 1, 1, 1>; };
template <> struct VariantCfg<14, MF_F64, 0> { using type = Cfg<1, 1, 4, 5, 1, 1, 1, 0, 1, 1>; };
template <> struct VariantCfg<14, MF_F64, 1> { using type = Cfg<1, 1, 4, 5, 1, 1, 1, 0, 1, 1, 1>; };
template <> struct VariantCfg<15, MF_F64, 0> { using type = Cfg<1, 1, 4, 8, 1, 1, 1, 0, 1, 1>; };
template <> struct VariantCfg<15, MF_F64, 1> { using type = Cfg<1, 1, 4, 8, 1, 1, 1, 0, 1, 1, 1>; };
template <> struct VariantCfg<16, MF_F64, 0> { using type = Cfg<1, 1, 4, 13, 1, 1, 1, 0, 1, 1>; };
template <> struct VariantCfg<16, MF_F64, 1> { using type = Cfg<1, 1, 4, 13, 1, 1, 1, 0, 1, 1, 1>; };
template <> struct VariantCfg<17, MF_F64, 0> { using type = Cfg<1, 1, 4, 18, 1, 1, 1, 0, 1, 1>; };
template <> struct VariantCfg<17, MF_F64, 1> { using type = Cfg<1, 1, 4, 18, 1, 1, 1, 0, 1, 1, 1>; };

template <int P, int PREC, int V>
struct Inst {
    using C = typename VariantCfg<P, family_of(PREC), V>::type;
    using S = Shape<P, PREC, C>;
    // workgroups of the instance (computed or supplied Jacobian terms) one CU holds at once
    static inline int resident_per_cu[2] = {1, 1};
    template <bool SUP> static const void *fn() { return reinterpret_cast<const void *>(&k_integrate<P, PREC, C, SUP>); }
    template <bool SUP> static hipError_t prepare_one()
    {
        hipError_t e = hipSuccess;
        if (S::lds_bytes > 65536)
            e = hipFuncSetAttribute(fn<SUP>(), hipFuncAttributeMaxDynamicSharedMemorySize, (int)S::lds_bytes);
        if (e != hipSuccess) return e;
        int blocks = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn<SUP>(), S::NT, S::lds_bytes);
        if (e != hipSuccess) return e;
        resident_per_cu[SUP] = blocks > 0 ? blocks : 1;
        return hipSuccess;
    }
    static hipError_t prepare()
    {
        const hipError_t e = prepare_one<false>();
        if constexpr (is_prism(P)) return e;  // prisms take no supplied Jacobian terms
        else return e != hipSuccess ? e : prepare_one<true>();
    }
    // a.nel is the exact element count, or an upper bound when a.seg supplies the count. The
    // grid is persistent: at most the workgroups the device holds at once.
    template <bool SUP> static hipError_t launch_one(const KArgs &a, hipStream_t s, int cus)
    {
        const int64_t groups = (a.nel + S::EG - 1) / S::EG;
        const int64_t total = groups * S::RT * S::CT;
        const int64_t cap = int64_t(cus) * resident_per_cu[SUP];
        const int64_t grid = total < cap ? total : cap;
        if (grid <= 0) return hipSuccess;
        hipLaunchKernelGGL((k_integrate<P, PREC, C, SUP>), dim3((unsigned)grid), dim3(S::NT), S::lds_bytes, s, a);
        return hipGetLastError();
    }
    static hipError_t launch(const KArgs &a, hipStream_t s, int cus)
    {
        if constexpr (is_prism(P)) return a.jac ? hipErrorInvalidValue : launch_one<false>(a, s, cus);
        else return a.jac ? launch_one<true>(a, s, cus) : launch_one<false>(a, s, cus);
    }
};

// Per-variant helpers that tolerate variants a family does not define.
template <int P, int PREC, int V>
constexpr bool has_variant() { return !std::is_void<typename VariantCfg<P, family_of(PREC), V>::type>::value; }

template <int P, int PREC, int V>
constexpr bool is_trilinear() { return std::is_same<typename VariantCfg<P, family_of(PREC), V>::type, TrilinearCfg>::value; }

// The variant of the vector-ALU kernel of (p, family), or -1 (p = 1 only).
constexpr int trilinear_variant(int p, int fam) { return p == 1 ? (fam == MF_F64 ? 1 : 5) : -1; }
static_assert(std::is_same<VariantCfg<1, MF_K16, trilinear_variant(1, MF_K16)>::type, TrilinearCfg>::value &&
                  std::is_same<VariantCfg<1, MF_F64, trilinear_variant(1, MF_F64)>::type, TrilinearCfg>::value,
              "trilinear_variant names the vector-ALU kernel");

template <int P, int PREC, int V>
hipError_t prepare_variant()
{
    if constexpr (is_trilinear<P, PREC, V>()) return hipSuccess;
    else if constexpr (has_variant<P, PREC, V>()) return Inst<P, PREC, V>::prepare();
    else return hipSuccess;
}

template <int P, int PREC, int V>
hipError_t launch_variant(const KArgs &a, hipStream_t s, int cus)
{
    if constexpr (is_trilinear<P, PREC, V>()) {
        using DT = typename std::conditional<PREC == PREC_F64, double, float>::type;
        return launch_trilinear<DT>(a, s, cus);
    } else if constexpr (has_variant<P, PREC, V>()) {
        return Inst<P, PREC, V>::launch(a, s, cus);
    } else {
        return hipErrorInvalidValue;
    }
}

// Whether a variant's epilogue can also write the transposed block (a.at_base, elasticity's
// lower blocks): from the staged image with an odd Ns (Shape::TRANS_EPI), or from the
// accumulators on the 32-wide families (Shape::TRANS_REG).
template <int P, int PREC, int V>
constexpr bool trans_epilogue()
{
    using Cf = typename VariantCfg<P, family_of(PREC), V>::type;
    if constexpr (std::is_void<Cf>::value || std::is_same<Cf, TrilinearCfg>::value) return false;
    else return Shape<P, PREC, Cf>::TRANS_EPI || Shape<P, PREC, Cf>::TRANS_REG;
}
template <int P, int PREC>
bool trans_pv(int v)
{
    switch (v) {
    case 0: return trans_epilogue<P, PREC, 0>();
    case 1: return trans_epilogue<P, PREC, 1>();
    case 2: return trans_epilogue<P, PREC, 2>();
    case 3: return trans_epilogue<P, PREC, 3>();
    case 4: return trans_epilogue<P, PREC, 4>();
    case 5: return trans_epilogue<P, PREC, 5>();
    case 6: return trans_epilogue<P, PREC, 6>();
    default: return false;
    }
}
template <int PREC>
bool trans_p(int p, int v)
{
    switch (p) {
    case 1: return trans_pv<1, PREC>(v);
    case 2: return trans_pv<2, PREC>(v);
    case 3: return trans_pv<3, PREC>(v);
    case 4: return trans_pv<4, PREC>(v);
    case 5: return trans_pv<5, PREC>(v);
    case 6: return trans_pv<6, PREC>(v);
    case 7: return trans_pv<7, PREC>(v);
    case 11: return trans_pv<11, PREC>(v);
    case 12: return trans_pv<12, PREC>(v);
    case 13: return trans_pv<13, PREC>(v);
    case 14: return trans_pv<14, PREC>(v);
    case 15: return trans_pv<15, PREC>(v);
    case 16: return trans_pv<16, PREC>(v);
    case 17: return trans_pv<17, PREC>(v);
    default: return false;
    }
}
inline bool trans_variant(int prec, int p, int v)
{
    switch (prec) {
    case PREC_F64: return trans_p<PREC_F64>(p, v);
    case PREC_F32: return trans_p<PREC_F32>(p, v);
    case PREC_BF16: return trans_p<PREC_BF16>(p, v);
    case PREC_SPLIT_BF16: return trans_p<PREC_SPLIT_BF16>(p, v);
    case PREC_SPLIT_F16: return trans_p<PREC_SPLIT_F16>(p, v);
    default: return false;
    }
}

template <int P, int PREC>
int count_variants()
{
    return has_variant<P, PREC, 0>() + has_variant<P, PREC, 1>() + has_variant<P, PREC, 2>() +
           has_variant<P, PREC, 3>() + has_variant<P, PREC, 4>() + has_variant<P, PREC, 5>() +
           has_variant<P, PREC, 6>();
}

template <int P, int PREC>
hipError_t prepare_p()
{
    hipError_t e = prepare_variant<P, PREC, 0>();
    if (e == hipSuccess) e = prepare_variant<P, PREC, 1>();
    if (e == hipSuccess) e = prepare_variant<P, PREC, 2>();
    if (e == hipSuccess) e = prepare_variant<P, PREC, 3>();
    if (e == hipSuccess) e = prepare_variant<P, PREC, 4>();
    if (e == hipSuccess) e = prepare_variant<P, PREC, 5>();
    if (e == hipSuccess) e = prepare_variant<P, PREC, 6>();
    return e;
}

template <int PREC>
hipError_t prepare_all()
{
    hipError_t e = hipSuccess;
    auto one = [&](hipError_t r) { if (e == hipSuccess) e = r; };
    one(prepare_p<1, PREC>()); one(prepare_p<2, PREC>()); one(prepare_p<3, PREC>());
    one(prepare_p<4, PREC>()); one(prepare_p<5, PREC>()); one(prepare_p<6, PREC>());
    one(prepare_p<7, PREC>());
    one(prepare_p<11, PREC>()); one(prepare_p<12, PREC>()); one(prepare_p<13, PREC>());
    one(prepare_p<14, PREC>()); one(prepare_p<15, PREC>()); one(prepare_p<16, PREC>());
    one(prepare_p<17, PREC>());
    return e;
}

template <int P, int PREC>
hipError_t launch_pv(int v, const KArgs &a, hipStream_t s, int cus)
{
    switch (v) {
    case 0: return launch_variant<P, PREC, 0>(a, s, cus);
    case 1: return launch_variant<P, PREC, 1>(a, s, cus);
    case 2: return launch_variant<P, PREC, 2>(a, s, cus);
    case 3: return launch_variant<P, PREC, 3>(a, s, cus);
    case 4: return launch_variant<P, PREC, 4>(a, s, cus);
    case 5: return launch_variant<P, PREC, 5>(a, s, cus);
    case 6: return launch_variant<P, PREC, 6>(a, s, cus);
    default: return hipErrorInvalidValue;
    }
}

template <int PREC>
hipError_t launch_p(int p, int v, const KArgs &a, hipStream_t s, int64_t cus)
{
    switch (p) {
    case 1: return launch_pv<1, PREC>(v, a, s, (int)cus);
    case 2: return launch_pv<2, PREC>(v, a, s, (int)cus);
    case 3: return launch_pv<3, PREC>(v, a, s, (int)cus);
    case 4: return launch_pv<4, PREC>(v, a, s, (int)cus);
    case 5: return launch_pv<5, PREC>(v, a, s, (int)cus);
    case 6: return launch_pv<6, PREC>(v, a, s, (int)cus);
    case 7: return launch_pv<7, PREC>(v, a, s, (int)cus);
    case 11: return launch_pv<11, PREC>(v, a, s, (int)cus);
    case 12: return launch_pv<12, PREC>(v, a, s, (int)cus);
    case 13: return launch_pv<13, PREC>(v, a, s, (int)cus);
    case 14: return launch_pv<14, PREC>(v, a, s, (int)cus);
    case 15: return launch_pv<15, PREC>(v, a, s, (int)cus);
    case 16: return launch_pv<16, PREC>(v, a, s, (int)cus);
    case 17: return launch_pv<17, PREC>(v, a, s, (int)cus);
    default: return hipErrorInvalidValue;
    }
}

template <int PREC>
int variants_p(int p)
{
    switch (p) {
    case 1: return count_variants<1, PREC>();
    case 2: return count_variants<2, PREC>();
    case 3: return count_variants<3, PREC>();
    case 4: return count_variants<4, PREC>();
    case 5: return count_variants<5, PREC>();
    case 6: return count_variants<6, PREC>();
    case 7: return count_variants<7, PREC>();
    case 11: return count_variants<11, PREC>();
    case 12: return count_variants<12, PREC>();
    case 13: return count_variants<13, PREC>();
    case 14: return count_variants<14, PREC>();
    case 15: return count_variants<15, PREC>();
    case 16: return count_variants<16, PREC>();
    case 17: return count_variants<17, PREC>();
    default: return 0;
    }
}

// Variant launched for each degree before any tuning (the fastest measured on MI355X at the
// plain-method and high-order workload sizes).
// p = 1 in ELEMENT mode (mode 0) runs the vector-ALU kernel.
constexpr int default_variant(int p, int fam, int mode)
{
    // prisms: the fastest measured per (family, degree, mode) on MI355X at the prism workload
    // sizes (fem_autotune over every variant); variant 2 (FP64: 1) is tile 0 that also writes
    // the transposed elasticity blocks
    if (is_prism(p)) {
        const int d = deg_of(p);
        constexpr int k16[2][8] = {{0, 1, 2, 2, 2, 2, 0, 1}, {0, 1, 2, 2, 2, 2, 2, 1}};
        constexpr int f32[2][8] = {{0, 1, 2, 1, 1, 2, 0, 0}, {0, 1, 2, 2, 1, 2, 2, 2}};
        constexpr int f64[2][8] = {{0, 0, 1, 1, 1, 0, 1, 0}, {0, 0, 1, 1, 1, 1, 1, 0}};
        const int m = mode == 2 ? 1 : 0;
        return fam == MF_F64 ? f64[m][d] : (fam == MF_F32 ? f32[m][d] : k16[m][d]);
    }
    if (p == 1 && mode == 0) return trilinear_variant(p, fam);
    if (p == 4 && mode == 2 && fam == MF_K16) return 4;  // tile 3 that also writes transposed blocks
    if (p == 4 && mode == 2 && fam == MF_F32) return 6;  // tile 5 that also writes transposed blocks
    if (mode == 2 && fam == MF_F64 && p >= 2) return p <= 4 ? 3 : 2;  // FP64 twins (below)
    if (mode == 2 && fam != MF_F64) {
        // the default tiles' twins that also write the transposed (lower) blocks
        if (p == 2 || p == 3 || p == 6) return 6;
        if (p == 5 || p == 7) return 5;
    }
    constexpr int f64[8] = {0, 0, 1, 1, 1, 1, 1, 1};
    if (fam == MF_F64) return f64[p];
    constexpr int k16[8] = {0, 3, 2, 1, 3, 4, 4, 4};
    constexpr int f32[8] = {0, 4, 2, 1, 5, 4, 4, 4};
    return fam == MF_F32 ? f32[p] : k16[p];
}

// The tiles compiled into the single-launch mixed-degree kernel: alternative t (0: the default,
// 1: the other) of degree p, as a variant number of the per-degree launches, or -1 where a
// degree has one. Only 256-thread tiles qualify (the kernel's workgroup size); the choice is made
// per (degree, precision, coefficient mode) at run time.
constexpr int mixed_tile(int p, int fam, int t)
{
    constexpr int f64[2][8] = {{0, 0, 1, 1, 1, 1, 1, 1}, {0, -1, 0, 0, 0, 0, 0, 0}};
    constexpr int k16[2][8] = {{0, 1, 1, 4, 3, 4, 4, 4}, {0, 0, 3, 2, 1, 1, 5, 1}};
    return fam == MF_F64 ? f64[t][p] : k16[t][p];
}
constexpr int mixed_tile_count(int p, int fam) { return mixed_tile(p, fam, 1) >= 0 ? 2 : 1; }

// The tile set of the single-launch mixed-degree kernel of a precision: C<P, t> is alternative t
// of degree P (a degree with one alternative repeats it).
template <int PREC>
struct MixedTiles {
    static constexpr int FAM = family_of(PREC);
    template <int P> static constexpr bool has_alt() { return mixed_tile_count(P, FAM) == 2; }
    template <int P, int T>
    using C = typename VariantCfg<P, FAM, mixed_tile(P, FAM, has_alt<P>() ? T : 0)>::type;
};

// The single-launch mixed-degree kernel of a precision.
template <int PREC>
struct MixedInst {
    using MT = MixedTiles<PREC>;
    template <int P, int T> using SP = Shape<P, PREC, typename MT::template C<P, T>>;
    static constexpr size_t max2(size_t x, size_t y) { return x > y ? x : y; }
    template <int P> static constexpr size_t lds_p() { return max2(SP<P, 0>::lds_bytes, SP<P, 1>::lds_bytes); }
    template <int P> static constexpr int64_t items_p()
    {
        return max2(SP<P, 0>::RT * SP<P, 0>::CT, SP<P, 1>::RT * SP<P, 1>::CT);
    }
    static constexpr size_t lds_bytes =
        max2(max2(max2(lds_p<1>(), lds_p<2>()), max2(lds_p<3>(), lds_p<4>())),
             max2(max2(lds_p<5>(), lds_p<6>()), lds_p<7>()));
    // work items per element, at most, over every degree and tile
    static constexpr int64_t per_el = max2(max2(max2(items_p<1>(), items_p<2>()), max2(items_p<3>(), items_p<4>())),
                                           max2(max2(items_p<5>(), items_p<6>()), items_p<7>()));
    static inline int resident_per_cu[2] = {1, 1};
    template <bool SUP> static const void *fn()
    {
        return reinterpret_cast<const void *>(&k_integrate_mixed<PREC, SUP, MT>);
    }
    template <bool SUP> static hipError_t prepare_one()
    {
        hipError_t e = hipSuccess;
        if (lds_bytes > 65536)
            e = hipFuncSetAttribute(fn<SUP>(), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        if (e != hipSuccess) return e;
        int blocks = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn<SUP>(), 256, lds_bytes);
        if (e != hipSuccess) return e;
        resident_per_cu[SUP] = blocks > 0 ? blocks : 1;
        return hipSuccess;
    }
    static hipError_t prepare()
    {
        const hipError_t e = prepare_one<false>();
        return e != hipSuccess ? e : prepare_one<true>();
    }
    // The bucket sizes are read on the device; the grid is the number of workgroups the device
    // holds at once, capped by an upper bound on the work items (every element in the bucket
    // with the most items per element).
    static hipError_t launch(const MixedKArgs &m, int64_t nel, hipStream_t s, int cus)
    {
        const int64_t bound = nel * per_el;
        const bool sup = m.deg[0].jac != nullptr;
        const int64_t cap = int64_t(cus) * resident_per_cu[sup];
        const int64_t grid = bound < cap ? bound : cap;
        if (grid <= 0) return hipSuccess;
        if (sup)
            hipLaunchKernelGGL((k_integrate_mixed<PREC, true, MT>), dim3((unsigned)grid), dim3(256), lds_bytes, s, m);
        else
            hipLaunchKernelGGL((k_integrate_mixed<PREC, false, MT>), dim3((unsigned)grid), dim3(256), lds_bytes, s, m);
        return hipGetLastError();
    }
};

}  // namespace fem
