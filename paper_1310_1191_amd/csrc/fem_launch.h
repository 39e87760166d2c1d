// fem_launch.h -- tile configurations per (degree, precision) and the launch of one degree.
#pragma once
#include "fem_kernel.h"

namespace fem {

// Work-item shapes. TM = 32 families (FP32, BF16, split): p = 1 packs 16 elements of 8 trial
// functions into 4 column blocks; p = 2, 3 put 4 and 2 elements side by side; p >= 4 tile one
// element. FP64 (TM = 16) uses the same scheme with 16-wide blocks.
template <int P, int FAM> struct DefaultCfg;
template <> struct DefaultCfg<1, MF_K16> { using type = Cfg<16, 1, 4, 1, 1, 2>; };
template <> struct DefaultCfg<2, MF_K16> { using type = Cfg<4, 1, 4, 1, 1, 2>; };
template <> struct DefaultCfg<3, MF_K16> { using type = Cfg<2, 1, 4, 2, 1, 2>; };
template <> struct DefaultCfg<4, MF_K16> { using type = Cfg<1, 1, 4, 4, 1, 2>; };
template <> struct DefaultCfg<5, MF_K16> { using type = Cfg<1, 1, 4, 4, 1, 1>; };
template <> struct DefaultCfg<6, MF_K16> { using type = Cfg<1, 1, 4, 6, 1>; };
template <> struct DefaultCfg<7, MF_K16> { using type = Cfg<1, 1, 4, 8, 1>; };
template <int P> struct DefaultCfg<P, MF_F32> { using type = typename DefaultCfg<P, MF_K16>::type; };
template <> struct DefaultCfg<1, MF_F64> { using type = Cfg<8, 1, 4, 1, 1, 2>; };
template <> struct DefaultCfg<2, MF_F64> { using type = Cfg<2, 1, 4, 2, 1, 2>; };
template <> struct DefaultCfg<3, MF_F64> { using type = Cfg<1, 1, 4, 4, 1, 2>; };
template <> struct DefaultCfg<4, MF_F64> { using type = Cfg<1, 1, 4, 8, 1>; };
template <> struct DefaultCfg<5, MF_F64> { using type = Cfg<1, 1, 4, 7, 1>; };
template <> struct DefaultCfg<6, MF_F64> { using type = Cfg<1, 1, 4, 8, 1>; };
template <> struct DefaultCfg<7, MF_F64> { using type = Cfg<1, 1, 4, 8, 1>; };

template <int P, int PREC>
struct Inst {
    using C = typename DefaultCfg<P, family_of(PREC)>::type;
    using S = Shape<P, PREC, C>;
    static void *fn() { return reinterpret_cast<void *>(&k_integrate<P, PREC, C>); }
    static hipError_t prepare()
    {
        if (S::lds_bytes > 65536)
            return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_integrate<P, PREC, C>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)S::lds_bytes);
        return hipSuccess;
    }
    // a.nel is the exact element count, or an upper bound when a.seg supplies the count.
    static hipError_t launch(const KArgs &a, hipStream_t s, int64_t grid_cap)
    {
        const int64_t groups = (a.nel + S::EG - 1) / S::EG;
        const int64_t total = groups * S::RT * S::CT;
        const int64_t grid = total < grid_cap ? total : grid_cap;
        if (grid <= 0) return hipSuccess;
        if (grid > 0x7fffffffLL) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_integrate<P, PREC, C>), dim3((unsigned)grid), dim3(S::NT), S::lds_bytes, s, a);
        return hipGetLastError();
    }
};


template <int PREC>
hipError_t prepare_all()
{
    hipError_t e;
    if ((e = Inst<1, PREC>::prepare()) != hipSuccess) return e;
    if ((e = Inst<2, PREC>::prepare()) != hipSuccess) return e;
    if ((e = Inst<3, PREC>::prepare()) != hipSuccess) return e;
    if ((e = Inst<4, PREC>::prepare()) != hipSuccess) return e;
    if ((e = Inst<5, PREC>::prepare()) != hipSuccess) return e;
    if ((e = Inst<6, PREC>::prepare()) != hipSuccess) return e;
    return Inst<7, PREC>::prepare();
}

template <int PREC>
hipError_t launch_p(int p, const KArgs &a, hipStream_t s, int64_t cap)
{
    switch (p) {
    case 1: return Inst<1, PREC>::launch(a, s, cap);
    case 2: return Inst<2, PREC>::launch(a, s, cap);
    case 3: return Inst<3, PREC>::launch(a, s, cap);
    case 4: return Inst<4, PREC>::launch(a, s, cap);
    case 5: return Inst<5, PREC>::launch(a, s, cap);
    case 6: return Inst<6, PREC>::launch(a, s, cap);
    case 7: return Inst<7, PREC>::launch(a, s, cap);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace fem
