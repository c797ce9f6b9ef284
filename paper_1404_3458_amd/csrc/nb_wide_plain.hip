// nb_wide_plain.hip -- instantiation and launch of the plain transform passes
// (W_PI, W_PF, W_PFM of nb_wide_impl.hpp): nb_fft, nb_ifft and nb_polymul
// over h > 256 points at shifts whose bits below h are clear, in two passes
// of up to 8 levels (Sec. 3.2 / 3.3).
#include "nb_wide_impl.hpp"

namespace nb {

template <int T, int KIND, int LD>
static hipError_t plain_launch_one(const WideArgs &a, const KPtrs &k, int ntiles, hipStream_t s)
{
    const size_t lds = WideLds<T, KIND, false>::BYTES;
    hipLaunchKernelGGL((k_wide<T, KIND, LD, false>), dim3(ntiles), dim3(NB_WIDE_THREADS(T)), lds, s, a, k.tw, k.B,
                       k.Binv, k.bits, k.rowtabs);
    return hipGetLastError();
}

template <int T, int KIND, int LD>
static hipError_t plain_prep_one()
{
    return hipFuncSetAttribute((const void *)k_wide<T, KIND, LD, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)WideLds<T, KIND, false>::BYTES);
}

template <int KIND, int LD>
static hipError_t plain_launch_T(int T, const WideArgs &a, const KPtrs &k, int ntiles, hipStream_t s)
{
    switch (T) {
    case 4: return plain_launch_one<4, KIND, LD>(a, k, ntiles, s);
    case 5: return plain_launch_one<5, KIND, LD>(a, k, ntiles, s);
    case 6: return plain_launch_one<6, KIND, LD>(a, k, ntiles, s);
    case 7: return plain_launch_one<7, KIND, LD>(a, k, ntiles, s);
    case 8: return plain_launch_one<8, KIND, LD>(a, k, ntiles, s);
    default: return hipErrorInvalidValue;
    }
}

template <int KIND, int LD>
static hipError_t plain_prep_T()
{
    hipError_t e = hipSuccess, f;
    if ((f = plain_prep_one<4, KIND, LD>()) != hipSuccess) e = f;
    if ((f = plain_prep_one<5, KIND, LD>()) != hipSuccess) e = f;
    if ((f = plain_prep_one<6, KIND, LD>()) != hipSuccess) e = f;
    if ((f = plain_prep_one<7, KIND, LD>()) != hipSuccess) e = f;
    if ((f = plain_prep_one<8, KIND, LD>()) != hipSuccess) e = f;
    return e;
}

template <int LD>
static hipError_t plain_launch_ld(int kind, int T, const WideArgs &a, const KPtrs &k, int ntiles, hipStream_t s)
{
    switch (kind) {
    case W_PI: return plain_launch_T<W_PI, LD>(T, a, k, ntiles, s);
    case W_PF: return plain_launch_T<W_PF, LD>(T, a, k, ntiles, s);
    case W_PFM: return plain_launch_T<W_PFM, LD>(T, a, k, ntiles, s);
    }
    return hipErrorInvalidValue;
}

hipError_t wide_plain_launch(int kind, int ld, int T, const WideArgs &a, const KPtrs &k, int ntiles, hipStream_t s)
{
    return ld == LD_VEC ? plain_launch_ld<LD_VEC>(kind, T, a, k, ntiles, s)
                        : plain_launch_ld<LD_SYM>(kind, T, a, k, ntiles, s);
}

hipError_t wide_plain_prepare()
{
    hipError_t e = hipSuccess, f;
    if ((f = plain_prep_T<W_PI, LD_VEC>()) != hipSuccess) e = f;
    if ((f = plain_prep_T<W_PI, LD_SYM>()) != hipSuccess) e = f;
    if ((f = plain_prep_T<W_PF, LD_VEC>()) != hipSuccess) e = f;
    if ((f = plain_prep_T<W_PF, LD_SYM>()) != hipSuccess) e = f;
    if ((f = plain_prep_T<W_PFM, LD_VEC>()) != hipSuccess) e = f;
    if ((f = plain_prep_T<W_PFM, LD_SYM>()) != hipSuccess) e = f;
    return e;
}

}  // namespace nb
