// nb_wide.hip -- instantiation and launch of the codec's pass kernels
// (nb_wide_impl.hpp); the plain transform passes are instantiated in
// nb_wide_plain.hip, so that the two compile in parallel.
#include "nb_wide_impl.hpp"

namespace nb {

template <int T, int KIND, int LD, bool PK>
static hipError_t wide_launch_one(const WideArgs &a, const KPtrs &k, int ntiles, hipStream_t s)
{
    if constexpr (PK && !packable(T, KIND)) {
        return hipErrorInvalidValue;
    } else {
        const size_t lds = WideLds<T, KIND, PK>::BYTES;
        hipLaunchKernelGGL((k_wide<T, KIND, LD, PK>), dim3(ntiles), dim3(NB_WIDE_THREADS_PK(T, PK)), lds, s, a, k.tw,
                           k.B, k.Binv, k.bits, k.rowtabs);
        return hipGetLastError();
    }
}

template <int T, int KIND, int LD, bool PK>
static hipError_t wide_prep_one()
{
    if constexpr (PK && !packable(T, KIND))
        return hipSuccess;
    else
        return hipFuncSetAttribute((const void *)k_wide<T, KIND, LD, PK>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)WideLds<T, KIND, PK>::BYTES);
}

template <int KIND, int LD, bool PK>
static hipError_t wide_launch_T(int T, const WideArgs &a, const KPtrs &k, int ntiles, hipStream_t s)
{
    switch (T) {
    case 4: return wide_launch_one<4, KIND, LD, PK>(a, k, ntiles, s);
    case 5: return wide_launch_one<5, KIND, LD, PK>(a, k, ntiles, s);
    case 6: return wide_launch_one<6, KIND, LD, PK>(a, k, ntiles, s);
    case 7: return wide_launch_one<7, KIND, LD, PK>(a, k, ntiles, s);
    case 8: return wide_launch_one<8, KIND, LD, PK>(a, k, ntiles, s);
    default: return hipErrorInvalidValue;
    }
}

template <int KIND, int LD, bool PK>
static hipError_t wide_prep_T()
{
    hipError_t e = hipSuccess, f;
    if ((f = wide_prep_one<4, KIND, LD, PK>()) != hipSuccess) e = f;
    if ((f = wide_prep_one<5, KIND, LD, PK>()) != hipSuccess) e = f;
    if ((f = wide_prep_one<6, KIND, LD, PK>()) != hipSuccess) e = f;
    if ((f = wide_prep_one<7, KIND, LD, PK>()) != hipSuccess) e = f;
    if ((f = wide_prep_one<8, KIND, LD, PK>()) != hipSuccess) e = f;
    return e;
}

template <int LD, bool PK>
static hipError_t wide_launch_ld(int kind, int T, const WideArgs &a, const KPtrs &k, int ntiles, hipStream_t s)
{
    switch (kind) {
    case W_E1: return wide_launch_T<W_E1, LD, PK>(T, a, k, ntiles, s);
    case W_E2: return wide_launch_T<W_E2, LD, PK>(T, a, k, ntiles, s);
    case W_E2F: return wide_launch_T<W_E2F, LD, PK>(T, a, k, ntiles, s);
    case W_E3: return wide_launch_T<W_E3, LD, PK>(T, a, k, ntiles, s);
    case W_D1: return wide_launch_T<W_D1, LD, PK>(T, a, k, ntiles, s);
    case W_D2: return wide_launch_T<W_D2, LD, PK>(T, a, k, ntiles, s);
    case W_D3: return wide_launch_T<W_D3, LD, PK>(T, a, k, ntiles, s);
    case W_DPM: return wide_launch_T<W_DPM, LD, PK>(T, a, k, ntiles, s);
    case W_D4: return wide_launch_T<W_D4, LD, PK>(T, a, k, ntiles, s);
    case W_D5: return wide_launch_T<W_D5, LD, PK>(T, a, k, ntiles, s);
    case W_DH: return wide_launch_T<W_DH, LD, PK>(T, a, k, ntiles, s);
    case W_DL: return wide_launch_T<W_DL, LD, PK>(T, a, k, ntiles, s);
    }
    return hipErrorInvalidValue;
}

bool wide_packable(int kind, int T) { return packable(T, kind); }

hipError_t wide_plain_launch(int kind, int ld, int T, const WideArgs &a, const KPtrs &k, int ntiles, hipStream_t s);
hipError_t wide_plain_prepare();

hipError_t wide_launch(int kind, int ld, int T, bool pk, const WideArgs &a, const KPtrs &k, int ntiles, hipStream_t s)
{
    if (ntiles <= 0)
        return hipSuccess;
    if (kind == W_PI || kind == W_PF || kind == W_PFM)
        return pk ? hipErrorInvalidValue : wide_plain_launch(kind, ld, T, a, k, ntiles, s);
    if (pk)
        return ld == LD_VEC ? wide_launch_ld<LD_VEC, true>(kind, T, a, k, ntiles, s)
                            : wide_launch_ld<LD_SYM, true>(kind, T, a, k, ntiles, s);
    return ld == LD_VEC ? wide_launch_ld<LD_VEC, false>(kind, T, a, k, ntiles, s)
                        : wide_launch_ld<LD_SYM, false>(kind, T, a, k, ntiles, s);
}

hipError_t wide_prepare()
{
    hipError_t e = hipSuccess, f;
#define NB_WPREP(K)                                                                                                \
    if ((f = wide_prep_T<K, LD_VEC, false>()) != hipSuccess) e = f;                                                \
    if ((f = wide_prep_T<K, LD_SYM, false>()) != hipSuccess) e = f;                                                \
    if ((f = wide_prep_T<K, LD_VEC, true>()) != hipSuccess) e = f;                                                 \
    if ((f = wide_prep_T<K, LD_SYM, true>()) != hipSuccess) e = f;
    NB_WPREP(W_E1) NB_WPREP(W_E2) NB_WPREP(W_E2F) NB_WPREP(W_E3) NB_WPREP(W_D1) NB_WPREP(W_D2) NB_WPREP(W_D3)
    NB_WPREP(W_DPM)
    NB_WPREP(W_D4) NB_WPREP(W_D5) NB_WPREP(W_DH) NB_WPREP(W_DL)
#undef NB_WPREP
    if ((f = wide_plain_prepare()) != hipSuccess)
        e = f;
    return e;
}

}  // namespace nb
