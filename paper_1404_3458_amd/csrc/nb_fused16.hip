// nb_fused16.hip -- instantiation of the fused kernels for GF(2^16).
#include "nb_fused_impl.hpp"

namespace nb {

hipError_t fused_prepare_16() { return fused_prepare_r<16>(); }

hipError_t fused_launch_16(int mode, int sh, int ld, int L, const FusedArgs &a, const KPtrs &k, int ntiles,
                          bool pr, hipStream_t s)
{
    return ld == LD_VEC ? launch_ld<16, LD_VEC>(mode, sh, L, a, k, ntiles, pr, s)
                        : launch_ld<16, LD_SYM>(mode, sh, L, a, k, ntiles, pr, s);
}

}  // namespace nb
