// nb_fused8.hip -- instantiation of the fused kernels for GF(2^8).
#include "nb_fused_impl.hpp"

namespace nb {

hipError_t fused_prepare_8() { return fused_prepare_r<8>(); }

hipError_t fused_launch_8(int mode, int sh, int ld, int L, const FusedArgs &a, const KPtrs &k, int ntiles,
                          bool pr, hipStream_t s)
{
    return ld == LD_VEC ? launch_ld<8, LD_VEC>(mode, sh, L, a, k, ntiles, pr, s)
                        : launch_ld<8, LD_SYM>(mode, sh, L, a, k, ntiles, pr, s);
}

}  // namespace nb
