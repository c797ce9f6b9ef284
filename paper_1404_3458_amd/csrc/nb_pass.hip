// nb_pass.hip -- multi-pass kernels for transform sizes h > 256 (up to 2^16).
//
// A pass applies up to five (forward) or four (inverse) consecutive levels
// lo .. lo+T-1 of the transform (Sec. 3.2 / 3.3) to every group of 2^T rows
// base + j 2^lo (base has no set bit in lo .. lo+T-1), reading the rows from
// global memory into registers
// and writing them back.  The group and the 256-column tile are uniform per
// workgroup, so the skew factors are wave-uniform as in the fused kernels.
// Rows may be multiplied by B_p before or after the levels (Sec. 4.2), and
// (GF(2^16)) by the rows of another array after them, symbol by symbol (the
// point-by-point product of Sec. 6.1, Table 1).
#include "nb_xform.hpp"

namespace nb {

__device__ __forceinline__ uint32_t group_base(uint32_t g, int lo, int T)
{
    return (g & ((1u << lo) - 1u)) | ((g >> lo) << (lo + T));
}

__device__ __forceinline__ const uint8_t *prow(const uint8_t *base, uint32_t t, uint64_t rb)
{
    return base + (uint64_t)t * rb;
}
__device__ __forceinline__ uint8_t *prow(uint8_t *base, uint32_t t, uint64_t rb)
{
    return base + (uint64_t)t * rb;
}

template <int R, int T, bool INV, bool GEN_L, int LD>
__global__ __launch_bounds__(64) void k_pass(PassArgs a, const uint32_t *__restrict__ p_tw,
                                             const uint32_t *__restrict__ p_B)
{
    constexpr int NW = Traits<R>::NW, NR = 1 << T;
    const TwGlobal<R> tw = {p_tw, a.l};
    const uint32_t g = blockIdx.x / (uint32_t)a.nct;
    const int ct = (int)(blockIdx.x % (uint32_t)a.nct);
    const uint32_t base = group_base(g, a.lo, T);
    const Lane ln = lane_of<R, LD>(ct, (int)threadIdx.x, a.col0, a.ncols);
    const uint64_t rb = a.row_bytes;
    uint32_t x[NR][NW];
#pragma unroll
    for (int j = 0; j < NR; j++) {
        const uint32_t p = base + ((uint32_t)j << a.lo);
        if ((int)p < a.src_rows)
            load_chunk<R, LD>(prow(a.src, p, rb), ln.off, ln.act, ln.nsym, x[j]);
        else
            zero_vec<R>(x[j]);
        if (a.pre_B)
            scale<R>(x[j], row_tab<R>(p_B, (int)p));
    }
    reg_levels<R, T, INV, (GEN_L ? SH_GENERAL : SH_ALIGNED), false>(x, base, a.lo, tw);
#pragma unroll
    for (int j = 0; j < NR; j++) {
        const uint32_t p = fresh(base + ((uint32_t)j << a.lo));
        if (a.post_B)
            scale<R>(x[j], row_tab<R>(p_B, (int)p));
        if constexpr (R == 16) {
            if (a.mul) {
                uint32_t m[NW];
                load_chunk<R, LD>(prow(a.mul, p, rb), ln.off, ln.act, ln.nsym, m);
                mul_symbols16<4>(x[j], m);
            }
        }
        if ((int)p >= a.dst_lo && (int)p < a.dst_hi)
            store_chunk<R, LD>(prow(a.dst, p - (uint32_t)a.dst_lo, rb), ln.off, ln.act, ln.nsym, x[j]);
    }
}

template <int R, int T, int LD>
__global__ __launch_bounds__(64) void k_dpart(DerivPassArgs a, const uint32_t *__restrict__ p_Binv)
{
    constexpr int NW = Traits<R>::NW, NR = 1 << T;
    const uint32_t g = blockIdx.x / (uint32_t)a.nct;
    const int ct = (int)(blockIdx.x % (uint32_t)a.nct);
    const uint32_t base = group_base(g, a.lo, T);
    const Lane ln = lane_of<R, LD>(ct, (int)threadIdx.x, a.col0, a.ncols);
    const uint64_t rb = a.row_bytes;
    uint32_t y[NR][NW];
#pragma unroll
    for (int j = 0; j < NR; j++)
        load_chunk<R, LD>(prow(a.y, base + ((uint32_t)j << a.lo), rb), ln.off, ln.act, ln.nsym, y[j]);
#pragma unroll
    for (int j = 0; j < NR; j++) {
        const uint32_t p = fresh(base + ((uint32_t)j << a.lo));
        uint32_t z[NW];
        if (a.first)
            zero_vec<R>(z);
        else
            load_chunk<R, LD>(prow(a.z, p, rb), ln.off, ln.act, ln.nsym, z);
#pragma unroll
        for (int lv = 0; lv < T; lv++)
            if (!((j >> lv) & 1))
#pragma unroll
                for (int w = 0; w < NW; w++)
                    z[w] ^= y[j + (1 << lv)][w];
        if (a.last) {
            scale<R>(z, row_tab<R>(p_Binv, (int)p));
            store_chunk<R, LD>(prow(a.out, p, rb), ln.off, ln.act, ln.nsym, z);
        } else {
            store_chunk<R, LD>(prow(a.z, p, rb), ln.off, ln.act, ln.nsym, z);
        }
    }
}

// ---------------------------------------------------------------- launchers

template <int R, bool INV, bool GEN_L, int LD>
static hipError_t pass_T(int T, const PassArgs &a, const KPtrs &k, uint32_t nblocks, hipStream_t s)
{
    switch (T) {
    case 0: hipLaunchKernelGGL((k_pass<R, 0, INV, GEN_L, LD>), dim3(nblocks), dim3(64), 0, s, a, k.tw, k.B); break;
    case 1: hipLaunchKernelGGL((k_pass<R, 1, INV, GEN_L, LD>), dim3(nblocks), dim3(64), 0, s, a, k.tw, k.B); break;
    case 2: hipLaunchKernelGGL((k_pass<R, 2, INV, GEN_L, LD>), dim3(nblocks), dim3(64), 0, s, a, k.tw, k.B); break;
    case 3: hipLaunchKernelGGL((k_pass<R, 3, INV, GEN_L, LD>), dim3(nblocks), dim3(64), 0, s, a, k.tw, k.B); break;
    case 4: hipLaunchKernelGGL((k_pass<R, 4, INV, GEN_L, LD>), dim3(nblocks), dim3(64), 0, s, a, k.tw, k.B); break;
    case 5:                     // forward passes only (an inverse one needs too many registers)
        if constexpr (!INV)
            hipLaunchKernelGGL((k_pass<R, 5, INV, GEN_L, LD>), dim3(nblocks), dim3(64), 0, s, a, k.tw, k.B);
        else
            return hipErrorInvalidValue;
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int R, int LD>
static hipError_t pass_r(int T, bool inv, bool gen_l, const PassArgs &a, const KPtrs &k, uint32_t nblocks,
                         hipStream_t s)
{
    if (inv)
        return gen_l ? pass_T<R, true, true, LD>(T, a, k, nblocks, s) : pass_T<R, true, false, LD>(T, a, k, nblocks, s);
    return gen_l ? pass_T<R, false, true, LD>(T, a, k, nblocks, s) : pass_T<R, false, false, LD>(T, a, k, nblocks, s);
}

hipError_t pass_launch(int r, int ld, int T, bool inv, bool gen_l, const PassArgs &a, const KPtrs &k,
                       uint32_t nblocks, hipStream_t s)
{
    if (nblocks == 0)
        return hipSuccess;
    if (r == 16)
        return ld == LD_VEC ? pass_r<16, LD_VEC>(T, inv, gen_l, a, k, nblocks, s)
                            : pass_r<16, LD_SYM>(T, inv, gen_l, a, k, nblocks, s);
    return ld == LD_VEC ? pass_r<8, LD_VEC>(T, inv, gen_l, a, k, nblocks, s)
                        : pass_r<8, LD_SYM>(T, inv, gen_l, a, k, nblocks, s);
}

template <int R, int LD>
static hipError_t dpart_T(int T, const DerivPassArgs &a, const KPtrs &k, uint32_t nblocks, hipStream_t s)
{
    switch (T) {
    case 1: hipLaunchKernelGGL((k_dpart<R, 1, LD>), dim3(nblocks), dim3(64), 0, s, a, k.Binv); break;
    case 2: hipLaunchKernelGGL((k_dpart<R, 2, LD>), dim3(nblocks), dim3(64), 0, s, a, k.Binv); break;
    case 3: hipLaunchKernelGGL((k_dpart<R, 3, LD>), dim3(nblocks), dim3(64), 0, s, a, k.Binv); break;
    case 4: hipLaunchKernelGGL((k_dpart<R, 4, LD>), dim3(nblocks), dim3(64), 0, s, a, k.Binv); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t dpart_launch(int r, int ld, int T, const DerivPassArgs &a, const KPtrs &k, uint32_t nblocks,
                        hipStream_t s)
{
    if (nblocks == 0)
        return hipSuccess;
    if (r == 16)
        return ld == LD_VEC ? dpart_T<16, LD_VEC>(T, a, k, nblocks, s) : dpart_T<16, LD_SYM>(T, a, k, nblocks, s);
    return ld == LD_VEC ? dpart_T<8, LD_VEC>(T, a, k, nblocks, s) : dpart_T<8, LD_SYM>(T, a, k, nblocks, s);
}

}  // namespace nb
