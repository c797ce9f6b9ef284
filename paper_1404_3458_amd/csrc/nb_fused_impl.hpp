// nb_fused_impl.hpp -- fused transform / derivative / encode / decode kernels
// for transform sizes h = 2^L <= 256: one launch per call, one read of the
// inputs and one write of the outputs.  Included by nb_fused16.hip and
// nb_fused8.hip, which instantiate it for one field size each.
//
// A workgroup owns a tile of 256 columns (64 lanes x 4 columns) of one stripe
// and all h rows of it.  Butterflies run in registers on groups of rows:
//   - "consecutive" groups: 16 rows 16g .. 16g+15, levels 0..3;
//   - "stride" groups: rows r0 + 16 j (r0 < 16), levels 4..L-1;
// and the tile is exchanged through LDS between the two groupings.  Lanes of
// a wave always share their rows, so every skew factor (which depends only
// on the level, the block and the shift, Sec. 3.2) is wave-uniform and its
// perm table is fetched with scalar loads.  For L <= 4 a single wave holds
// the whole transform in registers and no LDS is used.
#pragma once
#include "nb_xform.hpp"

namespace nb {

enum Mode { M_FFT = 0, M_IFFT = 1, M_DERIV = 2, M_ENC = 3, M_DEC = 4 };

__device__ __forceinline__ const uint8_t *row_ptr(const uint8_t *base, uint32_t t, uint64_t rb)
{
    return base + (uint64_t)t * rb;
}
__device__ __forceinline__ uint8_t *row_ptr(uint8_t *base, uint32_t t, uint64_t rb)
{
    return base + (uint64_t)t * rb;
}

// Decode step 2 (eq. hatF(l)) for one point: received symbols times Pi(omega_p);
// erased, virtual and never-stored points are zero.  Surviving rows are
// copied to the output when decoding out of place.
template <int R, int LD>
__device__ __forceinline__ void dec_load(uint32_t *v, int p, const DevStripe &st, const Lane &ln,
                                         const uint32_t *__restrict__ bits, const uint32_t *__restrict__ rowtab)
{
    constexpr int TS = Traits<R>::TS;
    const bool rcv = point_bit(bits, p);
    const uint32_t tr = rcv ? (uint32_t)point_row(p, st) : 0u;
    uint32_t raw[Traits<R>::NW];
    load_chunk<R, LD>(row_ptr(st.in, tr, st.row_bytes), ln.off, ln.act && rcv, ln.nsym, raw);
    if (st.copy_survivors)
        store_chunk<R, LD>(row_ptr(st.out, tr, st.row_bytes), ln.off, ln.act && rcv, ln.nsym, raw);
    zero_vec<R>(v);
    if (rcv)
        Ops<R>::mac(v, raw, Ops<R>::prep(rowtab + (size_t)TS * p));
    __builtin_amdgcn_sched_barrier(0);
}

// Decode step 6 (eq. F(j)) for one point: erased stored rows get
// Phi^d[p] / Pi'(omega_p).
template <int R, int LD>
__device__ __forceinline__ void dec_store(const uint32_t *v, int p_, const DevStripe &st, const Lane &ln,
                                          const uint32_t *__restrict__ bits, const uint32_t *__restrict__ rowtab)
{
    constexpr int TS = Traits<R>::TS;
    const int p = (int)fresh((uint32_t)p_);
    if (point_bit(bits + bitmap_words(st.np), p)) {
        const int t = point_row(p, st);
        uint32_t o[Traits<R>::NW];
        zero_vec<R>(o);
        Ops<R>::mac(o, v, Ops<R>::prep(rowtab + (size_t)TS * p));
        store_chunk<R, LD>(row_ptr(st.out, (uint32_t)t, st.row_bytes), ln.off, ln.act, ln.nsym, o);
    }
    __builtin_amdgcn_sched_barrier(0);
}

// Sec. 4.2 on rows all held in registers: d^d = B d, coefficient of X_j is
// the sum of d^d_{j + 2^l} over the clear bits l of j, divided by B_j.
template <int R, int L>
__device__ __forceinline__ void deriv_regs(uint32_t (*x)[Traits<R>::NW], const Tabs &tb)
{
    constexpr int NW = Traits<R>::NW, TS = Traits<R>::TS, NR = 1 << L;
    uint32_t y[NR][NW];
#pragma unroll
    for (int j = 0; j < NR; j++) {
#pragma unroll
        for (int w = 0; w < NW; w++)
            y[j][w] = x[j][w];
        if (j)
            scale<R>(y[j], tb.B + (size_t)TS * fresh(j));     // B_0 = 1
    }
#pragma unroll
    for (int j = 0; j < NR; j++) {
        zero_vec<R>(x[j]);
#pragma unroll
        for (int lv = 0; lv < L; lv++)
            if (!((j >> lv) & 1))
#pragma unroll
                for (int w = 0; w < NW; w++)
                    x[j][w] ^= y[j + (1 << lv)][w];
        if (j && j + 1 < NR)
            scale<R>(x[j], tb.Binv + (size_t)TS * fresh(j));  // 1/B_0 = 1; row NR-1 is 0
    }
}

#define NB_FUSED_PARAMS                                                                                       \
    FusedArgs a, const uint32_t *__restrict__ p_tw, const uint32_t *__restrict__ p_one,                       \
        const uint32_t *__restrict__ p_B, const uint32_t *__restrict__ p_Binv,                                \
        const uint32_t *__restrict__ p_bits, const uint32_t *__restrict__ p_rowtabs

// ------------------------------------------------------------------ L <= 4

template <int R, int L, int MODE, int SH, int LD>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_small(NB_FUSED_PARAMS)
{
    constexpr int NW = Traits<R>::NW, NR = 1 << L;
    const int tile = blockIdx.x;
    const int s = find_stripe(a.stripes, a.nstripes, tile);
    const DevStripe st = a.stripes[s];
    const Lane ln = lane_of<R, LD>(tile - st.tile0, (int)threadIdx.x, st.col0, st.ncols);
    const uint64_t rb = st.row_bytes;
    const Tabs tb = {p_tw, p_one, p_B, p_Binv};
    const uint32_t *__restrict__ bits = p_bits + st.bits_off;
    const uint32_t *__restrict__ rowtab = p_rowtabs + st.rowtab_off;
    uint32_t x[NR][NW];

    if (MODE == M_FFT || MODE == M_IFFT || MODE == M_DERIV) {
#pragma unroll
        for (int j = 0; j < NR; j++)
            load_chunk<R, LD>(row_ptr(st.in, j, rb), ln.off, ln.act, ln.nsym, x[j]);
        if (MODE == M_FFT)
            reg_levels<R, L, false, SH, true>(x, 0, 0, a.l, tb);
        else if (MODE == M_IFFT)
            reg_levels<R, L, true, SH, true>(x, 0, 0, a.l, tb);
        else
            deriv_regs<R, L>(x, tb);
#pragma unroll
        for (int j = 0; j < NR; j++)
            store_chunk<R, LD>(row_ptr(st.out, fresh(j), rb), ln.off, ln.act, ln.nsym, x[j]);
    } else if (MODE == M_ENC) {
        // Algorithm 1: M_bar = inverse transform of the (zero-padded) message,
        // then one forward transform per parity block at shift blk * k'.
#pragma unroll
        for (int j = 0; j < NR; j++)
            load_chunk<R, LD>(row_ptr(st.in, j, rb), ln.off, ln.act && j < st.k, ln.nsym, x[j]);
        reg_levels<R, L, true, SH_ZERO, true>(x, 0, 0, 0u, tb);
        const int nblocks = st.np / st.kp;
        const int npar = st.n - st.k;
        for (int blk = 1; blk < nblocks; blk++) {
            uint32_t y[NR][NW];
#pragma unroll
            for (int j = 0; j < NR; j++)
#pragma unroll
                for (int w = 0; w < NW; w++)
                    y[j][w] = x[j][w];
            reg_levels<R, L, false, SH_ALIGNED, true>(y, 0, 0, (uint32_t)(blk * NR), tb);
#pragma unroll
            for (int j = 0; j < NR; j++) {
                const int t = (blk - 1) * NR + j;
                if (t < npar)
                    store_chunk<R, LD>(row_ptr(st.out, fresh(t), rb), ln.off, ln.act, ln.nsym, y[j]);
            }
        }
    } else {  // M_DEC with n' = NR
#pragma unroll
        for (int p = 0; p < NR; p++)
            dec_load<R, LD>(x[p], p, st, ln, bits, rowtab);
        reg_levels<R, L, true, SH_ZERO, true>(x, 0, 0, 0u, tb);     // step 3
        deriv_regs<R, L>(x, tb);                             // step 4
        reg_levels<R, L, false, SH_ZERO, true>(x, 0, 0, 0u, tb);    // step 5
#pragma unroll
        for (int p = 0; p < NR; p++)                         // step 6
            dec_store<R, LD>(x[p], p, st, ln, bits, rowtab);
    }
}

// ------------------------------------------------------------------ 5 <= L <= 8

template <int R, int L, int MODE, int SH, int LD>
__global__ __launch_bounds__(64 << (L - 4)) __attribute__((amdgpu_waves_per_eu(4))) void k_tiled(NB_FUSED_PARAMS)
{
    constexpr int NW = Traits<R>::NW, TS = Traits<R>::TS;
    constexpr int L2 = L - 4;            // levels of the stride phase
    constexpr int NR2 = 1 << L2;         // rows per stride group
    constexpr int GPW = 16 >> L2;        // stride groups per wave (waves = 2^L2)
    extern __shared__ uint32_t lds[];    // [2^L rows][64 lanes][NW]

    const int lane = (int)threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int tile = blockIdx.x;
    const int s = find_stripe(a.stripes, a.nstripes, tile);
    const DevStripe st = a.stripes[s];
    const Lane ln = lane_of<R, LD>(tile - st.tile0, lane, st.col0, st.ncols);
    const uint64_t rb = st.row_bytes;
    const Tabs tb = {p_tw, p_one, p_B, p_Binv};
    const uint32_t *__restrict__ bits = p_bits + st.bits_off;
    const uint32_t *__restrict__ rowtab = p_rowtabs + st.rowtab_off;

    auto lds_put = [&](int row, const uint32_t *v) {
        uint32_t *p = lds + ((size_t)row * 64 + lane) * NW;
        if (NW == 2)
            *reinterpret_cast<uint2 *>(p) = make_uint2(v[0], v[NW - 1]);
        else
            p[0] = v[0];
    };
    auto lds_get = [&](int row, uint32_t *v) {
        const uint32_t *p = lds + ((size_t)row * 64 + lane) * NW;
        if (NW == 2) {
            const uint2 t = *reinterpret_cast<const uint2 *>(p);
            v[0] = t.x;
            v[NW - 1] = t.y;
        } else {
            v[0] = p[0];
        }
    };

    const int g = wave;                       // consecutive group of this wave
    uint32_t x[16][NW];                       // consecutive-phase registers
    uint32_t y[GPW][NR2][NW];                 // stride-phase registers

    if (MODE == M_FFT) {
#pragma unroll
        for (int u = 0; u < GPW; u++) {
            const int r0 = wave * GPW + u;
#pragma unroll
            for (int j = 0; j < NR2; j++)
                load_chunk<R, LD>(row_ptr(st.in, r0 + 16 * j, rb), ln.off, ln.act, ln.nsym, y[u][j]);
            reg_levels<R, L2, false, SH, true>(y[u], (uint32_t)r0, 4, a.l, tb);
#pragma unroll
            for (int j = 0; j < NR2; j++)
                lds_put(r0 + 16 * j, y[u][j]);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 16; j++)
            lds_get(16 * g + j, x[j]);
        reg_levels<R, 4, false, SH, false>(x, (uint32_t)(16 * g), 0, a.l, tb);
#pragma unroll
        for (int j = 0; j < 16; j++)
            store_chunk<R, LD>(row_ptr(st.out, fresh(16 * g + j), rb), ln.off, ln.act, ln.nsym, x[j]);
        return;
    }

    if (MODE == M_DERIV) {
        // Sec. 4.2 on consecutive groups: partners 2^l with l < 4 are in the
        // wave's registers, those with l >= 4 are read from LDS.
#pragma unroll
        for (int j = 0; j < 16; j++) {
            const int p = 16 * g + j;
            load_chunk<R, LD>(row_ptr(st.in, p, rb), ln.off, ln.act, ln.nsym, x[j]);
            if (p)
                scale<R>(x[j], tb.B + (size_t)TS * p);
            lds_put(p, x[j]);
        }
        __syncthreads();
        uint32_t z[16][NW];
#pragma unroll
        for (int j = 0; j < 16; j++) {
            zero_vec<R>(z[j]);
#pragma unroll
            for (int lv = 0; lv < 4; lv++)
                if (!((j >> lv) & 1))
#pragma unroll
                    for (int w = 0; w < NW; w++)
                        z[j][w] ^= x[j + (1 << lv)][w];
        }
#pragma unroll
        for (int lv = 0; lv < L2; lv++) {
            if (!((g >> lv) & 1)) {
                const int pg = g + (1 << lv);
#pragma unroll
                for (int j = 0; j < 16; j++) {
                    uint32_t v[NW];
                    lds_get(16 * pg + j, v);
#pragma unroll
                    for (int w = 0; w < NW; w++)
                        z[j][w] ^= v[w];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < 16; j++) {
            const int p = (int)fresh(16 * g + j);
            if (p)
                scale<R>(z[j], tb.Binv + (size_t)TS * p);
            store_chunk<R, LD>(row_ptr(st.out, p, rb), ln.off, ln.act, ln.nsym, z[j]);
        }
        return;
    }

    // ---- phase 1 (consecutive groups): input and inverse levels 0..3
#pragma unroll
    for (int j = 0; j < 16; j++) {
        const int p = 16 * g + j;
        if (MODE == M_IFFT) {
            load_chunk<R, LD>(row_ptr(st.in, p, rb), ln.off, ln.act, ln.nsym, x[j]);
        } else if (MODE == M_ENC) {
            // rows k .. k'-1 are the zero padding of a shortened message
            load_chunk<R, LD>(row_ptr(st.in, p, rb), ln.off, ln.act && p < st.k, ln.nsym, x[j]);
        } else {
            dec_load<R, LD>(x[j], p, st, ln, bits, rowtab);
        }
    }
    reg_levels<R, 4, true, (MODE == M_IFFT ? SH : SH_ZERO), false>(x, (uint32_t)(16 * g), 0,
                                                                   MODE == M_IFFT ? a.l : 0u, tb);
#pragma unroll
    for (int j = 0; j < 16; j++)
        lds_put(16 * g + j, x[j]);
    __syncthreads();

    // ---- phase 2 (stride groups): inverse levels 4..L-1
#pragma unroll
    for (int u = 0; u < GPW; u++) {
        const int r0 = wave * GPW + u;
#pragma unroll
        for (int j = 0; j < NR2; j++)
            lds_get(r0 + 16 * j, y[u][j]);
        reg_levels<R, L2, true, (MODE == M_IFFT ? SH : SH_ZERO), true>(y[u], (uint32_t)r0, 4,
                                                                      MODE == M_IFFT ? a.l : 0u, tb);
    }

    if (MODE == M_IFFT) {
#pragma unroll
        for (int u = 0; u < GPW; u++) {
            const int r0 = wave * GPW + u;
#pragma unroll
            for (int j = 0; j < NR2; j++)
                store_chunk<R, LD>(row_ptr(st.out, fresh(r0 + 16 * j), rb), ln.off, ln.act, ln.nsym, y[u][j]);
        }
        return;
    }

    if (MODE == M_ENC) {
        const int nblocks = st.np / st.kp;
        const int npar = st.n - st.k;
        for (int blk = 1; blk < nblocks; blk++) {
            const uint32_t lsh = (uint32_t)(blk << L);
            if (blk > 1)
                __syncthreads();      // the previous block's phase-3 reads are done
#pragma unroll
            for (int u = 0; u < GPW; u++) {
                const int r0 = wave * GPW + u;
                uint32_t z[NR2][NW];
#pragma unroll
                for (int j = 0; j < NR2; j++)
#pragma unroll
                    for (int w = 0; w < NW; w++)
                        z[j][w] = y[u][j][w];
                reg_levels<R, L2, false, SH_ALIGNED, true>(z, (uint32_t)r0, 4, lsh, tb);
#pragma unroll
                for (int j = 0; j < NR2; j++)
                    lds_put(r0 + 16 * j, z[j]);
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < 16; j++)
                lds_get(16 * g + j, x[j]);
            reg_levels<R, 4, false, SH_ALIGNED, false>(x, (uint32_t)(16 * g), 0, lsh, tb);
#pragma unroll
            for (int j = 0; j < 16; j++) {
                const int t = (blk - 1) * (1 << L) + 16 * g + j;
                if (t < npar)
                    store_chunk<R, LD>(row_ptr(st.out, fresh(t), rb), ln.off, ln.act, ln.nsym, x[j]);
            }
        }
        return;
    }

    // ---- M_DEC: step 4 (derivative) across the two groupings, then step 5.
#pragma unroll
    for (int u = 0; u < GPW; u++) {
        const int r0 = wave * GPW + u;
#pragma unroll
        for (int j = 0; j < NR2; j++) {
            const int p = r0 + 16 * j;
            if (p)
                scale<R>(y[u][j], tb.B + (size_t)TS * p);
            lds_put(p, y[u][j]);
        }
    }
    __syncthreads();
    uint32_t z[GPW][NR2][NW];
#pragma unroll
    for (int u = 0; u < GPW; u++) {
        const int r0 = wave * GPW + u;
#pragma unroll
        for (int j = 0; j < NR2; j++) {
            zero_vec<R>(z[u][j]);
#pragma unroll
            for (int lv = 0; lv < L2; lv++)              // partners 16 * 2^lv away
                if (!((j >> lv) & 1))
#pragma unroll
                    for (int w = 0; w < NW; w++)
                        z[u][j][w] ^= y[u][j + (1 << lv)][w];
        }
#pragma unroll
        for (int lv = 0; lv < 4; lv++) {                 // partners 2^lv away
            if (!((r0 >> lv) & 1)) {
                const int pr = r0 + (1 << lv);
#pragma unroll
                for (int j = 0; j < NR2; j++) {
                    uint32_t v[NW];
                    lds_get(pr + 16 * j, v);
#pragma unroll
                    for (int w = 0; w < NW; w++)
                        z[u][j][w] ^= v[w];
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < GPW; u++) {
        const int r0 = wave * GPW + u;
#pragma unroll
        for (int j = 0; j < NR2; j++) {
            const int p = r0 + 16 * j;
            if (p)
                scale<R>(z[u][j], tb.Binv + (size_t)TS * p);
        }
        reg_levels<R, L2, false, SH_ZERO, true>(z[u], (uint32_t)r0, 4, 0u, tb);
#pragma unroll
        for (int j = 0; j < NR2; j++)
            lds_put(r0 + 16 * j, z[u][j]);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; j++)
        lds_get(16 * g + j, x[j]);
    reg_levels<R, 4, false, SH_ZERO, false>(x, (uint32_t)(16 * g), 0, 0u, tb);
#pragma unroll
    for (int j = 0; j < 16; j++)
        dec_store<R, LD>(x[j], 16 * g + j, st, ln, bits, rowtab);
}

// ------------------------------------------------------------------ launchers

template <int R, int L, int MODE, int SH, int LD>
static hipError_t launch_one(const FusedArgs &a, const KPtrs &k, int ntiles, hipStream_t stream)
{
    if (ntiles <= 0)
        return hipSuccess;
    if (L <= 4) {
        hipLaunchKernelGGL((k_small<R, (L <= 4 ? L : 4), MODE, SH, LD>), dim3(ntiles), dim3(64), 0, stream, a,
                           k.tw, k.one, k.B, k.Binv, k.bits, k.rowtabs);
    } else {
        constexpr int LL = L > 4 ? L : 5;
        const size_t lds = (size_t)(1u << LL) * 64 * Traits<R>::NW * 4;
        hipLaunchKernelGGL((k_tiled<R, LL, MODE, SH, LD>), dim3(ntiles), dim3(64 << (LL - 4)), lds, stream, a,
                           k.tw, k.one, k.B, k.Binv, k.bits, k.rowtabs);
    }
    return hipGetLastError();
}

template <int R, int L, int MODE, int SH, int LD>
static hipError_t prep_one()
{
    if (L > 4) {
        constexpr int LL = L > 4 ? L : 5;
        const int lds = (int)((1u << LL) * 64 * Traits<R>::NW * 4);
        return hipFuncSetAttribute((const void *)k_tiled<R, LL, MODE, SH, LD>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    }
    return hipSuccess;
}

template <int R, int MODE, int SH, int LD>
static hipError_t launch_L(int L, const FusedArgs &a, const KPtrs &k, int ntiles, hipStream_t s)
{
    switch (L) {
    case 0: return launch_one<R, 0, MODE, SH, LD>(a, k, ntiles, s);
    case 1: return launch_one<R, 1, MODE, SH, LD>(a, k, ntiles, s);
    case 2: return launch_one<R, 2, MODE, SH, LD>(a, k, ntiles, s);
    case 3: return launch_one<R, 3, MODE, SH, LD>(a, k, ntiles, s);
    case 4: return launch_one<R, 4, MODE, SH, LD>(a, k, ntiles, s);
    case 5: return launch_one<R, 5, MODE, SH, LD>(a, k, ntiles, s);
    case 6: return launch_one<R, 6, MODE, SH, LD>(a, k, ntiles, s);
    case 7: return launch_one<R, 7, MODE, SH, LD>(a, k, ntiles, s);
    case 8: return launch_one<R, 8, MODE, SH, LD>(a, k, ntiles, s);
    default: return hipErrorInvalidValue;
    }
}

template <int R, int MODE, int SH, int LD>
static hipError_t prep_L()
{
    hipError_t e = hipSuccess, f;
    if ((f = prep_one<R, 5, MODE, SH, LD>()) != hipSuccess) e = f;
    if ((f = prep_one<R, 6, MODE, SH, LD>()) != hipSuccess) e = f;
    if ((f = prep_one<R, 7, MODE, SH, LD>()) != hipSuccess) e = f;
    if ((f = prep_one<R, 8, MODE, SH, LD>()) != hipSuccess) e = f;
    return e;
}

template <int R, int LD>
static hipError_t launch_ld(int mode, int sh, int L, const FusedArgs &a, const KPtrs &k, int ntiles, hipStream_t s)
{
    switch (mode) {
    case M_FFT:
        return sh == SH_ZERO ? launch_L<R, M_FFT, SH_ZERO, LD>(L, a, k, ntiles, s)
             : sh == SH_ALIGNED ? launch_L<R, M_FFT, SH_ALIGNED, LD>(L, a, k, ntiles, s)
                                : launch_L<R, M_FFT, SH_GENERAL, LD>(L, a, k, ntiles, s);
    case M_IFFT:
        return sh == SH_ZERO ? launch_L<R, M_IFFT, SH_ZERO, LD>(L, a, k, ntiles, s)
             : sh == SH_ALIGNED ? launch_L<R, M_IFFT, SH_ALIGNED, LD>(L, a, k, ntiles, s)
                                : launch_L<R, M_IFFT, SH_GENERAL, LD>(L, a, k, ntiles, s);
    case M_DERIV: return launch_L<R, M_DERIV, SH_ZERO, LD>(L, a, k, ntiles, s);
    case M_ENC: return launch_L<R, M_ENC, SH_ZERO, LD>(L, a, k, ntiles, s);
    case M_DEC: return launch_L<R, M_DEC, SH_ZERO, LD>(L, a, k, ntiles, s);
    }
    return hipErrorInvalidValue;
}

template <int R>
static hipError_t fused_prepare_r()
{
    hipError_t e = hipSuccess, f;
#define NB_PREP(M, SHM, LD) if ((f = prep_L<R, M, SHM, LD>()) != hipSuccess) e = f;
    NB_PREP(M_FFT, SH_ZERO, LD_VEC) NB_PREP(M_FFT, SH_ALIGNED, LD_VEC) NB_PREP(M_FFT, SH_GENERAL, LD_VEC)
    NB_PREP(M_IFFT, SH_ZERO, LD_VEC) NB_PREP(M_IFFT, SH_ALIGNED, LD_VEC) NB_PREP(M_IFFT, SH_GENERAL, LD_VEC)
    NB_PREP(M_DERIV, SH_ZERO, LD_VEC) NB_PREP(M_ENC, SH_ZERO, LD_VEC) NB_PREP(M_DEC, SH_ZERO, LD_VEC)
    NB_PREP(M_FFT, SH_ZERO, LD_SYM) NB_PREP(M_FFT, SH_ALIGNED, LD_SYM) NB_PREP(M_FFT, SH_GENERAL, LD_SYM)
    NB_PREP(M_IFFT, SH_ZERO, LD_SYM) NB_PREP(M_IFFT, SH_ALIGNED, LD_SYM) NB_PREP(M_IFFT, SH_GENERAL, LD_SYM)
    NB_PREP(M_DERIV, SH_ZERO, LD_SYM) NB_PREP(M_ENC, SH_ZERO, LD_SYM) NB_PREP(M_DEC, SH_ZERO, LD_SYM)
#undef NB_PREP
    return e;
}

}  // namespace nb
