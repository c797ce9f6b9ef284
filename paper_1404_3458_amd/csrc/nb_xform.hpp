// nb_xform.hpp -- register-level transform helpers shared by the fused
// (h <= 256) and multi-pass (h > 256) kernels.
//
// Level order and butterflies follow Sec. 3.2 (forward: levels lg h - 1 down
// to 0, a += s b then b += a) and Sec. 3.3 (inverse: levels 0 up, b += a then
// a += s b), with Delta_i^m(omega_c + omega_l) stored at index c + m, so rows
// come out in natural order.
#pragma once
#include "nb_device.hpp"
#include "nb_internal.hpp"

namespace nb {

__device__ __forceinline__ int find_stripe(const DevStripe *__restrict__ st, int n, int tile)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (st[mid].tile0 <= tile)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// How the shift l of a transform is known to the kernel:
//   SH_ZERO     l = 0: the factor of block c = 0 is zero at every level;
//   SH_ALIGNED  h divides l and l != 0: no factor is zero, and bit i of l is
//               clear for every level i < lg h;
//   SH_GENERAL  any l.
enum { SH_ZERO = 0, SH_ALIGNED = 1, SH_GENERAL = 2 };

// Skew factor W_i(omega_c + omega_l) / W_i(omega_{2^i}) for a block c (bits
// <= i clear): by additivity (Lemma 1) it is the table entry of level i at
// (c xor l) >> (i + 1), plus 1 when bit i of l is set (W_i(v_i) normalises to 1).
template <int R, int SH>
struct Twiddle {
    static constexpr int TS = Traits<R>::TS;
    uint32_t buf[SH == SH_GENERAL ? TS : 1];
    __device__ __forceinline__ const uint32_t *get(const Tabs &tb, int i, uint32_t c, uint32_t l)
    {
        const uint32_t off = (1u << R) - (1u << (R - i));
        // an opaque index: the same factor loaded by two transforms of a kernel
        // is loaded twice instead of being kept live in between
        const uint32_t *t = tb.tw + (size_t)TS * fresh(off + ((c ^ l) >> (i + 1)));
        if (SH == SH_GENERAL && ((l >> i) & 1u)) {
#pragma unroll
            for (int u = 0; u < TS; u++)
                buf[u] = t[u] ^ tb.one[u];
            return buf;
        }
        return t;
    }
};

template <int R, bool INV>
__device__ __forceinline__ void bfly(uint32_t *a, uint32_t *b, const typename Ops<R>::Tab &T, bool zero)
{
    constexpr int NW = Traits<R>::NW;
    if (!INV) {
        if (!zero)
            Ops<R>::mac(a, b, T);
#pragma unroll
        for (int w = 0; w < NW; w++)
            b[w] ^= a[w];
    } else {
#pragma unroll
        for (int w = 0; w < NW; w++)
            b[w] ^= a[w];
        if (!zero)
            Ops<R>::mac(a, b, T);
    }
}

// T levels on 2^T rows in registers; x[j] is global row base + (j << LO),
// where base has no set bit in positions LO .. LO+T-1.  A zero factor only
// occurs at shift 0 for block c = 0; the multiply is skipped there when
// CT_BASE says that base has no bit at or above LO (so that block 0 of the
// group is block 0 of the transform, known at compile time).  Elsewhere a
// zero factor is simply multiplied (its table is all zero), which avoids a
// data-dependent branch around the butterflies.
template <int R, int T, bool INV, int SH, bool CT_BASE>
__device__ __forceinline__ void reg_levels(uint32_t (*x)[Traits<R>::NW], uint32_t base, int LO, uint32_t l,
                                           const Tabs &tb)
{
    constexpr int NR = 1 << T;
    Twiddle<R, SH> tw;
#pragma unroll
    for (int tt = 0; tt < T; tt++) {
        const int t = INV ? tt : T - 1 - tt;
        const int i = LO + t;
#pragma unroll
        for (int blk = 0; blk < NR; blk += 2 << t) {
            const bool zero = SH == SH_ZERO && CT_BASE && blk == 0;
            if (zero) {
                const typename Ops<R>::Tab tab = {};
#pragma unroll
                for (int m = 0; m < (1 << t); m++)
                    bfly<R, INV>(x[blk + m], x[blk + m + (1 << t)], tab, true);
            } else {
                const uint32_t c = (base & ~((2u << i) - 1u)) | ((uint32_t)blk << LO);
                const typename Ops<R>::Tab tab = Ops<R>::prep(tw.get(tb, i, c, l));
#pragma unroll
                for (int m = 0; m < (1 << t); m++)
                    bfly<R, INV>(x[blk + m], x[blk + m + (1 << t)], tab, false);
            }
            // keep each block's factor table live only while it is used
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// x <- s_row * x for a row whose perm table is t.
template <int R>
__device__ __forceinline__ void scale(uint32_t *x, const uint32_t *t)
{
    constexpr int NW = Traits<R>::NW;
    uint32_t acc[NW];
#pragma unroll
    for (int w = 0; w < NW; w++)
        acc[w] = 0;
    Ops<R>::mac(acc, x, Ops<R>::prep(t));
#pragma unroll
    for (int w = 0; w < NW; w++)
        x[w] = acc[w];
    __builtin_amdgcn_sched_barrier(0);
}

// Stored row of point p of the mother code, -1 for a virtual zero point,
// -2 for a point that is never stored.
__device__ __forceinline__ int point_row(int p, const DevStripe &st)
{
    if (p < st.k)
        return p;
    if (p < st.kp)
        return -1;
    const int t = st.k + (p - st.kp);
    return t < st.n ? t : -2;
}

// Bit p of a point bitmap (read with scalar loads).
__device__ __forceinline__ bool point_bit(const uint32_t *__restrict__ bm, int p)
{
    return (bm[p >> 5] >> (p & 31)) & 1u;
}

__device__ __forceinline__ int bitmap_words(int np) { return (np + 31) >> 5; }

template <int R>
__device__ __forceinline__ void zero_vec(uint32_t *v)
{
#pragma unroll
    for (int w = 0; w < Traits<R>::NW; w++)
        v[w] = 0;
}

}  // namespace nb
