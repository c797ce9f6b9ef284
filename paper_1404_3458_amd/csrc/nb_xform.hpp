// nb_xform.hpp -- register-level transform helpers shared by the fused
// (h <= 256) and multi-pass (h > 256) kernels.
//
// Level order and butterflies follow Sec. 3.2 (forward: levels lg h - 1 down
// to 0, a += s b then b += a) and Sec. 3.3 (inverse: levels 0 up, b += a then
// a += s b), with Delta_i^m(omega_c + omega_l) stored at index c + m, so rows
// come out in natural order.
#pragma once
#include <type_traits>

#include "nb_device.hpp"
#include "nb_internal.hpp"

namespace nb {

// Stripe descriptors are written by the host only; a kernel that stores to
// global memory before reading one reads it through the constant address
// space, so that the reads stay scalar loads.  (The host pass of a kernel
// body sees plain pointers.)
#if defined(__HIP_DEVICE_COMPILE__)
typedef const __attribute__((address_space(4))) DevStripe ConstStripe;
#else
typedef const DevStripe ConstStripe;
#endif

__device__ __forceinline__ ConstStripe *const_stripes(const DevStripe *p)
{
    return (ConstStripe *)p;
}

template <class P>
__device__ __forceinline__ int find_stripe(P st, int n, int tile)
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

// The same for a launch of one workgroup per tile over ntiles tiles: the
// stripe at the tile's share of the stripe count is tried first (it is
// the right one when the stripes have equal tile counts, with both loads
// in flight at once), the search only when it is not.
template <class P>
__device__ __forceinline__ int find_stripe_guess(P st, int n, int tile, int ntiles)
{
    const int g = (int)((int64_t)tile * n / ntiles);
    const int lo = st[g].tile0, hi = g + 1 < n ? st[g + 1].tile0 : ntiles;
    if (lo <= tile && tile < hi)
        return g;
    return find_stripe(st, n, tile);
}

// How the shift l of a transform is known to the kernel:
//   SH_ZERO     l = 0: the factor of block c = 0 is zero at every level;
//   SH_ALIGNED  h divides l and l != 0: no factor is zero, and bit i of l is
//               clear for every level i < lg h;
//   SH_GENERAL  any l.
enum { SH_ZERO = 0, SH_ALIGNED = 1, SH_GENERAL = 2 };

// Skew factor W_i(omega_c + omega_l) / W_i(omega_{2^i}) for a block c (bits
// <= i clear): by additivity (Lemma 1) it is the table entry of level i at
// (c xor l) >> (i + 1), plus 1 when bit i of l is set (W_i(v_i) normalises to
// 1).  The "plus 1" is applied as an extra a += b in the butterfly, so a
// factor source only ever yields plain table entries.

// Factor source reading whole perm tables from global memory.
template <int R>
struct TwGlobal {
    static constexpr int TS = Traits<R>::TS;
    typedef typename Ops<R>::Tab Tab;
    const uint32_t *__restrict__ tw;
    uint32_t l;
    __device__ __forceinline__ uint32_t plus1(int i) const { return ((l >> i) & 1u) ? ~0u : 0u; }
    __device__ __forceinline__ typename Ops<R>::Tab tab(int i, uint32_t c) const
    {
        const uint32_t off = (1u << R) - (1u << (R - i));
        // an opaque index: the same factor fetched by two transforms of a
        // kernel is fetched twice instead of being kept live in between
        return Ops<R>::prep(tw + (size_t)TS * fresh(off + ((c ^ l) >> (i + 1))));
    }
};

// Factor source for a group of 2^LT rows gbase + (j << lo) (gbase has no bit
// in lo .. lo+LT-1) transformed at shift l, whose local levels i < LT are the
// global levels lo + i.  The V words were staged in LDS by stage_levels
// (local level i at entries 2^LT - 2^(LT-i) + q); the S words are read from
// global memory.  A whole transform is the group lo = 0, gbase = 0.
template <int R, int LT>
struct TwLds {
    static constexpr int TS = Traits<R>::TS, NV = Ops<R>::NV;
    typedef typename Ops<R>::Tab Tab;
    const uint32_t *__restrict__ tw;
    uint32_t l;
    const uint32_t *vt;
    uint32_t lo = 0, gbase = 0;
    __device__ __forceinline__ uint32_t plus1(int i) const { return ((l >> (lo + i)) & 1u) ? ~0u : 0u; }
    __device__ __forceinline__ typename Ops<R>::Tab tab(int i, uint32_t c) const
    {
        const int I = (int)lo + i;
        const uint32_t off = (1u << R) - (1u << (R - I));
        const uint32_t cg = gbase | (c << lo);
        const uint32_t q = ((c ^ (l >> lo)) & ((1u << LT) - 1u)) >> (i + 1);
        const uint32_t e = fresh((1u << LT) - (1u << (LT - i)) + q);
        return Ops<R>::prep_lds(vt + NV * e, tw + (size_t)TS * fresh(off + ((cg ^ l) >> (I + 1))));
    }
};

// The same factors with every word of a table staged in LDS (stage_levels
// with WPE = TAB16) and read per lane: for a wave whose two halves hold rows
// of different blocks (GF(2^16) only).
template <int LT>
struct TwLdsV {
    typedef Tab16V Tab;
    uint32_t l;
    const uint32_t *vt;
    uint32_t lo = 0;
    __device__ __forceinline__ uint32_t plus1(int i) const { return ((l >> (lo + i)) & 1u) ? ~0u : 0u; }
    __device__ __forceinline__ Tab tab(int i, uint32_t c) const
    {
        const uint32_t q = ((c ^ (l >> lo)) & ((1u << LT) - 1u)) >> (i + 1);
        return tab_lds_all(vt + TAB16 * ((1u << LT) - (1u << (LT - i)) + q));
    }
};

// Cooperative copy (all threads of the block) of the first WPE words (the V
// words by default, the whole table with WPE = TAB16) of the factor tables
// TwLds / TwLdsV read: local level i holds the 2^(LT-i-1) entries starting at
// table index 2^r - 2^(r-lo-i) + (((gbase ^ l) >> (lo + LT)) << (LT - i - 1)).
template <int R, int LT, int WPE = Ops<R>::NV>
__device__ __forceinline__ void stage_levels(uint32_t *vt, const uint32_t *__restrict__ tw, uint32_t l, int tid,
                                             int nthreads, uint32_t lo = 0, uint32_t gbase = 0)
{
    constexpr int TS = Traits<R>::TS, NV = WPE, H = 1 << LT;
    // 16-byte pieces when every table (and the staged copy) is 16-byte aligned
    typedef typename std::conditional<(TS % 4 == 0 && NV % 4 == 0), uint4, uint2>::type Piece;
    constexpr int PW = sizeof(Piece) / 4, PER = NV / PW;     // words per piece, pieces per entry
    const uint32_t hi = (gbase ^ l) >> (lo + LT);
    for (int u = tid; u < (H - 1) * PER; u += nthreads) {
        const int e = u / PER, w = u % PER;
        const int m = H - 1 - e;                       // in [2^(LT-i-1), 2^(LT-i) - 1]
        const int i = LT - 1 - (31 - __builtin_clz((unsigned)m));
        const int q = e - (H - (H >> i));
        const int I = (int)lo + i;
        const uint32_t g = (1u << R) - (1u << (R - I)) + (hi << (LT - i - 1)) + (uint32_t)q;
        const Piece v = *reinterpret_cast<const Piece *>(tw + (size_t)TS * g + PW * w);
        *reinterpret_cast<Piece *>(vt + NV * e + PW * w) = v;
    }
}

// Cooperative copy of the first WPE words of `count` perm tables: entries
// first + (j << lo) of src for j < count.
template <int R, int WPE = Ops<R>::NV>
__device__ __forceinline__ void stage_rows(uint32_t *vt, const uint32_t *__restrict__ src, int count, int tid,
                                           int nthreads, uint32_t lo = 0, uint32_t first = 0)
{
    constexpr int TS = Traits<R>::TS, NV = WPE;
    typedef typename std::conditional<(TS % 4 == 0 && NV % 4 == 0), uint4, uint2>::type Piece;
    constexpr int PW = sizeof(Piece) / 4, PER = NV / PW;
    for (int u = tid; u < count * PER; u += nthreads) {
        const int e = u / PER, w = u % PER;
        const size_t g = (size_t)first + ((size_t)e << lo);
        const Piece v = *reinterpret_cast<const Piece *>(src + (size_t)TS * g + PW * w);
        *reinterpret_cast<Piece *>(vt + NV * e + PW * w) = v;
    }
}

// Perm table of row j of a per-row table (B_j, 1/B_j or a locator table),
// from global memory only or with the V words from LDS.
template <int R>
__device__ __forceinline__ typename Ops<R>::Tab row_tab(const uint32_t *__restrict__ g, int j)
{
    return Ops<R>::prep(g + (size_t)Traits<R>::TS * fresh((uint32_t)j));
}
template <int R>
__device__ __forceinline__ typename Ops<R>::Tab row_tab(const uint32_t *__restrict__ g, const uint32_t *vt, int j)
{
    const uint32_t jj = fresh((uint32_t)j);
    return Ops<R>::prep_lds(vt + Ops<R>::NV * jj, g + (size_t)Traits<R>::TS * jj);
}
// The same for a table staged at a different position: LDS entry jl, global
// entry jg.
template <int R>
__device__ __forceinline__ typename Ops<R>::Tab row_tab(const uint32_t *__restrict__ g, const uint32_t *vt, int jl,
                                                        uint32_t jg)
{
    const uint32_t jj = fresh((uint32_t)jl);
    return Ops<R>::prep_lds(vt + Ops<R>::NV * jj, g + (size_t)Traits<R>::TS * fresh(jg));
}

// One butterfly; m1 (all ones or zero, wave-uniform) adds the "plus 1" of the
// factor.
template <int R, bool INV>
__device__ __forceinline__ void bfly(uint32_t *a, uint32_t *b, const typename Ops<R>::Tab &T, bool zero,
                                     uint32_t m1)
{
    constexpr int NW = Traits<R>::NW;
    if (!INV) {
        if (!zero)
            Ops<R>::mac(a, b, T);
#pragma unroll
        for (int w = 0; w < NW; w++) {
            a[w] ^= b[w] & m1;
            b[w] ^= a[w];
        }
    } else {
#pragma unroll
        for (int w = 0; w < NW; w++)
            b[w] ^= a[w];
        if (!zero)
            Ops<R>::mac(a, b, T);
#pragma unroll
        for (int w = 0; w < NW; w++)
            a[w] ^= b[w] & m1;
    }
}

// Block k of the butterfly blocks of T levels on 2^T rows, in execution
// order (levels T-1 .. 0 forward, 0 .. T-1 inverse; blocks by first row).
template <int T, bool INV>
constexpr int block_level(int k)
{
    for (int tt = 0; tt < T; tt++) {
        const int t = INV ? tt : T - 1 - tt;
        const int nb = (1 << T) >> (t + 1);
        if (k < nb)
            return t;
        k -= nb;
    }
    return 0;
}
template <int T, bool INV>
constexpr int block_row(int k)
{
    for (int tt = 0; tt < T; tt++) {
        const int t = INV ? tt : T - 1 - tt;
        const int nb = (1 << T) >> (t + 1);
        if (k < nb)
            return k * (2 << t);
        k -= nb;
    }
    return 0;
}

// T levels on 2^T rows in registers; x[j] is global row base + (j << LO),
// where base has no set bit in positions LO .. LO+T-1.  A zero factor only
// occurs at shift 0 for block c = 0; the multiply is skipped there when
// CT_BASE says that base has no bit at or above LO (so that block 0 of the
// group is block 0 of the transform, known at compile time).  Elsewhere a
// zero factor is simply multiplied (its table is all zero), which avoids a
// data-dependent branch around the butterflies.  TW is the factor source;
// the factor of the next block is fetched while a block is computed.
// Pruning (forward only): bit j of `need` (wave-uniform) says that output
// row j is used; a block none of whose rows is used is skipped, its rows
// left undefined.  The default keeps every block at no cost.
template <int R, int T, bool INV, int SH, bool CT_BASE, class TW>
__device__ __forceinline__ void reg_levels(uint32_t (*x)[Traits<R>::NW], uint32_t base, int LO, const TW &tw,
                                           uint64_t need = ~0ull)
{
    typedef typename TW::Tab Tab;
    constexpr int NW = Traits<R>::NW, NB = (1 << T) - 1;
    static_assert(T <= 6, "a 64-bit row mask");
    auto used = [&](int t, int blk) {
        const uint64_t span = (2u << t) >= 64u ? ~0ull : ((1ull << (2u << t)) - 1ull);
        return ((need >> blk) & span) != 0ull;
    };
    auto fetch = [&](int k) -> Tab {
        const int t = block_level<T, INV>(k), blk = block_row<T, INV>(k);
        if (SH == SH_ZERO && CT_BASE && blk == 0)
            return Tab{};
        if (!used(t, blk))
            return Tab{};
        const int i = LO + t;
        const uint32_t c = (base & ~((2u << i) - 1u)) | ((uint32_t)blk << LO);
        return tw.tab(i, c);
    };
    auto work = [&](int k, const Tab &tab) {
        const int t = block_level<T, INV>(k), blk = block_row<T, INV>(k);
        if (!used(t, blk))
            return;
        const bool zero = SH == SH_ZERO && CT_BASE && blk == 0;
        const uint32_t m1 = SH == SH_GENERAL ? tw.plus1(t + LO) : 0u;
#pragma unroll
        for (int m = 0; m < (1 << t); m++) {
            bfly<R, INV>(x[blk + m], x[blk + m + (1 << t)], tab, zero, m1);
            pin<NW>(x[blk + m]);
        }
    };
    if (NB > 0)
        pipelined<Tab, NB>(fetch, work);
}

// x <- s_row * x for a row whose perm table is T.
template <int R>
__device__ __forceinline__ void scale(uint32_t *x, const typename Ops<R>::Tab &T)
{
    constexpr int NW = Traits<R>::NW;
    uint32_t acc[NW];
#pragma unroll
    for (int w = 0; w < NW; w++)
        acc[w] = 0;
    Ops<R>::mac(acc, x, T);
#pragma unroll
    for (int w = 0; w < NW; w++)
        x[w] = acc[w];
    pin<NW>(x);
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

__device__ __forceinline__ const uint8_t *row_ptr(const uint8_t *base, uint32_t t, uint64_t rb)
{
    return base + (uint64_t)t * rb;
}
__device__ __forceinline__ uint8_t *row_ptr(uint8_t *base, uint32_t t, uint64_t rb)
{
    return base + (uint64_t)t * rb;
}

// Decode step 2 (eq. hatF(l)), first half: fetch the received row of point
// p (zeros when the point has none) and copy it to the output when decoding
// out of place.  Returns whether the point was received.
template <int R, int LD>
__device__ __forceinline__ bool dec_fetch(uint32_t *raw, int p, const DevStripe &st, const Lane &ln,
                                          const uint32_t *__restrict__ bits)
{
    const bool rcv = point_bit(bits, p);
    const uint32_t tr = rcv ? (uint32_t)point_row(p, st) : 0u;
    load_chunk<R, LD>(row_ptr(st.in, tr, st.row_bytes), ln.off, ln.act && rcv, ln.nsym, raw);
    if (st.copy_survivors)
        store_chunk<R, LD>(row_ptr(st.out, tr, st.row_bytes), ln.off, ln.act && rcv, ln.nsym, raw);
    return rcv;
}

// Second half: x <- Pi(omega_p) x for a received point (x is zero otherwise).
template <int R>
__device__ __forceinline__ void dec_weigh(uint32_t *x, bool rcv, const typename Ops<R>::Tab &T)
{
    if (rcv)
        scale<R>(x, T);
}

// Decode step 6 (eq. F(j)) for one point: erased stored rows get
// Phi^d[p] / Pi'(omega_p); tabf(p) yields the point's perm table.  UNI:
// the point is the same for the whole wave (else per lane).  NT: stored
// non-temporally (see store_chunk).
template <int R, int LD, bool UNI = true, bool NT = false, class TABF>
__device__ __forceinline__ void dec_store(const uint32_t *v, int p_, const DevStripe &st, const Lane &ln,
                                          const uint32_t *__restrict__ bits, const TABF &tabf)
{
    const int p = UNI ? (int)fresh((uint32_t)p_) : p_;
    if (point_bit(bits + bitmap_words(st.np), p)) {
        const int t = point_row(p, st);
        uint32_t o[Traits<R>::NW];
        zero_vec<R>(o);
        Ops<R>::mac(o, v, tabf(p));
        store_chunk<R, LD, NT>(row_ptr(st.out, (uint32_t)t, st.row_bytes), ln.off, ln.act, ln.nsym, o);
    }
}

}  // namespace nb
