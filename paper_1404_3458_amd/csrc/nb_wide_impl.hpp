// nb_wide_impl.hpp -- passes of up to 8 levels for the codec on transforms over
// h = 2^N > 256 points (GF(2^16) only: GF(2^8) never exceeds 256 points),
// batched over stripes.
//
// The N levels are split into a low part of T1 = ceil(N/2) levels, applied
// to groups of 2^T1 consecutive rows, and a high part of T2 = N - T1 levels,
// applied to groups of 2^T2 rows at stride 2^T1 (Sec. 3.2 / 3.3: level i
// pairs rows j and j + 2^i, so a group holding every row that differs in
// bits lo .. lo+T-1 can apply those levels alone).  Inside a workgroup a
// group of 2^T rows is handled like a whole small transform of the fused
// kernels: 16-row register groups, an LDS transpose, the other levels on
// stride-16 register groups, with the factors' vector words staged in LDS.
//
// Pass kinds (one launch each, over every stripe of the call with this N):
//   encode (Algorithm 1; coefficients A, k' rows):
//     W_E1   low levels of the inverse transform of the zero-padded message
//     W_E2   high levels of that inverse, then the high levels of the forward
//            transform of parity block 1 (shift k'); the coefficients are also
//            kept when later blocks need them
//     W_E2F  high levels of the forward transform of block blk >= 2
//     W_E3   low levels of block blk's forward transform; parity rows written
//   decode (Algorithm 2; n' rows):
//     W_D1   step 2 (received rows times Pi) and low inverse levels
//     W_D2   high inverse levels, d^d = B (.) coefficients (Sec. 4.2), and the
//            derivative's partial sums over the high bits
//     W_D3   the partial sums over the low bits, plus those of the other
//            passes, over B_j
//     W_DPM  (pipelines of three or four parts) the partial sums over the bits
//            of a middle part, added to those of W_D2
// Pipelines of more than two parts run the middle parts' inverse levels as
// W_E1 passes and their forward levels as W_E2F (encode) or W_D4 (decode)
// passes, in place on the same buffers.
//     W_D4   high forward levels
//     W_D5   low forward levels and step 6 (erased rows over Pi')
//   decode of a two-part pipeline, three passes (W_D1, W_DH, W_DL):
//     The derivative of Sec. 4.2 is Binv (.) S (.) B with S the sum over the
//     bits l of the shifts j <- j + 2^l.  B_j is the product of W'_l over the
//     set bits of j, so it factors into a low-bit and a high-bit part, S is
//     the sum of a low-bit and a high-bit part, and the derivative splits
//     into D_lo + D_hi, each acting on one part of the row index only.  The
//     high levels of both transforms act on the high index alone (their
//     factors depend only on the high bits), so
//       Psi[D Psi^-1[Phi]] = Psi_lo[ Psi_hi D_hi Psi_hi^-1 A + D_lo A ],
//     where A = Psi_lo^-1[Phi] is what W_D1 writes and Psi_lo, Psi_lo^-1 are
//     the low levels (per high index, at that index's shift).
//     W_DH   high inverse levels, D_hi, high forward levels: U
//     W_DL   U + D_lo A, low forward levels and step 6
//   plain transforms (nb_fft / nb_ifft / nb_polymul over h > 256 points at a
//   shift l whose bits below h are clear; two parts):
//     W_PI   one part of the inverse transform at shift l
//     W_PF   one part of the forward transform at shift l; rows >= dst_rows
//            are not written
//     W_PFM  the same, each output row first multiplied symbol by symbol by
//            the same row of src2 (the product of Sec. 6.1)
// Every pass reads and writes its rows once, non-temporally: the rows
// streaming through an XCD's L2 would otherwise evict the factor and
// locator tables each workgroup re-reads.
#pragma once
#include "nb_xform.hpp"

namespace nb {

enum WideKind {
    W_E1 = 0, W_E2 = 1, W_E2F = 2, W_E3 = 3, W_D1 = 4, W_D2 = 5, W_D3 = 6, W_D4 = 7, W_D5 = 8, W_DPM = 9,
    W_DH = 10, W_DL = 11, W_PI = 12, W_PF = 13, W_PFM = 14
};

__device__ __forceinline__ int find_wide(const WideStripe *__restrict__ st, int n, int tile)
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

__device__ __forceinline__ const uint8_t *wrow(const uint8_t *b, uint32_t t, uint64_t rb) { return b + (uint64_t)t * rb; }
__device__ __forceinline__ uint8_t *wrow(uint8_t *b, uint32_t t, uint64_t rb) { return b + (uint64_t)t * rb; }

// Groups of up to 2^WREG rows are held whole in the registers of one wave
// (no LDS exchange, no barrier); larger ones are exchanged through an LDS
// tile between 16-row register groups and stride-16 groups.  (One-wave
// groups of 32 rows were measured slower than the tiled ones: they need up
// to 190 registers, leaving two or three waves per SIMD.)
constexpr int WREG = 4;

// Rows of at most 128 symbols fill only half of a wave (32 lanes of 4
// columns).  For them a tiled pass can run "packed": a workgroup of half the
// waves, each wave's two halves holding the rows of two of the original
// waves (virtual wave 2 w + half).  The halves then multiply by different
// constants, so every table is staged whole in LDS and read per lane
// (Tab16V) instead of V words from LDS plus S words from scalar loads.
// Packed passes exist for the kinds of the two-part pipelines.
__host__ __device__ constexpr bool packable(int T, int kind)
{
    return T > WREG && (kind == W_E1 || kind == W_E2 || kind == W_E3 || kind == W_D1 || kind == W_DH || kind == W_DL);
}

// Table access of a pass: uniform tables (V words staged in LDS, S words read
// with scalar loads), or per-lane tables staged whole (packed passes).
template <bool PK> struct WTab;
template <> struct WTab<false> {
    typedef Tab16 Tab;
    static constexpr int WPE = VW16;                // staged words per table
    template <int T> using Tw = TwLds<16, T>;
    __device__ static __forceinline__ Tab row(const uint32_t *__restrict__ g, const uint32_t *vt, int jl, uint32_t jg)
    {
        return row_tab<16>(g, vt, jl, jg);
    }
    template <int T>
    __device__ static __forceinline__ Tw<T> tw(const uint32_t *p_tw, uint32_t l, const uint32_t *vt, uint32_t lo,
                                               uint32_t gbase)
    {
        return {p_tw, l, vt, lo, gbase};
    }
    __device__ static __forceinline__ uint32_t uni(uint32_t v) { return fresh(v); }
};
template <> struct WTab<true> {
    typedef Tab16V Tab;
    static constexpr int WPE = TAB16;
    template <int T> using Tw = TwLdsV<T>;
    __device__ static __forceinline__ Tab row(const uint32_t *__restrict__, const uint32_t *vt, int jl, uint32_t)
    {
        return tab_lds_all(vt + TAB16 * jl);
    }
    template <int T>
    __device__ static __forceinline__ Tw<T> tw(const uint32_t *, uint32_t l, const uint32_t *vt, uint32_t lo, uint32_t)
    {
        return {l, vt, lo};
    }
    __device__ static __forceinline__ uint32_t uni(uint32_t v) { return v; }   // per lane: no broadcast
};

// LDS of a pass: the group tile, then the staged words of the factor tables
// (a second set for W_E2's forward part) and of the per-point tables.
// Half-tile exchange: plain passes on groups of 32 to 128 rows hold a tile
// of one word per row and lane and move the two words of each row in two
// rounds, which halves the tile and lets more workgroups share a CU (the
// partial-sum passes of longer pipelines keep the whole tile).
__host__ __device__ constexpr bool half_tile(int T, int kind, bool pk)
{
    return !pk && T >= 5 && T <= 7 && kind != W_D2 && kind != W_D3 && kind != W_DPM;
}

template <int T, int KIND, bool PK = false>
struct WideLds {
    static constexpr int R = 16, H = 1 << T, NV = WTab<PK>::WPE, NW = Traits<R>::NW;
    static constexpr bool HALF = half_tile(T, KIND, PK);
    static constexpr int TILE = T > WREG ? H * (PK ? 32 : 64) * (HALF ? 1 : NW) : 0;
    static constexpr int EX = (KIND == W_D3 || KIND == W_DPM) ? 0 : H - 1;
    static constexpr int EX2 = KIND == W_E2 ? H - 1 : 0;
    static constexpr int EB = (KIND == W_D2 || KIND == W_D3) ? H : (KIND == W_DH || KIND == W_DL) ? 2 * H : 0;
    static constexpr int ERT = (KIND == W_D1 || KIND == W_D5 || KIND == W_DL) ? H : 0;
    static constexpr size_t BYTES = 4 * ((size_t)TILE + (size_t)NV * (EX + EX2 + EB + ERT));
    static_assert(BYTES <= 160 * 1024, "pass tile and tables exceed the LDS of a workgroup");
};

#define NB_WIDE_THREADS(T) ((T) > WREG ? (64 << ((T) - 4)) : 64)
#define NB_WIDE_THREADS_PK(T, PK) (NB_WIDE_THREADS(T) >> ((PK) ? 1 : 0))

// W_DH and W_DL on one group of 2^T rows (the rows gbase + (p << lo)):
// x holds a wave's consecutive rows (16 g + j, or all rows when the group is
// not tiled), y its stride groups (rows r0 + 16 j); cb / my are the wave's and
// the lane's views of the LDS tile.  The part's derivative factors are
// B_(p << lo) and its inverse (staged at vb / vbi), local index p.  PK: a
// packed pass (wave and g are then per-lane virtual wave indices).
template <int T, int KIND, int LD, bool PK, bool HALF, class TW, class STAGE>
__device__ __forceinline__ void split_decode_pass(uint32_t (*x)[2], uint32_t (*y)[T > WREG ? (1 << (T - 4)) : 1][2],
                                                  const WideStripe &ws, const DevStripe &st, const Lane &ln,
                                                  uint32_t gbase, uint32_t lo, int wave, int g, uint32_t *cb,
                                                  uint32_t *my, const uint32_t *__restrict__ bits,
                                                  const uint32_t *__restrict__ rowtab,
                                                  const uint32_t *__restrict__ p_B,
                                                  const uint32_t *__restrict__ p_Binv, const uint32_t *vb,
                                                  const uint32_t *vbi, const uint32_t *vrt, const TW &tw,
                                                  const STAGE &stage_tables)
{
    constexpr int R = 16, NW = 2, H = 1 << T;
    typedef WTab<PK> WT;
    typedef typename WT::Tab Tab;
    constexpr bool TILED = T > WREG;
    static_assert(TILED || !PK, "packed passes are tiled");
    constexpr int L2 = TILED ? T - 4 : 0, NR2 = 1 << L2, GPW = TILED ? 16 >> L2 : 1;
    // tile row stride in words (HALF: one word per lane, cb / my then point
    // at that layout)
    constexpr int RS = HALF ? 64 : (PK ? 32 : 64) * NW;
    const uint64_t rb = st.row_bytes;
    auto grow = [&](int p) -> uint32_t { return gbase + ((uint32_t)p << lo); };
    auto lds_put = [&](uint32_t *base, int rows, const uint32_t *v) {
        *reinterpret_cast<uint2 *>(base + RS * rows) = make_uint2(v[0], v[1]);
    };
    auto lds_get = [&](const uint32_t *base, int rows, uint32_t *v) {
        const uint2 t = *reinterpret_cast<const uint2 *>(base + RS * rows);
        v[0] = t.x;
        v[1] = t.y;
    };
    auto xorv = [&](uint32_t *a, const uint32_t *b) {
        a[0] ^= b[0];
        a[1] ^= b[1];
    };

    if constexpr (!TILED) {
        // the whole group in one wave's registers
        uint32_t a[H][NW];
#pragma unroll
        for (int j = 0; j < H; j++) {
            load_chunk<R, LD, true>(wrow(ws.src, grow(j), rb), ln.off, ln.act, ln.nsym, x[j]);
            if (KIND == W_DL)
                load_chunk<R, LD, true>(wrow(ws.src2, grow(j), rb), ln.off, ln.act, ln.nsym, a[j]);
        }
        stage_tables();
        uint32_t (*d)[NW] = KIND == W_DH ? x : a;
        if (KIND == W_DH)
            reg_levels<R, T, true, SH_ZERO, false>(x, 0u, 0, tw);
        // d = B (.) rows, then in place, rows in ascending order: the sum of
        // d over the rows p + 2^l with bit l of p clear, over B_p
        pipelined<Tab, H>([&](int j) { return WT::row(p_B, vb, j, (uint32_t)j << lo); },
                          [&](int j, const Tab &t) {
                              if (j)
                                  scale<R>(d[j], t);
                          });
#pragma unroll
        for (int j = 0; j < H; j++) {
            uint32_t z[NW] = {0u, 0u};
#pragma unroll
            for (int l = 0; l < T; l++)
                if (!((j >> l) & 1))
                    xorv(z, d[j + (1 << l)]);
            d[j][0] = z[0];
            d[j][1] = z[1];
        }
        pipelined<Tab, H>([&](int j) { return WT::row(p_Binv, vbi, j, (uint32_t)j << lo); },
                          [&](int j, const Tab &t) {
                              if (j && j + 1 < H)
                                  scale<R>(d[j], t);
                              if (KIND == W_DL)
                                  xorv(x[j], d[j]);
                          });
        reg_levels<R, T, false, SH_ZERO, false>(x, 0u, 0, tw);
        if (KIND == W_DH) {
#pragma unroll
            for (int j = 0; j < H; j++)
                store_chunk<R, LD, true>(wrow(ws.dst, WT::uni(grow(j)), rb), ln.off, ln.act, ln.nsym, x[j]);
        } else {
            pipelined<Tab, H>([&](int j) { return WT::row(rowtab, vrt, j, grow(j)); },
                              [&](int j, const Tab &t) {
                                  dec_store<R, LD>(x[j], (int)grow(j), st, ln, bits, [&](int) { return t; });
                              });
        }
    } else {
        // stride layout for the derivative: the partners 16 * 2^l away are in
        // a wave's registers, those 2^l away (l < 4) in other waves' rows of
        // the LDS tile
        uint32_t a[GPW][NR2][NW];                    // W_DL: the rows of A; W_DH: unused
        uint32_t (*d)[NR2][NW] = KIND == W_DH ? y : a;
        if (KIND == W_DH) {
#pragma unroll
            for (int j = 0; j < 16; j++)
                load_chunk<R, LD, true>(wrow(ws.src, grow(16 * g + j), rb), ln.off, ln.act, ln.nsym, x[j]);
            stage_tables();
            reg_levels<R, 4, true, SH_ZERO, false>(x, (uint32_t)(16 * g), 0, tw);
            if constexpr (HALF) {
#pragma unroll
                for (int w = 0; w < NW; w++) {
                    if (w)
                        __syncthreads();
#pragma unroll
                    for (int j = 0; j < 16; j++)
                        cb[RS * j] = x[j][w];
                    __syncthreads();
#pragma unroll
                    for (int u = 0; u < GPW; u++)
#pragma unroll
                        for (int j = 0; j < NR2; j++)
                            y[u][j][w] = my[RS * (wave * GPW + u + 16 * j)];
                }
            } else {
#pragma unroll
                for (int j = 0; j < 16; j++)
                    lds_put(cb, j, x[j]);
                __syncthreads();
#pragma unroll
                for (int u = 0; u < GPW; u++)
#pragma unroll
                    for (int j = 0; j < NR2; j++)
                        lds_get(my + RS * (wave * GPW + u), 16 * j, y[u][j]);
            }
#pragma unroll
            for (int u = 0; u < GPW; u++)
                reg_levels<R, L2, true, SH_ZERO, false>(y[u], (uint32_t)(wave * GPW + u), 4, tw);
        } else {
#pragma unroll
            for (int u = 0; u < GPW; u++) {
                const int r0 = wave * GPW + u;
#pragma unroll
                for (int j = 0; j < NR2; j++) {
                    load_chunk<R, LD, true>(wrow(ws.src, grow(r0 + 16 * j), rb), ln.off, ln.act, ln.nsym, y[u][j]);
                    load_chunk<R, LD, true>(wrow(ws.src2, grow(r0 + 16 * j), rb), ln.off, ln.act, ln.nsym, a[u][j]);
                }
            }
            stage_tables();
        }
        // d = B (.) rows; each wave rewrites only its own tile rows, which it
        // alone has read, so no barrier is needed before the writes
#pragma unroll
        for (int u = 0; u < GPW; u++) {
            const int r0 = wave * GPW + u;
            pipelined<Tab, NR2>([&](int j) { return WT::row(p_B, vb, r0 + 16 * j, (uint32_t)(r0 + 16 * j) << lo); },
                                [&](int j, const Tab &t) {
                                    if (r0 + 16 * j)
                                        scale<R>(d[u][j], t);
                                    if constexpr (!HALF)
                                        lds_put(my + RS * r0, 16 * j, d[u][j]);
                                });
        }
        // the sums over the rows p + 2^l with bit l of p clear: partners
        // 16 * 2^l away in registers, 2^l away (l < 4) in other waves' tile
        // rows; in place, j ascending: row j's sum reads only rows above it
        if constexpr (HALF) {
#pragma unroll
            for (int w = 0; w < NW; w++) {
                if (w)
                    __syncthreads();
#pragma unroll
                for (int u = 0; u < GPW; u++)
#pragma unroll
                    for (int j = 0; j < NR2; j++)
                        my[RS * (wave * GPW + u + 16 * j)] = d[u][j][w];
                __syncthreads();
#pragma unroll
                for (int u = 0; u < GPW; u++) {
                    const int r0 = wave * GPW + u;
#pragma unroll
                    for (int j = 0; j < NR2; j++) {
                        uint32_t z = 0u;
#pragma unroll
                        for (int l = 0; l < L2; l++)
                            if (!((j >> l) & 1))
                                z ^= d[u][j + (1 << l)][w];
#pragma unroll
                        for (int l = 0; l < 4; l++)
                            if (!((r0 >> l) & 1))
                                z ^= my[RS * (r0 + (1 << l) + 16 * j)];
                        d[u][j][w] = z;
                    }
                }
            }
        } else {
            __syncthreads();
#pragma unroll
            for (int u = 0; u < GPW; u++) {
                const int r0 = wave * GPW + u;
#pragma unroll
                for (int j = 0; j < NR2; j++) {
                    uint32_t z[NW] = {0u, 0u};
#pragma unroll
                    for (int l = 0; l < L2; l++)
                        if (!((j >> l) & 1))
                            xorv(z, d[u][j + (1 << l)]);
#pragma unroll
                    for (int l = 0; l < 4; l++) {
                        if (!((r0 >> l) & 1)) {
                            uint32_t v[NW];
                            lds_get(my + RS * r0, (1 << l) + 16 * j, v);
                            xorv(z, v);
                        }
                    }
                    d[u][j][0] = z[0];
                    d[u][j][1] = z[1];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < GPW; u++) {
            const int r0 = wave * GPW + u;
            pipelined<Tab, NR2>([&](int j) { return WT::row(p_Binv, vbi, r0 + 16 * j,
                                                               (uint32_t)(r0 + 16 * j) << lo); },
                                [&](int j, const Tab &t) {
                                    if (r0 + 16 * j && r0 + 16 * j + 1 < H)
                                        scale<R>(d[u][j], t);
                                    if (KIND == W_DL)
                                        xorv(y[u][j], d[u][j]);
                                });
            reg_levels<R, L2, false, SH_ZERO, false>(y[u], (uint32_t)r0, 4, tw);
        }
        __syncthreads();                             // every partner read is done
        if constexpr (HALF) {
#pragma unroll
            for (int w = 0; w < NW; w++) {
                if (w)
                    __syncthreads();
#pragma unroll
                for (int u = 0; u < GPW; u++)
#pragma unroll
                    for (int j = 0; j < NR2; j++)
                        my[RS * (wave * GPW + u + 16 * j)] = y[u][j][w];
                __syncthreads();
#pragma unroll
                for (int j = 0; j < 16; j++)
                    x[j][w] = cb[RS * j];
            }
        } else {
#pragma unroll
            for (int u = 0; u < GPW; u++)
#pragma unroll
                for (int j = 0; j < NR2; j++)
                    lds_put(my + RS * (wave * GPW + u), 16 * j, y[u][j]);
            __syncthreads();
        }
        if (KIND == W_DL) {
            // only the 16 consecutive rows that hold an erased stored point
            // need the last levels
            const uint32_t *__restrict__ sbm = bits + bitmap_words(st.np);
            const uint32_t p0 = grow(16 * g);
            const uint32_t need = (sbm[p0 >> 5] >> (p0 & 31)) & 0xFFFFu;
            if (PK ? !__builtin_amdgcn_ballot_w64(need != 0u) : !fresh(need))
                return;
        }
        if constexpr (!HALF) {
#pragma unroll
            for (int j = 0; j < 16; j++)
                lds_get(cb, j, x[j]);
        }
        reg_levels<R, 4, false, SH_ZERO, false>(x, (uint32_t)(16 * g), 0, tw);
        if (KIND == W_DH) {
#pragma unroll
            for (int j = 0; j < 16; j++)
                store_chunk<R, LD, true>(wrow(ws.dst, WT::uni(grow(16 * g + j)), rb), ln.off, ln.act, ln.nsym, x[j]);
        } else {
            pipelined<Tab, 16>([&](int j) { return WT::row(rowtab, vrt, 16 * g + j, grow(16 * g + j)); },
                               [&](int j, const Tab &t) {
                                   dec_store<R, LD, !PK>(x[j], (int)grow(16 * g + j), st, ln, bits,
                                                         [&](int) { return t; });
                               });
        }
    }
}

// Waves per SIMD the register allocation aims at: packed passes two (one
// workgroup per CU holds their whole group), half-tile passes five (except
// the two kinds that would spill there), others four.
__host__ __device__ constexpr int wide_waves(int T, int kind, bool pk)
{
    return pk ? 2 : (half_tile(T, kind, pk) && kind != W_E2 && kind != W_DL) ? 5 : 4;
}

template <int T, int KIND, int LD, bool PK>
__global__ __launch_bounds__(NB_WIDE_THREADS_PK(T, PK)) __attribute__((amdgpu_waves_per_eu(wide_waves(T, KIND, PK))))
void k_wide(
    WideArgs a, const uint32_t *__restrict__ p_tw, const uint32_t *__restrict__ p_B,
    const uint32_t *__restrict__ p_Binv, const uint32_t *__restrict__ p_bits, const uint32_t *__restrict__ p_rowtabs)
{
    constexpr int R = 16;
    typedef WideLds<T, KIND, PK> LY;
    typedef WTab<PK> WT;
    typedef typename WT::Tab Tab;
    static_assert(!PK || packable(T, KIND), "no packed variant of this pass");
    constexpr int NW = Traits<R>::NW, NV = WT::WPE, H = 1 << T;
    constexpr bool TILED = T > WREG;               // LDS exchange between two register groupings
    constexpr int TA = TILED ? 4 : T;              // levels of the consecutive (register) phase
    constexpr int L2 = TILED ? T - 4 : 0;          // levels of the stride phase
    constexpr int NR2 = 1 << L2;
    constexpr int GPW = TILED ? 16 >> L2 : 1;
    constexpr int NT = NB_WIDE_THREADS_PK(T, PK);
    constexpr int NX = 1 << TA;                    // rows of a consecutive register group
    constexpr bool INV_FIRST = KIND == W_E1 || KIND == W_E2 || KIND == W_D1 || KIND == W_D2 || KIND == W_PI;
    constexpr bool PSUM = KIND == W_D3 || KIND == W_DPM;     // partial sums of the derivative
    constexpr bool FWD = KIND == W_E2 || KIND == W_E2F || KIND == W_E3 || KIND == W_D4 || KIND == W_D5 ||
                         KIND == W_PF || KIND == W_PFM;
    constexpr int SHF = (KIND == W_D4 || KIND == W_D5) ? SH_ZERO : SH_ALIGNED;   // forward-part shift

    extern __shared__ uint32_t lds[];
    uint32_t *const vX = lds + LY::TILE;
    uint32_t *const vX2 = vX + NV * LY::EX;
    uint32_t *const vB = vX2 + NV * LY::EX2;
    uint32_t *const vRT = vB + NV * LY::EB;

    const int tid = (int)threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int vw = PK ? 2 * wave + (lane >> 5) : wave;     // (virtual) wave of this lane's rows
    const int tile = blockIdx.x;
    const int s = find_wide(a.stripes, a.nstripes, tile);
    const WideStripe ws = a.stripes[s];
    const DevStripe &st = ws.st;
    const DoneStamp done = {a.ts};
    const int rel = tile - ws.tile0;
    const uint32_t gi = (uint32_t)(rel / ws.nct);
    const int ct = rel % ws.nct;
    const uint32_t lo = (uint32_t)a.lo;
    const uint32_t gbase = (gi & ((1u << lo) - 1u)) | ((gi >> lo) << (lo + T));
    const Lane ln = PK ? lane_of<R, LD>(0, 32 * ct + (lane & 31), st.col0, st.ncols)
                       : lane_of<R, LD>(ct, lane, st.col0, st.ncols);
    const uint64_t rb = st.row_bytes;
    const uint32_t *__restrict__ bits = p_bits + st.bits_off;
    const uint32_t *__restrict__ rowtab = p_rowtabs + st.rowtab_off;
    auto grow = [&](int p) -> uint32_t { return gbase + ((uint32_t)p << lo); };

    // Pruning: a consecutive group none of whose rows is written has nothing
    // to compute in the last pass (decode: no erased stored point, encode:
    // rows past the stored parity).  The test is workgroup-uniform.
    if (KIND == W_D5 || KIND == W_DL) {
        const uint32_t *__restrict__ sbm = bits + bitmap_words(st.np);
        uint32_t any = 0;
        for (uint32_t w = gbase >> 5; w <= (gbase + H - 1) >> 5; w++)
            any |= sbm[w];
        if (H < 32)
            any = (any >> (gbase & 31)) & ((1u << (H & 31)) - 1u);
        if (!fresh(any))
            return;
    }
    if (KIND == W_E3 && (int)gbase >= ws.dst_rows)
        return;

    // the inverse part runs at shift 0; the forward part at shift blk * k'
    // (encode) or 0 (decode)
    const uint32_t lf = (KIND == W_E2) ? (uint32_t)st.kp
                      : (KIND == W_E2F || KIND == W_E3) ? (uint32_t)a.blk * (uint32_t)st.kp
                      : (KIND == W_PF || KIND == W_PFM) ? a.l : 0u;
    const uint32_t li = KIND == W_PI ? a.l : 0u;   // the inverse part's shift
    const auto twI = WT::template tw<T>(p_tw, li, vX, lo, gbase);
    const auto twF = WT::template tw<T>(p_tw, lf, KIND == W_E2 ? vX2 : vX, lo, gbase);

    constexpr bool HALF = LY::HALF;                // tile of one word per row and lane
    constexpr int RS = HALF ? 64 : (PK ? 32 : 64) * NW;       // tile row stride in words
    uint32_t *const my = lds + (PK ? (lane & 31) : lane) * (HALF ? 1 : NW);
    auto lds_put = [&](uint32_t *base, int rows, const uint32_t *v) {
        uint32_t *p = base + RS * rows;
        *reinterpret_cast<uint2 *>(p) = make_uint2(v[0], v[1]);
    };
    auto lds_get = [&](const uint32_t *base, int rows, uint32_t *v) {
        const uint2 t = *reinterpret_cast<const uint2 *>(base + RS * rows);
        v[0] = t.x;
        v[1] = t.y;
    };
    auto stage_tables = [&]() {
        if (LY::EX)
            stage_levels<R, T, NV>(vX, p_tw, INV_FIRST ? li : lf, tid, NT, lo, gbase);
        if (LY::EX2)
            stage_levels<R, T, NV>(vX2, p_tw, lf, tid, NT, lo, gbase);
        if (KIND == W_D2)
            stage_rows<R, NV>(vB, p_B, H, tid, NT, lo, gbase);
        if (KIND == W_D3)
            stage_rows<R, NV>(vB, p_Binv, H, tid, NT, lo, gbase);
        if (KIND == W_DH || KIND == W_DL) {          // the part's own factors: entries j << lo
            stage_rows<R, NV>(vB, p_B, H, tid, NT, lo, 0u);
            stage_rows<R, NV>(vB + NV * H, p_Binv, H, tid, NT, lo, 0u);
        }
        if (LY::ERT)
            stage_rows<R, NV>(vRT, rowtab, H, tid, NT, lo, gbase);
        __syncthreads();
    };

    const int g = vw;                               // consecutive register group of this wave
    uint32_t *const cb = my + RS * 16 * g;
    uint32_t x[NX][NW];                             // consecutive-phase registers (local rows NX g + j)
    uint32_t y[GPW][NR2][NW];                       // stride-phase registers (local rows r0 + 16 j)
    auto xrow = [&](int j) { return NX * g + j; };
    // The two register groupings through the LDS tile: consecutive rows x
    // to stride groups y, and back (each wave first writes the tile rows it
    // alone has read, so no barrier is needed before the first writes).
    auto to_stride = [&]() {
        if constexpr (HALF) {
#pragma unroll
            for (int w = 0; w < NW; w++) {
                if (w)
                    __syncthreads();
#pragma unroll
                for (int j = 0; j < 16; j++)
                    cb[RS * j] = x[j][w];
                __syncthreads();
#pragma unroll
                for (int u = 0; u < GPW; u++)
#pragma unroll
                    for (int j = 0; j < NR2; j++)
                        y[u][j][w] = my[RS * (vw * GPW + u + 16 * j)];
            }
        } else {
#pragma unroll
            for (int j = 0; j < 16; j++)
                lds_put(cb, j, x[j]);
            __syncthreads();
#pragma unroll
            for (int u = 0; u < GPW; u++)
#pragma unroll
                for (int j = 0; j < NR2; j++)
                    lds_get(my + RS * (vw * GPW + u), 16 * j, y[u][j]);
        }
    };
    auto to_consecutive = [&]() {
        if constexpr (HALF) {
#pragma unroll
            for (int w = 0; w < NW; w++) {
                if (w)
                    __syncthreads();
#pragma unroll
                for (int u = 0; u < GPW; u++)
#pragma unroll
                    for (int j = 0; j < NR2; j++)
                        my[RS * (vw * GPW + u + 16 * j)] = y[u][j][w];
                __syncthreads();
#pragma unroll
                for (int j = 0; j < 16; j++)
                    x[j][w] = cb[RS * j];
            }
        } else {
#pragma unroll
            for (int u = 0; u < GPW; u++)
#pragma unroll
                for (int j = 0; j < NR2; j++)
                    lds_put(my + RS * (vw * GPW + u), 16 * j, y[u][j]);
            __syncthreads();
#pragma unroll
            for (int j = 0; j < 16; j++)
                lds_get(cb, j, x[j]);
        }
    };

    // Rows of the data once it sits in stride registers (TILED) or in x.
    auto store_data = [&](uint8_t *d) {
        if constexpr (TILED) {
#pragma unroll
            for (int u = 0; u < GPW; u++)
#pragma unroll
                for (int j = 0; j < NR2; j++)
                    store_chunk<R, LD, true>(wrow(d, WT::uni(grow(vw * GPW + u + 16 * j)), rb), ln.off, ln.act, ln.nsym,
                                       y[u][j]);
        } else {
#pragma unroll
            for (int j = 0; j < NX; j++)
                store_chunk<R, LD, true>(wrow(d, WT::uni(grow(j)), rb), ln.off, ln.act, ln.nsym, x[j]);
        }
    };

    if constexpr (KIND == W_DH || KIND == W_DL) {
        split_decode_pass<T, KIND, LD, PK, HALF>(x, y, ws, st, ln, gbase, lo, vw, g, cb, my, bits, rowtab, p_B, p_Binv,
                                            vB, vB + NV * H, vRT, twI, stage_tables);
        return;
    }

    // ------------------------------------------------ input
    bool rcv[NX];
    if (INV_FIRST || PSUM || !TILED) {
#pragma unroll
        for (int j = 0; j < NX; j++) {
            const uint32_t p = grow(xrow(j));
            if (KIND == W_D1)
                rcv[j] = dec_fetch<R, LD>(x[j], (int)p, st, ln, bits);
            else
                load_chunk<R, LD, true>(wrow(ws.src, p, rb), ln.off, ln.act && (int)p < ws.src_rows, ln.nsym, x[j]);
        }
    } else {
        if constexpr (TILED) {
#pragma unroll
            for (int u = 0; u < GPW; u++)
#pragma unroll
                for (int j = 0; j < NR2; j++) {
                    const uint32_t p = grow(vw * GPW + u + 16 * j);
                    load_chunk<R, LD, true>(wrow(ws.src, p, rb), ln.off, ln.act && (int)p < ws.src_rows, ln.nsym, y[u][j]);
                }
        }
    }
    stage_tables();

    if (PSUM && !TILED) {
        // z_p = partial sums of W_D2 + sum over clear local bits l of p of
        // y_{p + 2^l}; the coefficient is z_p / B_p (Sec. 4.2).  Rows in
        // chunks of 16, so that the partial sums need no second copy of the
        // group in registers.
#pragma unroll
        for (int c = 0; c < NX; c += 16) {
            constexpr int NC = NX < 16 ? NX : 16;
            uint32_t z[NC][NW];
#pragma unroll
            for (int j = 0; j < NC; j++)
                load_chunk<R, LD, true>(wrow(ws.src2, grow(c + j), rb), ln.off, ln.act, ln.nsym, z[j]);
#pragma unroll
            for (int j = 0; j < NC; j++)
#pragma unroll
                for (int lv = 0; lv < TA; lv++)
                    if (!(((c + j) >> lv) & 1))
#pragma unroll
                        for (int w = 0; w < NW; w++)
                            z[j][w] ^= x[c + j + (1 << lv)][w];
            if (KIND == W_DPM) {
#pragma unroll
                for (int j = 0; j < NC; j++)
                    store_chunk<R, LD, true>(wrow(ws.dst, WT::uni(grow(c + j)), rb), ln.off, ln.act, ln.nsym, z[j]);
            } else {
                pipelined<Tab, NC>([&](int j) { return WT::row(p_Binv, vB, c + j, grow(c + j)); },
                                   [&](int j, const Tab &t) {
                                       const uint32_t p = grow(c + j);
                                       if (p)
                                           scale<R>(z[j], t);
                                       store_chunk<R, LD, true>(wrow(ws.dst, WT::uni(p), rb), ln.off, ln.act, ln.nsym, z[j]);
                                   });
            }
        }
        return;
    }
    if (PSUM) {
        // as above, for a tiled group: the partners 2^l away with l < 4 are
        // in this wave's registers, the others in the LDS tile
        uint32_t z[NX][NW];
#pragma unroll
        for (int j = 0; j < NX; j++)
            load_chunk<R, LD, true>(wrow(ws.src2, grow(xrow(j)), rb), ln.off, ln.act, ln.nsym, z[j]);
#pragma unroll
        for (int j = 0; j < NX; j++)
#pragma unroll
            for (int lv = 0; lv < TA; lv++)
                if (!((j >> lv) & 1))
#pragma unroll
                    for (int w = 0; w < NW; w++)
                        z[j][w] ^= x[j + (1 << lv)][w];
        if constexpr (TILED) {
#pragma unroll
            for (int j = 0; j < 16; j++)
                lds_put(cb, j, x[j]);
            __syncthreads();
#pragma unroll
            for (int lv = 0; lv < L2; lv++) {
                if (!((g >> lv) & 1)) {
#pragma unroll
                    for (int j = 0; j < 16; j++) {
                        uint32_t v[NW];
                        lds_get(cb, 16 * (1 << lv) + j, v);
#pragma unroll
                        for (int w = 0; w < NW; w++)
                            z[j][w] ^= v[w];
                    }
                }
            }
        }
        if (KIND == W_DPM) {
#pragma unroll
            for (int j = 0; j < NX; j++)
                store_chunk<R, LD, true>(wrow(ws.dst, WT::uni(grow(xrow(j))), rb), ln.off, ln.act, ln.nsym, z[j]);
        } else {
            pipelined<Tab, NX>([&](int j) { return WT::row(p_Binv, vB, xrow(j), grow(xrow(j))); },
                               [&](int j, const Tab &t) {
                                   const uint32_t p = grow(xrow(j));
                                   if (p)
                                       scale<R>(z[j], t);
                                   store_chunk<R, LD, true>(wrow(ws.dst, WT::uni(p), rb), ln.off, ln.act, ln.nsym, z[j]);
                               });
        }
        return;
    }

    if (INV_FIRST) {
        if (KIND == W_D1)
            pipelined<Tab, NX>([&](int j) { return WT::row(rowtab, vRT, xrow(j), grow(xrow(j))); },
                               [&](int j, const Tab &t) { dec_weigh<R>(x[j], rcv[j], t); });
        reg_levels<R, TA, true, SH_ZERO, false>(x, (uint32_t)(NX * g), 0, twI);
        if constexpr (TILED) {
            to_stride();
#pragma unroll
            for (int u = 0; u < GPW; u++)
                reg_levels<R, L2, true, SH_ZERO, false>(y[u], (uint32_t)(vw * GPW + u), 4, twI);
        }
        if (KIND == W_E1 || KIND == W_D1 || KIND == W_PI) {
            store_data(ws.dst);
            return;
        }
        if (KIND == W_E2 && ws.dst2)                // coefficients read again by later blocks
            store_data(ws.dst2);
        if (KIND == W_D2) {
            // d^d = B (.) coefficients, stored; then each point's partial sum
            // over the clear local bits (the transform's high bits).  Each
            // wave rewrites only the tile rows it read itself, so no barrier
            // is needed before the exchange.
            if constexpr (TILED) {
#pragma unroll
                for (int u = 0; u < GPW; u++) {
                    const int r0 = vw * GPW + u;
                    pipelined<Tab, NR2>([&](int j) { return WT::row(p_B, vB, r0 + 16 * j, grow(r0 + 16 * j)); },
                                        [&](int j, const Tab &t) {
                                            if (grow(r0 + 16 * j))
                                                scale<R>(y[u][j], t);
                                            lds_put(my + RS * r0, 16 * j, y[u][j]);
                                        });
                }
                store_data(ws.dst);
                __syncthreads();
#pragma unroll
                for (int u = 0; u < GPW; u++) {
                    const int r0 = vw * GPW + u;
#pragma unroll
                    for (int j = 0; j < NR2; j++) {
                        uint32_t z[NW];
                        zero_vec<R>(z);
#pragma unroll
                        for (int lv = 0; lv < L2; lv++)          // local partners 16 * 2^lv away
                            if (!((j >> lv) & 1))
#pragma unroll
                                for (int w = 0; w < NW; w++)
                                    z[w] ^= y[u][j + (1 << lv)][w];
#pragma unroll
                        for (int lv = 0; lv < 4; lv++) {         // local partners 2^lv away
                            if (!((r0 >> lv) & 1)) {
                                uint32_t v[NW];
                                lds_get(my + RS * r0, (1 << lv) + 16 * j, v);
#pragma unroll
                                for (int w = 0; w < NW; w++)
                                    z[w] ^= v[w];
                            }
                        }
                        store_chunk<R, LD, true>(wrow(ws.dst2, WT::uni(grow(r0 + 16 * j)), rb), ln.off, ln.act, ln.nsym,
                                           z);
                    }
                }
            } else {
                pipelined<Tab, NX>([&](int j) { return WT::row(p_B, vB, j, grow(j)); },
                                   [&](int j, const Tab &t) {
                                       if (grow(j))
                                           scale<R>(x[j], t);
                                   });
                store_data(ws.dst);
#pragma unroll
                for (int j = 0; j < NX; j++) {
                    uint32_t z[NW];
                    zero_vec<R>(z);
#pragma unroll
                    for (int lv = 0; lv < TA; lv++)
                        if (!((j >> lv) & 1))
#pragma unroll
                            for (int w = 0; w < NW; w++)
                                z[w] ^= x[j + (1 << lv)][w];
                    store_chunk<R, LD, true>(wrow(ws.dst2, WT::uni(grow(j)), rb), ln.off, ln.act, ln.nsym, z);
                }
            }
            return;
        }
        // W_E2 continues with the forward transform of parity block 1, whose
        // highest levels start from the stride layout left in registers; each
        // wave again rewrites only its own tile rows before the barrier.
    }

    if (FWD) {
        if constexpr (TILED) {
#pragma unroll
            for (int u = 0; u < GPW; u++)
                reg_levels<R, L2, false, SHF, false>(y[u], (uint32_t)(vw * GPW + u), 4, twF);
            to_consecutive();
        }
        reg_levels<R, TA, false, SHF, false>(x, (uint32_t)(NX * g), 0, twF);
        if (KIND == W_D5) {
            pipelined<Tab, NX>([&](int j) { return WT::row(rowtab, vRT, xrow(j), grow(xrow(j))); },
                               [&](int j, const Tab &t) {
                                   dec_store<R, LD, !PK>(x[j], (int)grow(xrow(j)), st, ln, bits, [&](int) { return t; });
                               });
            return;
        }
#pragma unroll
        for (int j = 0; j < NX; j++) {
            const uint32_t p = grow(xrow(j));
            if ((int)p < ws.dst_rows) {
                if (KIND == W_PFM) {                 // times row p of src2, symbol by symbol
                    uint32_t m[NW];
                    load_chunk<R, LD, true>(wrow(ws.src2, WT::uni(p), rb), ln.off, ln.act, ln.nsym, m);
                    mul_symbols16<4>(x[j], m);
                }
                store_chunk<R, LD, true>(wrow(ws.dst, WT::uni(p), rb), ln.off, ln.act, ln.nsym, x[j]);
            }
        }
    }
}

}  // namespace nb
