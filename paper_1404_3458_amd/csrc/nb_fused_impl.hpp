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
// on the level, the block and the shift, Sec. 3.2) is wave-uniform.  Each
// workgroup first copies the vector-operand words of every perm table it
// will use into LDS (read back as broadcasts); the scalar-operand words are
// read with scalar loads.  For L <= 4 a single wave holds the whole
// transform in registers and no LDS is used.
#pragma once
#include "nb_xform.hpp"

namespace nb {

// M_ENC2: encode of a code with exactly one parity block (n' = 2 k').
enum Mode { M_FFT = 0, M_IFFT = 1, M_DERIV = 2, M_ENC = 3, M_DEC = 4, M_ENC2 = 5 };

// Sec. 4.2 on rows all held in registers: d^d = B d, coefficient of X_j is
// the sum of d^d_{j + 2^l} over the clear bits l of j, divided by B_j.
template <int R, int L>
__device__ __forceinline__ void deriv_regs(uint32_t (*x)[Traits<R>::NW], const Tabs &tb)
{
    constexpr int NW = Traits<R>::NW, NR = 1 << L;
    uint32_t y[NR][NW];
#pragma unroll
    for (int j = 0; j < NR; j++) {
#pragma unroll
        for (int w = 0; w < NW; w++)
            y[j][w] = x[j][w];
        if (j)
            scale<R>(y[j], row_tab<R>(tb.B, j));     // B_0 = 1
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
            scale<R>(x[j], row_tab<R>(tb.Binv, j));  // 1/B_0 = 1; row NR-1 is 0
    }
}

#define NB_FUSED_PARAMS                                                                                       \
    FusedArgs a, const uint32_t *__restrict__ p_tw, const uint32_t *__restrict__ p_B,                         \
        const uint32_t *__restrict__ p_Binv, const uint32_t *__restrict__ p_bits,                             \
        const uint32_t *__restrict__ p_rowtabs

// ------------------------------------------------------------------ L <= 4

// PR: the pruned variant, for stripes some of whose forward-transform
// outputs are never used (encode: parity rows of a shortened code that are
// not stored; decode: groups of 16 points without an erased stored row).
template <int R, int L, int MODE, int SH, int LD, bool PR = false>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(MODE == M_ENC || MODE == M_ENC2 ? 3 : 4))) void k_small(
    NB_FUSED_PARAMS)
{
    constexpr int NW = Traits<R>::NW, NR = 1 << L;
    const int tile = blockIdx.x;
    const int s = find_stripe_guess(a.stripes, a.nstripes, tile, (int)gridDim.x);
    const DevStripe st = a.stripes[s];
    const Lane ln = lane_of<R, LD>(tile - st.tile0, (int)threadIdx.x, st.col0, st.ncols);
    const DoneStamp done = {a.ts};
    const uint64_t rb = st.row_bytes;
    const Tabs tb = {p_tw, p_B, p_Binv};
    const uint32_t *__restrict__ bits = p_bits + st.bits_off;
    const uint32_t *__restrict__ rowtab = p_rowtabs + st.rowtab_off;
    const TwGlobal<R> tw = {p_tw, a.l};
    const TwGlobal<R> tw0 = {p_tw, 0u};
    uint32_t x[NR][NW];

    if (MODE == M_FFT || MODE == M_IFFT || MODE == M_DERIV) {
#pragma unroll
        for (int j = 0; j < NR; j++)
            load_chunk<R, LD>(row_ptr(st.in, j, rb), ln.off, ln.act, ln.nsym, x[j]);
        if (MODE == M_FFT)
            reg_levels<R, L, false, SH, true>(x, 0, 0, tw);
        else if (MODE == M_IFFT)
            reg_levels<R, L, true, SH, true>(x, 0, 0, tw);
        else
            deriv_regs<R, L>(x, tb);
#pragma unroll
        for (int j = 0; j < NR; j++)
            store_chunk<R, LD>(row_ptr(st.out, fresh(j), rb), ln.off, ln.act, ln.nsym, x[j]);
    } else if (MODE == M_ENC || MODE == M_ENC2) {
        // Algorithm 1: M_bar = inverse transform of the (zero-padded) message,
        // then one forward transform per parity block at shift blk * k'.
#pragma unroll
        for (int j = 0; j < NR; j++)
            load_chunk<R, LD>(row_ptr(st.in, j, rb), ln.off, ln.act && j < st.k, ln.nsym, x[j]);
        reg_levels<R, L, true, SH_ZERO, true>(x, 0, 0, tw0);
        const int nblocks = st.np / st.kp;
        const int npar = st.n - st.k;
        // only the stored parity rows are computed (pruned forward transforms)
        for (int blk = 1; blk < nblocks && (!PR || (blk - 1) * NR < npar); blk++) {
            uint32_t y[NR][NW];
#pragma unroll
            for (int j = 0; j < NR; j++)
#pragma unroll
                for (int w = 0; w < NW; w++)
                    y[j][w] = x[j][w];
            const TwGlobal<R> twb = {p_tw, (uint32_t)(blk * NR)};
            const int nout = npar - (blk - 1) * NR;
            reg_levels<R, L, false, SH_ALIGNED, true>(y, 0, 0, twb, !PR || nout >= 32 ? ~0u : (1u << nout) - 1u);
#pragma unroll
            for (int j = 0; j < NR; j++) {
                const int t = (blk - 1) * NR + j;
                if (t < npar)
                    store_chunk<R, LD>(row_ptr(st.out, fresh(t), rb), ln.off, ln.act, ln.nsym, y[j]);
            }
        }
    } else {  // M_DEC with n' = NR
        auto tabf = [&](int p) { return row_tab<R>(rowtab, p); };
#pragma unroll
        for (int p = 0; p < NR; p++) {
            const bool rcv = dec_fetch<R, LD>(x[p], p, st, ln, bits);
            dec_weigh<R>(x[p], rcv, tabf(p));
        }
        reg_levels<R, L, true, SH_ZERO, true>(x, 0, 0, tw0);      // step 3
        deriv_regs<R, L>(x, tb);                                  // step 4
        reg_levels<R, L, false, SH_ZERO, true>(x, 0, 0, tw0);     // step 5
#pragma unroll
        for (int p = 0; p < NR; p++)                              // step 6
            dec_store<R, LD>(x[p], p, st, ln, bits, tabf);
    }
}

// ------------------------------------------------------------------ 5 <= L <= 8

// LDS of k_tiled: the tile (2^L rows x 64 lanes x NW dwords), then the V words
// of every perm table the kernel multiplies by, staged once per workgroup.
// HALF: the encode of a code with one parity block over at most 2^7 points
// exchanges the tile one dword of each lane's symbol group at a time (two
// rounds per exchange), so the LDS holds half a tile: 40 KB per workgroup,
// which lets four workgroups (32 waves) share a CU instead of two.
template <int R, int L, int MODE>
struct TiledLds {
    static constexpr int H = 1 << L, NV = Ops<R>::NV, NW = Traits<R>::NW;
    static constexpr bool HALF = R == 16 && MODE == M_ENC2 && L <= 7;
    static constexpr int TILE = H * 64 * (HALF ? 1 : NW);               // dwords
    static constexpr int EX = MODE == M_DERIV ? 0 : H - 1;               // factors of the main transform
    static constexpr int EY = MODE == M_ENC ? 2 * (H - 1) : MODE == M_ENC2 ? H - 1 : 0;  // parity blocks
    static constexpr int EB = (MODE == M_DERIV || MODE == M_DEC) ? H : 0;  // B_j, and as many 1/B_j
    static constexpr int ERT = MODE == M_DEC ? H : 0;                    // per-point locator tables
    static constexpr size_t BYTES = 4 * ((size_t)TILE + (size_t)NV * (EX + EY + 2 * EB + ERT));
    static_assert(BYTES <= 160 * 1024, "tile and tables exceed the LDS of a workgroup");
};

// Algorithm 2 steps 2-6 on one tile of 2^L points whose received rows are
// in x (zeros for the other points) and whose tables are staged: the
// weighting by Pi, the inverse transform (16-row register groups, LDS
// transpose, stride-16 groups), the derivative across both groupings, the
// forward transform and the division of erased rows by Pi'.
template <int R, int L>
struct DecTile {
    typedef TiledLds<R, L, M_DEC> LY;
    typedef typename Ops<R>::Tab Tab;
    static constexpr int NW = Traits<R>::NW, NV = Ops<R>::NV, H = 1 << L;
    static constexpr int L2 = L - 4, NR2 = 1 << L2, GPW = 16 >> L2, RS = 64 * NW;
    uint32_t *lds;
    const uint32_t *__restrict__ p_tw;
    const uint32_t *__restrict__ p_B;
    const uint32_t *__restrict__ p_Binv;
    int wave, lane;

    __device__ __forceinline__ uint32_t *vX() const { return lds + LY::TILE; }
    __device__ __forceinline__ uint32_t *vB() const { return vX() + NV * LY::EX; }
    __device__ __forceinline__ uint32_t *vBi() const { return vB() + NV * LY::EB; }
    __device__ __forceinline__ uint32_t *vRT() const { return vBi() + NV * LY::EB; }
    __device__ __forceinline__ uint32_t *slot(int row) const { return lds + (size_t)row * RS + lane * NW; }
    __device__ __forceinline__ void put(int row, const uint32_t *v) const
    {
        uint32_t *p = slot(row);
        if (NW == 2)
            *reinterpret_cast<uint2 *>(p) = make_uint2(v[0], v[NW - 1]);
        else
            p[0] = v[0];
    }
    __device__ __forceinline__ void get(int row, uint32_t *v) const
    {
        const uint32_t *p = slot(row);
        if (NW == 2) {
            const uint2 t = *reinterpret_cast<const uint2 *>(p);
            v[0] = t.x;
            v[NW - 1] = t.y;
        } else {
            v[0] = p[0];
        }
    }

    template <int LD, bool PR>
    __device__ __forceinline__ void run(uint32_t (*x)[Traits<R>::NW], const bool *rcv, const DevStripe &st,
                                        const Lane &ln, const uint32_t *__restrict__ bits,
                                        const uint32_t *__restrict__ rowtab) const
    {
        run<LD, PR, false>(x, rcv, st, ln, bits, rowtab, [] {});
    }

    // after_read: called once this wave has read its consecutive rows for the
    // last phase, from which point no other wave reads its tile rows (rows
    // 16 g .. 16 g + 15) of this tile again.  NT: the decoded rows are
    // stored non-temporally.
    template <int LD, bool PR, bool NT, class AFTER>
    __device__ __forceinline__ void run(uint32_t (*x)[Traits<R>::NW], const bool *rcv, const DevStripe &st,
                                        const Lane &ln, const uint32_t *__restrict__ bits,
                                        const uint32_t *__restrict__ rowtab, const AFTER &after_read) const
    {
        const int g = wave;
        const TwLds<R, L> twX = {p_tw, 0u, vX()};
        uint32_t *const vb = vB(), *const vbi = vBi(), *const vrt = vRT();
        // step 2 and the inverse levels 0..3 on the consecutive group
        pipelined<Tab, 16>([&](int j) { return row_tab<R>(rowtab, vrt, 16 * g + j); },
                           [&](int j, const Tab &t) { dec_weigh<R>(x[j], rcv[j], t); });
        reg_levels<R, 4, true, SH_ZERO, false>(x, (uint32_t)(16 * g), 0, twX);
#pragma unroll
        for (int j = 0; j < 16; j++)
            put(16 * g + j, x[j]);
        __syncthreads();
        // inverse levels 4..L-1 on the stride groups, then d^d = B (.) coefficients
        uint32_t y[GPW][NR2][NW];
#pragma unroll
        for (int u = 0; u < GPW; u++) {
            const int r0 = wave * GPW + u;
#pragma unroll
            for (int j = 0; j < NR2; j++)
                get(r0 + 16 * j, y[u][j]);
            reg_levels<R, L2, true, SH_ZERO, true>(y[u], (uint32_t)r0, 4, twX);
            pipelined<Tab, NR2>([&](int j) { return row_tab<R>(p_B, vb, r0 + 16 * j); },
                                [&](int j, const Tab &t) {
                                    if (r0 + 16 * j)
                                        scale<R>(y[u][j], t);
                                    put(r0 + 16 * j, y[u][j]);
                                });
        }
        __syncthreads();
        // step 4: partners 16 * 2^lv away are in registers, 2^lv away in LDS
        uint32_t z[GPW][NR2][NW];
#pragma unroll
        for (int u = 0; u < GPW; u++) {
            const int r0 = wave * GPW + u;
#pragma unroll
            for (int j = 0; j < NR2; j++) {
                zero_vec<R>(z[u][j]);
#pragma unroll
                for (int lv = 0; lv < L2; lv++)
                    if (!((j >> lv) & 1))
#pragma unroll
                        for (int w = 0; w < NW; w++)
                            z[u][j][w] ^= y[u][j + (1 << lv)][w];
            }
#pragma unroll
            for (int lv = 0; lv < 4; lv++) {
                if (!((r0 >> lv) & 1)) {
#pragma unroll
                    for (int j = 0; j < NR2; j++) {
                        uint32_t v[NW];
                        get(r0 + (1 << lv) + 16 * j, v);
#pragma unroll
                        for (int w = 0; w < NW; w++)
                            z[u][j][w] ^= v[w];
                    }
                }
            }
        }
        __syncthreads();
        // Step 5 is pruned to the outputs step 6 uses: bit j of `used` says
        // that consecutive group j (points 16 j .. 16 j + 15) holds an erased
        // stored point; the other groups' forward levels are skipped.
        constexpr uint32_t ALL = NR2 >= 32 ? ~0u : (1u << NR2) - 1u;
        uint32_t used = ALL;
        if (PR) {
            const uint32_t *__restrict__ sbm = bits + bitmap_words(st.np);
            used = 0;
#pragma unroll
            for (int j = 0; j < NR2; j++)
                used |= ((sbm[(16 * j) >> 5] >> ((16 * j) & 31)) & 0xFFFFu) ? (1u << j) : 0u;
            used = fresh(used);
        }
        // coefficients over B_j, step 5's levels L-1..4
#pragma unroll
        for (int u = 0; u < GPW; u++) {
            const int r0 = wave * GPW + u;
            pipelined<Tab, NR2>([&](int j) { return row_tab<R>(p_Binv, vbi, r0 + 16 * j); },
                                [&](int j, const Tab &t) {
                                    if (r0 + 16 * j)
                                        scale<R>(z[u][j], t);
                                });
            reg_levels<R, L2, false, SH_ZERO, true>(z[u], (uint32_t)r0, 4, twX, used);
#pragma unroll
            for (int j = 0; j < NR2; j++)
                if ((used >> j) & 1u)
                    put(r0 + 16 * j, z[u][j]);
        }
        __syncthreads();
        if (PR && !((used >> g) & 1u))
            return;
#pragma unroll
        for (int j = 0; j < 16; j++)
            get(16 * g + j, x[j]);
        after_read();
        // levels 3..0 and step 6
        reg_levels<R, 4, false, SH_ZERO, false>(x, (uint32_t)(16 * g), 0, twX);
        pipelined<Tab, 16>([&](int j) { return row_tab<R>(rowtab, vrt, 16 * g + j); },
                           [&](int j, const Tab &t) {
                               dec_store<R, LD, true, NT>(x[j], 16 * g + j, st, ln, bits,
                                                          [&](int) { return t; });
                           });
    }
};

// M_ENC keeps the coefficients in registers across the parity blocks: below
// 2^8 points its workgroup has at most 8 waves, so it may use the registers
// of two waves per SIMD instead of spilling.  The half-tile encodes (HALF)
// are held to six waves per SIMD (at most 80 registers), so that three
// workgroups share a CU: a SIMD issues VALU work at close to its peak rate
// only with more than four waves to pick from.  Their pruned variants keep
// four (they would spill at six).
template <int R, int L, int MODE, int SH, int LD, bool PR = false>
__global__ __launch_bounds__(64 << (L - 4)) __attribute__((amdgpu_waves_per_eu(
    MODE == M_ENC && L < 8 ? 2 : (TiledLds<R, L, MODE>::HALF && !PR) ? 6 : 4))) void k_tiled(NB_FUSED_PARAMS)
{
    typedef TiledLds<R, L, MODE> LY;
    typedef typename Ops<R>::Tab Tab;
    constexpr int NW = Traits<R>::NW, NV = Ops<R>::NV, H = 1 << L;
    constexpr int L2 = L - 4;            // levels of the stride phase
    constexpr int NR2 = 1 << L2;         // rows per stride group
    constexpr int GPW = 16 >> L2;        // stride groups per wave (waves = 2^L2)
    constexpr int NT = 64 << L2;         // threads
    extern __shared__ uint32_t lds[];    // [2^L rows][64 lanes][NW], then the staged tables
    uint32_t *const vX = lds + LY::TILE;
    uint32_t *const vY = vX + NV * LY::EX;
    uint32_t *const vB = vY + NV * LY::EY;
    uint32_t *const vBi = vB + NV * LY::EB;
    uint32_t *const vRT = vBi + NV * LY::EB;

    const int tid = (int)threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int tile = blockIdx.x;
    const int s = find_stripe_guess(a.stripes, a.nstripes, tile, (int)gridDim.x);
    const DevStripe st = a.stripes[s];
    const Lane ln = lane_of<R, LD>(tile - st.tile0, lane, st.col0, st.ncols);
    const DoneStamp done = {a.ts};
    const uint64_t rb = st.row_bytes;
    const uint32_t *__restrict__ bits = p_bits + st.bits_off;
    const uint32_t *__restrict__ rowtab = p_rowtabs + st.rowtab_off;
    const uint32_t lx = (MODE == M_FFT || MODE == M_IFFT) ? a.l : 0u;
    const TwLds<R, L> twX = {p_tw, lx, vX};

    // LDS row slots of this lane: rows are RS dwords apart; callers pass a
    // group base (a lane slot of the group's first row) and a compile-time
    // row offset, so accesses are one base register plus an immediate.
    constexpr int RS = 64 * NW;
    uint32_t *const my = lds + lane * NW;
    auto lds_put = [&](uint32_t *base, int rows, const uint32_t *v) {
        uint32_t *p = base + RS * rows;
        if (NW == 2)
            *reinterpret_cast<uint2 *>(p) = make_uint2(v[0], v[NW - 1]);
        else
            p[0] = v[0];
    };
    auto lds_get = [&](const uint32_t *base, int rows, uint32_t *v) {
        const uint32_t *p = base + RS * rows;
        if (NW == 2) {
            const uint2 t = *reinterpret_cast<const uint2 *>(p);
            v[0] = t.x;
            v[NW - 1] = t.y;
        } else {
            v[0] = p[0];
        }
    };
    // Called by every thread after the first row loads are issued: copies
    // the tables and makes them visible to the whole workgroup.
    auto stage_tables = [&]() {
        if (MODE != M_DERIV)
            stage_levels<R, L>(vX, p_tw, lx, tid, NT);
        if (MODE == M_ENC && st.np > H)                 // parity block 1 (shift 2^L) into buffer 1
            stage_levels<R, L>(vY + NV * (H - 1), p_tw, 1u << L, tid, NT);
        if (MODE == M_ENC2)                             // the parity block (shift 2^L)
            stage_levels<R, L>(vY, p_tw, 1u << L, tid, NT);
        if (LY::EB) {
            stage_rows<R>(vB, p_B, H, tid, NT);
            stage_rows<R>(vBi, p_Binv, H, tid, NT);
        }
        if (MODE == M_DEC)
            stage_rows<R>(vRT, rowtab, H, tid, NT);
        __syncthreads();
    };

    const int g = wave;                       // consecutive group of this wave
    uint32_t *const cb = my + RS * 16 * g;    // its first row
    uint32_t x[16][NW];                       // consecutive-phase registers
    uint32_t y[GPW][NR2][NW];                 // stride-phase registers

    if (MODE == M_FFT) {
#pragma unroll
        for (int u = 0; u < GPW; u++)
#pragma unroll
            for (int j = 0; j < NR2; j++)
                load_chunk<R, LD>(row_ptr(st.in, wave * GPW + u + 16 * j, rb), ln.off, ln.act, ln.nsym, y[u][j]);
        stage_tables();
#pragma unroll
        for (int u = 0; u < GPW; u++) {
            const int r0 = wave * GPW + u;
            reg_levels<R, L2, false, SH, true>(y[u], (uint32_t)r0, 4, twX);
#pragma unroll
            for (int j = 0; j < NR2; j++)
                lds_put(my + RS * r0, 16 * j, y[u][j]);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 16; j++)
            lds_get(cb, j, x[j]);
        reg_levels<R, 4, false, SH, false>(x, (uint32_t)(16 * g), 0, twX);
#pragma unroll
        for (int j = 0; j < 16; j++)
            store_chunk<R, LD>(row_ptr(st.out, fresh(16 * g + j), rb), ln.off, ln.act, ln.nsym, x[j]);
        return;
    }

    if (MODE == M_DERIV) {
        // Sec. 4.2 on consecutive groups: partners 2^l with l < 4 are in the
        // wave's registers, those with l >= 4 are read from LDS.
#pragma unroll
        for (int j = 0; j < 16; j++)
            load_chunk<R, LD>(row_ptr(st.in, 16 * g + j, rb), ln.off, ln.act, ln.nsym, x[j]);
        stage_tables();
        pipelined<Tab, 16>([&](int j) { return row_tab<R>(p_B, vB, 16 * g + j); },
                           [&](int j, const Tab &t) {
                               if (16 * g + j)
                                   scale<R>(x[j], t);
                               lds_put(cb, j, x[j]);
                           });
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
        pipelined<Tab, 16>([&](int j) { return row_tab<R>(p_Binv, vBi, 16 * g + j); },
                           [&](int j, const Tab &t) {
                               const int p = (int)fresh(16 * g + j);
                               if (p)
                                   scale<R>(z[j], t);
                               store_chunk<R, LD>(row_ptr(st.out, p, rb), ln.off, ln.act, ln.nsym, z[j]);
                           });
        return;
    }

    // ---- phase 1 (consecutive groups): input and inverse levels 0..3
    bool rcv[16];
#pragma unroll
    for (int j = 0; j < 16; j++) {
        const int p = 16 * g + j;
        if (MODE == M_IFFT) {
            load_chunk<R, LD>(row_ptr(st.in, p, rb), ln.off, ln.act, ln.nsym, x[j]);
        } else if (MODE == M_ENC || MODE == M_ENC2) {
            // rows k .. k'-1 are the zero padding of a shortened message
            load_chunk<R, LD>(row_ptr(st.in, p, rb), ln.off, ln.act && p < st.k, ln.nsym, x[j]);
        } else {
            rcv[j] = dec_fetch<R, LD>(x[j], p, st, ln, bits);
        }
    }
    stage_tables();
    if (MODE == M_DEC) {
        const DecTile<R, L> dt = {lds, p_tw, p_B, p_Binv, wave, lane};
        dt.template run<LD, PR>(x, rcv, st, ln, bits, rowtab);
        return;
    }
    reg_levels<R, 4, true, (MODE == M_IFFT ? SH : SH_ZERO), false>(x, (uint32_t)(16 * g), 0, twX);
    if constexpr (LY::HALF) {
        // two rounds through half a tile: row t, lane l at dword 64 t + l
        uint32_t *const hl = lds + lane;
#pragma unroll
        for (int w = 0; w < NW; w++) {
            if (w)
                __syncthreads();                     // the previous round's words are read
#pragma unroll
            for (int j = 0; j < 16; j++)
                hl[64 * (16 * g + j)] = x[j][w];
            __syncthreads();
#pragma unroll
            for (int u = 0; u < GPW; u++)
#pragma unroll
                for (int j = 0; j < NR2; j++)
                    y[u][j][w] = hl[64 * (wave * GPW + u + 16 * j)];
        }
    } else {
#pragma unroll
        for (int j = 0; j < 16; j++)
            lds_put(cb, j, x[j]);
        __syncthreads();
    }

    // ---- phase 2 (stride groups): inverse levels 4..L-1
#pragma unroll
    for (int u = 0; u < GPW; u++) {
        const int r0 = wave * GPW + u;
        if constexpr (!LY::HALF) {
#pragma unroll
            for (int j = 0; j < NR2; j++)
                lds_get(my + RS * r0, 16 * j, y[u][j]);
        }
        reg_levels<R, L2, true, (MODE == M_IFFT ? SH : SH_ZERO), true>(y[u], (uint32_t)r0, 4, twX);
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

    if (MODE == M_ENC2) {
        // the one parity block at shift 2^L, transformed in place; of a
        // shortened code only the first npar rows are stored, so the stride
        // groups compute only the blocks of rows 16 j with j < ceil(npar/16)
        // and only the waves holding such rows run the consecutive levels
        const TwLds<R, L> twY = {p_tw, 1u << L, vY};
        const int npar = st.n - st.k;
        const int ng = PR ? (npar + 15) >> 4 : NR2;      // consecutive groups with stored rows
        const uint32_t need = ng >= NR2 ? ~0u : (1u << ng) - 1u;
#pragma unroll
        for (int u = 0; u < GPW; u++) {
            const int r0 = wave * GPW + u;
            reg_levels<R, L2, false, SH_ALIGNED, true>(y[u], (uint32_t)r0, 4, twY, need);
            if constexpr (!LY::HALF) {
#pragma unroll
                for (int j = 0; j < NR2; j++)
                    if (!PR || j < ng)
                        lds_put(my + RS * r0, 16 * j, y[u][j]);
            }
        }
        if constexpr (LY::HALF) {
            // each wave rewrites only the rows it read itself, so the first
            // round needs no barrier before its writes
            uint32_t *const hl = lds + lane;
#pragma unroll
            for (int w = 0; w < NW; w++) {
                if (w)
                    __syncthreads();
#pragma unroll
                for (int u = 0; u < GPW; u++)
#pragma unroll
                    for (int j = 0; j < NR2; j++)
                        if (!PR || j < ng)
                            hl[64 * (wave * GPW + u + 16 * j)] = y[u][j][w];
                __syncthreads();
                if (!PR || g < ng) {
#pragma unroll
                    for (int j = 0; j < 16; j++)
                        x[j][w] = hl[64 * (16 * g + j)];
                }
            }
        } else {
            __syncthreads();
        }
        if (PR && g >= ng)
            return;
        if constexpr (!LY::HALF) {
#pragma unroll
            for (int j = 0; j < 16; j++)
                lds_get(cb, j, x[j]);
        }
        reg_levels<R, 4, false, SH_ALIGNED, false>(x, (uint32_t)(16 * g), 0, twY);
#pragma unroll
        for (int j = 0; j < 16; j++) {
            const int t = 16 * g + j;
            if (t < npar)
                store_chunk<R, LD>(row_ptr(st.out, fresh(t), rb), ln.off, ln.act, ln.nsym, x[j]);
        }
        return;
    }

    if (MODE == M_ENC) {
        const int nblocks = st.np >> L;
        const int npar = st.n - st.k;
        // parity blocks and rows past the stored ones are not computed
        for (int blk = 1; blk < nblocks && (!PR || (blk - 1) * H < npar); blk++) {
            const int ng = PR ? (npar - (blk - 1) * H + 15) >> 4 : NR2;
            const uint32_t need = ng >= NR2 ? ~0u : (1u << ng) - 1u;
            const uint32_t lsh = (uint32_t)(blk << L);
            const TwLds<R, L> twY = {p_tw, lsh, vY + NV * (H - 1) * (blk & 1)};
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
                reg_levels<R, L2, false, SH_ALIGNED, true>(z, (uint32_t)r0, 4, twY, need);
#pragma unroll
                for (int j = 0; j < NR2; j++)
                    if (!PR || j < ng)
                        lds_put(my + RS * r0, 16 * j, z[j]);
            }
            __syncthreads();
            // the next block's factors go to the other buffer, last read by
            // block blk - 1 before the barrier above
            if (blk + 1 < nblocks && (!PR || blk * H < npar))
                stage_levels<R, L>(vY + NV * (H - 1) * ((blk + 1) & 1), p_tw, (uint32_t)((blk + 1) << L), tid, NT);
            if (!PR || g < ng) {
#pragma unroll
                for (int j = 0; j < 16; j++)
                    lds_get(cb, j, x[j]);
                reg_levels<R, 4, false, SH_ALIGNED, false>(x, (uint32_t)(16 * g), 0, twY);
#pragma unroll
                for (int j = 0; j < 16; j++) {
                    const int t = (blk - 1) * H + 16 * g + j;
                    if (t < npar)
                        store_chunk<R, LD>(row_ptr(st.out, fresh(t), rb), ln.off, ln.act, ln.nsym, x[j]);
                }
            }
        }
        return;
    }

}

// Decode (Algorithm 2 steps 2-6) of 2^L-point stripes with vector-aligned
// rows, persistent: one workgroup per LDS slot of the device walks a
// contiguous range of tiles.  The transform and derivative tables are staged
// once, the per-point locator tables when the stripe changes, and while a
// wave computes the last phase of one tile the received rows of its part of
// the next tile travel from global memory straight into its (then unused)
// tile rows (global_load_lds, no registers), so that the next tile starts
// from LDS instead of waiting for HBM.  A copied tile row holds the row's
// 512 bytes in memory order (lane l's chunk at dwords 2l, 2l + 1).  Rows
// are read and written non-temporally: each XCD streams about as many row
// bytes per tile as its L2 holds, which otherwise evicts the table words
// every tile re-reads (they came back as extra 64-byte HBM reads, about a
// sixth of the row bytes, and slower scalar loads).  Only launches without
// completion stamps (one stamp slot per workgroup would span several
// stripes) and without pruning.
template <int R, int L>
__global__ __launch_bounds__(64 << (L - 4)) __attribute__((amdgpu_waves_per_eu(4))) void k_dec_persist(
    NB_FUSED_PARAMS, int ntiles)
{
    static_assert(R == 16, "GF(2^16) rows of 4-byte dwords");
    typedef TiledLds<R, L, M_DEC> LY;
    constexpr int NW = Traits<R>::NW, NV = Ops<R>::NV, H = 1 << L, NT = 64 << (L - 4), RS = 64 * NW;
    extern __shared__ uint32_t lds[];
    uint32_t *const vX = lds + LY::TILE;
    uint32_t *const vB = vX + NV * LY::EX;
    uint32_t *const vBi = vB + NV * LY::EB;
    uint32_t *const vRT = vBi + NV * LY::EB;
    const int tid = (int)threadIdx.x;
    // workgroup b takes tiles [t0, t1): ntiles / G each, one more for the
    // first ntiles % G
    const int G = (int)gridDim.x, b = (int)blockIdx.x, q = ntiles / G, rm = ntiles % G;
    const int t0 = b * q + (b < rm ? b : rm);
    const int t1 = t0 + q + (b < rm ? 1 : 0);

    // Copies the received rows of tile t's consecutive group of this wave
    // into the wave's tile rows, in two 256-byte halves: in the first, lane l
    // copies dword l of the row (half of chunk l / 2), in the second dword
    // 64 + l (half of chunk 32 + l / 2); a chunk past the stripe's columns is
    // not copied.
    ConstStripe *const cst = const_stripes(a.stripes);
    auto issue = [&](int t, int si, int g, int lane) {
        const DevStripe st = cst[si];
        const Lane la = lane_of<R, LD_VEC>(t - st.tile0, lane >> 1, st.col0, st.ncols);
        const Lane lb = lane_of<R, LD_VEC>(t - st.tile0, 32 + (lane >> 1), st.col0, st.ncols);
        const uint32_t half = 4u * (uint32_t)(lane & 1);
        const uint32_t *__restrict__ bits = p_bits + st.bits_off;
#pragma unroll
        for (int j = 0; j < 16; j++) {
            const int p = 16 * g + j;
            if (point_bit(bits, p)) {
                const uint8_t *row = row_ptr(st.in, (uint32_t)point_row(p, st), st.row_bytes) + half;
                uint32_t *dst = lds + (size_t)p * RS;
                // cache policy 2: non-temporal
                if (la.act)
                    __builtin_amdgcn_global_load_lds((const void *)(row + la.off),
                                                     (__attribute__((address_space(3))) void *)dst, 4, 0, 2);
                if (lb.act)
                    __builtin_amdgcn_global_load_lds((const void *)(row + lb.off),
                                                     (__attribute__((address_space(3))) void *)(dst + 64), 4, 0,
                                                     2);
            }
        }
    };
    // stripes are in tile order: the stripe of the next tile is this one or
    // a later one (past any without tiles), so one search at the start
    int s = t0 < t1 ? find_stripe(cst, a.nstripes, t0) : 0;
    if (t0 < t1)
        issue(t0, s, __builtin_amdgcn_readfirstlane(tid >> 6), tid & 63);
    stage_levels<R, L>(vX, p_tw, 0u, tid, NT);
    stage_rows<R>(vB, p_B, H, tid, NT);
    stage_rows<R>(vBi, p_Binv, H, tid, NT);
    int cur = -1;                                // stripe whose locator tables are staged
    for (int tile = t0; tile < t1; tile++) {
        // wave and lane pass through an empty asm per tile, so that the
        // compiler recomputes the hundred addresses and table indices derived
        // from them inside the loop instead of keeping them live across it
        int g = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
        asm volatile("" : "+s"(g), "+v"(lane));
        const DecTile<R, L> dt = {lds, p_tw, p_B, p_Binv, g, lane};
        const DevStripe st = cst[s];
        const Lane ln = lane_of<R, LD_VEC>(tile - st.tile0, lane, st.col0, st.ncols);
        const uint32_t *__restrict__ bits = p_bits + st.bits_off;
        const uint32_t *__restrict__ rowtab = p_rowtabs + st.rowtab_off;
        if (s != cur) {
            __syncthreads();                     // every wave is done with the previous tables
            stage_rows<R>(vRT, rowtab, H, tid, NT);
            __syncthreads();
            cur = s;
        }
        uint32_t x[16][NW];
        bool rcv[16];
        __builtin_amdgcn_s_waitcnt(0x0F70);      // vmcnt(0): this wave's row copies have landed
        asm volatile("" ::: "memory");
        // one per-lane base; the rows sit at constant offsets from it
        const uint2 *const mine = reinterpret_cast<const uint2 *>(lds + (size_t)(16 * g) * RS) + lane;
#pragma unroll
        for (int j = 0; j < 16; j++) {
            const int p = 16 * g + j;
            rcv[j] = point_bit(bits, p);
            if (rcv[j]) {
                // chunks past the stripe's columns were not copied: zero
                const uint2 w = mine[j * (RS / 2)];
                Ops<R>::unpack(ln.act ? w.x : 0u, ln.act ? w.y : 0u, x[j]);
            } else {
                zero_vec<R>(x[j]);
            }
        }
        if (st.copy_survivors) {
#pragma unroll
            for (int j = 0; j < 16; j++) {
                const int p = 16 * g + j;
                if (rcv[j])
                    store_chunk<R, LD_VEC, true>(row_ptr(st.out, (uint32_t)point_row(p, st), st.row_bytes), ln.off,
                                                 ln.act, ln.nsym, x[j]);
            }
        }
        const int nx = tile + 1;
        int s2 = s;
        while (s2 + 1 < a.nstripes && cst[s2 + 1].tile0 <= nx)
            s2++;
        dt.template run<LD_VEC, false, true>(x, rcv, st, ln, bits, rowtab, [&] {
            if (nx < t1) {
                // this wave's reads of its tile rows have returned before the
                // copies into them start
                __builtin_amdgcn_s_waitcnt(0xC07F); // lgkmcnt(0)
                asm volatile("" ::: "memory");
                issue(nx, s2, g, lane);
                asm volatile("" ::: "memory");
            }
        });
        s = s2;
    }
}

// Workgroups of k_dec_persist that fit one CU at once.
template <int L>
constexpr int dec_persist_per_cu()
{
    return (int)((160 * 1024) / TiledLds<16, L, M_DEC>::BYTES);
}

// ------------------------------------------------------------------ launchers

// Modes with a pruned variant.
constexpr bool can_prune(int mode) { return mode == M_ENC || mode == M_ENC2 || mode == M_DEC; }

// Encodes over 2^8 points with several parity blocks run as pass pipelines
// (the host never sends them here), so that variant is not built.
template <int R, int L, int MODE>
constexpr bool fused_built() { return !(MODE == M_ENC && L >= 8); }

// Compute units of the current device (cached per device).
static int device_cus()
{
    static int cus[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return 0;
    if (!cus[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
            cus[dev] = v;
    }
    return cus[dev];
}

template <int R, int L, int MODE, int SH, int LD, bool PR>
static hipError_t launch_pr(const FusedArgs &a, const KPtrs &k, int ntiles, hipStream_t stream)
{
    if constexpr (!fused_built<R, L, MODE>())
        return hipErrorInvalidValue;
    else if constexpr (R == 16 && MODE == M_DEC && LD == LD_VEC && !PR && L >= 7) {
        // persistent when there is more than one round of workgroups and no
        // completion stamps are asked for
        const int slots = device_cus() * dec_persist_per_cu<L>();
        const size_t lds = TiledLds<R, L, MODE>::BYTES;
        if (!a.ts && slots > 0 && ntiles > slots) {
            hipLaunchKernelGGL((k_dec_persist<R, L>), dim3(slots), dim3(64 << (L - 4)), lds, stream, a, k.tw, k.B,
                               k.Binv, k.bits, k.rowtabs, ntiles);
        } else {
            hipLaunchKernelGGL((k_tiled<R, L, MODE, SH, LD, PR>), dim3(ntiles), dim3(64 << (L - 4)), lds, stream, a,
                               k.tw, k.B, k.Binv, k.bits, k.rowtabs);
        }
    } else if (L <= 4) {
        hipLaunchKernelGGL((k_small<R, (L <= 4 ? L : 4), MODE, SH, LD, PR>), dim3(ntiles), dim3(64), 0, stream, a,
                           k.tw, k.B, k.Binv, k.bits, k.rowtabs);
    } else {
        constexpr int LL = L > 4 ? L : 5;
        const size_t lds = TiledLds<R, LL, MODE>::BYTES;
        hipLaunchKernelGGL((k_tiled<R, LL, MODE, SH, LD, PR>), dim3(ntiles), dim3(64 << (LL - 4)), lds, stream, a,
                           k.tw, k.B, k.Binv, k.bits, k.rowtabs);
    }
    return hipGetLastError();
}

template <int R, int L, int MODE, int SH, int LD>
static hipError_t launch_one(const FusedArgs &a, const KPtrs &k, int ntiles, bool pr, hipStream_t stream)
{
    if (ntiles <= 0)
        return hipSuccess;
    if constexpr (can_prune(MODE))
        if (pr)
            return launch_pr<R, L, MODE, SH, LD, true>(a, k, ntiles, stream);
    return launch_pr<R, L, MODE, SH, LD, false>(a, k, ntiles, stream);
}

template <int R, int L, int MODE, int SH, int LD>
static hipError_t prep_one()
{
    if constexpr (!fused_built<R, L, MODE>())
        return hipSuccess;
    else if (L > 4) {
        constexpr int LL = L > 4 ? L : 5;
        hipError_t e = hipFuncSetAttribute((const void *)k_tiled<R, LL, MODE, SH, LD, false>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)TiledLds<R, LL, MODE>::BYTES);
        if constexpr (can_prune(MODE)) {
            const hipError_t f = hipFuncSetAttribute((const void *)k_tiled<R, LL, MODE, SH, LD, true>,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)TiledLds<R, LL, MODE>::BYTES);
            if (e == hipSuccess)
                e = f;
        }
        if constexpr (R == 16 && MODE == M_DEC && LD == LD_VEC && LL >= 7) {
            const hipError_t f = hipFuncSetAttribute((const void *)k_dec_persist<R, LL>,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)TiledLds<R, LL, MODE>::BYTES);
            if (e == hipSuccess)
                e = f;
        }
        return e;
    }
    return hipSuccess;
}

template <int R, int MODE, int SH, int LD>
static hipError_t launch_L(int L, const FusedArgs &a, const KPtrs &k, int ntiles, bool pr, hipStream_t s)
{
    switch (L) {
    case 0: return launch_one<R, 0, MODE, SH, LD>(a, k, ntiles, pr, s);
    case 1: return launch_one<R, 1, MODE, SH, LD>(a, k, ntiles, pr, s);
    case 2: return launch_one<R, 2, MODE, SH, LD>(a, k, ntiles, pr, s);
    case 3: return launch_one<R, 3, MODE, SH, LD>(a, k, ntiles, pr, s);
    case 4: return launch_one<R, 4, MODE, SH, LD>(a, k, ntiles, pr, s);
    case 5: return launch_one<R, 5, MODE, SH, LD>(a, k, ntiles, pr, s);
    case 6: return launch_one<R, 6, MODE, SH, LD>(a, k, ntiles, pr, s);
    case 7: return launch_one<R, 7, MODE, SH, LD>(a, k, ntiles, pr, s);
    case 8: return launch_one<R, 8, MODE, SH, LD>(a, k, ntiles, pr, s);
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
static hipError_t launch_ld(int mode, int sh, int L, const FusedArgs &a, const KPtrs &k, int ntiles, bool pr,
                            hipStream_t s)
{
    switch (mode) {
    case M_FFT:
        return sh == SH_ZERO ? launch_L<R, M_FFT, SH_ZERO, LD>(L, a, k, ntiles, pr, s)
             : sh == SH_ALIGNED ? launch_L<R, M_FFT, SH_ALIGNED, LD>(L, a, k, ntiles, pr, s)
                                : launch_L<R, M_FFT, SH_GENERAL, LD>(L, a, k, ntiles, pr, s);
    case M_IFFT:
        return sh == SH_ZERO ? launch_L<R, M_IFFT, SH_ZERO, LD>(L, a, k, ntiles, pr, s)
             : sh == SH_ALIGNED ? launch_L<R, M_IFFT, SH_ALIGNED, LD>(L, a, k, ntiles, pr, s)
                                : launch_L<R, M_IFFT, SH_GENERAL, LD>(L, a, k, ntiles, pr, s);
    case M_DERIV: return launch_L<R, M_DERIV, SH_ZERO, LD>(L, a, k, ntiles, pr, s);
    case M_ENC: return launch_L<R, M_ENC, SH_ZERO, LD>(L, a, k, ntiles, pr, s);
    case M_ENC2: return launch_L<R, M_ENC2, SH_ZERO, LD>(L, a, k, ntiles, pr, s);
    case M_DEC: return launch_L<R, M_DEC, SH_ZERO, LD>(L, a, k, ntiles, pr, s);
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
    NB_PREP(M_ENC2, SH_ZERO, LD_VEC) NB_PREP(M_ENC2, SH_ZERO, LD_SYM)
    NB_PREP(M_FFT, SH_ZERO, LD_SYM) NB_PREP(M_FFT, SH_ALIGNED, LD_SYM) NB_PREP(M_FFT, SH_GENERAL, LD_SYM)
    NB_PREP(M_IFFT, SH_ZERO, LD_SYM) NB_PREP(M_IFFT, SH_ALIGNED, LD_SYM) NB_PREP(M_IFFT, SH_GENERAL, LD_SYM)
    NB_PREP(M_DERIV, SH_ZERO, LD_SYM) NB_PREP(M_ENC, SH_ZERO, LD_SYM) NB_PREP(M_DEC, SH_ZERO, LD_SYM)
#undef NB_PREP
    return e;
}

}  // namespace nb
