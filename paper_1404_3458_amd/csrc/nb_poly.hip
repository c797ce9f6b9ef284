// nb_poly.hip -- polynomial operations in the novel basis beyond the
// transforms (Sec. 6.1 and its Table 1): the zero padding and the
// point-by-point product of the product algorithm (for products over at most
// 256 points; above, the transform passes read the unpadded operands and
// multiply in their last pass), the degree, and the conversion between the
// novel basis and the monomial basis.
//
// Every kernel works on column tiles of 256 columns (64 lanes x 4 columns)
// of row-major stripes, like the transform kernels; a workgroup of one wave
// handles one row (or one output row) of one tile unless noted.
//
// Conversion.  X_{i + 2^(t-1)} = X_i * What_{t-1} for i < 2^(t-1) (Definition
// 1: X_i is the product of the What_j over the set bits j of i), so the
// polynomial of a block of 2^t consecutive novel-basis coefficients is
// lo(x) + What_{t-1}(x) hi(x), lo and hi being the polynomials of its two
// halves.  What_{t-1} is linearized: its monomials sit at the degrees 2^m,
// m < t (it is W_{t-1} scaled, and W_j has monomials only at powers of two),
// so with w_m its coefficients:
//   novel -> monomial, level t = 1 .. lg h (ping-pong between two buffers):
//     out[j] = lo[j] + sum_m w_m hi[j - 2^m]        (lo[j] = 0 for j >= 2^(t-1))
//   monomial -> novel, level t = lg h .. 1 (in place): the division of the
//   block P by What_{t-1},
//     hi[e] = (P[h' + e] + sum_{m < t-1, 2^m > e} w_m hi[e + h' - 2^m]) / w_{t-1}
//     lo[j] = P[j] + sum_{m < t-1, 2^m <= j} w_m hi[j - 2^m]        (h' = 2^(t-1))
//   where hi[e] only needs entries at least h'/2 above e: the ranges
//   [h'/2, h'), [h'/4, h'/2), ..., [1, 2), [0, 1) are computed one after the
//   other, each entirely in parallel, and lo last.
// Levels t <= 8 only mix rows of the same block of 256 consecutive rows:
// k_conv_up_tile and k_conv_down_tile run all of them for one block and one
// column tile in one workgroup, with the block in LDS and a barrier where the
// one-level kernels need a launch (the levels above 8 keep those).
#include "nb_xform.hpp"

namespace nb {

__device__ __forceinline__ const uint8_t *qrow(const uint8_t *b, uint32_t t, uint64_t rb) { return b + (uint64_t)t * rb; }
__device__ __forceinline__ uint8_t *qrow(uint8_t *b, uint32_t t, uint64_t rb) { return b + (uint64_t)t * rb; }

// dst rows [0, rows): src rows below src_rows, zero above.
template <int R, int LD>
__global__ __launch_bounds__(64) void k_poly_pad(PolyArgs a)
{
    constexpr int NW = Traits<R>::NW;
    const uint32_t p = fresh(blockIdx.x / (uint32_t)a.nct);
    const int ct = (int)(blockIdx.x % (uint32_t)a.nct);
    const Lane ln = lane_of<R, LD>(ct, (int)threadIdx.x, a.col0, a.ncols);
    uint32_t x[NW];
    load_chunk<R, LD>(qrow(a.src, p, a.row_bytes), ln.off, ln.act && (int)p < a.src_rows, ln.nsym, x);
    store_chunk<R, LD>(qrow(a.dst, p, a.row_bytes), ln.off, ln.act, ln.nsym, x);
}

// Product of two field elements through the logarithm tables (alpha = 2);
// GF(2^8) only (GF(2^16) multiplies by shift and add, gf16_mul2).
__device__ __forceinline__ uint32_t mul_log(uint32_t x, uint32_t y, const uint32_t *__restrict__ lg,
                                            const uint32_t *__restrict__ ex, uint32_t M)
{
    if (!x || !y)
        return 0u;
    uint32_t e = lg[x] + lg[y];
    e = e >= M ? e - M : e;
    return ex[e];
}

// dst[p] <- dst[p] * src2[p] symbol by symbol, rows [0, rows).
template <int R, int LD>
__global__ __launch_bounds__(64) void k_poly_mul(PolyArgs a, const uint32_t *__restrict__ lg,
                                                 const uint32_t *__restrict__ ex)
{
    constexpr int NW = Traits<R>::NW;
    constexpr uint32_t M = (1u << R) - 1u;
    const uint32_t p = fresh(blockIdx.x / (uint32_t)a.nct);
    const int ct = (int)(blockIdx.x % (uint32_t)a.nct);
    const Lane ln = lane_of<R, LD>(ct, (int)threadIdx.x, a.col0, a.ncols);
    uint32_t x[NW], y[NW];
    load_chunk<R, LD>(qrow(a.dst, p, a.row_bytes), ln.off, ln.act, ln.nsym, x);
    load_chunk<R, LD>(qrow(a.src2, p, a.row_bytes), ln.off, ln.act, ln.nsym, y);
    if (R == 16) {
        mul_symbols16(x, y);
    } else {
        uint32_t o = 0;
#pragma unroll
        for (int s = 0; s < 4; s++)
            o |= mul_log((x[0] >> (8 * s)) & 0xFFu, (y[0] >> (8 * s)) & 0xFFu, lg, ex, M) << (8 * s);
        x[0] = o;
    }
    store_chunk<R, LD>(qrow(a.dst, p, a.row_bytes), ln.off, ln.act, ln.nsym, x);
}

// deg[c] = the last of the rows [0, rows) whose symbol c is nonzero, -1 if
// none (deg X_j = j, Sec. 6.1).  One workgroup of four waves per column tile:
// wave w scans the rows w, w + 4, ...; the four results meet in LDS.
template <int R, int LD>
__global__ __launch_bounds__(256) void k_poly_degree(PolyArgs a)
{
    constexpr int NW = Traits<R>::NW;
    __shared__ int32_t best[4][64][4];
    const int lane = (int)threadIdx.x & 63;
    const int wave = (int)threadIdx.x >> 6;
    const int ct = (int)blockIdx.x;
    const Lane ln = lane_of<R, LD>(ct, lane, a.col0, a.ncols);
    int32_t b[4] = {-1, -1, -1, -1};
#pragma unroll 8
    for (int p = wave; p < a.rows; p += 4) {
        uint32_t x[NW];
        load_chunk<R, LD>(qrow(a.src, (uint32_t)p, a.row_bytes), ln.off, ln.act, ln.nsym, x);
        const uint32_t any = NW == 2 ? (x[0] | x[NW - 1]) : x[0];
#pragma unroll
        for (int s = 0; s < 4; s++)
            if ((any >> (8 * s)) & 0xFFu)
                b[s] = p;
    }
#pragma unroll
    for (int s = 0; s < 4; s++)
        best[wave][lane][s] = b[s];
    __syncthreads();
    if (wave == 0 && ln.act) {
        const int c = a.col0 + 4 * (ct * 64 + lane);
#pragma unroll
        for (int s = 0; s < 4; s++) {
            const int32_t v = max(max(best[0][lane][s], best[1][lane][s]), max(best[2][lane][s], best[3][lane][s]));
            if (s < ln.nsym)
                a.deg[c + s] = v;
        }
    }
}

// novel -> monomial, one level (out of place): output row p of src's blocks
// of 2^t rows.  wt: perm tables of the coefficients w_{j,m} of What_j at
// entry 16 j + m.
template <int R, int LD>
__global__ __launch_bounds__(64) void k_conv_up(PolyArgs a, const uint32_t *__restrict__ wt)
{
    constexpr int NW = Traits<R>::NW;
    const uint32_t p = fresh(blockIdx.x / (uint32_t)a.nct);
    const int ct = (int)(blockIdx.x % (uint32_t)a.nct);
    const Lane ln = lane_of<R, LD>(ct, (int)threadIdx.x, a.col0, a.ncols);
    const int t = a.t;
    const uint32_t hh = 1u << (t - 1);
    const uint32_t c = p & ~((2u << (t - 1)) - 1u), j = p - c;
    const uint64_t rb = a.row_bytes;
    uint32_t acc[NW];
    load_chunk<R, LD>(qrow(a.src, p, rb), ln.off, ln.act && j < hh, ln.nsym, acc);
    for (int m = 0; m < t; m++) {
        const uint32_t s = 1u << m;
        if (j >= s && j - s < hh) {
            uint32_t v[NW];
            load_chunk<R, LD>(qrow(a.src, fresh(c + hh + j - s), rb), ln.off, ln.act, ln.nsym, v);
            Ops<R>::mac(acc, v, row_tab<R>(wt, 16 * (t - 1) + m));
        }
    }
    store_chunk<R, LD>(qrow(a.dst, p, rb), ln.off, ln.act, ln.nsym, acc);
}

// monomial -> novel, one step of level t (in place on dst): quotient entries
// [e0, e1) of every block, or (e1 == 0) the remainders.  wt as above, with the
// tables of 1 / w_{j,j} at entry 256 + j.
template <int R, int LD>
__global__ __launch_bounds__(64) void k_conv_down(PolyArgs a, const uint32_t *__restrict__ wt)
{
    constexpr int NW = Traits<R>::NW;
    const int t = a.t;
    const uint32_t hh = 1u << (t - 1);
    const uint32_t span = a.e1 ? (uint32_t)(a.e1 - a.e0) : hh;   // entries per block of this step
    const uint32_t q = fresh(blockIdx.x / (uint32_t)a.nct);
    const int ct = (int)(blockIdx.x % (uint32_t)a.nct);
    const uint32_t c = (q / span) << t, i = q % span;
    const Lane ln = lane_of<R, LD>(ct, (int)threadIdx.x, a.col0, a.ncols);
    const uint64_t rb = a.row_bytes;
    uint32_t acc[NW];
    if (a.e1) {
        const uint32_t e = (uint32_t)a.e0 + i;
        load_chunk<R, LD>(qrow(a.dst, fresh(c + hh + e), rb), ln.off, ln.act, ln.nsym, acc);
        for (int m = 0; m < t - 1; m++) {
            const uint32_t s = 1u << m;
            if (s > e) {
                uint32_t v[NW];
                load_chunk<R, LD>(qrow(a.dst, fresh(c + hh + e + hh - s), rb), ln.off, ln.act, ln.nsym, v);
                Ops<R>::mac(acc, v, row_tab<R>(wt, 16 * (t - 1) + m));
            }
        }
        scale<R>(acc, row_tab<R>(wt, 256 + (t - 1)));
        store_chunk<R, LD>(qrow(a.dst, fresh(c + hh + e), rb), ln.off, ln.act, ln.nsym, acc);
    } else {
        const uint32_t j = i;
        load_chunk<R, LD>(qrow(a.dst, fresh(c + j), rb), ln.off, ln.act, ln.nsym, acc);
        for (int m = 0; m < t - 1; m++) {
            const uint32_t s = 1u << m;
            if (s <= j) {
                uint32_t v[NW];
                load_chunk<R, LD>(qrow(a.dst, fresh(c + hh + j - s), rb), ln.off, ln.act, ln.nsym, v);
                Ops<R>::mac(acc, v, row_tab<R>(wt, 16 * (t - 1) + m));
            }
        }
        store_chunk<R, LD>(qrow(a.dst, fresh(c + j), rb), ln.off, ln.act, ln.nsym, acc);
    }
}

// The levels 1 .. LB of the conversion of one block of 2^LB <= 256 rows
// (lg of the rows in a.t) and one column tile, the block held in LDS (row r
// at tile row r, one word pair per lane); wave w owns the rows w + 16 i.
constexpr int CONV_TILE_ROWS = 256;
constexpr int CONV_TILE_THREADS = 1024;

// The What tables of the levels t <= 8 (w_{t-1,m} at 8 (t-1) + m, m < t,
// and 1 / w_{t-1,t-1} at 64 + t - 1): GF(2^16) stages them whole in LDS
// once per workgroup (the division steps are short and dependent, so table
// latency is on their critical path); GF(2^8) reads them from global memory.
constexpr int CONV_TABS = 72;

template <int R> struct ConvTabs;
template <> struct ConvTabs<16> {
    static constexpr int WORDS = CONV_TABS * TAB16;
    const uint32_t *lt;
    __device__ static void stage(uint32_t *lt, const uint32_t *__restrict__ wt, int tid, int nthreads)
    {
        for (int u = tid; u < CONV_TABS * (TAB16 / 4); u += nthreads) {
            const int e = u / (TAB16 / 4), w = u % (TAB16 / 4);
            const int src = e < 64 ? 16 * (e / 8) + e % 8 : 256 + (e - 64);
            *reinterpret_cast<uint4 *>(lt + TAB16 * e + 4 * w) =
                *reinterpret_cast<const uint4 *>(wt + (size_t)TAB16 * src + 4 * w);
        }
    }
    __device__ __forceinline__ Tab16V w(int t, int m) const { return tab_lds_all(lt + TAB16 * (8 * (t - 1) + m)); }
    __device__ __forceinline__ Tab16V inv(int t) const { return tab_lds_all(lt + TAB16 * (64 + t - 1)); }
};
template <> struct ConvTabs<8> {
    static constexpr int WORDS = 0;
    const uint32_t *wt;
    __device__ static void stage(uint32_t *, const uint32_t *__restrict__, int, int) {}
    __device__ __forceinline__ Tab8 w(int t, int m) const { return row_tab<8>(wt, 16 * (t - 1) + m); }
    __device__ __forceinline__ Tab8 inv(int t) const { return row_tab<8>(wt, 256 + (t - 1)); }
};

template <int R>
__device__ __forceinline__ ConvTabs<R> conv_tabs(const uint32_t *lt, const uint32_t *__restrict__ wt)
{
    if constexpr (R == 16)
        return {lt};
    else
        return {wt};
}

template <int R>
struct ConvTile {
    static constexpr int NW = Traits<R>::NW, RS = 64 * NW;
    uint32_t *my;             // this lane's word(s) of tile row 0
    __device__ __forceinline__ void put(int r, const uint32_t *v) const
    {
        if (NW == 2)
            *reinterpret_cast<uint2 *>(my + RS * r) = make_uint2(v[0], v[NW - 1]);
        else
            my[RS * r] = v[0];
    }
    __device__ __forceinline__ void get(int r, uint32_t *v) const
    {
        if (NW == 2) {
            const uint2 t = *reinterpret_cast<const uint2 *>(my + RS * r);
            v[0] = t.x;
            v[NW - 1] = t.y;
        } else {
            v[0] = my[RS * r];
        }
    }
};

// novel -> monomial, levels 1 .. LB of each block: reads the block's rows
// of a.src, writes them to a.dst (which may be a.src).
template <int R, int LD>
__global__ __launch_bounds__(CONV_TILE_THREADS) void k_conv_up_tile(PolyArgs a, const uint32_t *__restrict__ wt)
{
    constexpr int NW = Traits<R>::NW, NI = CONV_TILE_ROWS / 16;
    extern __shared__ uint32_t lds[];
    const int tid = (int)threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const uint32_t blk = blockIdx.x / (uint32_t)a.nct;
    const int ct = (int)(blockIdx.x % (uint32_t)a.nct);
    const Lane ln = lane_of<R, LD>(ct, lane, a.col0, a.ncols);
    const int LB = a.t, B = 1 << LB;
    const uint32_t base = blk << LB;
    const uint64_t rb = a.row_bytes;
    const ConvTile<R> tl = {lds + lane * NW};
    uint32_t *const lt = lds + CONV_TILE_ROWS * 64 * NW;
    ConvTabs<R>::stage(lt, wt, tid, CONV_TILE_THREADS);
    const ConvTabs<R> tabs = conv_tabs<R>(lt, wt);
    uint32_t acc[NI][NW];
#pragma unroll
    for (int i = 0; i < NI; i++) {
        const int r = wave + 16 * i;
        if (r < B) {
            load_chunk<R, LD>(qrow(a.src, fresh(base + (uint32_t)r), rb), ln.off, ln.act, ln.nsym, acc[i]);
            tl.put(r, acc[i]);
        }
    }
    __syncthreads();
    for (int t = 1; t <= LB; t++) {
        const int hh = 1 << (t - 1);
        // out[j] = lo[j] + sum_m w_m hi[j - 2^m] within each block of 2^t rows
#pragma unroll
        for (int i = 0; i < NI; i++) {
            const int r = wave + 16 * i, j = r & (2 * hh - 1);
            if (r < B && j >= hh)
                zero_vec<R>(acc[i]);
        }
        for (int m = 0; m < t; m++) {
            const int s = 1 << m;
            const auto tab = tabs.w(t, m);
#pragma unroll
            for (int i = 0; i < NI; i++) {
                const int r = wave + 16 * i, j = r & (2 * hh - 1);
                if (r < B && j >= s && j - s < hh) {
                    uint32_t v[NW];
                    tl.get(r - j + hh + j - s, v);
                    Ops<R>::mac(acc[i], v, tab);
                }
            }
        }
        __syncthreads();                          // every row of the level read
#pragma unroll
        for (int i = 0; i < NI; i++) {
            const int r = wave + 16 * i;
            if (r < B)
                tl.put(r, acc[i]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < NI; i++) {
        const int r = wave + 16 * i;
        if (r < B)
            store_chunk<R, LD>(qrow(a.dst, fresh(base + (uint32_t)r), rb), ln.off, ln.act, ln.nsym, acc[i]);
    }
}

// monomial -> novel, levels LB .. 1 of each block, in place on a.dst: per
// level the quotient ranges top first, then the remainders, a barrier after
// each (the entries of one range read only entries of higher ranges).
template <int R, int LD>
__global__ __launch_bounds__(CONV_TILE_THREADS) void k_conv_down_tile(PolyArgs a, const uint32_t *__restrict__ wt)
{
    constexpr int NW = Traits<R>::NW, NI = CONV_TILE_ROWS / 16;
    extern __shared__ uint32_t lds[];
    const int tid = (int)threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const uint32_t blk = blockIdx.x / (uint32_t)a.nct;
    const int ct = (int)(blockIdx.x % (uint32_t)a.nct);
    const Lane ln = lane_of<R, LD>(ct, lane, a.col0, a.ncols);
    const int LB = a.t, B = 1 << LB;
    const uint32_t base = blk << LB;
    const uint64_t rb = a.row_bytes;
    const ConvTile<R> tl = {lds + lane * NW};
    uint32_t *const lt = lds + CONV_TILE_ROWS * 64 * NW;
    ConvTabs<R>::stage(lt, wt, tid, CONV_TILE_THREADS);
    const ConvTabs<R> tabs = conv_tabs<R>(lt, wt);
#pragma unroll
    for (int i = 0; i < NI; i++) {
        const int r = wave + 16 * i;
        if (r < B) {
            uint32_t v[NW];
            load_chunk<R, LD>(qrow(a.dst, fresh(base + (uint32_t)r), rb), ln.off, ln.act, ln.nsym, v);
            tl.put(r, v);
        }
    }
    __syncthreads();
    for (int t = LB; t >= 1; t--) {
        const int hh = 1 << (t - 1), nblk = B >> t;
        const auto inv = tabs.inv(t);
        for (int e1 = hh; e1 > 0; e1 >>= 1) {
            const int e0 = e1 >> 1, span = e1 - e0;
            for (int q = wave; q < nblk * span; q += 16) {
                const int c = (q / span) << t, e = e0 + q % span;
                uint32_t acc[NW];
                tl.get(c + hh + e, acc);
                for (int m = 0; m < t - 1; m++) {
                    const int s = 1 << m;
                    if (s > e) {
                        uint32_t v[NW];
                        tl.get(c + hh + e + hh - s, v);
                        Ops<R>::mac(acc, v, tabs.w(t, m));
                    }
                }
                scale<R>(acc, inv);
                tl.put(c + hh + e, acc);
            }
            __syncthreads();
        }
        if (t > 1) {                               // remainders (t = 1: the coefficient itself)
            for (int q = wave; q < nblk * hh; q += 16) {
                const int c = (q / hh) << t, j = q % hh;
                uint32_t acc[NW];
                tl.get(c + j, acc);
                for (int m = 0; m < t - 1; m++) {
                    const int s = 1 << m;
                    if (s <= j) {
                        uint32_t v[NW];
                        tl.get(c + hh + j - s, v);
                        Ops<R>::mac(acc, v, tabs.w(t, m));
                    }
                }
                tl.put(c + j, acc);
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int i = 0; i < NI; i++) {
        const int r = wave + 16 * i;
        if (r < B) {
            uint32_t v[NW];
            tl.get(r, v);
            store_chunk<R, LD>(qrow(a.dst, fresh(base + (uint32_t)r), rb), ln.off, ln.act, ln.nsym, v);
        }
    }
}

// ------------------------------------------------------------------ launchers

enum PolyKernel { PK_PAD = 0, PK_MUL = 1, PK_DEGREE = 2, PK_UP = 3, PK_DOWN = 4, PK_UP_TILE = 5, PK_DOWN_TILE = 6 };

template <int R>
constexpr size_t conv_tile_lds() { return (size_t)4 * (CONV_TILE_ROWS * 64 * Traits<R>::NW + ConvTabs<R>::WORDS); }

template <int R, int LD>
static hipError_t poly_launch_rld(int kind, const PolyArgs &a, const uint32_t *t1, const uint32_t *t2,
                                  uint32_t nblocks, hipStream_t s)
{
    if (nblocks == 0)
        return hipSuccess;
    switch (kind) {
    case PK_PAD: hipLaunchKernelGGL((k_poly_pad<R, LD>), dim3(nblocks), dim3(64), 0, s, a); break;
    case PK_MUL: hipLaunchKernelGGL((k_poly_mul<R, LD>), dim3(nblocks), dim3(64), 0, s, a, t1, t2); break;
    case PK_DEGREE: hipLaunchKernelGGL((k_poly_degree<R, LD>), dim3(nblocks), dim3(256), 0, s, a); break;
    case PK_UP: hipLaunchKernelGGL((k_conv_up<R, LD>), dim3(nblocks), dim3(64), 0, s, a, t1); break;
    case PK_DOWN: hipLaunchKernelGGL((k_conv_down<R, LD>), dim3(nblocks), dim3(64), 0, s, a, t1); break;
    case PK_UP_TILE:
        hipLaunchKernelGGL((k_conv_up_tile<R, LD>), dim3(nblocks), dim3(CONV_TILE_THREADS), conv_tile_lds<R>(), s, a,
                           t1);
        break;
    case PK_DOWN_TILE:
        hipLaunchKernelGGL((k_conv_down_tile<R, LD>), dim3(nblocks), dim3(CONV_TILE_THREADS), conv_tile_lds<R>(), s,
                           a, t1);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// kind: PK_*; t1, t2: the log and exp tables (PK_MUL) or the What tables
// (PK_UP, PK_DOWN); nblocks as each kernel expects.
template <int R, int LD>
static hipError_t conv_prep_rld()
{
    hipError_t e = hipFuncSetAttribute((const void *)k_conv_up_tile<R, LD>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)conv_tile_lds<R>());
    const hipError_t f = hipFuncSetAttribute((const void *)k_conv_down_tile<R, LD>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)conv_tile_lds<R>());
    return e != hipSuccess ? e : f;
}

// LDS limits of the block-tile conversion kernels (once per device).
hipError_t poly_prepare()
{
    hipError_t e = hipSuccess, f;
    if ((f = conv_prep_rld<16, LD_VEC>()) != hipSuccess) e = f;
    if ((f = conv_prep_rld<16, LD_SYM>()) != hipSuccess) e = f;
    if ((f = conv_prep_rld<8, LD_VEC>()) != hipSuccess) e = f;
    if ((f = conv_prep_rld<8, LD_SYM>()) != hipSuccess) e = f;
    return e;
}

hipError_t poly_launch(int r, int ld, int kind, const PolyArgs &a, const uint32_t *t1, const uint32_t *t2,
                       uint32_t nblocks, hipStream_t s)
{
    if (r == 16)
        return ld == LD_VEC ? poly_launch_rld<16, LD_VEC>(kind, a, t1, t2, nblocks, s)
                            : poly_launch_rld<16, LD_SYM>(kind, a, t1, t2, nblocks, s);
    return ld == LD_VEC ? poly_launch_rld<8, LD_VEC>(kind, a, t1, t2, nblocks, s)
                        : poly_launch_rld<8, LD_SYM>(kind, a, t1, t2, nblocks, s);
}

}  // namespace nb
