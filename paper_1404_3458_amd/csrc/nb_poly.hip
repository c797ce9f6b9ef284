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

// ------------------------------------------------------------------ launchers

enum PolyKernel { PK_PAD = 0, PK_MUL = 1, PK_DEGREE = 2, PK_UP = 3, PK_DOWN = 4 };

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
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// kind: PK_*; t1, t2: the log and exp tables (PK_MUL) or the What tables
// (PK_UP, PK_DOWN); nblocks as each kernel expects.
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
