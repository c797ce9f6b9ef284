// nb_internal.hpp -- structures shared by the host launcher code and the
// kernels of librs_nb.so (not part of the public ABI).
//
// Read-only tables reach the kernels as separate __restrict__ pointer
// parameters (never through memory), so the compiler can prove that the
// kernel's own stores do not clobber them and fetches the wave-uniform
// entries with scalar loads.  Per-stripe masks and locator tables are
// addressed by offsets from such parameters for the same reason.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace nb {

// Device-resident method tables (built once by rs_init).
struct Tabs {
    const uint32_t *__restrict__ tw;     // perm tables of the skew factors, 2^r - 1 entries
    const uint32_t *__restrict__ B;      // perm tables of B_j, 2^r entries (Sec. 4.2, eq. B)
    const uint32_t *__restrict__ Binv;   // perm tables of 1 / B_j
};

// Host-side bundle of every read-only pointer a kernel receives as a
// separate parameter.
struct KPtrs {
    const uint32_t *tw, *B, *Binv;
    const uint32_t *bits;      // decode: point bitmaps, stripe s at DevStripe::bits_off
    const uint32_t *rowtabs;   // decode: locator perm tables, stripe s at DevStripe::rowtab_off
};

// One stripe of a launch.  A tile is 256 columns (64 lanes x 4 columns)
// starting at column col0 + 256 * (tile - tile0).
struct DevStripe {
    const uint8_t *in;        // encode: k message rows; decode: n shard rows; xform: data
    uint8_t *out;             // encode: n - k parity rows; decode: n rows; xform: data
    uint64_t bits_off;        // decode: dword offset of the point bitmaps: W = ceil(n'/32)
                              // words "received" (point has a surviving stored row),
                              // then W words "erased" (point has an erased stored row)
    uint64_t rowtab_off;      // decode: dword offset of the n' per-point perm tables
    uint64_t row_bytes;
    int32_t n, k, kp, np;     // stored shape and mother shape
    int32_t ncols;            // symbols per row
    int32_t tile0;            // index of this stripe's first tile in the launch
    int32_t col0;             // first column covered by this launch
    int32_t copy_survivors;   // decode with out != in
    int32_t sid;              // index of the stripe in the call (completion timestamps)
};

struct FusedArgs {
    const DevStripe *stripes;
    int32_t nstripes;
    uint32_t l;               // shift of the plain transforms
    uint64_t *ts;             // completion stamp slots of this launch (one per workgroup), or null
};

// Multi-pass (h > 256) kernels: one launch applies up to 4 levels.  The
// grid is 1-D: block b handles group b / nct and column tile b % nct.
struct PassArgs {
    const uint8_t *src;       // rows read (row p; rows >= src_rows read as zero)
    uint8_t *dst;             // rows written (row p -> dst row p - dst_lo if in range)
    uint64_t row_bytes;
    int32_t src_rows;
    int32_t dst_lo, dst_hi;
    int32_t ncols;
    int32_t lo;               // lowest level of this pass
    int32_t col0;             // first column covered by this launch
    uint32_t l;
    int32_t nct;              // column tiles (of 256 columns) per group
    int32_t pre_B;            // multiply rows by B_p before the levels
    int32_t post_B;           // multiply rows by B_p after the levels
    const uint8_t *mul;       // GF(2^16): output row p times row p of mul, symbol by symbol (null: none)
};

// Polynomial operations of Sec. 6.1, Table 1 (nb_poly.hip): padding, point-by-point
// product, degree and basis conversion; each kernel reads the fields it needs.
struct PolyArgs {
    const uint8_t *src;       // rows read
    const uint8_t *src2;      // the second operand (point-by-point product)
    uint8_t *dst;             // rows written
    int32_t *deg;             // degree, one entry per column
    uint64_t row_bytes;
    int32_t ncols, col0, nct; // columns, first column of the launch, its column tiles
    int32_t rows;             // rows of the operation
    int32_t src_rows;         // padding: rows copied, the rest written as zero
    int32_t t;                // conversion level (blocks of 2^t rows)
    int32_t e0, e1;           // division: quotient entries [e0, e1) of each block; e1 == 0: the remainder
};

// Derivative partial pass (Sec. 4.2 split over level ranges): for the rows
// p of each group, z_p (+)= sum of y_{p + 2^l} over the levels l of the pass
// with bit l of p clear.  first: z is written instead of accumulated.
// last: the total is multiplied by 1 / B_p and written to `out`.
struct DerivPassArgs {
    const uint8_t *y;
    uint8_t *z;
    uint8_t *out;
    uint64_t row_bytes;
    int32_t ncols, lo, nct;   // nct: column tiles per group
    int32_t col0, first, last;
};

// One stripe (column part) of a launch of 8-level passes over a transform of
// n' or k' = 2^N > 256 points.  Groups are 2^T rows gbase + (j << lo) of the
// transform; tile t of the launch is group (t - tile0) / nct, column tile
// (t - tile0) % nct.
struct WideStripe {
    DevStripe st;             // decode: shards, output, point bitmaps and tables
    const uint8_t *src;       // rows read (row = point index); rows >= src_rows read as zero
    uint8_t *dst;             // rows written; rows >= dst_rows are not written
    const uint8_t *src2;      // decode derivative: partial sums read (W_D3, W_DPM) or the low part's rows A (W_DL)
    uint8_t *dst2;            // decode derivative: partial sums written; encode: coefficients kept
    int32_t src_rows, dst_rows;
    int32_t tile0, nct;
};

struct WideArgs {
    const WideStripe *stripes;
    int32_t nstripes;
    int32_t lo;               // groups are rows gbase + (j << lo)
    int32_t blk;              // encode: parity block, transformed at shift blk * k'
    uint32_t l;               // plain transform passes: the shift
    uint64_t *ts;             // completion stamp slots of this launch (one per workgroup), or null
};

// One pass of the multi-workgroup locator of one stripe (k_loc_pass).
struct LocPassArgs {
    const DevStripe *stripe;
    uint32_t *v;              // n' residues
    int32_t r, lo, T, kind;
};

struct LocatorArgs {
    const DevStripe *stripes;
    int r;
};

}  // namespace nb
