// nb_device.hpp -- device primitives for the gfx950 codec kernels.
//
// Data layout in registers ("byte-sliced"): a lane owns 4 adjacent columns of
// a row.  For r = 16 the 4 symbols are held as two dwords, L = their four low
// bytes and H = their four high bytes; for r = 8 one dword holds the four
// byte symbols.  Field addition is XOR on these words.
//
// Multiplication by a constant s that every column of a row shares (the skew
// factors of Sec. 3.2, the B table of Sec. 4.2, the locator values of the
// appendix) uses v_perm_b32 as an 8-entry byte lookup: each byte of a symbol
// is split into bit groups of 3, 3 and 2 bits, and s * (group << offset) is
// looked up per group and per output byte, then XOR-ed (the product is
// GF(2)-linear in the multiplicand).  A constant's lookup tables ("perm
// table") take 20 dwords for r = 16 and 5 (stored as 8) for r = 8.
//
// v_perm_b32 reads 8 table bytes from a (hi, lo) dword pair and can take only
// one scalar operand, so every 3-bit group table has one word that must sit
// in a vector register (its entries 0-3, "V words") and one that can stay
// scalar (entries 4-7, "S words"); the 2-bit group tables have 4 entries and
// are one S word, with the selector itself as the ignored high operand.
// Layout, r = 16 (tables numbered by input byte L/H, group, output byte):
//   [0..7]   V words: gL0->L, gL0->H, gL1->L, gL1->H, gH0->L, gH0->H, gH1->L, gH1->H
//   [8..15]  S words of the same eight tables, same order
//   [16..19] 2-bit tables: gL2->L, gL2->H, gH2->L, gH2->H
// r = 8: [0..1] V words of g0, g1; [2..3] their S words; [4] the 2-bit table.
// Entry e of a table occupies byte (e mod 4) of the word holding it.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nb {

constexpr int TAB16 = 20;   // dwords per perm table, r = 16
constexpr int TAB8 = 8;     // dwords per perm table, r = 8 (5 used)

template <int R> struct Traits;
template <> struct Traits<16> { static constexpr int NW = 2, TS = TAB16, SYM = 2; };
template <> struct Traits<8> { static constexpr int NW = 1, TS = TAB8, SYM = 1; };

__host__ __device__ inline uint32_t field_poly(int r) { return r == 8 ? 0x11Du : 0x1100Bu; }

// a * x in GF(2^r)
__host__ __device__ inline uint32_t gf_times_x(uint32_t a, int r)
{
    a <<= 1;
    return ((a >> r) & 1u) ? (a ^ field_poly(r)) : a;
}

// General product, right-to-left over the bits of b with the multiplicand
// doubled (and reduced) at each step.  Used only by table builders.
__host__ __device__ inline uint32_t gf_mul(uint32_t a, uint32_t b, int r)
{
    uint32_t acc = 0;
    while (b) {
        if (b & 1u)
            acc ^= a;
        a = gf_times_x(a, r);
        b >>= 1;
    }
    return acc;
}

__host__ __device__ inline uint32_t gf_pow(uint32_t a, uint32_t e, int r)
{
    uint32_t acc = 1;
    while (e) {
        if (e & 1u)
            acc = gf_mul(acc, a, r);
        a = gf_mul(a, a, r);
        e >>= 1;
    }
    return acc;
}

// Inverse through Fermat: a^(2^r - 2).
__host__ __device__ inline uint32_t gf_inv(uint32_t a, int r)
{
    return gf_pow(a, (1u << r) - 2u, r);
}

// Build the perm table of constant s (layout in the file comment); R fixed
// at compile time, so that every loop unrolls and a local `out` stays in
// registers.
template <int R>
__device__ __forceinline__ void build_perm_table_r(uint32_t s, uint32_t *out)
{
    uint32_t px[R];                  // s * x^t
    px[0] = s;
#pragma unroll
    for (int t = 1; t < R; t++)
        px[t] = gf_times_x(px[t - 1], R);
    constexpr int nbytes = R / 8;
#pragma unroll
    for (int b = 0; b < nbytes; b++) {
#pragma unroll
        for (int g = 0; g < 3; g++) {
            const int nbits = g == 2 ? 2 : 3;
            const int shift = 8 * b + 3 * g;
            uint32_t lo_out[2] = {0, 0}, hi_out[2] = {0, 0};
#pragma unroll
            for (int e = 0; e < (1 << nbits); e++) {
                uint32_t prod = 0;
#pragma unroll
                for (int u = 0; u < nbits; u++)
                    if ((e >> u) & 1)
                        prod ^= px[shift + u];
                lo_out[e >> 2] |= (prod & 0xFFu) << (8 * (e & 3));
                hi_out[e >> 2] |= ((prod >> 8) & 0xFFu) << (8 * (e & 3));
            }
            if (R == 16) {
                if (g < 2) {
                    const int v = 4 * b + 2 * g;          // table index among the eight
                    out[v] = lo_out[0];
                    out[8 + v] = lo_out[1];
                    out[v + 1] = hi_out[0];
                    out[8 + v + 1] = hi_out[1];
                } else {
                    out[16 + 2 * b] = lo_out[0];
                    out[16 + 2 * b + 1] = hi_out[0];
                }
            } else {
                if (g < 2) {
                    out[g] = lo_out[0];
                    out[2 + g] = lo_out[1];
                } else {
                    out[4] = lo_out[0];
                }
            }
        }
    }
    if (R == 8) {
        out[5] = out[6] = out[7] = 0;
    }
}

__device__ inline void build_perm_table(uint32_t s, int r, uint32_t *out)
{
    if (r == 16)
        build_perm_table_r<16>(s, out);
    else
        build_perm_table_r<8>(s, out);
}

// The perm table of s built in registers and stored at out (16-byte aligned)
// as 16-byte pieces.
template <int R>
__device__ __forceinline__ void store_perm_table(uint32_t s, uint32_t *out)
{
    constexpr int TS = R == 16 ? 20 : 8;
    uint32_t t[TS];
    build_perm_table_r<R>(s, t);
#pragma unroll
    for (int i = 0; i < TS / 4; i++)
        reinterpret_cast<uint4 *>(out)[i] = make_uint4(t[4 * i], t[4 * i + 1], t[4 * i + 2], t[4 * i + 3]);
}

// ---------------------------------------------------------------- hot ops

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ uint32_t prm(uint32_t hi, uint32_t lo, uint32_t sel)
{
    return __builtin_amdgcn_perm(hi, lo, sel);
}

constexpr int VW16 = 8;     // V words per table, r = 16
constexpr int VW8 = 2;      // V words per table, r = 8

constexpr int SW16 = 12;    // S words per table, r = 16
constexpr int SW8 = 3;      // S words per table, r = 8

// A constant's perm table as the multiply reads it: the V words in vector
// registers (read from LDS, or copied from scalar registers) and the S words
// in scalar registers (uniform loads).
template <int NV, int NS>
struct TabT {
    uint32_t v[NV];
    uint32_t s[NS];
};
typedef TabT<VW16, SW16> Tab16;
typedef TabT<VW8, SW8> Tab8;

// a ^= s * b for 4 symbols, r = 16 (S word u is table word 8 + u).
__device__ __forceinline__ void mac16(uint32_t &aL, uint32_t &aH, uint32_t bL, uint32_t bH, const Tab16 &T)
{
    const uint32_t m3 = 0x07070707u, m2 = 0x03030303u;
    const uint32_t s0 = bL & m3, s1 = (bL >> 3) & m3, s2 = (bL >> 6) & m2;
    const uint32_t s3 = bH & m3, s4 = (bH >> 3) & m3, s5 = (bH >> 6) & m2;
    const uint32_t *v = T.v, *t = T.s;
    aL = xor3(aL, prm(t[0], v[0], s0), prm(t[2], v[2], s1));
    aH = xor3(aH, prm(t[1], v[1], s0), prm(t[3], v[3], s1));
    aL = xor3(aL, prm(s2, t[8], s2), prm(t[4], v[4], s3));
    aH = xor3(aH, prm(s2, t[9], s2), prm(t[5], v[5], s3));
    aL = xor3(aL, prm(t[6], v[6], s4), prm(s5, t[10], s5));
    aH = xor3(aH, prm(t[7], v[7], s4), prm(s5, t[11], s5));
}

// a ^= s * b for 4 symbols, r = 8 (S word u is table word 2 + u).
__device__ __forceinline__ void mac8(uint32_t &a, uint32_t b, const Tab8 &T)
{
    const uint32_t m3 = 0x07070707u, m2 = 0x03030303u;
    const uint32_t s0 = b & m3, s1 = (b >> 3) & m3, s2 = (b >> 6) & m2;
    a = xor3(a, prm(T.s[0], T.v[0], s0), prm(T.s[1], T.v[1], s1));
    a ^= prm(s2, T.s[2], s2);
}

// Table read whole from global memory with uniform loads.
template <int NV, int NS>
__device__ __forceinline__ TabT<NV, NS> tab_global(const uint32_t *__restrict__ t)
{
    TabT<NV, NS> r;
#pragma unroll
    for (int u = 0; u < NV; u++)
        r.v[u] = t[u];
#pragma unroll
    for (int u = 0; u < NS; u++)
        r.s[u] = t[NV + u];
    return r;
}

// Table with the V words read from LDS (all lanes read the same address) and
// the S words read from global memory with uniform loads.
template <int NV, int NS>
__device__ __forceinline__ TabT<NV, NS> tab_lds(const uint32_t *lds_v, const uint32_t *__restrict__ t)
{
    TabT<NV, NS> r;
    if (NV == 8) {
        const uint4 a = *reinterpret_cast<const uint4 *>(lds_v);
        const uint4 b = *reinterpret_cast<const uint4 *>(lds_v + 4);
        r.v[0] = a.x; r.v[1] = a.y; r.v[2] = a.z; r.v[3] = a.w;
        r.v[NV > 4 ? 4 : 0] = b.x; r.v[NV > 5 ? 5 : 0] = b.y; r.v[NV > 6 ? 6 : 0] = b.z; r.v[NV > 7 ? 7 : 0] = b.w;
    } else {
        const uint2 a = *reinterpret_cast<const uint2 *>(lds_v);
        r.v[0] = a.x;
        r.v[NV > 1 ? 1 : 0] = a.y;
    }
#pragma unroll
    for (int u = 0; u < NS; u++)
        r.s[u] = t[NV + u];
    return r;
}

// Marks a table as needed here: its loads complete at this point of the
// program (a wait is placed here), not where the multiply first uses it.
template <int NV, int NS>
__device__ __forceinline__ void touch(const TabT<NV, NS> &T)
{
    if (NV == 8)
        asm volatile("" ::"v"(T.v[0]), "v"(T.v[1]), "v"(T.v[2 % NV]), "v"(T.v[3 % NV]), "v"(T.v[4 % NV]),
                     "v"(T.v[5 % NV]), "v"(T.v[6 % NV]), "v"(T.v[7 % NV]));
    else
        asm volatile("" ::"v"(T.v[0]), "v"(T.v[NV - 1]));
#pragma unroll
    for (int u = 0; u < NS; u++)
        asm volatile("" ::"s"(T.s[u]));
}

template <int R> struct Ops;

// A GF(2^16) perm table whose every word is a per-lane value (both halves
// of a wave may multiply by different constants): read whole from LDS, the
// "S words" then sit in vector registers too.  The multiply is unchanged;
// only the registers its operands live in differ.
struct Tab16V : Tab16 {
};

__device__ __forceinline__ void touch(const Tab16V &T)
{
    asm volatile("" ::"v"(T.v[0]), "v"(T.v[1]), "v"(T.v[2]), "v"(T.v[3]), "v"(T.v[4]), "v"(T.v[5]), "v"(T.v[6]),
                 "v"(T.v[7]));
    asm volatile("" ::"v"(T.s[0]), "v"(T.s[1]), "v"(T.s[2]), "v"(T.s[3]), "v"(T.s[4]), "v"(T.s[5]), "v"(T.s[6]),
                 "v"(T.s[7]), "v"(T.s[8]), "v"(T.s[9]), "v"(T.s[10]), "v"(T.s[11]));
}

// All TAB16 words of a table staged in LDS (16-byte aligned), per lane.
__device__ __forceinline__ Tab16V tab_lds_all(const uint32_t *p)
{
    Tab16V r;
    const uint4 a = *reinterpret_cast<const uint4 *>(p);
    const uint4 b = *reinterpret_cast<const uint4 *>(p + 4);
    const uint4 c = *reinterpret_cast<const uint4 *>(p + 8);
    const uint4 d = *reinterpret_cast<const uint4 *>(p + 12);
    const uint4 e = *reinterpret_cast<const uint4 *>(p + 16);
    r.v[0] = a.x; r.v[1] = a.y; r.v[2] = a.z; r.v[3] = a.w;
    r.v[4] = b.x; r.v[5] = b.y; r.v[6] = b.z; r.v[7] = b.w;
    r.s[0] = c.x; r.s[1] = c.y; r.s[2] = c.z; r.s[3] = c.w;
    r.s[4] = d.x; r.s[5] = d.y; r.s[6] = d.z; r.s[7] = d.w;
    r.s[8] = e.x; r.s[9] = e.y; r.s[10] = e.z; r.s[11] = e.w;
    return r;
}

template <> struct Ops<16> {
    static constexpr int NW = 2, NV = VW16, NS = SW16;
    typedef Tab16 Tab;
    __device__ static __forceinline__ Tab prep(const uint32_t *t) { return tab_global<NV, NS>(t); }
    __device__ static __forceinline__ Tab prep_lds(const uint32_t *v, const uint32_t *t) { return tab_lds<NV, NS>(v, t); }
    __device__ static __forceinline__ void mac(uint32_t *a, const uint32_t *b, const Tab &T)
    {
        mac16(a[0], a[1], b[0], b[1], T);
    }
    // packed symbols (two little-endian u16 per dword) -> byte-sliced
    __device__ static __forceinline__ void unpack(uint32_t w0, uint32_t w1, uint32_t *v)
    {
        v[0] = prm(w1, w0, 0x06040200u);
        v[1] = prm(w1, w0, 0x07050301u);
    }
    __device__ static __forceinline__ void pack(const uint32_t *v, uint32_t &w0, uint32_t &w1)
    {
        w0 = prm(v[1], v[0], 0x05010400u);
        w1 = prm(v[1], v[0], 0x07030602u);
    }
};

template <> struct Ops<8> {
    static constexpr int NW = 1, NV = VW8, NS = SW8;
    typedef Tab8 Tab;
    __device__ static __forceinline__ Tab prep(const uint32_t *t) { return tab_global<NV, NS>(t); }
    __device__ static __forceinline__ Tab prep_lds(const uint32_t *v, const uint32_t *t) { return tab_lds<NV, NS>(v, t); }
    __device__ static __forceinline__ void mac(uint32_t *a, const uint32_t *b, const Tab &T)
    {
        mac8(a[0], b[0], T);
    }
};

// Global-address-space views of row pointers: loads and stores then use an
// SGPR row base plus a 32-bit VGPR lane offset (and immediate offsets)
// instead of 64-bit flat addresses.
typedef __attribute__((address_space(1))) uint8_t gu8;
typedef __attribute__((address_space(1))) uint16_t gu16;
typedef __attribute__((address_space(1))) uint32_t gu32;
typedef __attribute__((address_space(1))) uint64_t gu64;
// The same accesses at any symbol alignment: the ROCm runtime runs global
// memory in unaligned-access mode, so an 8-byte (4-byte) access at a 2-byte
// (1-byte) aligned address is one global_load/store_dwordx2 (dword) of
// exactly the bytes named.
typedef uint64_t __attribute__((aligned(2))) u64_a2;
typedef uint32_t __attribute__((aligned(1))) u32_a1;
typedef __attribute__((address_space(1))) u64_a2 gu64_a2;
typedef __attribute__((address_space(1))) u32_a1 gu32_a1;

// How a lane reaches its 4 symbols of a row:
//   LD_VEC  one 8-byte (r = 16) or 4-byte (r = 8) access; rows are aligned
//           and only full chunks are touched;
//   LD_SYM  only symbol alignment is required: a full chunk is one access at
//           symbol alignment, the last partial chunk one access per symbol,
//           bounded by nsym.
enum { LD_VEC = 0, LD_SYM = 1 };

// Uniform value the compiler must treat as freshly computed, so that row
// pointers derived from it are rebuilt where used instead of being kept
// live in scalar registers from one phase of a kernel to the next.
__device__ __forceinline__ uint32_t fresh(uint32_t v)
{
    v = __builtin_amdgcn_readfirstlane(v);
    asm volatile("" : "+s"(v));
    return v;
}

// Marks the values of v as computed at this point of the program: a later
// fresh() (from which table addresses are derived) is ordered after it, so
// a table fetch placed after the marker cannot be issued before the work
// that produced v, which bounds how many tables are in flight.
template <int NW>
__device__ __forceinline__ void pin(const uint32_t *v)
{
    if (NW == 2)
        asm volatile("" ::"v"(v[0]), "v"(v[NW - 1]));
    else
        asm volatile("" ::"v"(v[0]));
}

// Each 16-bit half of v replaced by all ones if its top bit is set, else 0
// (a packed arithmetic shift by 15; op_sel_hi:[0,1] makes the high half also
// take its shift count from the low half of the inline constant.  Written
// out so that the compiler keeps the masks as data rather than turning the
// ANDs below into selects).
__device__ __forceinline__ uint32_t top_mask16x2(uint32_t v)
{
    uint32_t r;
    asm("v_pk_ashrrev_i16 %0, 15, %1 op_sel_hi:[0,1]" : "=v"(r) : "v"(v));
    return r;
}

// Products of the GF(2^16) symbols in the two 16-bit halves of a and b:
// shift and add over the bits of b, highest first, reducing by
// x^16 = x^12 + x^3 + x + 1 after every shift (about 6 lane-ops per bit for
// both halves, no memory traffic; both factors vary, so the per-constant
// lookup tables of the transforms do not apply).
// U: unroll factor of the 16 steps (a caller that multiplies many rows
// inside an unrolled loop keeps the steps rolled, or that loop would be left
// rolled and its register arrays moved to scratch memory).
template <int U = 16>
__device__ __forceinline__ uint32_t gf16_mul2(uint32_t a, uint32_t b)
{
    typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
    uint32_t acc = 0u, bv = b;
#pragma unroll U
    for (int i = 0; i < 16; i++) {
        const uint32_t carry = top_mask16x2(acc);
        acc = __builtin_bit_cast(uint32_t, (u16x2)(__builtin_bit_cast(u16x2, acc) << 1)) ^ (carry & 0x100B100Bu);
        acc ^= a & top_mask16x2(bv);
        bv = __builtin_bit_cast(uint32_t, (u16x2)(__builtin_bit_cast(u16x2, bv) << 1));
    }
    return acc;
}

// x (4 GF(2^16) symbols, byte-sliced) <- x times y symbol by symbol.
template <int U = 16>
__device__ __forceinline__ void mul_symbols16(uint32_t *x, const uint32_t *y)
{
    uint32_t xw0, xw1, yw0, yw1;
    Ops<16>::pack(x, xw0, xw1);
    Ops<16>::pack(y, yw0, yw1);
    Ops<16>::unpack(gf16_mul2<U>(xw0, yw0), gf16_mul2<U>(xw1, yw1), x);
}

// Completion stamp of a workgroup: when an object of this type goes out of
// scope (every return of a kernel), the first lane of each wave raises
// slots[blockIdx.x] to the device's real-time counter with a vector atomic,
// so that the slot ends as the time its last wave finished.  Every
// workgroup has a slot of its own (atomics on one address serialize).
struct DoneStamp {
    uint64_t *slots;
    __device__ __forceinline__ ~DoneStamp()
    {
        if (slots && (threadIdx.x & 63u) == 0u)
            atomicMax((unsigned long long *)(slots + blockIdx.x), (unsigned long long)__builtin_amdgcn_s_memrealtime());
    }
};

// Step k of the loop is instantiated once per k (template recursion rather
// than an unroll pragma, which the compiler may decline for long loops; a
// loop left rolled would index the register arrays at run time and move them
// to scratch memory).
template <class Tab, int K, int N>
struct PipeStep {
    template <class F, class W>
    __device__ static __forceinline__ void run(const F &fetch, const W &work, Tab &cur)
    {
        // wait for table K (fetched a block ago) before issuing table K + 1,
        // so that the wait, which covers every outstanding scalar and LDS
        // load, never includes the fetch that should overlap block K
        touch(cur);
        asm volatile("" ::: "memory");
        Tab nxt = cur;
        if (K + 1 < N)
            nxt = fetch(K + 1);
        asm volatile("" ::: "memory");
        work(K, cur);
        cur = nxt;
        PipeStep<Tab, K + 1, N>::run(fetch, work, cur);
    }
};
template <class Tab, int N>
struct PipeStep<Tab, N, N> {
    template <class F, class W>
    __device__ static __forceinline__ void run(const F &, const W &, Tab &)
    {
    }
};

// Runs work(k, table_k) for k < N with table k + 1 fetched before work k, so
// that one table fetch is in flight while a block is computed; work ends
// with pin() on what it produced.
// Two tables in flight: table K + 2 is fetched while block K is computed and
// table K + 1 is still arriving (per-lane tables come from LDS, five loads
// each, in waves that have few others to hide their latency behind).
template <class Tab, int K, int N>
struct PipeStep2 {
    template <class F, class W>
    __device__ static __forceinline__ void run(const F &fetch, const W &work, Tab &cur, Tab &nxt)
    {
        touch(cur);
        asm volatile("" ::: "memory");
        Tab far = cur;
        if (K + 2 < N)
            far = fetch(K + 2);
        asm volatile("" ::: "memory");
        work(K, cur);
        PipeStep2<Tab, K + 1, N>::run(fetch, work, nxt, far);
    }
};
template <class Tab, int N>
struct PipeStep2<Tab, N, N> {
    template <class F, class W>
    __device__ static __forceinline__ void run(const F &, const W &, Tab &, Tab &)
    {
    }
};

template <class Tab> struct PipeDepth { static constexpr int D = 1; };
template <> struct PipeDepth<Tab16V> { static constexpr int D = 2; };

template <class Tab, int N, class F, class W>
__device__ __forceinline__ void pipelined(const F &fetch, const W &work)
{
    if constexpr (PipeDepth<Tab>::D == 2 && N > 1) {
        Tab cur = fetch(0);
        Tab nxt = fetch(1);
        PipeStep2<Tab, 0, N>::run(fetch, work, cur, nxt);
    } else {
        Tab cur = fetch(0);
        PipeStep<Tab, 0, N>::run(fetch, work, cur);
    }
}

// Load this lane's chunk (byte offset `off` in the row) into byte-sliced
// registers; inactive lanes and symbols >= nsym read zero.  NT: a streamed
// input the launch reads once; a full GF(2^16) chunk is then read
// non-temporally, so that it does not push the tables the launch keeps
// re-reading out of L2.
template <int R, int LD, bool NT = false>
__device__ __forceinline__ void load_chunk(const uint8_t *row_, uint32_t off, bool act, int nsym, uint32_t *v)
{
    const gu8 *row = (const gu8 *)row_ + off;
    // LD_SYM: a full chunk in one access at symbol alignment; a partial one
    // per symbol
    if (R == 16) {
        uint32_t w0 = 0, w1 = 0;
        if (act) {
            if (LD == LD_VEC) {
                const uint64_t t = NT ? __builtin_nontemporal_load((const gu64 *)row) : *(const gu64 *)row;
                w0 = (uint32_t)t;
                w1 = (uint32_t)(t >> 32);
            } else if (nsym == 4) {
                const uint64_t t = NT ? __builtin_nontemporal_load((const gu64_a2 *)row) : *(const gu64_a2 *)row;
                w0 = (uint32_t)t;
                w1 = (uint32_t)(t >> 32);
            } else {
                const gu16 *r16 = (const gu16 *)row;
                const uint32_t s0 = r16[0];
                const uint32_t s1 = nsym > 1 ? (uint32_t)r16[1] : 0u;
                const uint32_t s2 = nsym > 2 ? (uint32_t)r16[2] : 0u;
                w0 = s0 | (s1 << 16);
                w1 = s2;
            }
        }
        Ops<16>::unpack(w0, w1, v);
    } else {
        uint32_t w = 0;
        if (act) {
            if (LD == LD_VEC) {
                w = *(const gu32 *)row;
            } else if (nsym == 4) {
                w = *(const gu32_a1 *)row;
            } else {
                w = row[0];
                if (nsym > 1) w |= (uint32_t)row[1] << 8;
                if (nsym > 2) w |= (uint32_t)row[2] << 16;
            }
        }
        v[0] = w;
    }
}
// NT: a streamed output that nothing in the launch reads again; a full
// GF(2^16) chunk is then stored non-temporally, so that it does not push
// the tables the launch keeps re-reading out of L2.
template <int R, int LD, bool NT = false>
__device__ __forceinline__ void store_chunk(uint8_t *row_, uint32_t off, bool act, int nsym, const uint32_t *v)
{
    if (!act)
        return;
    gu8 *row = (gu8 *)row_ + off;
    if (R == 16) {
        uint32_t w0, w1;
        Ops<16>::pack(v, w0, w1);
        if (LD == LD_VEC) {
            const uint64_t t = (uint64_t)w0 | ((uint64_t)w1 << 32);
            if (NT)
                __builtin_nontemporal_store(t, (gu64 *)row);
            else
                *(gu64 *)row = t;
        } else if (nsym == 4) {
            const uint64_t t = (uint64_t)w0 | ((uint64_t)w1 << 32);
            if (NT)
                __builtin_nontemporal_store(t, (gu64_a2 *)row);
            else
                *(gu64_a2 *)row = t;
        } else {
            gu16 *r16 = (gu16 *)row;
            r16[0] = (uint16_t)w0;
            if (nsym > 1) r16[1] = (uint16_t)(w0 >> 16);
            if (nsym > 2) r16[2] = (uint16_t)w1;
        }
    } else {
        const uint32_t w = v[0];
        if (LD == LD_VEC) {
            *(gu32 *)row = w;
        } else if (nsym == 4) {
            *(gu32_a1 *)row = w;
        } else {
            row[0] = (uint8_t)w;
            if (nsym > 1) row[1] = (uint8_t)(w >> 8);
            if (nsym > 2) row[2] = (uint8_t)(w >> 16);
        }
    }
}
// Per-lane view of a tile: byte offset of the lane's chunk, whether the lane
// holds real columns, and how many of its 4 symbols exist.
struct Lane {
    uint32_t off;
    bool act;
    int nsym;
};

// Chunk q of a launch covers columns col0 + 4q .. col0 + 4q + 3.  LD_VEC
// launches only touch chunks that lie entirely below ncols; LD_SYM launches
// also serve the last partial chunk.
template <int R, int LD>
__device__ __forceinline__ Lane lane_of(int tile_rel, int lane, int col0, int ncols)
{
    Lane ln;
    constexpr uint32_t SB = R / 8;
    const int c = col0 + 4 * (tile_rel * 64 + lane);
    ln.off = (uint32_t)c * SB;
    ln.nsym = ncols - c < 4 ? ncols - c : 4;
    ln.act = LD == LD_VEC ? ln.nsym == 4 : ln.nsym > 0;
    return ln;
}

}  // namespace nb
