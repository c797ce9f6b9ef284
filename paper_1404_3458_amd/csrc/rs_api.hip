// rs_api.hip -- host side of librs_nb.so: context and tables, argument
// validation, per-stream scratch, launch planning (fused kernels for
// transform sizes <= 256, multi-pass kernels above), and the C ABI of
// include/rs.h.
#include "rs.h"
#include "nb_device.hpp"
#include "nb_internal.hpp"

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <mutex>
#include <new>
#include <vector>

#include <emmintrin.h>

namespace nb {
hipError_t init_tables(int r, const uint32_t *d_basis, uint32_t *d_Wv, uint32_t *d_S, uint32_t *d_wp,
                       uint32_t *d_skew, uint32_t *d_B, uint32_t *d_Binv, uint32_t *d_exp, uint32_t *d_log,
                       uint32_t *d_FL, uint32_t *d_tw_tab, uint32_t *d_B_tab, uint32_t *d_Binv_tab,
                       hipStream_t s);
hipError_t init_prepare(int r);
hipError_t locator_launch(const LocatorArgs &a, const KPtrs &k, const uint32_t *fwht_L, const uint32_t *expt,
                          int nstripes, int max_np, hipStream_t s);
hipError_t loc_pass_launch(const LocPassArgs &a, const KPtrs &k, const uint32_t *fwht_L, const uint32_t *expt,
                           int ngroups, hipStream_t s);
hipError_t fused_prepare_16();
hipError_t fused_prepare_8();
hipError_t poly_launch(int r, int ld, int kind, const PolyArgs &a, const uint32_t *t1, const uint32_t *t2,
                       uint32_t nblocks, hipStream_t s);
hipError_t perm_tables(int r, const uint32_t *vals, uint32_t count, uint32_t *tabs, hipStream_t s);
hipError_t stamp_start(uint64_t *ts, uint64_t *slots, size_t nslots, hipStream_t s);
hipError_t stamp_reduce(uint64_t *ts, const uint64_t *slots, const uint32_t *seg_ptr, const uint32_t *segs,
                        int nstripes, hipStream_t s);
enum { PK_PAD = 0, PK_MUL = 1, PK_DEGREE = 2, PK_UP = 3, PK_DOWN = 4, PK_UP_TILE = 5, PK_DOWN_TILE = 6 };
constexpr int CONV_TILE_L = 8;      // the block-tile conversion kernels cover the levels of 256-row blocks
hipError_t fused_launch_16(int mode, int sh, int ld, int L, const FusedArgs &a, const KPtrs &k, int ntiles,
                           bool pr, hipStream_t s);
hipError_t fused_launch_8(int mode, int sh, int ld, int L, const FusedArgs &a, const KPtrs &k, int ntiles,
                          bool pr, hipStream_t s);
hipError_t pass_launch(int r, int ld, int T, bool inv, bool gen_l, const PassArgs &a, const KPtrs &k,
                       uint32_t nblocks, hipStream_t s);
hipError_t dpart_launch(int r, int ld, int T, const DerivPassArgs &a, const KPtrs &k, uint32_t nblocks,
                        hipStream_t s);
hipError_t wide_launch(int kind, int ld, int T, bool pk, const WideArgs &a, const KPtrs &k, int ntiles, hipStream_t s);
bool wide_packable(int kind, int T);
hipError_t wide_prepare();
hipError_t poly_prepare();
}  // namespace nb

using namespace nb;

namespace {

// MODE_ENC2: encode of a code with one parity block (n' = 2 k')
enum { MODE_FFT = 0, MODE_IFFT = 1, MODE_DERIV = 2, MODE_ENC = 3, MODE_DEC = 4, MODE_ENC2 = 5 };
constexpr int FUSED_MAX_L = 8;      // fused single-launch kernels cover h <= 256
// Levels per plain transform pass (k_pass): a forward pass of 5 levels (32
// rows of a lane in registers, about 100 VGPRs) beats a 4-level and a
// 1-level pass; an inverse one needs about 175 VGPRs (two waves per SIMD)
// and loses to them.
constexpr int PASS_MAX_T_FWD = 5, PASS_MAX_T_INV = 4;
constexpr int LOC_ONE_WG_MAX = 4096; // larger mother codes use the multi-workgroup locator
// pass kinds of nb_wide.hip
enum { W_E1 = 0, W_E2 = 1, W_E2F = 2, W_E3 = 3, W_D1 = 4, W_D2 = 5, W_D3 = 6, W_D4 = 7, W_D5 = 8, W_DPM = 9,
       W_DH = 10, W_DL = 11, W_PI = 12, W_PF = 13, W_PFM = 14 };
// scratch of the 8-level pass pipelines: stripes are processed in chunks
// whose scratch fits this budget (a stripe larger than it runs alone)
constexpr size_t WIDE_SCRATCH_BUDGET = (size_t)2 << 30;
// Pinned host ring through which each call's descriptors reach the device.
// Every upload occupies a byte range until the event recorded after its copy
// completes; the host waits only when the ring is full, so it can run many
// calls ahead of the device.
struct Staging {
    uint8_t *host = nullptr;
    size_t cap = 0;
    size_t head = 0;                 // next byte to hand out
    struct Rec {
        size_t begin, end;
        hipEvent_t ev;
    };
    std::deque<Rec> live;            // uploads in flight, oldest first
    std::vector<hipEvent_t> pool;    // completed events for reuse
};

constexpr size_t STAGING_MIN = (size_t)4 << 20;

struct Scratch {
    hipStream_t stream = nullptr;
    void *dev = nullptr;             // descriptors, masks, locator tables
    size_t dev_cap = 0;
    void *big = nullptr;             // rows of the multi-pass pipelines
    size_t big_cap = 0;
    Staging stg;
};

int ilog2(long v)
{
    int t = 0;
    while ((1L << t) < v)
        t++;
    return t;
}

bool is_pow2(long v) { return v > 0 && (v & (v - 1)) == 0; }
long pow2ceil(long v)
{
    long p = 1;
    while (p < v)
        p <<= 1;
    return p;
}
size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

struct rs_ctx {
    int r = 0;
    int device = 0;
    uint32_t basis[16] = {};
    void *d_mem = nullptr;
    uint32_t *d_basis, *d_Wv, *d_S, *d_wp, *d_skew, *d_B, *d_Binv, *d_exp, *d_log, *d_FL;
    uint32_t *d_tw_tab, *d_B_tab, *d_Binv_tab;
    uint32_t *d_wh, *d_wh_tab;  // What_j monomial coefficients (16 j + m) and 1 / leading (256 + j); perm tables
    KPtrs kp;           // method tables (masks / rowtabs filled per call)
    void *d_static = nullptr;  // this device's static_scratch (rs_decode_static)
    std::mutex mu;
    std::vector<Scratch *> scratch;
    int sticky = RS_OK;
    // schedules of the pass pipelines per (op, N): the level counts of the
    // parts, low part first, one per 4-bit field; 0 = two parts, ceil(N / 2) low
    std::atomic<int> sched[2][17] = {};
    std::atomic<int> tile[2][17] = {};             // column tiles of the pass pipelines (rs_schedule_set_tile)
};

namespace {

struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) {
            ok = false;
            return;
        }
        if (prev != dev && hipSetDevice(dev) != hipSuccess)
            ok = false;
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev)
            (void)hipSetDevice(prev);
    }
};

int dev_err(rs_ctx *ctx, hipError_t e)
{
    if (e == hipSuccess)
        return RS_OK;
    ctx->sticky = RS_EDEVICE;
    return RS_EDEVICE;
}

Scratch *get_scratch(rs_ctx *ctx, hipStream_t s)
{
    for (Scratch *sc : ctx->scratch)
        if (sc->stream == s)
            return sc;
    Scratch *sc = new (std::nothrow) Scratch();
    if (!sc)
        return nullptr;
    sc->stream = s;
    ctx->scratch.push_back(sc);
    return sc;
}

// Grow a device buffer; the stream's earlier work may still read the old one.
int ensure_dev(Scratch *sc, void **buf, size_t *cap, size_t need)
{
    if (need <= *cap)
        return RS_OK;
    if (*buf) {
        if (hipStreamSynchronize(sc->stream) != hipSuccess)
            return RS_EDEVICE;
        (void)hipFree(*buf);
        *buf = nullptr;
        *cap = 0;
    }
    size_t want = std::max(need, (size_t)1 << 20);
    if (hipMalloc(buf, want) != hipSuccess) {
        *buf = nullptr;
        return RS_ENOMEM;
    }
    *cap = want;
    return RS_OK;
}

// Wait for the oldest in-flight upload of the ring and recycle its event.
int staging_retire_oldest(Staging &g)
{
    Staging::Rec r = g.live.front();
    g.live.pop_front();
    const hipError_t e = hipEventSynchronize(r.ev);
    g.pool.push_back(r.ev);
    return e == hipSuccess ? RS_OK : RS_EDEVICE;
}

// Copy `bytes` of host data to `dst` (device) through the pinned ring.
int stage_upload(Scratch *sc, const void *src, size_t bytes, void *dst)
{
    if (!bytes)
        return RS_OK;
    Staging &g = sc->stg;
    const size_t need = align_up(bytes, 256);
    if (need > g.cap) {                           // grow: drain, then reallocate
        while (!g.live.empty())
            if (staging_retire_oldest(g))
                return RS_EDEVICE;
        if (g.host)
            (void)hipHostFree(g.host);
        g.host = nullptr;
        g.cap = 0;
        g.head = 0;
        const size_t want = std::max(need, STAGING_MIN);
        if (hipHostMalloc((void **)&g.host, want, hipHostMallocDefault) != hipSuccess) {
            g.host = nullptr;
            return RS_ENOMEM;
        }
        g.cap = want;
    }
    const size_t begin = g.head + need <= g.cap ? g.head : 0;
    auto overlaps = [&]() {
        for (const Staging::Rec &r : g.live)
            if (r.begin < begin + need && begin < r.end)
                return true;
        return false;
    };
    while (!g.live.empty() && overlaps())
        if (staging_retire_oldest(g))
            return RS_EDEVICE;
    hipEvent_t ev = nullptr;
    if (!g.pool.empty()) {
        ev = g.pool.back();
        g.pool.pop_back();
    } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        return RS_EDEVICE;
    }
    std::memcpy(g.host + begin, src, bytes);
    if (hipMemcpyAsync(dst, g.host + begin, bytes, hipMemcpyHostToDevice, sc->stream) != hipSuccess ||
        hipEventRecord(ev, sc->stream) != hipSuccess) {
        g.pool.push_back(ev);
        return RS_EDEVICE;
    }
    g.live.push_back({begin, begin + need, ev});
    g.head = begin + need;
    return RS_OK;
}

int sym_bytes(const rs_ctx *ctx) { return ctx->r / 8; }

bool vec_aligned(const rs_ctx *ctx, const void *a, const void *b, size_t rb)
{
    const size_t al = ctx->r == 16 ? 8 : 4;
    return ((uintptr_t)a % al == 0) && ((uintptr_t)b % al == 0) && (rb % al == 0);
}

int mother_shape(const rs_ctx *ctx, int n, int k, int *kp, int *np)
{
    if (k < 1 || n <= k)
        return RS_ESHAPE;
    long k2 = pow2ceil(k), n2 = pow2ceil(k2 + (long)n - k);
    if (n2 > (1L << ctx->r))
        return RS_ESHAPE;
    *kp = (int)k2;
    *np = (int)n2;
    return RS_OK;
}

// One stripe of a codec call after validation.
struct Plan {
    DevStripe ds;       // col0 / tile0 / offsets filled when launches are planned
    int L;              // lg of the transform size (k' for encode, n' for decode)
    int erasures;
    bool decoding;
    bool aligned;       // rows and bases allow LD_VEC accesses
    bool prune;         // fused kernels: some outputs of a forward transform are unused (set by validate_stripe)
    size_t mask_src;    // offset of the stripe's mask in the caller's mask array
};

// Column ranges of a stripe and the access variant each is launched with:
// aligned rows use LD_VEC on the full 4-column chunks and LD_SYM on the last
// partial chunk; unaligned rows use LD_SYM throughout.
struct ColPart {
    int ld;
    int col0;
    int ntiles;
    long chunks;        // 4-column chunks of the part
};

int ntiles_of_chunks(long chunks) { return (int)((chunks + 63) / 64); }

// The column parts of a row range: whole chunks of 4 columns read with vector
// loads plus a ragged tail read per symbol, or one per-symbol part when the
// rows are not aligned; at most two, held inline (this runs once per stripe
// of every call, so it allocates nothing).
struct ColParts {
    ColPart p[2];
    int n = 0;
    const ColPart *begin() const { return p; }
    const ColPart *end() const { return p + n; }
    size_t size() const { return (size_t)n; }
    const ColPart &operator[](size_t i) const { return p[i]; }
};

ColParts col_parts(bool aligned, int ncols)
{
    ColParts v;
    if (ncols <= 0)
        return v;
    if (!aligned) {
        v.p[v.n++] = {LD_SYM, 0, ntiles_of_chunks((ncols + 3) / 4), (ncols + 3) / 4};
        return v;
    }
    const int full = ncols / 4;
    if (full)
        v.p[v.n++] = {LD_VEC, 0, ntiles_of_chunks(full), full};
    if (ncols % 4)
        v.p[v.n++] = {LD_SYM, 4 * full, 1, 1};
    return v;
}

int validate_stripe(rs_ctx *ctx, const rs_stripe_desc &d, bool decode, const uint8_t *mask, Plan &pl)
{
    const int sym = sym_bytes(ctx);
    int kp, np;
    int rc = mother_shape(ctx, d.n, d.k, &kp, &np);
    if (rc)
        return rc;
    if (d.row_bytes % (uint64_t)sym)
        return RS_EALIGN;
    if (d.row_bytes && (!d.in || !d.out))
        return RS_EINVAL;
    if (d.row_bytes / sym > (uint64_t)INT32_MAX / 2)
        return RS_ESHAPE;
    std::memset(&pl.ds, 0, sizeof(pl.ds));
    pl.ds.in = (const uint8_t *)d.in;
    pl.ds.out = (uint8_t *)d.out;
    pl.ds.row_bytes = d.row_bytes;
    pl.ds.n = d.n;
    pl.ds.k = d.k;
    pl.ds.kp = kp;
    pl.ds.np = np;
    pl.ds.ncols = (int32_t)(d.row_bytes / sym);
    pl.ds.copy_survivors = decode && d.in != d.out ? 1 : 0;
    pl.ds.sid = 0;                                    // set by build_codec
    pl.aligned = vec_aligned(ctx, d.in, d.out, d.row_bytes);
    pl.L = ilog2(decode ? np : kp);
    pl.erasures = 0;
    pl.decoding = decode;
    pl.prune = false;
    if (decode) {
        if (!mask)
            return RS_EINVAL;
        int e = 0;
        for (int t = 0; t < d.n; t++)
            e += mask[t] != 0;
        if (e > d.n - d.k)
            return RS_ETOOMANY;
        pl.erasures = e;
        // a group of 16 points without an erased stored row leaves its
        // outputs of decode step 5 unused
        if (np >= 32)
            for (int g = 0; g < np / 16 && !pl.prune; g++) {
                bool any = false;
                for (int p = 16 * g; p < 16 * g + 16 && !any; p++) {
                    const int row = p < d.k ? p : (p >= kp && p - kp < d.n - d.k ? d.k + (p - kp) : -1);
                    any = row >= 0 && mask[row];
                }
                pl.prune = !any;
            }
    } else {
        // parity rows that are not stored (shortened codes)
        pl.prune = d.n - d.k < np - kp;
    }
    return RS_OK;
}

// ------------------------------------------------------------------ multi-pass pipelines

// Apply levels [0, L) (inverse) or [L-1 .. 0] (forward) to h = 2^L rows with
// passes of up to 4 levels.  The first pass reads `src` (src_rows rows, the
// rest zero), every pass writes `work`, except that the last pass writes
// rows [dst_lo, dst_hi) to `final_dst` when it is given.
int run_plain_tiled(rs_ctx *ctx, Scratch *sc, hipStream_t s, bool inv, int L, uint32_t l, const uint8_t *src,
                    int src_rows, uint8_t *work, uint8_t *final_dst, int dst_hi, uint64_t rb, int ncols, bool aligned,
                    const uint8_t *mul_last);

int run_passes(rs_ctx *ctx, Scratch *sc, hipStream_t s, bool inv, bool gen_l, int L, uint32_t l, const uint8_t *src,
               int src_rows, uint8_t *work, uint8_t *final_dst, int dst_lo, int dst_hi, uint64_t rb,
               int ncols, bool aligned, bool pre_B_first, bool post_B_last, const uint8_t *mul_last = nullptr)
{
    // GF(2^16) transforms at a shift with no bit below h: two passes of up to
    // 8 levels on LDS tiles instead of register-only passes of 4 or 5
    if (ctx->r == 16 && sc && L > FUSED_MAX_L && !gen_l && !pre_B_first && !post_B_last && dst_lo == 0)
        return run_plain_tiled(ctx, sc, s, inv, L, l, src, src_rows, work, final_dst, dst_hi, rb, ncols, aligned,
                               mul_last);
    // the L levels in as few passes as possible, as even as possible (e.g.
    // forward 13 = 5 + 4 + 4): every pass reads and writes all h rows, so the
    // pass count sets the traffic
    std::vector<std::pair<int, int>> chunks;   // (lo, T)
    const int maxT = inv ? PASS_MAX_T_INV : PASS_MAX_T_FWD;
    const int np_ = (L + maxT - 1) / maxT;
    std::vector<int> Ts;
    for (int i = 0; i < np_; i++)
        Ts.push_back(L / np_ + (i < L % np_ ? 1 : 0));
    if (inv) {
        int lo = 0;
        for (int T : Ts) {
            chunks.push_back({lo, T});
            lo += T;
        }
    } else {
        int top = L;
        for (int T : Ts) {
            chunks.push_back({top - T, T});
            top -= T;
        }
    }
    if (chunks.empty())
        chunks.push_back({0, 0});
    const int h = 1 << L;
    const ColParts parts = col_parts(aligned, ncols);
    for (size_t c = 0; c < chunks.size(); c++) {
        const bool first = c == 0, last = c + 1 == chunks.size();
        for (const ColPart &cp : parts) {
            PassArgs a;
            std::memset(&a, 0, sizeof(a));
            a.src = first ? src : work;
            a.src_rows = first ? src_rows : h;
            if (last && final_dst) {
                a.dst = final_dst;
                a.dst_lo = dst_lo;
                a.dst_hi = dst_hi;
            } else {
                a.dst = work;
                a.dst_lo = 0;
                a.dst_hi = h;
            }
            a.row_bytes = rb;
            a.ncols = ncols;
            a.lo = chunks[c].first;
            a.col0 = cp.col0;
            a.l = l;
            a.pre_B = first && pre_B_first;
            a.post_B = last && post_B_last;
            a.mul = last ? mul_last : nullptr;
            a.nct = cp.ntiles;
            const int T = chunks[c].second;
            const uint32_t nblocks = (uint32_t)((h >> T) * cp.ntiles);
            if (dev_err(ctx, pass_launch(ctx->r, cp.ld, T, inv, gen_l, a, ctx->kp, nblocks, s)))
                return RS_EDEVICE;
        }
    }
    return RS_OK;
}

// A plain transform over h = 2^L rows (8 < L <= 16) at a shift l with no bit
// below h, in two passes of the codec's pass kernels (Sec. 3.2 / 3.3): the
// low T1 = ceil(L/2) levels on groups of 2^T1 consecutive rows and the high
// ones on groups at stride 2^T1, the inverse low part first, the forward high
// part first.  The first pass reads src (rows >= src_rows as zero), the
// passes work in `work`, and the last one writes rows [0, dst_hi) of
// final_dst when it is given, each multiplied symbol by symbol by the same
// row of mul_last when that is given.
int run_plain_tiled(rs_ctx *ctx, Scratch *sc, hipStream_t s, bool inv, int L, uint32_t l, const uint8_t *src,
                    int src_rows, uint8_t *work, uint8_t *final_dst, int dst_hi, uint64_t rb, int ncols, bool aligned,
                    const uint8_t *mul_last)
{
    const int h = 1 << L, T1 = (L + 1) / 2, T2 = L - T1;
    const int lo_of[2] = {inv ? 0 : T1, inv ? T1 : 0}, T_of[2] = {inv ? T1 : T2, inv ? T2 : T1};
    struct Launch {
        int kind, ld, T, lo, ntiles;
        size_t first;
    };
    WideStripe descs[4];
    Launch launches[4];
    int nl = 0;
    const ColParts parts = col_parts(aligned, ncols);
    for (int c = 0; c < 2; c++) {
        const bool first = c == 0, last = c == 1;
        for (const ColPart &cp : parts) {
            WideStripe &w = descs[nl];
            std::memset(&w, 0, sizeof(w));
            w.st.row_bytes = rb;
            w.st.ncols = ncols;
            w.st.col0 = cp.col0;
            w.st.n = w.st.kp = w.st.np = h;
            w.src = first ? src : work;
            w.src_rows = first ? src_rows : h;
            w.dst = last && final_dst ? final_dst : work;
            w.dst_rows = last && final_dst ? dst_hi : h;
            w.src2 = last ? mul_last : nullptr;
            w.tile0 = 0;
            w.nct = cp.ntiles;
            launches[nl] = {inv ? W_PI : (last && mul_last ? W_PFM : W_PF), cp.ld, T_of[c], lo_of[c],
                            (h >> T_of[c]) * cp.ntiles, (size_t)nl};
            nl++;
        }
    }
    int rc = ensure_dev(sc, &sc->dev, &sc->dev_cap, sizeof(WideStripe) * nl);
    if (!rc)
        rc = stage_upload(sc, descs, sizeof(WideStripe) * nl, sc->dev);
    if (rc)
        return rc;
    for (int i = 0; i < nl; i++) {
        WideArgs wa;
        wa.stripes = (const WideStripe *)sc->dev + launches[i].first;
        wa.nstripes = 1;
        wa.lo = launches[i].lo;
        wa.blk = 0;
        wa.l = l;
        wa.ts = nullptr;
        if (dev_err(ctx, wide_launch(launches[i].kind, launches[i].ld, launches[i].T, false, wa, ctx->kp,
                                     launches[i].ntiles, s)))
            return RS_EDEVICE;
    }
    return RS_OK;
}

// Multiply every one of h rows by B_p in place (a pass with no levels).
int scale_rows_B(rs_ctx *ctx, hipStream_t s, uint8_t *d, int h, uint64_t rb, int ncols, bool aligned)
{
    for (const ColPart &cp : col_parts(aligned, ncols)) {
        PassArgs a;
        std::memset(&a, 0, sizeof(a));
        a.src = d;
        a.src_rows = h;
        a.dst = d;
        a.dst_hi = h;
        a.row_bytes = rb;
        a.ncols = ncols;
        a.col0 = cp.col0;
        a.post_B = 1;
        a.nct = cp.ntiles;
        if (dev_err(ctx, pass_launch(ctx->r, cp.ld, 0, false, false, a, ctx->kp, (uint32_t)(h * cp.ntiles), s)))
            return RS_EDEVICE;
    }
    return RS_OK;
}

// Derivative of h = 2^L rows held in y (already multiplied by B): z gets the
// partial sums level range by level range; the last range writes
// (sum) / B_p into out.
int run_deriv_passes(rs_ctx *ctx, hipStream_t s, int L, const uint8_t *y, uint8_t *z, uint8_t *out,
                     uint64_t rb, int ncols, bool aligned)
{
    const int h = 1 << L;
    for (int lo = 0; lo < L; lo += 4) {
        const int T = std::min(4, L - lo);
        for (const ColPart &cp : col_parts(aligned, ncols)) {
            DerivPassArgs a;
            std::memset(&a, 0, sizeof(a));
            a.y = y;
            a.z = z;
            a.out = out;
            a.row_bytes = rb;
            a.ncols = ncols;
            a.lo = lo;
            a.nct = cp.ntiles;
            a.col0 = cp.col0;
            a.first = lo == 0;
            a.last = lo + T >= L;
            if (dev_err(ctx, dpart_launch(ctx->r, cp.ld, T, a, ctx->kp, (uint32_t)((h >> T) * cp.ntiles), s)))
                return RS_EDEVICE;
        }
    }
    return RS_OK;
}

// Zero one row (the derivative of a constant) with a no-level pass that
// reads nothing, so that the call records no memset node.
int fill_zero(rs_ctx *ctx, hipStream_t s, uint8_t *data, uint64_t rb)
{
    const int ncols = (int)(rb / sym_bytes(ctx));
    for (const ColPart &cp : col_parts(vec_aligned(ctx, data, data, rb), ncols)) {
        PassArgs a;
        std::memset(&a, 0, sizeof(a));
        a.src = data;
        a.src_rows = 0;
        a.dst = data;
        a.dst_hi = 1;
        a.row_bytes = rb;
        a.ncols = ncols;
        a.col0 = cp.col0;
        a.nct = cp.ntiles;
        if (dev_err(ctx, pass_launch(ctx->r, cp.ld, 0, false, false, a, ctx->kp, (uint32_t)cp.ntiles, s)))
            return RS_EDEVICE;
    }
    return RS_OK;
}

int big_scratch(Scratch *sc, size_t need, uint8_t **p)
{
    int rc = ensure_dev(sc, &sc->big, &sc->big_cap, need);
    *p = (uint8_t *)sc->big;
    return rc;
}

// pr: the kernel variant that skips unused outputs (encode and decode only).
hipError_t fused_launch(int r, int mode, int sh, int ld, int L, const FusedArgs &a, const KPtrs &k, int ntiles,
                        bool pr, hipStream_t s)
{
    return r == 16 ? fused_launch_16(mode, sh, ld, L, a, k, ntiles, pr, s)
                   : fused_launch_8(mode, sh, ld, L, a, k, ntiles, pr, s);
}

// An encode whose mother code has a single parity block (n' = 2 k') runs a
// kernel variant without the loop over parity blocks.
bool one_parity_block(const Plan &p) { return !p.decoding && p.ds.np == 2 * p.ds.kp; }

// Stripes whose transforms run as pass pipelines: more than 256 points, and
// encodes over 256 points with several parity blocks (the fused kernel
// would keep the coefficients of a 1024-thread workgroup in registers across
// the blocks, which does not fit).
bool runs_wide(const Plan &p) { return p.L > FUSED_MAX_L || (p.L == FUSED_MAX_L && !p.decoding && !one_parity_block(p)); }

// Stripes of one fused launch share the transform size, the row access
// variant and the kernel variant.
int launch_key(const Plan &p, int ld)
{
    return ((p.L * 2 + ld) * 2 + (one_parity_block(p) ? 1 : 0)) * 2 + (p.prune ? 1 : 0);
}

// One launch unit: a column part of one stripe.
struct Entry {
    int plan;
    ColPart cp;
    int key;           // launch_key of the pair, computed once
};

// ------------------------------------------------------------------ 8-level pass pipelines

// One launch of the pass pipelines: descriptors [first, first + count) of
// the uploaded array.
struct WideLaunch {
    int kind, ld, T, lo, blk;
    bool pk;                     // packed: rows of at most 32 chunks, two row sets per wave
    size_t first, count;
    int ntiles;
};

struct WidePlan {
    std::vector<WideStripe> descs;
    std::vector<WideLaunch> launches;
    size_t scratch = 0;          // bytes of scratch the largest chunk needs
};

// Scratch rows a stripe needs (encode: coefficients unless they can live in
// the parity rows, plus one parity block unless it is stored whole; decode:
// n' transform rows and n' partial-sum rows).
size_t wide_scratch_rows(const Plan &p)
{
    const DevStripe &d = p.ds;
    if (p.decoding)
        return 2 * (size_t)d.np;
    const int npar = d.n - d.k;
    const int nblocks = d.np / d.kp;
    if (nblocks == 2 && npar == d.kp)
        return 0;
    return 2 * (size_t)d.kp;
}

void unpack_parts(int v, int N, int *parts, int *nparts);

// Split the wide stripes (plan indices, all runs_wide) into
// chunks, lay out their scratch from `scratch_base` (null while sizing) and
// list the launches: per chunk and transform size, every pass kind in order,
// one launch per row-access variant.
void plan_wide(const std::vector<Plan> &plans, const std::vector<int> &idx, bool decode, uint8_t *scratch_base,
               const int *sched, const int *tile_cols, WidePlan &wp)
{
    wp.descs.clear();
    wp.launches.clear();
    wp.scratch = 0;
    // chunks in plan order
    std::vector<std::pair<size_t, size_t>> chunks;     // [begin, end) into idx
    size_t cur = 0, begin = 0;
    for (size_t q = 0; q < idx.size(); q++) {
        const Plan &p = plans[idx[q]];
        const size_t need = wide_scratch_rows(p) * p.ds.row_bytes;
        if (q > begin && cur + need > WIDE_SCRATCH_BUDGET) {
            chunks.push_back({begin, q});
            begin = q;
            cur = 0;
        }
        cur += need;
        wp.scratch = std::max(wp.scratch, cur);
    }
    if (begin < idx.size())
        chunks.push_back({begin, idx.size()});

    for (const auto &ch : chunks) {
        // scratch of each stripe of the chunk
        std::vector<uint8_t *> sA(ch.second - ch.first), sZ(ch.second - ch.first);
        size_t off = 0;
        for (size_t q = ch.first; q < ch.second; q++) {
            const Plan &p = plans[idx[q]];
            const size_t rows = wide_scratch_rows(p);
            const size_t half = rows / 2 * p.ds.row_bytes;
            sA[q - ch.first] = rows ? scratch_base + off : nullptr;
            sZ[q - ch.first] = rows ? scratch_base + off + half : nullptr;
            off += rows * p.ds.row_bytes;
        }
        // transform sizes present in the chunk
        std::vector<int> Ns;
        for (size_t q = ch.first; q < ch.second; q++)
            if (std::find(Ns.begin(), Ns.end(), plans[idx[q]].L) == Ns.end())
                Ns.push_back(plans[idx[q]].L);
        std::sort(Ns.begin(), Ns.end());
        for (int N : Ns) {
            int parts[4], m = 0;
            unpack_parts(sched[N], N, parts, &m);
            int los[4] = {0, 0, 0, 0};
            for (int i = 1; i < m; i++)
                los[i] = los[i - 1] + parts[i - 1];
            const int T1 = parts[0], TH = parts[m - 1], LH = los[m - 1];
            int max_blocks = 2;
            for (size_t q = ch.first; q < ch.second; q++)
                if (plans[idx[q]].L == N)
                    max_blocks = std::max(max_blocks, plans[idx[q]].ds.np / plans[idx[q]].ds.kp);
            // (kind, lo, T, blk, middle part) sequence: the low part, the
            // middle parts (pipelines of three or four parts), the high part
            struct Step { int kind, lo, T, blk; bool mid; };
            std::vector<Step> steps;
            if (decode && m == 2) {
                // three passes: the derivative split into its low-bit and
                // high-bit parts (see nb_wide.hip)
                steps.push_back({W_D1, 0, T1, 0, false});
                steps.push_back({W_DH, LH, TH, 0, false});
                steps.push_back({W_DL, 0, T1, 0, false});
            } else if (decode) {
                steps.push_back({W_D1, 0, T1, 0, false});
                for (int i = 1; i + 1 < m; i++)
                    steps.push_back({W_E1, los[i], parts[i], 0, true});
                steps.push_back({W_D2, LH, TH, 0, false});
                for (int i = m - 2; i >= 1; i--)
                    steps.push_back({W_DPM, los[i], parts[i], 0, true});
                steps.push_back({W_D3, 0, T1, 0, false});
                steps.push_back({W_D4, LH, TH, 0, false});
                for (int i = m - 2; i >= 1; i--)
                    steps.push_back({W_D4, los[i], parts[i], 0, true});
                steps.push_back({W_D5, 0, T1, 0, false});
            } else {
                steps.push_back({W_E1, 0, T1, 0, false});
                for (int i = 1; i + 1 < m; i++)
                    steps.push_back({W_E1, los[i], parts[i], 0, true});
                for (int b = 1; b < max_blocks; b++) {
                    steps.push_back({b == 1 ? W_E2 : W_E2F, LH, TH, b, false});
                    for (int i = m - 2; i >= 1; i--)
                        steps.push_back({W_E2F, los[i], parts[i], b, true});
                    steps.push_back({W_E3, 0, T1, b, false});
                }
            }
            for (const Step &stp : steps) {
                // one launch per row-access variant, plain or packed (parts
                // of at most 32 chunks, which fill half a wave)
                for (int var = 0; var < 4; var++) {
                    const int ld = var & 1;
                    const bool pk = var >> 1;
                    if (pk && !wide_packable(stp.kind, stp.T))
                        continue;
                    WideLaunch wl;
                    wl.kind = stp.kind;
                    wl.ld = ld;
                    wl.pk = pk;
                    wl.T = stp.T;
                    wl.lo = stp.lo;
                    wl.blk = stp.blk;
                    wl.first = wp.descs.size();
                    int tiles = 0;
                    for (size_t q = ch.first; q < ch.second; q++) {
                        const Plan &p = plans[idx[q]];
                        if (p.L != N)
                            continue;
                        const DevStripe &d = p.ds;
                        const int npar = d.n - d.k;
                        const int nblocks = d.np / d.kp;
                        if (!decode && (stp.blk >= nblocks || (stp.blk - 1) * d.kp >= npar))
                            continue;
                        const uint64_t rb = d.row_bytes;
                        uint8_t *A = sA[q - ch.first], *Z = sZ[q - ch.first];
                        const bool in_parity = !decode && A == nullptr;   // (2k', k') code, not shortened
                        uint8_t *coef = in_parity ? d.out : A;
                        // parity block b goes straight to its rows when they are all stored
                        auto block_buf = [&](int b) -> uint8_t * {
                            if (in_parity)
                                return d.out;
                            return (size_t)b * d.kp <= (size_t)npar ? d.out + (size_t)(b - 1) * d.kp * rb : Z;
                        };
                        WideStripe w;
                        std::memset(&w, 0, sizeof(w));
                        w.st = d;
                        w.src_rows = decode ? d.np : d.kp;
                        w.dst_rows = decode ? d.np : d.kp;
                        switch (stp.kind) {
                        case W_E1:
                            if (decode) {                       // a middle part's inverse levels
                                w.src = A;
                                w.dst = A;
                            } else {
                                w.src = stp.mid ? coef : d.in;
                                w.src_rows = stp.mid ? d.kp : d.k;
                                w.dst = coef;
                            }
                            break;
                        case W_E2:
                            w.src = coef;
                            w.dst2 = nblocks > 2 ? coef : nullptr;
                            w.dst = block_buf(1);
                            break;
                        case W_E2F:
                            w.src = stp.mid ? block_buf(stp.blk) : coef;
                            w.dst = block_buf(stp.blk);
                            break;
                        case W_E3:
                            w.src = block_buf(stp.blk);
                            w.dst = d.out + (size_t)(stp.blk - 1) * d.kp * rb;
                            w.dst_rows = std::min(d.kp, npar - (stp.blk - 1) * d.kp);
                            break;
                        case W_D1: w.dst = A; break;
                        case W_D2: w.src = A; w.dst = A; w.dst2 = Z; break;
                        case W_D3: w.src = A; w.src2 = Z; w.dst = A; break;
                        case W_DPM: w.src = A; w.src2 = Z; w.dst = Z; break;
                        case W_D4: w.src = A; w.dst = A; break;
                        case W_D5: w.src = A; break;
                        case W_DH: w.src = A; w.dst = Z; break;
                        case W_DL: w.src = Z; w.src2 = A; break;
                        }
                        for (const ColPart &cp : col_parts(p.aligned, d.ncols)) {
                            // packed 128-column tiles: by default for parts of at
                            // most 32 chunks, else as the schedule's tile says
                            const int tc = tile_cols[N];
                            const bool part_pk = wide_packable(stp.kind, stp.T) &&
                                                 (tc == 128 || (tc == 0 && cp.chunks <= 32));
                            if (cp.ld != ld || part_pk != pk)
                                continue;
                            WideStripe e = w;
                            e.st.col0 = cp.col0;
                            e.nct = part_pk ? (int)((cp.chunks + 31) / 32) : cp.ntiles;
                            e.tile0 = tiles;
                            tiles += (1 << (N - stp.T)) * e.nct;
                            wp.descs.push_back(e);
                        }
                    }
                    wl.count = wp.descs.size() - wl.first;
                    wl.ntiles = tiles;
                    if (wl.count)
                        wp.launches.push_back(wl);
                }
            }
        }
    }
}

// A codec call turned into device work: the image of its device arena
// (descriptors, locator stripes, point bitmaps, pass descriptors; then room
// for the locator tables and residues the kernels write) and the list of
// launches.  Built on the host from the call's arguments; executed by
// exec_codec on any stream, with the arena at any device address.
struct FusedLaunch {
    int mode, ld, L;
    bool prune;                // the pruned kernel variant
    size_t first, count;       // entries of the descriptor array
    int ntiles;
};

struct LocLarge {
    size_t q;                  // index in the locator stripes
    int N;
    size_t v_off;              // dword offset of its residues
};

struct CodecPlan {
    bool decode = false;
    std::vector<uint8_t> host;                 // arena image (host_bytes)
    size_t dev_bytes = 0;
    size_t off_loc = 0, off_bits = 0, off_wide = 0, off_rt = 0, off_locv = 0;
    std::vector<FusedLaunch> fused;
    std::vector<std::pair<int32_t, int32_t>> ent_tiles;  // (stripe, first tile) of each fused entry
    int m_small = 0, max_np = 1;
    std::vector<LocLarge> loc_large;
    WidePlan wp;
    // decode stripes without erasures, copied when out != in
    std::vector<std::pair<uint8_t *, const uint8_t *>> copies;
    std::vector<size_t> copy_bytes;
    bool empty() const { return fused.empty() && wp.launches.empty() && copies.empty() && m_small == 0 && loc_large.empty(); }
};

// Scratch of the pass pipelines: get(need, &base) yields `need` bytes of
// device memory, or an error code.
typedef std::function<int(size_t, uint8_t **)> ScratchFn;

// The point bitmaps of one stripe: bit p of rx (received) or er (erased) for
// every stored row; message row t is point t, parity row t point k' + t - k.
// 16 rows at a time where the points of a run start on a word boundary.
static void pack_points(const uint8_t *mk, int t0, int count, int pt0, uint32_t *rx, uint32_t *er)
{
    int i = 0;
    if ((pt0 & 31) == 0) {
        const __m128i zero = _mm_setzero_si128();
        for (; i + 16 <= count; i += 16) {
            const __m128i v = _mm_loadu_si128(reinterpret_cast<const __m128i *>(mk + t0 + i));
            const uint32_t z = (uint32_t)_mm_movemask_epi8(_mm_cmpeq_epi8(v, zero));   // bit j: row not erased
            const int pt = pt0 + i;
            rx[pt >> 5] |= z << (pt & 31);
            er[pt >> 5] |= (~z & 0xFFFFu) << (pt & 31);
        }
    }
    for (; i < count; i++) {
        const int pt = pt0 + i;
        uint32_t *w = mk[t0 + i] ? er : rx;
        w[pt >> 5] |= 1u << (pt & 31);
    }
}

// Validate the call and build its plan.  get_scratch is called once, with
// the size the pass pipelines need, when they need any (an empty function:
// such calls fail with RS_ESHAPE).
int build_codec(rs_ctx *ctx, const rs_stripe_desc *descs, const uint8_t *masks, int count, bool decode,
                const ScratchFn &get_scratch, CodecPlan &cp)
{
    if (!ctx || (count > 0 && !descs) || count < 0)
        return RS_EINVAL;
    if (decode && count > 0 && !masks)
        return RS_EINVAL;
    cp = CodecPlan();
    cp.decode = decode;
    std::vector<Plan> plans((size_t)count);
    size_t mask_total = 0;
    for (int i = 0; i < count; i++) {
        const uint8_t *m = decode ? masks + mask_total : nullptr;
        int rc = validate_stripe(ctx, descs[i], decode, m, plans[i]);
        if (rc)
            return rc;
        plans[i].ds.sid = i;
        plans[i].mask_src = mask_total;
        if (decode)
            mask_total += (size_t)descs[i].n;
    }

    // Active stripes: with columns and, for decode, at least one erasure.
    std::vector<int> act;
    for (int i = 0; i < count; i++) {
        const Plan &p = plans[i];
        if (p.ds.ncols == 0)
            continue;
        if (decode && p.erasures == 0) {
            if (p.ds.copy_survivors) {
                cp.copies.push_back({p.ds.out, p.ds.in});
                cp.copy_bytes.push_back((size_t)p.ds.n * p.ds.row_bytes);
            }
            continue;
        }
        act.push_back(i);
    }
    const int m = (int)act.size();
    const int ts = ctx->r == 16 ? TAB16 : TAB8;

    // Per-stripe device data (decode): point bitmaps and locator tables.
    size_t bit_words = 0, rt_dwords = 0;
    for (int q = 0; q < m; q++) {
        Plan &p = plans[act[q]];
        if (decode) {
            p.ds.bits_off = bit_words;
            bit_words += 2 * (size_t)((p.ds.np + 31) / 32);
            p.ds.rowtab_off = rt_dwords;
            rt_dwords += (size_t)p.ds.np * ts;
        }
    }
    // Fused-path entries, grouped by launch key.
    std::vector<Entry> ents;
    for (int q = 0; q < m; q++) {
        const Plan &p = plans[act[q]];
        if (runs_wide(p))
            continue;
        for (const ColPart &c : col_parts(p.aligned, p.ds.ncols))
            ents.push_back({act[q], c, launch_key(p, c.ld)});
    }
    std::stable_sort(ents.begin(), ents.end(), [](const Entry &x, const Entry &y) { return x.key < y.key; });
    const int ne = (int)ents.size();
    std::vector<DevStripe> eds((size_t)ne);
    for (int j = 0; j < ne;) {
        const Plan &pj = plans[ents[j].plan];
        const int key = ents[j].key;
        int e = j, tiles = 0;
        while (e < ne && ents[e].key == key) {
            eds[e] = plans[ents[e].plan].ds;
            eds[e].col0 = ents[e].cp.col0;
            eds[e].tile0 = tiles;
            cp.ent_tiles.push_back({eds[e].sid, tiles});
            tiles += ents[e].cp.ntiles;
            e++;
        }
        FusedLaunch fl;
        fl.mode = decode ? MODE_DEC : (one_parity_block(pj) ? MODE_ENC2 : MODE_ENC);
        fl.ld = ents[j].cp.ld;
        fl.L = pj.L;
        fl.prune = pj.prune;
        fl.first = (size_t)j;
        fl.count = (size_t)(e - j);
        fl.ntiles = tiles;
        cp.fused.push_back(fl);
        j = e;
    }
    // Locator descriptors: those with a one-workgroup locator first; the
    // others get a residue array each.
    std::vector<DevStripe> lds_;
    size_t locv_words = 0;
    for (int pass = 0; decode && pass < 2; pass++)
        for (int q = 0; q < m; q++) {
            const DevStripe &d = plans[act[q]].ds;
            if ((d.np <= LOC_ONE_WG_MAX) != (pass == 0))
                continue;
            if (pass == 0) {
                cp.m_small++;
                cp.max_np = std::max(cp.max_np, d.np);
            } else {
                cp.loc_large.push_back({lds_.size(), ilog2(d.np), locv_words});
                locv_words += (size_t)d.np;
            }
            lds_.push_back(d);
        }
    // Stripes over more than 256 points: 8-level pass pipelines.
    std::vector<int> widx;
    for (int q = 0; q < m; q++)
        if (runs_wide(plans[act[q]]))
            widx.push_back(act[q]);
    if (!widx.empty()) {
        int sc[17], tl[17];
        for (int N = 0; N < 17; N++) {
            sc[N] = ctx->sched[decode ? 1 : 0][N].load(std::memory_order_relaxed);
            tl[N] = ctx->tile[decode ? 1 : 0][N].load(std::memory_order_relaxed);
        }
        plan_wide(plans, widx, decode, nullptr, sc, tl, cp.wp);        // sizes the scratch
        if (cp.wp.scratch) {
            uint8_t *base = nullptr;
            const int rc = get_scratch ? get_scratch(cp.wp.scratch, &base) : RS_ESHAPE;
            if (rc)
                return rc;
            plan_wide(plans, widx, decode, base, sc, tl, cp.wp);
        }
    }

    // Arena: [entries | locator stripes | point bitmaps | pass descriptors |
    // locator tables | locator residues]; the first four are uploaded.
    cp.off_loc = align_up(sizeof(DevStripe) * ne, 256);
    cp.off_bits = align_up(cp.off_loc + sizeof(DevStripe) * lds_.size(), 256);
    cp.off_wide = align_up(cp.off_bits + bit_words * 4, 256);
    cp.off_rt = align_up(cp.off_wide + sizeof(WideStripe) * cp.wp.descs.size(), 256);
    cp.off_locv = align_up(cp.off_rt + rt_dwords * 4, 256);
    cp.dev_bytes = cp.off_locv + locv_words * 4;
    cp.host.assign(cp.off_rt, 0);
    if (ne)
        std::memcpy(cp.host.data(), eds.data(), sizeof(DevStripe) * ne);
    if (!cp.wp.descs.empty())
        std::memcpy(cp.host.data() + cp.off_wide, cp.wp.descs.data(), sizeof(WideStripe) * cp.wp.descs.size());
    if (decode) {
        if (!lds_.empty())
            std::memcpy(cp.host.data() + cp.off_loc, lds_.data(), sizeof(DevStripe) * lds_.size());
        uint32_t *bits = (uint32_t *)(cp.host.data() + cp.off_bits);
        for (int q = 0; q < m; q++) {
            const Plan &p = plans[act[q]];
            const uint8_t *mk = masks + p.mask_src;
            const int W = (p.ds.np + 31) / 32;
            uint32_t *rx = bits + p.ds.bits_off, *er = rx + W;
            pack_points(mk, 0, p.ds.k, 0, rx, er);
            pack_points(mk, p.ds.k, p.ds.n - p.ds.k, p.ds.kp, rx, er);
        }
    }
    return RS_OK;
}

// Completion stamps of a plan: one slot per workgroup of every fused and
// pass-pipeline launch (the kernels raise their workgroup's slot as its
// waves finish) and, per stripe, the slot ranges of the workgroups that work
// on it, which a last kernel reduces into the caller's timestamps.
struct StampMap {
    uint8_t *dev = nullptr;             // slots | seg_ptr | segs
    uint64_t *slots = nullptr;
    const uint32_t *seg_ptr = nullptr;  // count + 1 offsets into segs (pairs)
    const uint32_t *segs = nullptr;     // [begin, end) slot ranges
    size_t nslots = 0;
    std::vector<size_t> fused_off, wide_off;  // first slot of each launch
};

// The slot ranges of a built plan of `count` stripes (host side of StampMap;
// reads the plan's entry lists, not its arena image, which a reusable plan
// drops once uploaded).  Within a launch, entry e covers workgroups
// tile0_e .. tile0_{e+1} - 1 (the last entry: up to the launch's workgroup
// count).
int stamp_ranges(const CodecPlan &cp, int count, StampMap &sm, std::vector<uint32_t> &seg_ptr,
                 std::vector<uint32_t> &segs)
{
    std::vector<std::vector<std::pair<size_t, size_t>>> per((size_t)count);
    size_t off = 0;
    auto add = [&](int sid, size_t b, size_t e) {
        if (e > b)
            per[(size_t)sid].push_back({off + b, off + e});
    };
    for (const FusedLaunch &fl : cp.fused) {
        sm.fused_off.push_back(off);
        for (size_t q = 0; q < fl.count; q++) {
            const std::pair<int32_t, int32_t> &t = cp.ent_tiles[fl.first + q];
            const size_t end = q + 1 < fl.count ? (size_t)cp.ent_tiles[fl.first + q + 1].second : (size_t)fl.ntiles;
            add(t.first, (size_t)t.second, end);
        }
        off += (size_t)fl.ntiles;
    }
    for (const WideLaunch &wl : cp.wp.launches) {
        sm.wide_off.push_back(off);
        for (size_t q = 0; q < wl.count; q++) {
            const WideStripe &w = cp.wp.descs[wl.first + q];
            const size_t end = q + 1 < wl.count ? (size_t)cp.wp.descs[wl.first + q + 1].tile0 : (size_t)wl.ntiles;
            add(w.st.sid, (size_t)w.tile0, end);
        }
        off += (size_t)wl.ntiles;
    }
    if (off > UINT32_MAX)
        return RS_EINVAL;
    sm.nslots = off;
    seg_ptr.assign(1, 0);
    segs.clear();
    for (const auto &v : per) {
        for (const auto &r : v) {
            segs.push_back((uint32_t)r.first);
            segs.push_back((uint32_t)r.second);
        }
        seg_ptr.push_back((uint32_t)(segs.size() / 2));
    }
    return RS_OK;
}

// Decode step 1 of a built plan: the erasure locator's per-point tables in
// the arena at `dev` (they depend only on the erasure patterns).
int run_locator(rs_ctx *ctx, const CodecPlan &cp, uint8_t *dev, hipStream_t stream)
{
    KPtrs kp = ctx->kp;
    kp.bits = (const uint32_t *)(dev + cp.off_bits);
    kp.rowtabs = (const uint32_t *)(dev + cp.off_rt);
    if (cp.decode) {
        LocatorArgs la;
        la.stripes = (const DevStripe *)(dev + cp.off_loc);
        la.r = ctx->r;
        if (dev_err(ctx, locator_launch(la, kp, ctx->d_FL, ctx->d_exp, cp.m_small, cp.max_np, stream)))
            return RS_EDEVICE;
        for (const LocLarge &ll : cp.loc_large) {
            const int T1 = (ll.N + 1) / 2, T2 = ll.N - T1;
            LocPassArgs pa;
            pa.stripe = la.stripes + ll.q;
            pa.v = (uint32_t *)(dev + cp.off_locv) + ll.v_off;
            pa.r = ctx->r;
            for (int kind = 0; kind < 3; kind++) {     // low, high, low (see k_loc_pass)
                pa.kind = kind;
                pa.lo = kind == 1 ? T1 : 0;
                pa.T = kind == 1 ? T2 : T1;
                if (dev_err(ctx, loc_pass_launch(pa, kp, ctx->d_FL, ctx->d_exp, 1 << (ll.N - pa.T), stream)))
                    return RS_EDEVICE;
            }
        }
    }
    return RS_OK;
}

// Queue a built plan on `stream` with its arena at `dev` (the uploaded part
// already in place).  Launches kernels and device-to-device copies only.
// sm, ts: completion stamps (ts[0] the launch start, ts[1 + i] stripe i's
// last workgroup), or null.  located: the locator's tables are already in
// the arena (a reusable plan computes them once).
int exec_codec(rs_ctx *ctx, const CodecPlan &cp, uint8_t *dev, hipStream_t stream, const StampMap *sm = nullptr,
               uint64_t *ts = nullptr, int nstripes = 0, bool located = false)
{
    if (sm && dev_err(ctx, stamp_start(ts, sm->slots, sm->nslots, stream)))
        return RS_EDEVICE;
    for (size_t i = 0; i < cp.copies.size(); i++)
        if (dev_err(ctx, hipMemcpyAsync(cp.copies[i].first, cp.copies[i].second, cp.copy_bytes[i],
                                        hipMemcpyDeviceToDevice, stream)))
            return RS_EDEVICE;
    KPtrs kp = ctx->kp;
    kp.bits = (const uint32_t *)(dev + cp.off_bits);
    kp.rowtabs = (const uint32_t *)(dev + cp.off_rt);
    if (!located) {
        const int rc = run_locator(ctx, cp, dev, stream);
        if (rc)
            return rc;
    }
    const DevStripe *d_ents = (const DevStripe *)dev;
    for (size_t i = 0; i < cp.fused.size(); i++) {
        const FusedLaunch &fl = cp.fused[i];
        FusedArgs fa;
        fa.stripes = d_ents + fl.first;
        fa.nstripes = (int)fl.count;
        fa.l = 0;
        fa.ts = sm ? sm->slots + sm->fused_off[i] : nullptr;
        if (dev_err(ctx, fused_launch(ctx->r, fl.mode, 0, fl.ld, fl.L, fa, kp, fl.ntiles, fl.prune, stream)))
            return RS_EDEVICE;
    }
    const WideStripe *d_wide = (const WideStripe *)(dev + cp.off_wide);
    for (size_t i = 0; i < cp.wp.launches.size(); i++) {
        const WideLaunch &wl = cp.wp.launches[i];
        WideArgs wa;
        wa.stripes = d_wide + wl.first;
        wa.nstripes = (int)wl.count;
        wa.lo = wl.lo;
        wa.blk = wl.blk;
        wa.l = 0;
        wa.ts = sm ? sm->slots + sm->wide_off[i] : nullptr;
        if (dev_err(ctx, wide_launch(wl.kind, wl.ld, wl.T, wl.pk, wa, kp, wl.ntiles, stream)))
            return RS_EDEVICE;
    }
    if (sm && dev_err(ctx, stamp_reduce(ts, sm->slots, sm->seg_ptr, sm->segs, nstripes, stream)))
        return RS_EDEVICE;
    return RS_OK;
}

int run_codec(rs_ctx *ctx, const rs_stripe_desc *descs, const uint8_t *masks, int count, bool decode,
              hipStream_t stream)
{
    if (!ctx)
        return RS_EINVAL;
    DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return RS_EDEVICE;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->sticky)
        return ctx->sticky;
    Scratch *sc = nullptr;
    // the stream's scratch, grown to what the pass pipelines need
    auto get_sc = [&](size_t need, uint8_t **base) -> int {
        if (!sc && !(sc = get_scratch(ctx, stream)))
            return RS_ENOMEM;
        return big_scratch(sc, need, base);
    };
    CodecPlan cp;
    int rc = build_codec(ctx, descs, masks, count, decode, get_sc, cp);
    if (rc)
        return rc;
    if (cp.empty())
        return RS_OK;
    if (!sc && !(sc = get_scratch(ctx, stream)))
        return RS_ENOMEM;
    rc = ensure_dev(sc, &sc->dev, &sc->dev_cap, cp.dev_bytes);
    if (rc)
        return rc;
    uint8_t *dev = (uint8_t *)sc->dev;
    rc = stage_upload(sc, cp.host.data(), cp.host.size(), dev);
    if (rc)
        return rc;
    return exec_codec(ctx, cp, dev, stream);
}

// The transform (mode MODE_FFT / MODE_IFFT / MODE_DERIV) of h rows of d in
// place, with the context locked and the stream's scratch at hand.
int xform_locked(rs_ctx *ctx, Scratch *sc, int mode, int h, uint32_t l, uint8_t *d, size_t rb, hipStream_t stream)
{
    const int L = ilog2(h);
    const int ncols = (int)(rb / sym_bytes(ctx));
    const bool aligned = vec_aligned(ctx, d, d, rb);
    // with h | l every factor is a plain table entry; otherwise bit i of l adds 1
    const bool gen_l = mode != MODE_DERIV && (l & (uint32_t)(h - 1)) != 0;
    if (mode == MODE_DERIV && L == 0)
        return fill_zero(ctx, stream, d, rb);
    if (L <= FUSED_MAX_L) {
        const ColParts parts = col_parts(aligned, ncols);
        std::vector<DevStripe> st(parts.size());
        for (size_t i = 0; i < parts.size(); i++) {
            std::memset(&st[i], 0, sizeof(DevStripe));
            st[i].in = d;
            st[i].out = d;
            st[i].row_bytes = rb;
            st[i].n = h;
            st[i].kp = st[i].np = h;
            st[i].ncols = ncols;
            st[i].col0 = parts[i].col0;
        }
        int rc = ensure_dev(sc, &sc->dev, &sc->dev_cap, sizeof(DevStripe) * parts.size());
        if (rc)
            return rc;
        rc = stage_upload(sc, st.data(), sizeof(DevStripe) * parts.size(), sc->dev);
        if (rc)
            return rc;
        for (size_t i = 0; i < parts.size(); i++) {
            FusedArgs fa;
            fa.stripes = (const DevStripe *)sc->dev + i;
            fa.nstripes = 1;
            fa.l = l;
            fa.ts = nullptr;
            const int sh = gen_l ? 2 : (l == 0 ? 0 : 1);
            if (dev_err(ctx, fused_launch(ctx->r, mode, sh, parts[i].ld, L, fa, ctx->kp, parts[i].ntiles, false, stream)))
                return RS_EDEVICE;
        }
        return RS_OK;
    }
    if (mode == MODE_FFT || mode == MODE_IFFT)
        return run_passes(ctx, sc, stream, mode == MODE_IFFT, gen_l, L, l, d, h, d, nullptr, 0, 0, rb, ncols, aligned,
                          false, false);
    // derivative: y = B d in place, partial sums into scratch, result / B back in place
    uint8_t *Z;
    int rc = big_scratch(sc, (size_t)h * rb, &Z);
    if (!rc)
        rc = scale_rows_B(ctx, stream, d, h, rb, ncols, aligned);
    if (!rc)
        rc = run_deriv_passes(ctx, stream, L, d, Z, d, rb, ncols, aligned);
    return rc;
}

int run_xform(rs_ctx *ctx, int mode, int h, uint32_t l, void *data, size_t rb, hipStream_t stream)
{
    if (!ctx)
        return RS_EINVAL;
    if (!is_pow2(h) || h > (1 << ctx->r))
        return RS_ESHAPE;
    if (l >= (1u << ctx->r))
        return RS_EINVAL;
    if (rb % (size_t)sym_bytes(ctx))
        return RS_EALIGN;
    if (rb == 0)
        return RS_OK;
    if (!data)
        return RS_EINVAL;
    if (rb / sym_bytes(ctx) > (size_t)INT32_MAX / 2)
        return RS_ESHAPE;
    DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return RS_EDEVICE;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->sticky)
        return ctx->sticky;
    Scratch *sc = get_scratch(ctx, stream);
    if (!sc)
        return RS_ENOMEM;
    return xform_locked(ctx, sc, mode, h, l, (uint8_t *)data, rb, stream);
}

bool basis_independent(int r, const uint32_t *b)
{
    uint32_t rows[16];
    for (int j = 0; j < r; j++) {
        if (b[j] >> r)
            return false;
        rows[j] = b[j];
    }
    int rank = 0;
    for (int bit = r - 1; bit >= 0; bit--) {
        int piv = -1;
        for (int j = rank; j < r; j++)
            if ((rows[j] >> bit) & 1u) {
                piv = j;
                break;
            }
        if (piv < 0)
            continue;
        std::swap(rows[rank], rows[piv]);
        for (int j = 0; j < r; j++)
            if (j != rank && ((rows[j] >> bit) & 1u))
                rows[j] ^= rows[rank];
        rank++;
    }
    return rank == r;
}

// ------------------------------------------------------------------ polynomial operations (Sec. 6.1, Table 1)

// Launch one nb_poly kernel over every column part of a call; per_tile:
// workgroups per column tile (rows of the operation, or 1 for the degree).
int poly_run(rs_ctx *ctx, hipStream_t s, int kind, PolyArgs a, bool aligned, uint32_t per_tile, const uint32_t *t1,
             const uint32_t *t2)
{
    for (const ColPart &cp : col_parts(aligned, a.ncols)) {
        a.col0 = cp.col0;
        a.nct = cp.ntiles;
        if (dev_err(ctx, poly_launch(ctx->r, cp.ld, kind, a, t1, t2, per_tile * (uint32_t)cp.ntiles, s)))
            return RS_EDEVICE;
    }
    return RS_OK;
}

PolyArgs poly_args(const void *src, const void *src2, void *dst, size_t rb, int ncols)
{
    PolyArgs a;
    std::memset(&a, 0, sizeof(a));
    a.src = (const uint8_t *)src;
    a.src2 = (const uint8_t *)src2;
    a.dst = (uint8_t *)dst;
    a.row_bytes = rb;
    a.ncols = ncols;
    return a;
}

bool ranges_overlap(const void *p, size_t pn, const void *q, size_t qn)
{
    const uintptr_t a = (uintptr_t)p, b = (uintptr_t)q;
    return a < b + qn && b < a + pn;
}

// Shared argument checks of the polynomial calls (rows: rows of the
// operand; pow2: rows must be a power of two).
int poly_check(const rs_ctx *ctx, long rows, bool pow2, size_t rb)
{
    if (!ctx)
        return RS_EINVAL;
    if (rows < 1 || rows > (1L << ctx->r) || (pow2 && !is_pow2(rows)))
        return RS_ESHAPE;
    if (rb % (size_t)sym_bytes(ctx))
        return RS_EALIGN;
    if (rb / sym_bytes(ctx) > (size_t)INT32_MAX / 2)
        return RS_ESHAPE;
    return RS_OK;
}

// Monomial coefficients of the normalized subspace polynomials What_j,
// j < r, for the basis conversion: W_0(x) = x and W_{j+1}(x) =
// W_j(x) (W_j(x) + W_j(v_j)) (Sec. 2.2; W_j is F2-linear, so
// W_j(x + v_j) = W_j(x) + W_j(v_j)), i.e. with W_j(x) = sum_m a_m x^(2^m)
// in characteristic 2, a'_m = a_{m-1}^2 + W_j(v_j) a_m; What_j = W_j / W_j(v_j).
// Entry 16 j + m holds the coefficient of x^(2^m) in What_j; entry 256 + j
// the inverse of its leading coefficient.
constexpr uint32_t WH_COUNT = 512;

void what_coefficients(int r, const uint32_t *basis, std::vector<uint32_t> &out)
{
    out.assign(WH_COUNT, 0u);
    uint32_t a[17] = {1u};
    for (int j = 0; j < r; j++) {
        uint32_t wv = 0, vp = basis[j];                 // W_j(v_j), vp = v_j^(2^m)
        for (int m = 0; m <= j; m++) {
            wv ^= gf_mul(a[m], vp, r);
            vp = gf_mul(vp, vp, r);
        }
        const uint32_t iv = gf_inv(wv, r);
        for (int m = 0; m <= j; m++)
            out[16 * j + m] = gf_mul(a[m], iv, r);
        out[256 + j] = gf_inv(out[16 * j + j], r);
        uint32_t nx[17] = {0u};
        for (int m = 0; m <= j + 1; m++)
            nx[m] = (m ? gf_mul(a[m - 1], a[m - 1], r) : 0u) ^ (m <= j ? gf_mul(wv, a[m], r) : 0u);
        std::memcpy(a, nx, sizeof(a));
    }
}

// A pass-pipeline schedule: the level counts of 2..4 parts (low part first),
// each 4..8, summing to N, for transforms over 2^N > 256 points (GF(2^16)).
bool schedule_ok(int r, int op, int N, const int *parts, int nparts)
{
    if (r != 16 || (op != RS_OP_ENCODE && op != RS_OP_DECODE) || N <= FUSED_MAX_L || N > 16)
        return false;
    if (nparts < 2 || nparts > 4 || !parts)
        return false;
    int sum = 0;
    for (int i = 0; i < nparts; i++) {
        if (parts[i] < 4 || parts[i] > 8)
            return false;
        sum += parts[i];
    }
    return sum == N;
}

int pack_parts(const int *parts, int nparts)
{
    int v = 0;
    for (int i = nparts - 1; i >= 0; i--)
        v = (v << 4) | parts[i];
    return v;
}

// The parts of a packed schedule; 0 is the default two-part split.
void unpack_parts(int v, int N, int *parts, int *nparts)
{
    if (!v) {
        parts[0] = (N + 1) / 2;
        parts[1] = N - parts[0];
        *nparts = 2;
        return;
    }
    int m = 0;
    while (v && m < 4) {
        parts[m++] = v & 15;
        v >>= 4;
    }
    *nparts = m;
}

// RS_NB_SCHEDULE: comma-separated "enc:N:P" / "dec:N:P" entries, P the low
// part's level count or the parts' counts joined by '/', low part first,
// optionally followed by ":C", the column tile (0, 128 or 256).
bool apply_schedule_env(rs_ctx *ctx)
{
    const char *env = std::getenv("RS_NB_SCHEDULE");
    if (!env || !*env)
        return true;
    const char *p = env;
    while (*p) {
        int op;
        if (!std::strncmp(p, "enc:", 4))
            op = RS_OP_ENCODE;
        else if (!std::strncmp(p, "dec:", 4))
            op = RS_OP_DECODE;
        else
            return false;
        p += 4;
        char *end;
        const long N = std::strtol(p, &end, 10);
        if (end == p || *end != ':' || N < 0 || N > 16)
            return false;
        p = end + 1;
        int parts[4], m = 0;
        while (true) {
            const long v = std::strtol(p, &end, 10);
            if (end == p || m == 4)
                return false;
            parts[m++] = (int)v;
            p = end;
            if (*p != '/')
                break;
            p++;
        }
        long cols = 0;                                  // optional ":C", the column tile
        if (*p == ':') {
            p++;
            cols = std::strtol(p, &end, 10);
            if (end == p || (cols != 0 && cols != 128 && cols != 256))
                return false;
            p = end;
        }
        if (*p && *p != ',')
            return false;
        if (*p)
            p++;
        if (m == 1) {                                   // the low part only
            parts[1] = (int)N - parts[0];
            m = 2;
        }
        if (!schedule_ok(ctx->r, op, (int)N, parts, m))
            return false;
        ctx->sched[op][N].store(pack_parts(parts, m));
        ctx->tile[op][N].store((int)cols);
    }
    return true;
}

}  // namespace

namespace nb {

// The checks a batched call makes on one descriptor, for callers that must
// refuse a bad stripe before it joins a batch (the serving loop).
int check_stripe(rs_ctx *ctx, const rs_stripe_desc &d, bool decode, const uint8_t *mask)
{
    if (!ctx)
        return RS_EINVAL;
    Plan pl;
    return validate_stripe(ctx, d, decode, mask, pl);
}

}  // namespace nb

// ------------------------------------------------------------------ decode without allocation
//
// rs_decode_static keeps its call arena (stripe descriptors, point bitmaps
// and the per-point tables the locator writes) in this fixed device array
// instead of the per-stream arena.  Each GPU holds its own copy of it; host
// code reaches it only through the address hipGetSymbolAddress returns for
// the device (the array's name is not a device address on the host).

namespace {

constexpr size_t STATIC_SCRATCH_BYTES = 32 << 10;
static __device__ __align__(256) uint8_t static_scratch[STATIC_SCRATCH_BYTES];

constexpr int STATIC_IMAGE_WORDS = 256;
struct StaticImage {
    uint32_t nwords;
    uint32_t w[STATIC_IMAGE_WORDS];
};

// The host-built part of the arena reaches the device as a kernel argument
// (no staging buffer, no host-to-device copy); vector stores only.
__global__ __launch_bounds__(64) void k_static_upload(StaticImage img, uint32_t *dst)
{
    for (uint32_t i = threadIdx.x; i < img.nwords; i += 64u)
        dst[i] = img.w[i];
}

std::mutex static_mu;
void *static_ptr[64];
bool static_done[64];

// Address of this device's static_scratch, looked up once per device with
// that device current (rs_init calls it); null on failure.
void *static_scratch_of(int device)
{
    if (device < 0 || device >= 64)
        return nullptr;
    std::lock_guard<std::mutex> lk(static_mu);
    if (!static_done[device]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(static_scratch)) != hipSuccess)
            return nullptr;
        static_ptr[device] = ptr;
        static_done[device] = true;
    }
    return static_ptr[device];
}

}  // namespace

// ------------------------------------------------------------------ C ABI

extern "C" {

__attribute__((visibility("default"))) int rs_init(int r, const uint32_t *basis, rs_ctx **out)
{
    if (!out)
        return RS_EINVAL;
    *out = nullptr;
    if (r != 8 && r != 16)
        return RS_EFIELD;
    uint32_t b[16];
    for (int j = 0; j < r; j++)
        b[j] = basis ? basis[j] : (1u << j);
    if (!basis_independent(r, b))
        return RS_EBASIS;
    rs_ctx *ctx = new (std::nothrow) rs_ctx();
    if (!ctx)
        return RS_ENOMEM;
    ctx->r = r;
    std::memcpy(ctx->basis, b, sizeof(uint32_t) * r);
    if (!apply_schedule_env(ctx)) {
        delete ctx;
        return RS_EINVAL;
    }
    if (hipGetDevice(&ctx->device) != hipSuccess) {
        delete ctx;
        return RS_EDEVICE;
    }
    ctx->d_static = static_scratch_of(ctx->device);
    if (!ctx->d_static) {
        delete ctx;
        return RS_EDEVICE;
    }
    static std::once_flag prep_once;
    static hipError_t prep_err = hipSuccess;
    std::call_once(prep_once, [] {
        hipError_t e1 = fused_prepare_16();
        hipError_t e2 = fused_prepare_8();
        hipError_t e3 = init_prepare(16);
        hipError_t e4 = wide_prepare();
        hipError_t e5 = poly_prepare();
        prep_err = e1 != hipSuccess ? e1
                 : e2 != hipSuccess ? e2
                 : e3 != hipSuccess ? e3
                 : e4 != hipSuccess ? e4 : e5;
    });
    if (prep_err != hipSuccess) {
        delete ctx;
        return RS_EDEVICE;
    }
    const size_t q = (size_t)1 << r;
    const int ts = r == 16 ? TAB16 : TAB8;
    // dword counts of every table, one allocation
    const size_t n_basis = 16, n_Wv = 256, n_S = 256, n_wp = 16, n_skew = q, n_B = q, n_Binv = q, n_exp = q,
                 n_log = q, n_FL = 2 * q, n_tw = ts * q, n_Bt = ts * q, n_Binvt = ts * q, n_wh = WH_COUNT,
                 n_wht = ts * WH_COUNT;
    const size_t sizes[] = {n_basis, n_Wv, n_S,  n_wp,   n_skew, n_B,  n_Binv, n_exp,
                            n_log,   n_FL, n_tw, n_Bt, n_Binvt, n_wh, n_wht};
    size_t total = 0;
    for (size_t s : sizes)
        total += align_up(s * 4, 256);
    if (hipMalloc(&ctx->d_mem, total) != hipSuccess) {
        delete ctx;
        return RS_ENOMEM;
    }
    uint32_t **dst[] = {&ctx->d_basis, &ctx->d_Wv,  &ctx->d_S,      &ctx->d_wp,    &ctx->d_skew,
                        &ctx->d_B,     &ctx->d_Binv, &ctx->d_exp,    &ctx->d_log,   &ctx->d_FL,
                        &ctx->d_tw_tab, &ctx->d_B_tab, &ctx->d_Binv_tab, &ctx->d_wh, &ctx->d_wh_tab};
    size_t off = 0;
    for (size_t i = 0; i < sizeof(sizes) / sizeof(sizes[0]); i++) {
        *dst[i] = (uint32_t *)((uint8_t *)ctx->d_mem + off);
        off += align_up(sizes[i] * 4, 256);
    }
    uint32_t hb[16] = {0};
    std::memcpy(hb, b, sizeof(uint32_t) * r);
    hipError_t e = hipMemcpy(ctx->d_basis, hb, sizeof(hb), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = init_tables(r, ctx->d_basis, ctx->d_Wv, ctx->d_S, ctx->d_wp, ctx->d_skew, ctx->d_B, ctx->d_Binv,
                        ctx->d_exp, ctx->d_log, ctx->d_FL, ctx->d_tw_tab, ctx->d_B_tab, ctx->d_Binv_tab, nullptr);
    std::vector<uint32_t> wh;
    what_coefficients(r, b, wh);
    if (e == hipSuccess)
        e = hipMemcpy(ctx->d_wh, wh.data(), sizeof(uint32_t) * WH_COUNT, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = perm_tables(r, ctx->d_wh, WH_COUNT, ctx->d_wh_tab, nullptr);
    if (e == hipSuccess)
        e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        (void)hipFree(ctx->d_mem);
        delete ctx;
        return RS_EDEVICE;
    }
    ctx->kp.tw = ctx->d_tw_tab;
    ctx->kp.B = ctx->d_B_tab;
    ctx->kp.Binv = ctx->d_Binv_tab;
    ctx->kp.bits = nullptr;
    ctx->kp.rowtabs = nullptr;
    *out = ctx;
    return RS_OK;
}

__attribute__((visibility("default"))) int rs_schedule_set_parts(rs_ctx *ctx, int op, int N, const int *parts,
                                                                 int nparts)
{
    if (!ctx)
        return RS_EINVAL;
    if (ctx->r != 16 || N <= FUSED_MAX_L || N > 16)
        return RS_ESHAPE;
    if (op != RS_OP_ENCODE && op != RS_OP_DECODE)
        return RS_EINVAL;
    if (nparts == 0) {
        ctx->sched[op][N].store(0);
        return RS_OK;
    }
    if (!schedule_ok(ctx->r, op, N, parts, nparts))
        return RS_EINVAL;
    ctx->sched[op][N].store(pack_parts(parts, nparts));
    return RS_OK;
}

__attribute__((visibility("default"))) int rs_schedule_set(rs_ctx *ctx, int op, int N, int T1)
{
    const int parts[2] = {T1, N - T1};
    return rs_schedule_set_parts(ctx, op, N, parts, T1 ? 2 : 0);
}

__attribute__((visibility("default"))) int rs_schedule_get_parts(rs_ctx *ctx, int op, int N, int *parts,
                                                                 int *nparts)
{
    if (!ctx || !parts || !nparts || (op != RS_OP_ENCODE && op != RS_OP_DECODE))
        return RS_EINVAL;
    if (ctx->r != 16 || N <= FUSED_MAX_L || N > 16)
        return RS_ESHAPE;
    unpack_parts(ctx->sched[op][N].load(), N, parts, nparts);
    return RS_OK;
}

__attribute__((visibility("default"))) int rs_schedule_set_tile(rs_ctx *ctx, int op, int N, int cols)
{
    if (!ctx)
        return RS_EINVAL;
    if (ctx->r != 16 || N <= FUSED_MAX_L || N > 16)
        return RS_ESHAPE;
    if ((op != RS_OP_ENCODE && op != RS_OP_DECODE) || (cols != 0 && cols != 128 && cols != 256))
        return RS_EINVAL;
    ctx->tile[op][N].store(cols);
    return RS_OK;
}

__attribute__((visibility("default"))) int rs_schedule_get_tile(rs_ctx *ctx, int op, int N, int *cols)
{
    if (!ctx || !cols || (op != RS_OP_ENCODE && op != RS_OP_DECODE))
        return RS_EINVAL;
    if (ctx->r != 16 || N <= FUSED_MAX_L || N > 16)
        return RS_ESHAPE;
    *cols = ctx->tile[op][N].load();
    return RS_OK;
}

__attribute__((visibility("default"))) int rs_schedule_get(rs_ctx *ctx, int op, int N, int *T1)
{
    if (!T1)
        return RS_EINVAL;
    int parts[4], m = 0;
    const int rc = rs_schedule_get_parts(ctx, op, N, parts, &m);
    if (!rc)
        *T1 = parts[0];
    return rc;
}

__attribute__((visibility("default"))) void rs_free(rs_ctx *ctx)
{
    if (!ctx)
        return;
    DeviceGuard guard(ctx->device);
    (void)hipDeviceSynchronize();
    for (Scratch *sc : ctx->scratch) {
        if (sc->dev)
            (void)hipFree(sc->dev);
        if (sc->big)
            (void)hipFree(sc->big);
        for (const Staging::Rec &r : sc->stg.live)
            (void)hipEventDestroy(r.ev);
        for (hipEvent_t ev : sc->stg.pool)
            (void)hipEventDestroy(ev);
        if (sc->stg.host)
            (void)hipHostFree(sc->stg.host);
        delete sc;
    }
    if (ctx->d_mem)
        (void)hipFree(ctx->d_mem);
    delete ctx;
}

__attribute__((visibility("default"))) int rs_encode(rs_ctx *ctx, int n, int k, const void *msg, void *parity,
                                                     size_t row_bytes, void *stream)
{
    rs_stripe_desc d;
    d.n = n;
    d.k = k;
    d.row_bytes = row_bytes;
    d.in = msg;
    d.out = parity;
    return run_codec(ctx, &d, nullptr, 1, false, (hipStream_t)stream);
}

__attribute__((visibility("default"))) int rs_decode(rs_ctx *ctx, int n, int k, const uint8_t *erasure_mask,
                                                     const void *shards, void *out, size_t row_bytes,
                                                     void *stream)
{
    rs_stripe_desc d;
    d.n = n;
    d.k = k;
    d.row_bytes = row_bytes;
    d.in = shards;
    d.out = out;
    return run_codec(ctx, &d, erasure_mask, 1, true, (hipStream_t)stream);
}

__attribute__((visibility("default"))) int rs_decode_static(rs_ctx *ctx, int n, int k, const uint8_t *erasure_mask,
                                                            const void *shards, void *out, size_t row_bytes,
                                                            void *stream)
{
    if (!ctx)
        return RS_EINVAL;
    int kp, np;
    int rc = mother_shape(ctx, n, k, &kp, &np);
    if (rc)
        return rc;
    if (np > 1 << FUSED_MAX_L)
        return RS_ESHAPE;                  // the pass pipelines need 2 n' rows of scratch
    rs_stripe_desc d;
    d.n = n;
    d.k = k;
    d.row_bytes = row_bytes;
    d.in = shards;
    d.out = out;
    CodecPlan cp;
    rc = build_codec(ctx, &d, erasure_mask, 1, true, ScratchFn(), cp);   // no pass pipelines: no scratch
    if (rc)
        return rc;
    if (cp.empty())
        return RS_OK;
    if (cp.dev_bytes > STATIC_SCRATCH_BYTES || cp.host.size() > sizeof(uint32_t) * STATIC_IMAGE_WORDS)
        return RS_ESHAPE;
    DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return RS_EDEVICE;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->sticky)
        return ctx->sticky;
    StaticImage img;
    std::memset(&img, 0, sizeof(img));
    img.nwords = (uint32_t)((cp.host.size() + 3) / 4);
    std::memcpy(img.w, cp.host.data(), cp.host.size());
    hipStream_t s = (hipStream_t)stream;
    uint8_t *dev = (uint8_t *)ctx->d_static;
    hipLaunchKernelGGL(k_static_upload, dim3(1), dim3(64), 0, s, img, (uint32_t *)dev);
    if (dev_err(ctx, hipGetLastError()))
        return RS_EDEVICE;
    return exec_codec(ctx, cp, dev, s);
}

__attribute__((visibility("default"))) int rs_encode_batch(rs_ctx *ctx, const rs_stripe_desc *descs, int count,
                                                           void *stream)
{
    return run_codec(ctx, descs, nullptr, count, false, (hipStream_t)stream);
}

__attribute__((visibility("default"))) int rs_decode_batch(rs_ctx *ctx, const rs_stripe_desc *descs,
                                                           const uint8_t *masks, int count, void *stream)
{
    return run_codec(ctx, descs, masks, count, true, (hipStream_t)stream);
}

__attribute__((visibility("default"))) int nb_fft(rs_ctx *ctx, int h, uint32_t l, void *data, size_t row_bytes,
                                                  void *stream)
{
    return run_xform(ctx, MODE_FFT, h, l, data, row_bytes, (hipStream_t)stream);
}

__attribute__((visibility("default"))) int nb_ifft(rs_ctx *ctx, int h, uint32_t l, void *data, size_t row_bytes,
                                                   void *stream)
{
    return run_xform(ctx, MODE_IFFT, h, l, data, row_bytes, (hipStream_t)stream);
}

__attribute__((visibility("default"))) int nb_derivative(rs_ctx *ctx, int h, void *data, size_t row_bytes,
                                                         void *stream)
{
    return run_xform(ctx, MODE_DERIV, h, 0, data, row_bytes, (hipStream_t)stream);
}

__attribute__((visibility("default"))) int nb_polymul(rs_ctx *ctx, int h, uint32_t l, const void *a, const void *b,
                                                      void *out, size_t row_bytes, void *stream_)
{
    const hipStream_t stream = (hipStream_t)stream_;
    int rc = poly_check(ctx, 2L * h, true, row_bytes);
    if (rc)
        return rc;
    if (l >= (1u << ctx->r))
        return RS_EINVAL;
    if (row_bytes == 0)
        return RS_OK;
    const size_t rb = row_bytes, in_bytes = (size_t)h * rb, out_bytes = 2 * in_bytes;
    if (!a || !b || !out || ranges_overlap(out, out_bytes, a, in_bytes) || ranges_overlap(out, out_bytes, b, in_bytes))
        return RS_EINVAL;
    DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return RS_EDEVICE;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->sticky)
        return ctx->sticky;
    Scratch *sc = get_scratch(ctx, stream);
    if (!sc)
        return RS_ENOMEM;
    uint8_t *Z;
    if ((rc = big_scratch(sc, out_bytes, &Z)))
        return rc;
    const int H = 2 * h, LH = ilog2(H), ncols = (int)(rb / sym_bytes(ctx));
    // A and B padded with zeros to 2h coefficients and transformed at 2h
    // points (into out and Z), multiplied point by point, transformed back
    if (LH > FUSED_MAX_L) {
        // pass pipelines: the first forward pass reads the h rows of the
        // operand and zeros above them, so no padding copy is needed
        const bool gen_l = (l & (uint32_t)(H - 1)) != 0;
        if ((rc = run_passes(ctx, sc, stream, false, gen_l, LH, l, (const uint8_t *)a, h, (uint8_t *)out, nullptr, 0, 0,
                             rb, ncols, vec_aligned(ctx, a, out, rb), false, false)))
            return rc;
        // B's last pass multiplies its values by A's, point by point, into out
        if ((rc = run_passes(ctx, sc, stream, false, gen_l, LH, l, (const uint8_t *)b, h, Z, (uint8_t *)out, 0, H, rb,
                             ncols, vec_aligned(ctx, b, Z, rb) && vec_aligned(ctx, out, out, rb), false, false,
                             (const uint8_t *)out)))
            return rc;
    } else {
        PolyArgs pa = poly_args(a, nullptr, out, rb, ncols);
        pa.rows = H;
        pa.src_rows = h;
        if ((rc = poly_run(ctx, stream, PK_PAD, pa, vec_aligned(ctx, a, out, rb), (uint32_t)H, nullptr, nullptr)))
            return rc;
        pa.src = (const uint8_t *)b;
        pa.dst = Z;
        if ((rc = poly_run(ctx, stream, PK_PAD, pa, vec_aligned(ctx, b, Z, rb), (uint32_t)H, nullptr, nullptr)))
            return rc;
        if ((rc = xform_locked(ctx, sc, MODE_FFT, H, l, (uint8_t *)out, rb, stream)))
            return rc;
        if ((rc = xform_locked(ctx, sc, MODE_FFT, H, l, Z, rb, stream)))
            return rc;
        PolyArgs pm = poly_args(nullptr, Z, out, rb, ncols);
        pm.rows = H;
        if ((rc = poly_run(ctx, stream, PK_MUL, pm, vec_aligned(ctx, out, Z, rb), (uint32_t)H, ctx->d_log,
                           ctx->d_exp)))
            return rc;
    }
    return xform_locked(ctx, sc, MODE_IFFT, H, l, (uint8_t *)out, rb, stream);
}

__attribute__((visibility("default"))) int nb_degree(rs_ctx *ctx, int h, const void *data, size_t row_bytes,
                                                     int32_t *deg, void *stream_)
{
    const hipStream_t stream = (hipStream_t)stream_;
    int rc = poly_check(ctx, h, false, row_bytes);
    if (rc)
        return rc;
    if (row_bytes == 0)
        return RS_OK;
    if (!data || !deg)
        return RS_EINVAL;
    DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return RS_EDEVICE;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->sticky)
        return ctx->sticky;
    PolyArgs pa = poly_args(data, nullptr, nullptr, row_bytes, (int)(row_bytes / sym_bytes(ctx)));
    pa.deg = deg;
    pa.rows = h;
    return poly_run(ctx, stream, PK_DEGREE, pa, vec_aligned(ctx, data, data, row_bytes), 1u, nullptr, nullptr);
}

// Shared body of the two conversions.
static int convert(rs_ctx *ctx, int h, void *data, size_t rb, hipStream_t stream, bool to_mono)
{
    int rc = poly_check(ctx, h, true, rb);
    if (rc)
        return rc;
    if (rb == 0 || h == 1)
        return RS_OK;                                    // X_0 = 1
    if (!data)
        return RS_EINVAL;
    DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return RS_EDEVICE;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->sticky)
        return ctx->sticky;
    const int L = ilog2(h), ncols = (int)(rb / sym_bytes(ctx));
    uint8_t *d = (uint8_t *)data;
    const bool aligned = vec_aligned(ctx, d, d, rb);
    if (to_mono) {
        Scratch *sc = get_scratch(ctx, stream);
        if (!sc)
            return RS_ENOMEM;
        uint8_t *Z;
        if ((rc = big_scratch(sc, (size_t)h * rb, &Z)))
            return rc;
        // levels 1 .. min(L, 8) in one launch, in place (each workgroup holds
        // its 256-row block in LDS); the higher ones level by level
        const int LB = std::min(L, CONV_TILE_L);
        PolyArgs pt = poly_args(d, nullptr, d, rb, ncols);
        pt.rows = h;
        pt.t = LB;
        if ((rc = poly_run(ctx, stream, PK_UP_TILE, pt, aligned, (uint32_t)(h >> LB), ctx->d_wh_tab, nullptr)))
            return rc;
        uint8_t *cur = d, *oth = Z;
        for (int t = LB + 1; t <= L; t++) {
            PolyArgs pa = poly_args(cur, nullptr, oth, rb, ncols);
            pa.rows = h;
            pa.t = t;
            if ((rc = poly_run(ctx, stream, PK_UP, pa, aligned, (uint32_t)h, ctx->d_wh_tab, nullptr)))
                return rc;
            std::swap(cur, oth);
        }
        if (cur != d) {                                  // odd level count: copy back
            PolyArgs pa = poly_args(cur, nullptr, d, rb, ncols);
            pa.rows = pa.src_rows = h;
            return poly_run(ctx, stream, PK_PAD, pa, aligned, (uint32_t)h, nullptr, nullptr);
        }
        return RS_OK;
    }
    const int LB = std::min(L, CONV_TILE_L);
    for (int t = L; t > LB; t--) {
        const int hh = 1 << (t - 1), nblk = h >> t;
        PolyArgs pa = poly_args(nullptr, nullptr, d, rb, ncols);
        pa.rows = h;
        pa.t = t;
        for (int e1 = hh; e1 > 0; e1 /= 2) {             // quotient ranges, top first
            pa.e1 = e1;
            pa.e0 = e1 / 2;
            if ((rc = poly_run(ctx, stream, PK_DOWN, pa, aligned, (uint32_t)(nblk * (pa.e1 - pa.e0)), ctx->d_wh_tab,
                               nullptr)))
                return rc;
        }
        if (t > 1) {                                     // remainders (t = 1: the coefficient itself)
            pa.e0 = pa.e1 = 0;
            if ((rc = poly_run(ctx, stream, PK_DOWN, pa, aligned, (uint32_t)(nblk * hh), ctx->d_wh_tab, nullptr)))
                return rc;
        }
    }
    // levels min(L, 8) .. 1 in one launch, each workgroup on its 256-row block
    PolyArgs pt = poly_args(nullptr, nullptr, d, rb, ncols);
    pt.rows = h;
    pt.t = LB;
    return poly_run(ctx, stream, PK_DOWN_TILE, pt, aligned, (uint32_t)(h >> LB), ctx->d_wh_tab, nullptr);
}

__attribute__((visibility("default"))) int nb_to_monomial(rs_ctx *ctx, int h, void *data, size_t row_bytes,
                                                          void *stream)
{
    return convert(ctx, h, data, row_bytes, (hipStream_t)stream, true);
}

__attribute__((visibility("default"))) int nb_from_monomial(rs_ctx *ctx, int h, void *data, size_t row_bytes,
                                                            void *stream)
{
    return convert(ctx, h, data, row_bytes, (hipStream_t)stream, false);
}

struct rs_plan {
    rs_ctx *ctx = nullptr;
    CodecPlan cp;
    uint8_t *arena = nullptr;
    uint8_t *scratch = nullptr;
    int count = 0;                // stripes of the batch
    uint64_t *ts = nullptr;       // completion timestamps (rs_plan_set_timestamps)
    StampMap *sm = nullptr;       // their slots, built on the first rs_plan_set_timestamps
    bool located = false;         // decode: the locator's tables were computed at creation
};

static int plan_batch(rs_ctx *ctx, const rs_stripe_desc *descs, const uint8_t *masks, int count, bool decode,
                      rs_plan **out)
{
    if (!ctx || !out)
        return RS_EINVAL;
    *out = nullptr;
    rs_plan *pl = new (std::nothrow) rs_plan();
    if (!pl)
        return RS_ENOMEM;
    pl->ctx = ctx;
    pl->count = count;
    DeviceGuard guard(ctx->device);
    int rc = guard.ok ? RS_OK : RS_EDEVICE;
    if (!rc)                                    // the plan's own scratch for its pass pipelines
        rc = build_codec(ctx, descs, masks, count, decode, [&](size_t need, uint8_t **base) -> int {
            if (hipMalloc((void **)&pl->scratch, need) != hipSuccess) {
                pl->scratch = nullptr;
                return RS_ENOMEM;
            }
            *base = pl->scratch;
            return RS_OK;
        }, pl->cp);
    if (!rc && pl->cp.dev_bytes) {
        if (hipMalloc((void **)&pl->arena, pl->cp.dev_bytes) != hipSuccess) {
            pl->arena = nullptr;
            rc = RS_ENOMEM;
        } else if (!pl->cp.host.empty() &&
                   hipMemcpy(pl->arena, pl->cp.host.data(), pl->cp.host.size(), hipMemcpyHostToDevice) !=
                       hipSuccess) {
            rc = RS_EDEVICE;
        }
    }
    if (!rc && decode && pl->cp.dev_bytes) {
        // the locator's tables depend only on the plan's fixed erasure
        // patterns: computed here once, so launches run the decode passes only
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
            rc = RS_EDEVICE;
        else {
            rc = run_locator(ctx, pl->cp, pl->arena, st);
            if (hipStreamSynchronize(st) != hipSuccess && !rc)
                rc = RS_EDEVICE;
            (void)hipStreamDestroy(st);
        }
        pl->located = rc == RS_OK;
    }
    if (rc) {
        if (pl->arena)
            (void)hipFree(pl->arena);
        if (pl->scratch)
            (void)hipFree(pl->scratch);
        delete pl;
        return rc;
    }
    pl->cp.host.clear();
    pl->cp.host.shrink_to_fit();
    *out = pl;
    return RS_OK;
}

__attribute__((visibility("default"))) int rs_plan_encode_batch(rs_ctx *ctx, const rs_stripe_desc *descs, int count,
                                                                rs_plan **out)
{
    return plan_batch(ctx, descs, nullptr, count, false, out);
}

__attribute__((visibility("default"))) int rs_plan_decode_batch(rs_ctx *ctx, const rs_stripe_desc *descs,
                                                                const uint8_t *masks, int count, rs_plan **out)
{
    return plan_batch(ctx, descs, masks, count, true, out);
}

__attribute__((visibility("default"))) int rs_plan_launch(rs_plan *plan, void *stream)
{
    if (!plan)
        return RS_EINVAL;
    rs_ctx *ctx = plan->ctx;
    DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return RS_EDEVICE;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (ctx->sticky)
            return ctx->sticky;
    }
    const StampMap *sm = plan->ts ? plan->sm : nullptr;
    if (plan->cp.empty()) {
        if (sm && (dev_err(ctx, stamp_start(plan->ts, sm->slots, sm->nslots, (hipStream_t)stream)) ||
                   dev_err(ctx, stamp_reduce(plan->ts, sm->slots, sm->seg_ptr, sm->segs, plan->count,
                                             (hipStream_t)stream))))
            return RS_EDEVICE;
        return RS_OK;
    }
    return exec_codec(ctx, plan->cp, plan->arena, (hipStream_t)stream, sm, plan->ts, plan->count, plan->located);
}

__attribute__((visibility("default"))) int rs_plan_set_timestamps(rs_plan *plan, uint64_t *dev_ts, int *clock_khz)
{
    if (!plan)
        return RS_EINVAL;
    DeviceGuard guard(plan->ctx->device);
    if (!guard.ok)
        return RS_EDEVICE;
    if (clock_khz && hipDeviceGetAttribute(clock_khz, hipDeviceAttributeWallClockRate, plan->ctx->device) != hipSuccess)
        return RS_EDEVICE;
    if (dev_ts && !plan->sm) {
        StampMap *sm = new (std::nothrow) StampMap();
        if (!sm)
            return RS_ENOMEM;
        std::vector<uint32_t> seg_ptr, segs;
        int rc = stamp_ranges(plan->cp, plan->count, *sm, seg_ptr, segs);
        if (rc) {
            delete sm;
            return rc;
        }
        const size_t b_slots = sm->nslots * sizeof(uint64_t), b_ptr = seg_ptr.size() * sizeof(uint32_t),
                     b_segs = segs.size() * sizeof(uint32_t);
        if (hipMalloc((void **)&sm->dev, b_slots + b_ptr + b_segs + 8) != hipSuccess) {
            (void)hipGetLastError();
            delete sm;
            return RS_ENOMEM;
        }
        sm->slots = (uint64_t *)sm->dev;
        sm->seg_ptr = (const uint32_t *)(sm->dev + b_slots);
        sm->segs = (const uint32_t *)(sm->dev + b_slots + b_ptr);
        if (hipMemcpy(sm->dev + b_slots, seg_ptr.data(), b_ptr, hipMemcpyHostToDevice) != hipSuccess ||
            (b_segs && hipMemcpy(sm->dev + b_slots + b_ptr, segs.data(), b_segs, hipMemcpyHostToDevice) != hipSuccess)) {
            (void)hipFree(sm->dev);
            delete sm;
            return RS_EDEVICE;
        }
        plan->sm = sm;
    }
    plan->ts = dev_ts;
    return RS_OK;
}

__attribute__((visibility("default"))) void rs_plan_free(rs_plan *plan)
{
    if (!plan)
        return;
    DeviceGuard guard(plan->ctx->device);
    (void)hipDeviceSynchronize();
    if (plan->arena)
        (void)hipFree(plan->arena);
    if (plan->scratch)
        (void)hipFree(plan->scratch);
    if (plan->sm) {
        (void)hipFree(plan->sm->dev);
        delete plan->sm;
    }
    delete plan;
}

__attribute__((visibility("default"))) int rs_sync(rs_ctx *ctx, void *stream)
{
    if (!ctx)
        return RS_EINVAL;
    DeviceGuard guard(ctx->device);
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
        ctx->sticky = RS_EDEVICE;
    return ctx->sticky;
}

__attribute__((visibility("default"))) int rs_get_table(rs_ctx *ctx, int which, uint32_t *host_out, size_t count)
{
    if (!ctx || !host_out)
        return RS_EINVAL;
    const size_t q = (size_t)1 << ctx->r;
    const uint32_t *src = nullptr;
    size_t len = 0;
    switch (which) {
    case RS_TAB_SKEW: src = ctx->d_skew; len = q - 1; break;
    case RS_TAB_B: src = ctx->d_B; len = q; break;
    case RS_TAB_BINV: src = ctx->d_Binv; len = q; break;
    case RS_TAB_LOG: src = ctx->d_log; len = q; break;
    case RS_TAB_EXP: src = ctx->d_exp; len = q; break;
    default: return RS_EINVAL;
    }
    if (count < len)
        return RS_EINVAL;
    DeviceGuard guard(ctx->device);
    if (hipMemcpy(host_out, src, len * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return RS_EDEVICE;
    return (int)len;
}

__attribute__((visibility("default"))) const char *rs_strerror(int code)
{
    switch (code) {
    case RS_OK: return "success";
    case RS_EINVAL: return "invalid argument";
    case RS_EFIELD: return "unsupported field (r must be 8 or 16)";
    case RS_EBASIS: return "basis is not F2-independent";
    case RS_ESHAPE: return "unsupported transform size or code shape";
    case RS_ETOOMANY: return "more erasures than parity symbols";
    case RS_EALIGN: return "row length is not a multiple of the symbol size";
    case RS_ENOMEM: return "out of memory";
    case RS_EDEVICE: return "device error";
    default: return "unknown error";
    }
}

}  // extern "C"
