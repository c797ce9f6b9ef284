// nb_init.hip -- device-side generation of the method tables (run once per
// context): subspace-polynomial values on the basis, the skew-factor table
// (Sec. 3.5), the derivative table B (Sec. 4.2, eq. B), log/exp and the
// Walsh-Hadamard transforms of the logarithm vectors L_N (appendix), and the
// perm tables of every constant the hot kernels multiply by.
#include "nb_device.hpp"
#include "nb_internal.hpp"

#include <algorithm>

namespace nb {

// One thread.  Wv[i*r + j] = W_i(v_j) through W_0(x) = x and
// W_{i+1}(x) = W_i(x) (W_i(x) + W_i(v_i)), which follows from the product
// definition (eq. w_j(x)) and additivity (Lemma 1): W_{i+1}(x) = W_i(x) W_i(x + v_i).
// S[i*r + j] = W_i(v_j) / W_i(v_i).  wp[i] = W_i'(x) / W_i(v_i) (eq. W-l),
// with the constant W_{i+1}' = W_i' W_i(v_i) obtained by differentiating the
// same recursion (W_0' = 1).
__global__ void k_init_basis(int r, const uint32_t *__restrict__ basis, uint32_t *__restrict__ Wv,
                             uint32_t *__restrict__ S, uint32_t *__restrict__ wp)
{
    if (threadIdx.x != 0 || blockIdx.x != 0)
        return;
    uint32_t w[16];
    for (int j = 0; j < r; j++)
        w[j] = basis[j];
    uint32_t dconst = 1;
    for (int i = 0; i < r; i++) {
        for (int j = 0; j < r; j++)
            Wv[i * r + j] = w[j];
        const uint32_t wvi = w[i];
        const uint32_t inv = gf_inv(wvi, r);
        for (int j = 0; j < r; j++)
            S[i * r + j] = gf_mul(w[j], inv, r);
        wp[i] = gf_mul(dconst, inv, r);
        dconst = gf_mul(dconst, wvi, r);
        for (int j = 0; j < r; j++)
            w[j] = gf_mul(w[j], w[j] ^ wvi, r);
    }
}

// Skew-factor table: entry (level i, block index b) = What_i(omega_{b 2^{i+1}}),
// flat offset 2^r - 2^{r-i} + b.  By additivity it is the XOR of
// What_i(v_{t+i+1}) over the set bits t of b.
__global__ void k_init_skew(int r, const uint32_t *__restrict__ S, uint32_t *__restrict__ skew)
{
    const uint32_t total = (1u << r) - 1u;
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
        int i = 0;
        while (e >= (1u << r) - (1u << (r - i - 1)))
            i++;
        const uint32_t b = e - ((1u << r) - (1u << (r - i)));
        uint32_t acc = 0;
        for (int t = 0; t + i + 1 < r; t++)
            if ((b >> t) & 1u)
                acc ^= S[i * r + t + i + 1];
        skew[e] = acc;
    }
}

// B_j = prod over the set bits t of j of W'_t (eq. B) and its inverse.
__global__ void k_init_B(int r, const uint32_t *__restrict__ wp, uint32_t *__restrict__ B,
                         uint32_t *__restrict__ Binv)
{
    const uint32_t total = 1u << r;
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < total; j += gridDim.x * blockDim.x) {
        uint32_t acc = 1;
        for (int t = 0; t < r; t++)
            if ((j >> t) & 1u)
                acc = gf_mul(acc, wp[t], r);
        B[j] = acc;
        Binv[j] = gf_inv(acc, r);
    }
}

// alpha^e for alpha = 2, and the discrete log (Log(0) = 0, appendix).
__global__ void k_init_logexp(int r, uint32_t *__restrict__ expt, uint32_t *__restrict__ logt)
{
    const uint32_t M = (1u << r) - 1u;
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e <= M; e += gridDim.x * blockDim.x) {
        if (e == M) {
            expt[M] = 1;
            logt[0] = 0;
            continue;
        }
        const uint32_t x = gf_pow(2u, e, r);
        expt[e] = x;
        logt[x] = e;
    }
}

__global__ void k_init_perm(int r, const uint32_t *__restrict__ vals, uint32_t count, uint32_t *__restrict__ tabs)
{
    const int ts = r == 16 ? TAB16 : TAB8;
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < count; e += gridDim.x * blockDim.x) {
        uint32_t t[TAB16];
        build_perm_table(vals[e], r, t);
        for (int u = 0; u < ts; u++)
            tabs[(size_t)ts * e + u] = t[u];
    }
}

// ---------------------------------------------------------------- Walsh-Hadamard mod 2^r - 1

__device__ __forceinline__ uint32_t addm(uint32_t a, uint32_t b, uint32_t M)
{
    const uint32_t s = a + b;
    return s >= M ? s - M : s;
}

__device__ __forceinline__ uint32_t subm(uint32_t a, uint32_t b, uint32_t M)
{
    return a >= b ? a - b : a + M - b;
}

__device__ __forceinline__ uint32_t mulm(uint32_t a, uint32_t b, int r)
{
    const uint32_t M = (1u << r) - 1u;
    uint32_t p = a * b;                        // a, b < 2^16: fits
    p = (p & M) + (p >> r);
    p = (p & M) + (p >> r);
    return p >= M ? p - M : p;
}

// In-place length-N Walsh-Hadamard transform of v (LDS) modulo M.
__device__ void fwht_lds(uint16_t *v, int N, uint32_t M)
{
    for (int len = 1; len < N; len <<= 1) {
        for (int idx = threadIdx.x; idx < N / 2; idx += blockDim.x) {
            const int i = ((idx & ~(len - 1)) << 1) | (idx & (len - 1));
            const uint32_t u = v[i], w = v[i + len];
            v[i] = (uint16_t)addm(u, w, M);
            v[i + len] = (uint16_t)subm(u, w, M);
        }
        __syncthreads();
    }
}

// Block t computes FWHT_N(L_N) for N = 2^t, L_N[u] = Log(omega_u) (Log(0) = 0),
// stored at FL + N - 1.
__global__ void k_init_fwhtL(int r, const uint32_t *__restrict__ basis, const uint32_t *__restrict__ logt,
                             uint32_t *__restrict__ FL)
{
    extern __shared__ uint16_t v16[];
    const int N = 1 << blockIdx.x;
    const uint32_t M = (1u << r) - 1u;
    for (int u = threadIdx.x; u < N; u += blockDim.x) {
        uint32_t w = 0;
        for (int j = 0; j < r; j++)
            if ((u >> j) & 1)
                w ^= basis[j];
        v16[u] = (uint16_t)(u ? logt[w] : 0u);
    }
    __syncthreads();
    fwht_lds(v16, N, M);
    for (int u = threadIdx.x; u < N; u += blockDim.x)
        FL[N - 1 + u] = v16[u];
}

// ---------------------------------------------------------------- locator (decode step 1)


// One block per stripe.  Log Pi(omega_p) (p not erased) and Log Pi'(omega_p)
// (p erased) for every point p < N of the mother code are the XOR convolution
// of the erasure indicator R with L_N, computed as
// FWHT(FWHT(R) * FWHT(L_N)) / N modulo 2^r - 1 (appendix, eq. Rnmathrmw; the
// division by N is the inverse transform's normalisation, 2^{r - lg N} mod
// 2^r - 1).  The stripe's per-point scale factors, Pi(omega_p) for survivors
// and 1 / Pi'(omega_p) for erasures, are written as perm tables.
__global__ void k_locator(LocatorArgs a, const uint32_t *__restrict__ p_bits, uint32_t *__restrict__ p_rowtabs,
                          const uint32_t *__restrict__ fwht_L, const uint32_t *__restrict__ expt)
{
    extern __shared__ uint16_t v16[];
    const DevStripe st = a.stripes[blockIdx.x];
    const int r = a.r;
    const int N = st.np;
    const uint32_t M = (1u << r) - 1u;
    const uint32_t *__restrict__ rxb = p_bits + st.bits_off;   // received points
    int lgN = 0;
    while ((1 << lgN) < N)
        lgN++;
    for (int p = threadIdx.x; p < N; p += blockDim.x) {
        // erased in the mother code: neither received nor a virtual zero
        const bool er = !((rxb[p >> 5] >> (p & 31)) & 1u) && !(p >= st.k && p < st.kp);
        v16[p] = er ? 1 : 0;
    }
    __syncthreads();
    fwht_lds(v16, N, M);
    const uint32_t *FLN = fwht_L + (N - 1);
    for (int p = threadIdx.x; p < N; p += blockDim.x)
        v16[p] = (uint16_t)mulm(v16[p], FLN[p], r);
    __syncthreads();
    fwht_lds(v16, N, M);
    const int sh = (r - lgN) % r;
    const int ts = r == 16 ? TAB16 : TAB8;
    uint32_t *out = p_rowtabs + st.rowtab_off;
    for (int p = threadIdx.x; p < N; p += blockDim.x) {
        uint32_t lg = v16[p];
        if (sh)
            lg = ((lg << sh) | (lg >> (r - sh))) & M;
        const bool er = !((rxb[p >> 5] >> (p & 31)) & 1u) && !(p >= st.k && p < st.kp);
        const uint32_t e = er ? (M - lg) % M : lg;
        if (r == 16)
            store_perm_table<16>(expt[e], out + (size_t)ts * p);
        else
            store_perm_table<8>(expt[e], out + (size_t)ts * p);
    }
}

// Locator for large n' (one stripe, many workgroups): the same two
// Walsh-Hadamard transforms as k_locator on a global array v of n' residues,
// in three passes over groups of 2^T1 consecutive points (the low levels)
// or of 2^T2 points at stride 2^T1 (the high levels).  The levels of a
// Walsh-Hadamard transform commute, so the second transform can take its
// high levels first, right after the pointwise product.  Kinds: 0 =
// indicator of erased points, then the first transform's low levels; 1 =
// its high levels, times FWHT(L_N), the second transform's high levels; 2 =
// the second transform's low levels, then the normalisation, exponentials
// and per-point perm tables as k_locator writes them.
__global__ __launch_bounds__(256) void k_loc_pass(LocPassArgs a, const uint32_t *__restrict__ p_bits,
                                                  uint32_t *__restrict__ p_rowtabs,
                                                  const uint32_t *__restrict__ fwht_L,
                                                  const uint32_t *__restrict__ expt)
{
    __shared__ uint32_t v[256];
    const DevStripe st = *a.stripe;
    const int r = a.r, T = a.T, lo = a.lo, H = 1 << T;
    const uint32_t M = (1u << r) - 1u;
    const uint32_t *__restrict__ rxb = p_bits + st.bits_off;
    const uint32_t gi = blockIdx.x;
    const uint32_t gbase = (gi & ((1u << lo) - 1u)) | ((gi >> lo) << (lo + T));
    auto erased = [&](uint32_t p) {
        return !((rxb[p >> 5] >> (p & 31)) & 1u) && !((int)p >= st.k && (int)p < st.kp);
    };
    for (int j = threadIdx.x; j < H; j += blockDim.x) {
        const uint32_t p = gbase + ((uint32_t)j << lo);
        v[j] = a.kind == 0 ? (erased(p) ? 1u : 0u) : a.v[p];
    }
    __syncthreads();
    auto levels = [&]() {
        for (int len = 1; len < H; len <<= 1) {
            for (int idx = threadIdx.x; idx < H / 2; idx += blockDim.x) {
                const int i = ((idx & ~(len - 1)) << 1) | (idx & (len - 1));
                const uint32_t u = v[i], w = v[i + len];
                v[i] = addm(u, w, M);
                v[i + len] = subm(u, w, M);
            }
            __syncthreads();
        }
    };
    levels();
    if (a.kind == 1) {
        const uint32_t *FLN = fwht_L + (st.np - 1);
        for (int j = threadIdx.x; j < H; j += blockDim.x)
            v[j] = mulm(v[j], FLN[gbase + ((uint32_t)j << lo)], r);
        __syncthreads();
        levels();
    }
    int lgN = 0;
    while ((1 << lgN) < st.np)
        lgN++;
    const int sh = (r - lgN) % r;
    const int ts = r == 16 ? TAB16 : TAB8;
    uint32_t *out = p_rowtabs + st.rowtab_off;
    for (int j = threadIdx.x; j < H; j += blockDim.x) {
        const uint32_t p = gbase + ((uint32_t)j << lo);
        uint32_t x = v[j];
        if (a.kind != 2) {
            a.v[p] = x;
            continue;
        }
        if (sh)
            x = ((x << sh) | (x >> (r - sh))) & M;
        const uint32_t e = erased(p) ? (M - x) % M : x % M;
        if (r == 16)
            store_perm_table<16>(expt[e], out + (size_t)ts * p);
        else
            store_perm_table<8>(expt[e], out + (size_t)ts * p);
    }
}

// ---------------------------------------------------------------- launchers

hipError_t init_tables(int r, const uint32_t *d_basis, uint32_t *d_Wv, uint32_t *d_S, uint32_t *d_wp,
                       uint32_t *d_skew, uint32_t *d_B, uint32_t *d_Binv, uint32_t *d_exp, uint32_t *d_log,
                       uint32_t *d_FL, uint32_t *d_tw_tab, uint32_t *d_B_tab, uint32_t *d_Binv_tab, hipStream_t s)
{
    const uint32_t q = 1u << r;
    hipLaunchKernelGGL(k_init_basis, dim3(1), dim3(64), 0, s, r, d_basis, d_Wv, d_S, d_wp);
    hipLaunchKernelGGL(k_init_skew, dim3(256), dim3(256), 0, s, r, (const uint32_t *)d_S, d_skew);
    hipLaunchKernelGGL(k_init_B, dim3(256), dim3(256), 0, s, r, (const uint32_t *)d_wp, d_B, d_Binv);
    hipLaunchKernelGGL(k_init_logexp, dim3(256), dim3(256), 0, s, r, d_exp, d_log);
    hipLaunchKernelGGL(k_init_fwhtL, dim3(r + 1), dim3(1024), (size_t)q * 2, s, r, d_basis,
                       (const uint32_t *)d_log, d_FL);
    hipLaunchKernelGGL(k_init_perm, dim3(256), dim3(256), 0, s, r, (const uint32_t *)d_skew, q - 1, d_tw_tab);
    hipLaunchKernelGGL(k_init_perm, dim3(256), dim3(256), 0, s, r, (const uint32_t *)d_B, q, d_B_tab);
    hipLaunchKernelGGL(k_init_perm, dim3(256), dim3(256), 0, s, r, (const uint32_t *)d_Binv, q, d_Binv_tab);
    return hipGetLastError();
}

// Start of a timed plan launch: ts[0] = the device's real-time counter, and
// the per-workgroup slots the kernels stamp are cleared.  A kernel rather
// than a memset, so that the launch can be captured in a graph.
__global__ void k_stamp_start(uint64_t *__restrict__ ts, uint64_t *__restrict__ slots, size_t nslots)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0)
        ts[0] = __builtin_amdgcn_s_memrealtime();
    for (; i < nslots; i += (size_t)gridDim.x * blockDim.x)
        slots[i] = 0ull;
}

hipError_t stamp_start(uint64_t *ts, uint64_t *slots, size_t nslots, hipStream_t s)
{
    const size_t blocks = (nslots + 255) / 256;
    hipLaunchKernelGGL(k_stamp_start, dim3(blocks < 1 ? 1 : blocks > 1024 ? 1024 : (unsigned)blocks), dim3(256), 0, s,
                       ts, slots, nslots);
    return hipGetLastError();
}

// End of a timed plan launch: ts[1 + i] = the latest stamp among the slots
// of the workgroups that worked on stripe i (slot ranges segs[2 j] ..
// segs[2 j + 1] - 1 for j in seg_ptr[i] .. seg_ptr[i + 1] - 1), 0 when there
// are none.  One workgroup per stripe.
__global__ __launch_bounds__(256) void k_stamp_reduce(uint64_t *__restrict__ ts, const uint64_t *__restrict__ slots,
                                                      const uint32_t *__restrict__ seg_ptr,
                                                      const uint32_t *__restrict__ segs)
{
    __shared__ uint64_t red[256];
    const int i = blockIdx.x, t = threadIdx.x;
    uint64_t m = 0;
    for (uint32_t j = seg_ptr[i]; j < seg_ptr[i + 1]; j++)
        for (uint32_t k = segs[2 * j] + t; k < segs[2 * j + 1]; k += 256)
            m = slots[k] > m ? slots[k] : m;
    red[t] = m;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h && red[t + h] > red[t])
            red[t] = red[t + h];
        __syncthreads();
    }
    if (t == 0)
        ts[1 + i] = red[0];
}

hipError_t stamp_reduce(uint64_t *ts, const uint64_t *slots, const uint32_t *seg_ptr, const uint32_t *segs,
                        int nstripes, hipStream_t s)
{
    if (nstripes <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_stamp_reduce, dim3(nstripes), dim3(256), 0, s, ts, slots, seg_ptr, segs);
    return hipGetLastError();
}

// Perm tables of `count` field elements (vals, device) into tabs.
hipError_t perm_tables(int r, const uint32_t *vals, uint32_t count, uint32_t *tabs, hipStream_t s)
{
    hipLaunchKernelGGL(k_init_perm, dim3(8), dim3(256), 0, s, r, vals, count, tabs);
    return hipGetLastError();
}

hipError_t init_prepare(int r)
{
    const int lds = (int)((1u << r) * 2);
    hipError_t e = hipFuncSetAttribute((const void *)k_init_fwhtL, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    hipError_t f = hipFuncSetAttribute((const void *)k_locator, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    return e != hipSuccess ? e : f;
}

hipError_t loc_pass_launch(const LocPassArgs &a, const KPtrs &k, const uint32_t *fwht_L, const uint32_t *expt,
                           int ngroups, hipStream_t s)
{
    hipLaunchKernelGGL(k_loc_pass, dim3(ngroups), dim3(256), 0, s, a, k.bits, (uint32_t *)k.rowtabs, fwht_L, expt);
    return hipGetLastError();
}

hipError_t locator_launch(const LocatorArgs &a, const KPtrs &k, const uint32_t *fwht_L, const uint32_t *expt,
                          int nstripes, int max_np, hipStream_t s)
{
    if (nstripes <= 0)
        return hipSuccess;
    // one butterfly per thread and level for the largest stripe (the kernel
    // loops over points and butterflies with the block's stride)
    const int threads = std::min(1024, std::max(64, (max_np / 2 + 63) / 64 * 64));
    hipLaunchKernelGGL(k_locator, dim3(nstripes), dim3(threads), (size_t)max_np * 2, s, a, k.bits,
                       (uint32_t *)k.rowtabs, fwht_L, expt);
    return hipGetLastError();
}

}  // namespace nb
