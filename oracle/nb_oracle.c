/*
 * nb_oracle.c -- plain, slow, obviously-correct CPU oracle for the novel
 * polynomial basis over GF(2^r), its O(h lg h) transform and inverse, the
 * formal derivative, and the (n, k) Reed-Solomon erasure codec built on them
 * (Lin, Chung, Han, "Novel Polynomial Basis and Its Application to
 * Reed-Solomon Erasure Codes", arXiv:1404.3458).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The GPU library never
 * links, includes or calls it, and it shares no code, table or constant
 * generator with the GPU library.
 *
 * Two tiers:
 *   - definitional: each quantity written out from its definition (naive
 *     products, naive O(h^2) evaluation, Lagrange interpolation, monomial
 *     expansion and term-by-term differentiation);
 *   - algorithmic: the paper's fast algorithms, step for step (Sec. 3.2 and
 *     3.3 transforms, Sec. 4 derivative, Algorithms 1 and 2, the appendix
 *     locator), with every factor computed from the definitional tier.
 *
 * Conventions the paper leaves open (fixed identically in the GPU library's
 * public header; the reasons are in the design notes):
 *   - field polynomial 0x11D for r = 8, 0x1100B for r = 16; primitive
 *     element alpha = 2 (used only by the locator's logarithms);
 *   - symbol t of a row is byte t (r = 8) or the little-endian 16-bit word at
 *     bytes 2t, 2t+1 (r = 16); bit b of a symbol is the coefficient of x^b;
 *   - basis v_0..v_{r-1}; NULL means v_j = 2^j, so omega_i = i;
 *   - code shortening for k or n not a power of two: k' = pow2ceil(k),
 *     n' = pow2ceil(k' + n - k); message rows are points omega_0..omega_{k-1},
 *     points omega_k..omega_{k'-1} hold virtual zeros, stored parity row t
 *     is point omega_{k'+t}; points omega_{k'+n-k}..omega_{n'-1} are never
 *     stored and count as erasures when decoding.
 *
 * Every function returns 0 on success and -1 on an invalid argument unless
 * it returns a field element.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EXPORT __attribute__((visibility("default")))

/* ------------------------------------------------------------------ */
/* Field GF(2^r) (Sec. 2.1).                                           */
/* ------------------------------------------------------------------ */

ORC_EXPORT uint32_t orc_field_poly(int r)
{
    return r == 8 ? 0x11Du : (r == 16 ? 0x1100Bu : 0u);
}

static int field_ok(int r) { return r == 8 || r == 16; }

/* Schoolbook carry-less product of two r-bit polynomials over GF(2),
 * followed by long-division reduction by the field polynomial. */
ORC_EXPORT uint32_t orc_mul(int r, uint32_t a, uint32_t b)
{
    uint32_t poly = orc_field_poly(r);
    uint32_t p = 0;
    for (int t = 0; t < r; t++)
        if ((b >> t) & 1u)
            p ^= a << t;
    for (int t = 2 * r - 2; t >= r; t--)
        if ((p >> t) & 1u)
            p ^= poly << (t - r);
    return p;
}

ORC_EXPORT uint32_t orc_pow(int r, uint32_t a, uint64_t e)
{
    uint32_t acc = 1, base = a;
    while (e) {
        if (e & 1u)
            acc = orc_mul(r, acc, base);
        base = orc_mul(r, base, base);
        e >>= 1;
    }
    return acc;
}

/* a^{-1} = a^{2^r - 2} (the multiplicative group has order 2^r - 1). */
ORC_EXPORT uint32_t orc_inv(int r, uint32_t a)
{
    return orc_pow(r, a, ((uint64_t)1 << r) - 2);
}

/* ------------------------------------------------------------------ */
/* Points omega_i (Sec. 2.1, eq. binaryrepresentation).                */
/* ------------------------------------------------------------------ */

static uint32_t basis_vec(const uint32_t *basis, int j)
{
    return basis ? basis[j] : (1u << j);
}

ORC_EXPORT uint32_t orc_omega(int r, const uint32_t *basis, uint32_t i)
{
    uint32_t w = 0;
    for (int j = 0; j < r; j++)
        if ((i >> j) & 1u)
            w ^= basis_vec(basis, j);
    return w;
}

/* ------------------------------------------------------------------ */
/* Subspace vanishing polynomial W_j (Sec. 2.2, eq. w_j(x)) and the    */
/* basis X_i (Sec. 2.3, eq. X_i(x)).                                   */
/* ------------------------------------------------------------------ */

/* W_j(x) = prod_{i < 2^j} (x + omega_i), evaluated by the naive product. */
ORC_EXPORT uint32_t orc_W(int r, const uint32_t *basis, int j, uint32_t x)
{
    uint32_t acc = 1;
    for (uint32_t i = 0; i < (1u << j); i++)
        acc = orc_mul(r, acc, x ^ orc_omega(r, basis, i));
    return acc;
}

/* W_j(x) / W_j(omega_{2^j}); omega_{2^j} = v_j. */
ORC_EXPORT uint32_t orc_What(int r, const uint32_t *basis, int j, uint32_t x)
{
    uint32_t norm = orc_W(r, basis, j, orc_omega(r, basis, 1u << j));
    return orc_mul(r, orc_W(r, basis, j, x), orc_inv(r, norm));
}

/* X_i(x) = prod over the set bits j of i of W_j(x) / W_j(omega_{2^j}). */
ORC_EXPORT uint32_t orc_X(int r, const uint32_t *basis, uint32_t i, uint32_t x)
{
    uint32_t acc = 1;
    for (int j = 0; j < r; j++)
        if ((i >> j) & 1u)
            acc = orc_mul(r, acc, orc_What(r, basis, j, x));
    return acc;
}

/* ------------------------------------------------------------------ */
/* Polynomials in the monomial basis (definitional tier helpers).      */
/* coef[t] is the coefficient of x^t.                                  */
/* ------------------------------------------------------------------ */

ORC_EXPORT uint32_t orc_poly_eval(int r, int len, const uint32_t *coef, uint32_t x)
{
    uint32_t acc = 0;
    for (int t = len - 1; t >= 0; t--)
        acc = orc_mul(r, acc, x) ^ coef[t];
    return acc;
}

/* out (len a + len b - 1 entries) = a * b */
static void poly_mul(int r, const uint32_t *a, int la, const uint32_t *b, int lb, uint32_t *out)
{
    memset(out, 0, sizeof(uint32_t) * (size_t)(la + lb - 1));
    for (int s = 0; s < la; s++)
        for (int t = 0; t < lb; t++)
            out[s + t] ^= orc_mul(r, a[s], b[t]);
}

/* Monomial coefficients of W_j: 2^j + 1 entries. */
ORC_EXPORT int orc_W_monomial(int r, const uint32_t *basis, int j, uint32_t *coef)
{
    if (!field_ok(r) || j < 0 || j >= r || !coef)
        return -1;
    int deg = 1 << j;
    memset(coef, 0, sizeof(uint32_t) * (size_t)(deg + 1));
    coef[0] = 1;
    for (int i = 0; i < deg; i++) {
        /* multiply the degree-i polynomial by (x + omega_i) */
        uint32_t w = orc_omega(r, basis, (uint32_t)i);
        for (int t = i + 1; t >= 1; t--)
            coef[t] = coef[t - 1] ^ orc_mul(r, w, coef[t]);
        coef[0] = orc_mul(r, w, coef[0]);
    }
    return 0;
}

/* Monomial coefficients of X_i: i + 1 entries (deg X_i = i). */
ORC_EXPORT int orc_X_monomial(int r, const uint32_t *basis, uint32_t i, uint32_t *coef)
{
    if (!field_ok(r) || !coef || i >= (1u << r))
        return -1;
    int cap = (int)i + 1;
    uint32_t *acc = calloc((size_t)cap + 1, sizeof(uint32_t));
    uint32_t *tmp = calloc((size_t)cap + 1, sizeof(uint32_t));
    uint32_t *wj = calloc((size_t)cap + 1, sizeof(uint32_t));
    if (!acc || !tmp || !wj) {
        free(acc); free(tmp); free(wj);
        return -1;
    }
    int len = 1;
    acc[0] = 1;
    for (int j = 0; j < r; j++) {
        if (!((i >> j) & 1u))
            continue;
        int dj = 1 << j;
        orc_W_monomial(r, basis, j, wj);
        uint32_t inv = orc_inv(r, orc_W(r, basis, j, orc_omega(r, basis, 1u << j)));
        for (int t = 0; t <= dj; t++)
            wj[t] = orc_mul(r, wj[t], inv);
        poly_mul(r, acc, len, wj, dj + 1, tmp);
        len += dj;
        memcpy(acc, tmp, sizeof(uint32_t) * (size_t)len);
    }
    memcpy(coef, acc, sizeof(uint32_t) * (size_t)cap);
    free(acc); free(tmp); free(wj);
    return 0;
}

/* [D_h](x) = sum_i d_i X_i(x) (Definition 1) rewritten in the monomial
 * basis: h coefficients. */
ORC_EXPORT int orc_to_monomial(int r, const uint32_t *basis, int h, const uint32_t *d, uint32_t *mono)
{
    if (!field_ok(r) || h < 1 || h > (1 << r) || !d || !mono)
        return -1;
    uint32_t *xi = calloc((size_t)h, sizeof(uint32_t));
    if (!xi)
        return -1;
    memset(mono, 0, sizeof(uint32_t) * (size_t)h);
    for (int i = 0; i < h; i++) {
        if (!d[i])
            continue;
        orc_X_monomial(r, basis, (uint32_t)i, xi);
        for (int t = 0; t <= i; t++)
            mono[t] ^= orc_mul(r, d[i], xi[t]);
    }
    free(xi);
    return 0;
}

/* Term-by-term formal derivative (proof of Lemma 3): c x^t -> c x^{t-1}
 * for odd t, 0 for even t.  out has len entries, out[len-1] = 0. */
ORC_EXPORT int orc_monomial_derivative(int r, int len, const uint32_t *mono, uint32_t *out)
{
    (void)r;
    if (len < 1 || !mono || !out)
        return -1;
    for (int t = 0; t < len; t++)
        out[t] = (t + 1 < len && ((t + 1) & 1)) ? mono[t + 1] : 0;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Transform Psi_h^l, definitional (Sec. 3, definition of Psi):        */
/* out[b] = [D_h](omega_b + omega_l) by naive evaluation.              */
/* ------------------------------------------------------------------ */

static int is_pow2(long v) { return v > 0 && (v & (v - 1)) == 0; }
static int ilog2(long v) { int t = 0; while ((1L << t) < v) t++; return t; }

ORC_EXPORT int orc_eval_naive(int r, const uint32_t *basis, int h, uint32_t l,
                              const uint32_t *d, uint32_t *out)
{
    if (!field_ok(r) || !is_pow2(h) || h > (1 << r) || l >= (1u << r) || !d || !out)
        return -1;
    int lg = ilog2(h);
    uint32_t *wh = calloc((size_t)(lg + 1), sizeof(uint32_t));
    if (!wh)
        return -1;
    for (int b = 0; b < h; b++) {
        uint32_t x = orc_omega(r, basis, (uint32_t)b) ^ orc_omega(r, basis, l);
        for (int j = 0; j < lg; j++)
            wh[j] = orc_What(r, basis, j, x);
        uint32_t acc = 0;
        for (int i = 0; i < h; i++) {
            uint32_t xi = 1;            /* X_i(x) from its factors */
            for (int j = 0; j < lg; j++)
                if ((i >> j) & 1)
                    xi = orc_mul(r, xi, wh[j]);
            acc ^= orc_mul(r, d[i], xi);
        }
        out[b] = acc;
    }
    free(wh);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Transform Psi_h^l, algorithmic (Sec. 3.2) and its inverse (Sec. 3.3).*/
/* In-place layout: Delta_i^m(omega_c + omega_l) lives at index c + m   */
/* (c a multiple of 2^i, m < 2^i), so the output is in natural order.   */
/* ------------------------------------------------------------------ */

/* Factor W_i(omega_c + omega_l) / W_i(omega_{2^i}) for every level i and
 * block c (a multiple of 2^{i+1}); precomputed as Sec. 3.2 allows.
 * Layout: level i starts at offset sum_{i' < i} h / 2^{i'+1}. */
static uint32_t *make_factors(int r, const uint32_t *basis, int h, uint32_t l)
{
    int lg = ilog2(h);
    uint32_t *f = calloc((size_t)(h > 1 ? h - 1 : 1), sizeof(uint32_t));
    if (!f)
        return NULL;
    uint32_t wl = orc_omega(r, basis, l);
    int off = 0;
    for (int i = 0; i < lg; i++) {
        int step = 2 << i;
        for (int c = 0; c < h; c += step)
            f[off + c / step] = orc_What(r, basis, i, orc_omega(r, basis, (uint32_t)c) ^ wl);
        off += h / step;
    }
    return f;
}

static void fft_core(int r, const uint32_t *basis, int h, uint32_t l, const uint32_t *f,
                     uint32_t *x, int64_t *counts)
{
    int lg = ilog2(h);
    uint32_t wl = orc_omega(r, basis, l);
    for (int i = lg - 1; i >= 0; i--) {
        int half = 1 << i, step = 2 << i;
        int off = h - (h >> i);          /* sum_{i' < i} h / 2^{i'+1} */
        for (int c = 0; c < h; c += step) {
            uint32_t s = f[off + c / step];
            int zero_point = (orc_omega(r, basis, (uint32_t)c) ^ wl) == 0;
            for (int m = 0; m < half; m++) {
                uint32_t a = x[c + m], b = x[c + m + half];
                if (!zero_point) {                       /* eq. Deltajimcoplusl */
                    a ^= orc_mul(r, s, b);
                    if (counts) { counts[0] += 1; counts[1] += 1; }
                }                                        /* else eq. Deltajim0 */
                b ^= a;                                  /* eq. Deltajimcoplusloplusi2 */
                if (counts) counts[0] += 1;
                x[c + m] = a;
                x[c + m + half] = b;
            }
        }
    }
}

static void ifft_core(int r, const uint32_t *basis, int h, uint32_t l, const uint32_t *f,
                      uint32_t *x, int64_t *counts)
{
    int lg = ilog2(h);
    uint32_t wl = orc_omega(r, basis, l);
    for (int i = 0; i < lg; i++) {
        int half = 1 << i, step = 2 << i;
        int off = h - (h >> i);
        for (int c = 0; c < h; c += step) {
            uint32_t s = f[off + c / step];
            int zero_point = (orc_omega(r, basis, (uint32_t)c) ^ wl) == 0;
            for (int m = 0; m < half; m++) {
                uint32_t a = x[c + m], b = x[c + m + half];
                b ^= a;                                  /* eq. Deltaj22imiomegacomegal */
                if (counts) counts[0] += 1;
                if (!zero_point) {                       /* eq. Deltaj22imomegacomegal */
                    a ^= orc_mul(r, s, b);
                    if (counts) { counts[0] += 1; counts[1] += 1; }
                }
                x[c + m] = a;
                x[c + m + half] = b;
            }
        }
    }
}

static int xform_args_ok(int r, int h, uint32_t l)
{
    return field_ok(r) && is_pow2(h) && h <= (1 << r) && l < (1u << r);
}

/* counts (optional): counts[0] += additions, counts[1] += multiplications */
ORC_EXPORT int orc_fft_vec(int r, const uint32_t *basis, int h, uint32_t l, uint32_t *x, int64_t *counts)
{
    if (!xform_args_ok(r, h, l) || !x)
        return -1;
    uint32_t *f = make_factors(r, basis, h, l);
    if (!f)
        return -1;
    fft_core(r, basis, h, l, f, x, counts);
    free(f);
    return 0;
}

ORC_EXPORT int orc_ifft_vec(int r, const uint32_t *basis, int h, uint32_t l, uint32_t *x, int64_t *counts)
{
    if (!xform_args_ok(r, h, l) || !x)
        return -1;
    uint32_t *f = make_factors(r, basis, h, l);
    if (!f)
        return -1;
    ifft_core(r, basis, h, l, f, x, counts);
    free(f);
    return 0;
}

/* Skew-factor table as the space-complexity paragraph (Sec. 3.5) counts it:
 * the h - 1 factors of an h-point transform, level-major. */
ORC_EXPORT int orc_factors(int r, const uint32_t *basis, int h, uint32_t l, uint32_t *out)
{
    if (!xform_args_ok(r, h, l) || !out)
        return -1;
    uint32_t *f = make_factors(r, basis, h, l);
    if (!f)
        return -1;
    memcpy(out, f, sizeof(uint32_t) * (size_t)(h - 1));
    free(f);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Formal derivative (Sec. 4).                                          */
/* ------------------------------------------------------------------ */

/* Normalised W'_l of eq. W-l: (prod_{j=1}^{2^l - 1} omega_j) / W_l(omega_{2^l}),
 * the numerator being the constant derivative of W_l given by Lemma 3. */
ORC_EXPORT uint32_t orc_Wprime_norm(int r, const uint32_t *basis, int l)
{
    uint32_t num = 1;
    for (uint32_t j = 1; j < (1u << l); j++)
        num = orc_mul(r, num, orc_omega(r, basis, j));
    uint32_t den = orc_W(r, basis, l, orc_omega(r, basis, 1u << l));
    return orc_mul(r, num, orc_inv(r, den));
}

/* eq. D'_h(x)-2: coefficient of X_j is sum_{l < lg h, bit l of j clear}
 * W'_l d_{j + 2^l}. */
ORC_EXPORT int orc_deriv_direct_vec(int r, const uint32_t *basis, int h, const uint32_t *d, uint32_t *out)
{
    if (!field_ok(r) || !is_pow2(h) || h > (1 << r) || !d || !out)
        return -1;
    int lg = ilog2(h);
    uint32_t wp[17];
    for (int l = 0; l < lg; l++)
        wp[l] = orc_Wprime_norm(r, basis, l);
    for (int j = 0; j < h; j++) {
        uint32_t acc = 0;
        for (int l = 0; l < lg; l++)
            if (!((j >> l) & 1))
                acc ^= orc_mul(r, wp[l], d[j + (1 << l)]);
        out[j] = acc;
    }
    return 0;
}

/* Sec. 4.2 (eqs. dimathrmd, XDhx3, B): B_i = prod_{j in I_i} W'_j,
 * d^d_i = d_i B_i, coefficient of X_j = (sum_{l not in I_j} d^d_{j+2^l}) / B_j. */
ORC_EXPORT int orc_deriv_B_vec(int r, const uint32_t *basis, int h, const uint32_t *d, uint32_t *out)
{
    if (!field_ok(r) || !is_pow2(h) || h > (1 << r) || !d || !out)
        return -1;
    int lg = ilog2(h);
    uint32_t wp[17];
    for (int l = 0; l < lg; l++)
        wp[l] = orc_Wprime_norm(r, basis, l);
    uint32_t *B = calloc((size_t)h, sizeof(uint32_t));
    uint32_t *dd = calloc((size_t)h, sizeof(uint32_t));
    if (!B || !dd) {
        free(B); free(dd);
        return -1;
    }
    for (int i = 0; i < h; i++) {
        uint32_t b = 1;
        for (int j = 0; j < lg; j++)
            if ((i >> j) & 1)
                b = orc_mul(r, b, wp[j]);
        B[i] = b;
        dd[i] = orc_mul(r, d[i], b);
    }
    for (int j = 0; j < h; j++) {
        uint32_t acc = 0;
        for (int l = 0; l < lg; l++)
            if (!((j >> l) & 1))
                acc ^= dd[j + (1 << l)];
        out[j] = orc_mul(r, acc, orc_inv(r, B[j]));
    }
    free(B); free(dd);
    return 0;
}

/* The table B itself (eq. B), h entries. */
ORC_EXPORT int orc_B_table(int r, const uint32_t *basis, int h, uint32_t *out)
{
    if (!field_ok(r) || !is_pow2(h) || h > (1 << r) || !out)
        return -1;
    int lg = ilog2(h);
    uint32_t wp[17];
    for (int l = 0; l < lg; l++)
        wp[l] = orc_Wprime_norm(r, basis, l);
    for (int i = 0; i < h; i++) {
        uint32_t b = 1;
        for (int j = 0; j < lg; j++)
            if ((i >> j) & 1)
                b = orc_mul(r, b, wp[j]);
        out[i] = b;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Row/column stripe helpers.  Row t starts at base + t * stride;      */
/* symbol c of a row at byte c (r = 8) or bytes 2c, 2c+1 little-endian. */
/* ------------------------------------------------------------------ */

static uint32_t get_sym(int r, const uint8_t *row, size_t c)
{
    if (r == 8)
        return row[c];
    return (uint32_t)row[2 * c] | ((uint32_t)row[2 * c + 1] << 8);
}

static void put_sym(int r, uint8_t *row, size_t c, uint32_t v)
{
    if (r == 8) {
        row[c] = (uint8_t)v;
    } else {
        row[2 * c] = (uint8_t)(v & 0xFF);
        row[2 * c + 1] = (uint8_t)(v >> 8);
    }
}

static int rows_xform(int r, const uint32_t *basis, int h, uint32_t l, uint8_t *data,
                      size_t stride, size_t ncols, int inverse)
{
    if (!xform_args_ok(r, h, l) || !data)
        return -1;
    uint32_t *f = make_factors(r, basis, h, l);
    uint32_t *x = calloc((size_t)h, sizeof(uint32_t));
    if (!f || !x) {
        free(f); free(x);
        return -1;
    }
    for (size_t c = 0; c < ncols; c++) {
        for (int t = 0; t < h; t++)
            x[t] = get_sym(r, data + (size_t)t * stride, c);
        if (inverse)
            ifft_core(r, basis, h, l, f, x, NULL);
        else
            fft_core(r, basis, h, l, f, x, NULL);
        for (int t = 0; t < h; t++)
            put_sym(r, data + (size_t)t * stride, c, x[t]);
    }
    free(f); free(x);
    return 0;
}

ORC_EXPORT int orc_fft_rows(int r, const uint32_t *basis, int h, uint32_t l, uint8_t *data,
                            size_t stride, size_t ncols)
{
    return rows_xform(r, basis, h, l, data, stride, ncols, 0);
}

ORC_EXPORT int orc_ifft_rows(int r, const uint32_t *basis, int h, uint32_t l, uint8_t *data,
                             size_t stride, size_t ncols)
{
    return rows_xform(r, basis, h, l, data, stride, ncols, 1);
}

ORC_EXPORT int orc_deriv_rows(int r, const uint32_t *basis, int h, uint8_t *data,
                              size_t stride, size_t ncols)
{
    if (!field_ok(r) || !is_pow2(h) || h > (1 << r) || !data)
        return -1;
    uint32_t *x = calloc((size_t)h, sizeof(uint32_t));
    uint32_t *y = calloc((size_t)h, sizeof(uint32_t));
    if (!x || !y) {
        free(x); free(y);
        return -1;
    }
    for (size_t c = 0; c < ncols; c++) {
        for (int t = 0; t < h; t++)
            x[t] = get_sym(r, data + (size_t)t * stride, c);
        orc_deriv_B_vec(r, basis, h, x, y);
        for (int t = 0; t < h; t++)
            put_sym(r, data + (size_t)t * stride, c, y[t]);
    }
    free(x); free(y);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Code shape with shortening (one sentence in Sec. 5; reading fixed    */
/* in the header comment).                                              */
/* ------------------------------------------------------------------ */

static long pow2ceil(long v) { long p = 1; while (p < v) p <<= 1; return p; }

ORC_EXPORT int orc_mother_shape(int r, int n, int k, int *kp, int *np)
{
    if (!field_ok(r) || k < 1 || n <= k)
        return -1;
    long k2 = pow2ceil(k);
    long n2 = pow2ceil(k2 + (long)n - k);
    if (n2 > (1L << r))
        return -1;
    if (kp) *kp = (int)k2;
    if (np) *np = (int)n2;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Algorithm 1 (encoding).                                              */
/* ------------------------------------------------------------------ */

ORC_EXPORT int orc_encode(int r, const uint32_t *basis, int n, int k, const uint8_t *msg,
                          uint8_t *parity, size_t stride, size_t ncols)
{
    int kp, np;
    if (orc_mother_shape(r, n, k, &kp, &np) || !msg || !parity)
        return -1;
    int nblocks = np / kp;
    uint32_t *f0 = make_factors(r, basis, kp, 0);
    uint32_t **fb = calloc((size_t)nblocks, sizeof(uint32_t *));
    uint32_t *mbar = calloc((size_t)kp, sizeof(uint32_t));
    uint32_t *blk = calloc((size_t)kp, sizeof(uint32_t));
    int ok = f0 && fb && mbar && blk;
    for (int i = 1; ok && i < nblocks; i++)
        ok = (fb[i] = make_factors(r, basis, kp, (uint32_t)(i * kp))) != NULL;
    if (ok) {
        for (size_t c = 0; c < ncols; c++) {
            for (int t = 0; t < kp; t++)
                mbar[t] = t < k ? get_sym(r, msg + (size_t)t * stride, c) : 0;
            ifft_core(r, basis, kp, 0, f0, mbar, NULL);             /* step 1 */
            for (int i = 1; i < nblocks; i++) {                     /* steps 2-4 */
                memcpy(blk, mbar, sizeof(uint32_t) * (size_t)kp);
                fft_core(r, basis, kp, (uint32_t)(i * kp), fb[i], blk, NULL);
                for (int j = 0; j < kp; j++) {
                    long t = (long)i * kp + j - kp;                 /* parity row */
                    if (t < n - k)
                        put_sym(r, parity + (size_t)t * stride, c, blk[j]);
                }
            }
        }
    }
    for (int i = 1; fb && i < nblocks; i++)
        free(fb[i]);
    free(fb); free(f0); free(mbar); free(blk);
    return ok ? 0 : -1;
}

/* Definitional encoder: Lagrange interpolation through the k' points
 * (omega_i, m_i), with m_i = 0 for the virtual rows, evaluated at the
 * parity points (Sec. 5, eq. F(i)=m_i). */
ORC_EXPORT int orc_encode_lagrange(int r, const uint32_t *basis, int n, int k, const uint8_t *msg,
                                   uint8_t *parity, size_t stride, size_t ncols)
{
    int kp, np;
    if (orc_mother_shape(r, n, k, &kp, &np) || !msg || !parity)
        return -1;
    for (size_t c = 0; c < ncols; c++) {
        for (int t = 0; t < n - k; t++) {
            uint32_t x = orc_omega(r, basis, (uint32_t)(kp + t));
            uint32_t acc = 0;
            for (int i = 0; i < k; i++) {          /* virtual zeros contribute 0 */
                uint32_t xi = orc_omega(r, basis, (uint32_t)i);
                uint32_t num = 1, den = 1;
                for (int u = 0; u < kp; u++) {
                    if (u == i)
                        continue;
                    uint32_t xu = orc_omega(r, basis, (uint32_t)u);
                    num = orc_mul(r, num, x ^ xu);
                    den = orc_mul(r, den, xi ^ xu);
                }
                uint32_t mi = get_sym(r, msg + (size_t)i * stride, c);
                acc ^= orc_mul(r, mi, orc_mul(r, num, orc_inv(r, den)));
            }
            put_sym(r, parity + (size_t)t * stride, c, acc);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Erasure locator (appendix).                                          */
/* ------------------------------------------------------------------ */

/* Walsh-Hadamard transform of length N over the integers modulo 2^r - 1
 * (the appendix notes all of its arithmetic may be done modulo 2^r - 1). */
ORC_EXPORT int orc_fwht_mod(int r, int N, uint32_t *v)
{
    if (!field_ok(r) || !is_pow2(N) || N > (1 << r) || !v)
        return -1;
    uint64_t M = ((uint64_t)1 << r) - 1;
    for (int len = 1; len < N; len <<= 1)
        for (int i = 0; i < N; i += 2 * len)
            for (int j = i; j < i + len; j++) {
                uint64_t u = v[j], w = v[j + len];
                v[j] = (uint32_t)((u + w) % M);
                v[j + len] = (uint32_t)((u + M - w) % M);
            }
    return 0;
}

/* Discrete logarithm to base alpha = 2 with Log(0) := 0 (appendix). */
static uint32_t *make_log(int r)
{
    uint32_t q = 1u << r;
    uint32_t *lg = calloc(q, sizeof(uint32_t));
    if (!lg)
        return NULL;
    uint32_t x = 1;
    for (uint32_t e = 0; e < q - 1; e++) {
        lg[x] = e;
        x = orc_mul(r, x, 2);
    }
    return lg;
}

/* Log Pi(omega_j) (j not erased) or Log Pi'(omega_j) (j erased) for all
 * j < N, as the XOR convolution of R and L computed with Walsh-Hadamard
 * transforms (appendix, eq. Rnmathrmw).  For N < 2^r the result is scaled
 * by N^{-1} = 2^{r - lg N} modulo 2^r - 1, the inverse transform's factor,
 * which equals 1 only when N = 2^r. */
ORC_EXPORT int orc_locator_fwht(int r, const uint32_t *basis, int N, const uint8_t *erased, uint32_t *logval)
{
    if (!field_ok(r) || !is_pow2(N) || N > (1 << r) || !erased || !logval)
        return -1;
    uint64_t M = ((uint64_t)1 << r) - 1;
    uint32_t *lg = make_log(r);
    uint32_t *L = calloc((size_t)N, sizeof(uint32_t));
    if (!lg || !L) {
        free(lg); free(L);
        return -1;
    }
    for (int t = 0; t < N; t++) {
        L[t] = t == 0 ? 0 : lg[orc_omega(r, basis, (uint32_t)t)];
        logval[t] = erased[t] ? 1 : 0;
    }
    orc_fwht_mod(r, N, L);
    orc_fwht_mod(r, N, logval);
    for (int t = 0; t < N; t++)
        logval[t] = (uint32_t)(((uint64_t)logval[t] * L[t]) % M);
    orc_fwht_mod(r, N, logval);
    uint64_t ninv = ((uint64_t)1 << (r - ilog2(N))) % M;
    for (int t = 0; t < N; t++)
        logval[t] = (uint32_t)((logval[t] * ninv) % M);
    free(lg); free(L);
    return 0;
}

/* Same quantities by direct products (appendix, eq. Pi'(j)2 and the
 * definition of Pi): val[j] = prod_{y in E, y != j} (omega_j + omega_y). */
ORC_EXPORT int orc_locator_direct(int r, const uint32_t *basis, int N, const uint8_t *erased, uint32_t *val)
{
    if (!field_ok(r) || !is_pow2(N) || N > (1 << r) || !erased || !val)
        return -1;
    for (int j = 0; j < N; j++) {
        uint32_t acc = 1, wj = orc_omega(r, basis, (uint32_t)j);
        for (int y = 0; y < N; y++)
            if (erased[y] && y != j)
                acc = orc_mul(r, acc, wj ^ orc_omega(r, basis, (uint32_t)y));
        val[j] = acc;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Algorithm 2 (erasure decoding).                                      */
/* ------------------------------------------------------------------ */

/* Map a stored row to its point of the mother code, and back. */
static long row_to_point(int k, int kp, long t) { return t < k ? t : (long)kp + (t - k); }

ORC_EXPORT int orc_decode(int r, const uint32_t *basis, int n, int k, const uint8_t *mask,
                          const uint8_t *shards, uint8_t *out, size_t stride, size_t ncols,
                          int locator)
{
    int kp, np;
    if (orc_mother_shape(r, n, k, &kp, &np) || !mask || !shards || !out)
        return -1;
    int e = 0;
    for (int t = 0; t < n; t++)
        e += mask[t] ? 1 : 0;
    if (e > n - k)
        return -2;
    /* point-indexed erasure set of the mother code */
    uint8_t *er = calloc((size_t)np, 1);
    long *point_row = calloc((size_t)np, sizeof(long));
    uint32_t *cst = calloc((size_t)np, sizeof(uint32_t));
    uint32_t *v = calloc((size_t)np, sizeof(uint32_t));
    uint32_t *vd = calloc((size_t)np, sizeof(uint32_t));
    uint32_t *f0 = make_factors(r, basis, np, 0);
    int ok = er && point_row && cst && v && vd && f0;
    if (!ok)
        goto done;
    for (long p = 0; p < np; p++)
        point_row[p] = -1;
    for (long t = 0; t < n; t++)
        point_row[row_to_point(k, kp, t)] = t;
    for (long p = 0; p < np; p++) {
        long t = point_row[p];
        if (t >= 0)
            er[p] = mask[t] ? 1 : 0;
        else
            er[p] = p >= k && p < kp ? 0 : 1;    /* virtual zero, or never stored */
    }
    /* step 1: Pi(omega_p) for p not erased, Pi'(omega_p) for p erased */
    if (locator == 0) {
        uint64_t M = ((uint64_t)1 << r) - 1;
        ok = orc_locator_fwht(r, basis, np, er, cst) == 0;
        uint32_t x = 1, q = 1u << r;
        uint32_t *ex = calloc(q, sizeof(uint32_t));
        ok = ok && ex;
        for (uint32_t i = 0; ok && i < q - 1; i++) {
            ex[i] = x;
            x = orc_mul(r, x, 2);
        }
        for (long p = 0; ok && p < np; p++)
            cst[p] = ex[cst[p] % M];
        free(ex);
    } else {
        ok = orc_locator_direct(r, basis, np, er, cst) == 0;
    }
    if (!ok)
        goto done;
    for (long p = 0; p < np; p++)
        if (er[p])
            cst[p] = orc_inv(r, cst[p]);              /* divisor of step 6 */
    for (size_t c = 0; c < ncols; c++) {
        for (long p = 0; p < np; p++) {               /* step 2, eq. hatF(l) */
            long t = point_row[p];
            uint32_t rx = (t >= 0 && !er[p]) ? get_sym(r, shards + (size_t)t * stride, c) : 0;
            v[p] = er[p] ? 0 : orc_mul(r, rx, cst[p]);
        }
        ifft_core(r, basis, np, 0, f0, v, NULL);      /* step 3 */
        orc_deriv_B_vec(r, basis, np, v, vd);         /* step 4 */
        fft_core(r, basis, np, 0, f0, vd, NULL);      /* step 5 */
        for (long t = 0; t < n; t++) {                /* step 6 */
            long p = row_to_point(k, kp, t);
            uint32_t val = mask[t] ? orc_mul(r, vd[p], cst[p])
                                   : get_sym(r, shards + (size_t)t * stride, c);
            put_sym(r, out + (size_t)t * stride, c, val);
        }
    }
done:
    free(er); free(point_row); free(cst); free(v); free(vd); free(f0);
    return ok ? 0 : -1;
}

/* Definitional decoder: Lagrange interpolation through the first k' known
 * points of the mother code (survivors and virtual zeros), evaluated at
 * the erased points (Sec. 5: any k un-erased symbols determine F). */
ORC_EXPORT int orc_decode_lagrange(int r, const uint32_t *basis, int n, int k, const uint8_t *mask,
                                   const uint8_t *shards, uint8_t *out, size_t stride, size_t ncols)
{
    int kp, np;
    if (orc_mother_shape(r, n, k, &kp, &np) || !mask || !shards || !out)
        return -1;
    int e = 0;
    for (int t = 0; t < n; t++)
        e += mask[t] ? 1 : 0;
    if (e > n - k)
        return -2;
    long *kpt = calloc((size_t)kp, sizeof(long));    /* known points */
    long *krow = calloc((size_t)kp, sizeof(long));   /* their stored row or -1 */
    if (!kpt || !krow) {
        free(kpt); free(krow);
        return -1;
    }
    int nk = 0;
    for (long p = 0; p < np && nk < kp; p++) {
        long t = -1;
        if (p < k)
            t = p;
        else if (p >= kp && p < (long)kp + (n - k))
            t = k + (p - kp);
        if (t >= 0 && !mask[t]) {
            kpt[nk] = p; krow[nk] = t; nk++;
        } else if (t < 0 && p >= k && p < kp) {
            kpt[nk] = p; krow[nk] = -1; nk++;        /* virtual zero */
        }
    }
    for (size_t c = 0; c < ncols; c++) {
        for (long t = 0; t < n; t++) {
            uint32_t val;
            if (!mask[t]) {
                val = get_sym(r, shards + (size_t)t * stride, c);
            } else {
                uint32_t x = orc_omega(r, basis, (uint32_t)row_to_point(k, kp, t));
                val = 0;
                for (int i = 0; i < nk; i++) {
                    if (krow[i] < 0)
                        continue;
                    uint32_t xi = orc_omega(r, basis, (uint32_t)kpt[i]);
                    uint32_t num = 1, den = 1;
                    for (int u = 0; u < nk; u++) {
                        if (u == i)
                            continue;
                        uint32_t xu = orc_omega(r, basis, (uint32_t)kpt[u]);
                        num = orc_mul(r, num, x ^ xu);
                        den = orc_mul(r, den, xi ^ xu);
                    }
                    uint32_t yi = get_sym(r, shards + (size_t)krow[i] * stride, c);
                    val ^= orc_mul(r, yi, orc_mul(r, num, orc_inv(r, den)));
                }
            }
            put_sym(r, out + (size_t)t * stride, c, val);
        }
    }
    free(kpt); free(krow);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Polynomial operations in the novel basis (Sec. 6.1, Table 1).       */
/* ------------------------------------------------------------------ */

/* Product in the monomial basis, schoolbook: out has la + lb - 1 entries. */
ORC_EXPORT int orc_poly_mul(int r, int la, const uint32_t *a, int lb, const uint32_t *b, uint32_t *out)
{
    if (!field_ok(r) || la < 1 || lb < 1 || !a || !b || !out)
        return -1;
    poly_mul(r, a, la, b, lb, out);
    return 0;
}

/* Row i of the table holds the i + 1 monomial coefficients of X_i
 * (Definition 1: the product of What_j over the set bits j of i), i < h;
 * entries above the diagonal are zero.  Row i is row i - 2^j times What_j
 * for the highest set bit j of i; What_j has nonzero monomials only at the
 * degrees 2^m (Sec. 2.2), and the product skips its zero coefficients. */
static uint32_t *x_table(int r, const uint32_t *basis, int h)
{
    uint32_t *t = calloc((size_t)h * (size_t)h, sizeof(uint32_t));
    uint32_t *wh = calloc((size_t)h + 1, sizeof(uint32_t));
    if (!t || !wh) {
        free(t); free(wh);
        return NULL;
    }
    t[0] = 1;                                       /* X_0 = 1 */
    for (int j = 0; (1 << j) < h; j++) {
        const int dj = 1 << j;
        if (orc_W_monomial(r, basis, j, wh)) {
            free(t); free(wh);
            return NULL;
        }
        const uint32_t inv = orc_inv(r, orc_W(r, basis, j, orc_omega(r, basis, (uint32_t)dj)));
        for (int m = 0; m <= dj; m++)
            wh[m] = orc_mul(r, wh[m], inv);
        for (int i = dj; i < 2 * dj && i < h; i++) {
            const uint32_t *src = t + (size_t)(i - dj) * h;   /* X_{i - 2^j}, degree i - 2^j */
            uint32_t *dst = t + (size_t)i * h;
            for (int m = 0; m <= dj; m++) {
                if (!wh[m])
                    continue;
                for (int e = 0; e <= i - dj; e++)
                    dst[e + m] ^= orc_mul(r, src[e], wh[m]);
            }
        }
    }
    free(wh);
    return t;
}

/* Monomial coefficients of sum_i d_i X_i from the table (as orc_to_monomial). */
static void to_mono_tab(int r, int h, const uint32_t *xt, const uint32_t *d, uint32_t *mono)
{
    memset(mono, 0, sizeof(uint32_t) * (size_t)h);
    for (int i = 0; i < h; i++)
        if (d[i])
            for (int t = 0; t <= i; t++)
                mono[t] ^= orc_mul(r, d[i], xt[(size_t)i * h + t]);
}

/* The inverse: X_i has degree exactly i (its factors are the nonzero-leading
 * W_j-hat), so the expansion is triangular; from the highest degree down,
 * d_j is the remaining coefficient of x^j over the leading coefficient of
 * X_j, and d_j X_j is then subtracted. */
static void from_mono_tab(int r, int h, const uint32_t *xt, const uint32_t *mono, uint32_t *d, uint32_t *work)
{
    memcpy(work, mono, sizeof(uint32_t) * (size_t)h);
    for (int j = h - 1; j >= 0; j--) {
        const uint32_t *xj = xt + (size_t)j * h;
        d[j] = orc_mul(r, work[j], orc_inv(r, xj[j]));
        if (d[j])
            for (int t = 0; t <= j; t++)
                work[t] ^= orc_mul(r, d[j], xj[t]);
    }
}

/* Novel-basis coefficients (h entries) of a polynomial of degree < h given
 * by its h monomial coefficients. */
ORC_EXPORT int orc_from_monomial(int r, const uint32_t *basis, int h, const uint32_t *mono, uint32_t *d)
{
    if (!field_ok(r) || h < 1 || h > (1 << r) || !mono || !d)
        return -1;
    uint32_t *xt = x_table(r, basis, h);
    uint32_t *work = calloc((size_t)h, sizeof(uint32_t));
    if (!xt || !work) {
        free(xt); free(work);
        return -1;
    }
    from_mono_tab(r, h, xt, mono, d, work);
    free(xt); free(work);
    return 0;
}

/* Degree of [D_h](x) (Sec. 6.1, Table 1): the largest j with d_j != 0, since
 * deg X_j = j; -1 for the zero polynomial. */
ORC_EXPORT int orc_degree(int h, const uint32_t *d)
{
    if (h < 1 || !d)
        return -2;
    for (int j = h - 1; j >= 0; j--)
        if (d[j])
            return j;
    return -1;
}

/* Sec. 6.1 (Table 1), product of [A_h] and [B_h]: both padded with zeros to 2h
 * coefficients, transformed by Psi_2h^l (Sec. 3.2), multiplied point by
 * point, and transformed back by the inverse (Sec. 3.3).  out: 2h entries,
 * the novel-basis coefficients of the product (the last one is zero). */
ORC_EXPORT int orc_polymul_fft(int r, const uint32_t *basis, int h, uint32_t l, const uint32_t *a, const uint32_t *b,
                               uint32_t *out)
{
    const int H = 2 * h;
    if (h < 1 || !xform_args_ok(r, H, l) || !a || !b || !out)
        return -1;
    uint32_t *f = make_factors(r, basis, H, l);
    uint32_t *tb = calloc((size_t)H, sizeof(uint32_t));
    if (!f || !tb) {
        free(f); free(tb);
        return -1;
    }
    memset(out, 0, sizeof(uint32_t) * (size_t)H);
    memcpy(out, a, sizeof(uint32_t) * (size_t)h);
    memcpy(tb, b, sizeof(uint32_t) * (size_t)h);
    fft_core(r, basis, H, l, f, out, NULL);
    fft_core(r, basis, H, l, f, tb, NULL);
    for (int j = 0; j < H; j++)
        out[j] = orc_mul(r, out[j], tb[j]);
    ifft_core(r, basis, H, l, f, out, NULL);
    free(f); free(tb);
    return 0;
}

/* Column-wise variants over row-major stripes (row t at data + t * stride):
 * a and b have h rows, out 2h rows. */
ORC_EXPORT int orc_polymul_rows(int r, const uint32_t *basis, int h, uint32_t l, const uint8_t *a,
                                const uint8_t *b, uint8_t *out, size_t stride, size_t ncols)
{
    if (h < 1 || !a || !b || !out)
        return -1;
    uint32_t *va = calloc((size_t)h, sizeof(uint32_t)), *vb = calloc((size_t)h, sizeof(uint32_t));
    uint32_t *vo = calloc((size_t)2 * h, sizeof(uint32_t));
    int rc = (va && vb && vo) ? 0 : -1;
    for (size_t c = 0; c < ncols && !rc; c++) {
        for (int t = 0; t < h; t++) {
            va[t] = get_sym(r, a + (size_t)t * stride, c);
            vb[t] = get_sym(r, b + (size_t)t * stride, c);
        }
        rc = orc_polymul_fft(r, basis, h, l, va, vb, vo);
        for (int t = 0; t < 2 * h && !rc; t++)
            put_sym(r, out + (size_t)t * stride, c, vo[t]);
    }
    free(va); free(vb); free(vo);
    return rc;
}

ORC_EXPORT int orc_degree_rows(int r, int h, const uint8_t *data, size_t stride, size_t ncols, int32_t *deg)
{
    if (!field_ok(r) || h < 1 || !data || !deg)
        return -1;
    for (size_t c = 0; c < ncols; c++) {
        deg[c] = -1;
        for (int j = h - 1; j >= 0; j--)
            if (get_sym(r, data + (size_t)j * stride, c)) {
                deg[c] = j;
                break;
            }
    }
    return 0;
}

/* In place, column by column: novel -> monomial (to_mono != 0) or back. */
ORC_EXPORT int orc_convert_rows(int r, const uint32_t *basis, int h, int to_mono, uint8_t *data, size_t stride,
                                size_t ncols)
{
    if (!field_ok(r) || h < 1 || h > (1 << r) || !data)
        return -1;
    uint32_t *xt = x_table(r, basis, h);
    uint32_t *v = calloc((size_t)h, sizeof(uint32_t)), *o = calloc((size_t)h, sizeof(uint32_t));
    uint32_t *work = calloc((size_t)h, sizeof(uint32_t));
    int rc = (xt && v && o && work) ? 0 : -1;
    for (size_t c = 0; c < ncols && !rc; c++) {
        for (int t = 0; t < h; t++)
            v[t] = get_sym(r, data + (size_t)t * stride, c);
        if (to_mono)
            to_mono_tab(r, h, xt, v, o);
        else
            from_mono_tab(r, h, xt, v, o, work);
        for (int t = 0; t < h; t++)
            put_sym(r, data + (size_t)t * stride, c, o[t]);
    }
    free(xt); free(v); free(o); free(work);
    return rc;
}
