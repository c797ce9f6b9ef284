"""Pins of the oracle's polynomial operations in the novel basis (Sec. 6.1, Table 1:
the product through 2h-point transforms, the degree, and the conversion
between the novel and the monomial basis), against facts the mathematics
fixes independently of the oracle's own formulas: values at field points by
naive evaluation of the basis polynomials, the schoolbook product in the
monomial basis, degrees of products, and identities."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.usefixtures("orc")


def rnd(r, n, seed, density=1.0):
    g = np.random.default_rng(seed)
    v = g.integers(0, 1 << r, n, dtype=np.uint32)
    if density < 1.0:
        v[g.random(n) > density] = 0
    return v


@pytest.mark.parametrize("r", [8, 16])
def test_poly_mul_values(r):
    for s in range(6):
        a, b = rnd(r, 1 + 3 * s, s), rnd(r, 2 + 5 * s, 100 + s)
        p = oracle.poly_mul(r, a, b)
        for x in rnd(r, 12, 200 + s):
            assert oracle.poly_eval(r, p, int(x)) == oracle.mul(r, oracle.poly_eval(r, a, int(x)),
                                                                oracle.poly_eval(r, b, int(x)))


@pytest.mark.parametrize("r,h", [(8, 1), (8, 16), (8, 64), (16, 2), (16, 32), (16, 128)])
def test_conversion_roundtrip_and_unit_vectors(r, h):
    d = rnd(r, h, h)
    assert (oracle.from_monomial(r, oracle.to_monomial(r, d)) == d).all()
    m = rnd(r, h, h + 1)
    assert (oracle.to_monomial(r, oracle.from_monomial(r, m)) == m).all()
    for i in sorted({0, min(1, h - 1), h // 2, h - 1}):
        xm = np.zeros(h, dtype=np.uint32)
        xm[:i + 1] = oracle.X_monomial(r, i)
        e = np.zeros(h, dtype=np.uint32)
        e[i] = 1
        assert (oracle.from_monomial(r, xm) == e).all()


def _values(r, d, shift):
    # naive evaluation of sum_i d_i X_i at omega_b + omega_shift, b < len(d)
    return oracle.eval_naive(r, d, shift)


@pytest.mark.parametrize("r,h,l", [(8, 1, 0), (8, 4, 8), (8, 16, 5), (8, 128, 0), (16, 1, 3), (16, 8, 16),
                                   (16, 32, 1000), (16, 64, 0), (16, 256, 40000)])
def test_polymul_is_the_product(r, h, l):
    a, b = rnd(r, h, 7 * h + l), rnd(r, h, 11 * h + l)
    c = oracle.polymul(r, a, b, l)
    assert len(c) == 2 * h and c[-1] == 0
    pad = lambda v: np.concatenate([v, np.zeros(h, dtype=np.uint32)])
    # values at 2h points of two different cosets, by definition (naive sums of X_i)
    for shift in {0, (l + 2 * h * 3) % (1 << r), (1 << r) - 2 * h}:
        va, vb, vc = _values(r, pad(a), shift), _values(r, pad(b), shift), _values(r, c, shift)
        assert all(int(vc[j]) == oracle.mul(r, int(va[j]), int(vb[j])) for j in range(2 * h)), shift
    if h <= 64:
        # and against the schoolbook product of the monomial expansions
        pm = oracle.poly_mul(r, oracle.to_monomial(r, a), oracle.to_monomial(r, b))
        assert (oracle.to_monomial(r, c)[:2 * h - 1] == pm).all()


@pytest.mark.parametrize("r", [8, 16])
def test_polymul_identities(r):
    h = 16
    a, b = rnd(r, h, 1), rnd(r, h, 2)
    assert (oracle.polymul(r, a, b, 3) == oracle.polymul(r, b, a, 3)).all()
    assert (oracle.polymul(r, a, b, 0) == oracle.polymul(r, a, b, 2 * h)).all()   # shift-independent result
    one = np.zeros(h, dtype=np.uint32)
    one[0] = 1                                                                    # X_0 = 1
    assert (oracle.polymul(r, a, one, 0) == np.concatenate([a, np.zeros(h, dtype=np.uint32)])).all()
    assert not oracle.polymul(r, a, np.zeros(h, dtype=np.uint32), 0).any()


@pytest.mark.parametrize("r", [8, 16])
def test_degree(r):
    h = 64
    assert oracle.degree(np.zeros(h, dtype=np.uint32)) == -1
    for s in range(8):
        d = rnd(r, h, s, density=0.3)
        d[h // 2 + s:] = 0
        m = oracle.to_monomial(r, d)
        nz = np.nonzero(m)[0]
        assert oracle.degree(d) == (int(nz[-1]) if len(nz) else -1)
        e = rnd(r, h, 50 + s, density=0.2)
        e[h // 4:] = 0
        if oracle.degree(d) >= 0 and oracle.degree(e) >= 0:
            # no zero divisors: degrees add
            c = oracle.polymul(r, d, e, 0)
            assert oracle.degree(c) == oracle.degree(d) + oracle.degree(e)


@pytest.mark.parametrize("r", [8, 16])
def test_row_variants_match_vectors(r):
    h, nc = 16, 5
    sb = r // 8
    g = np.random.default_rng(9)
    A = g.integers(0, 256, (h, nc * sb), dtype=np.uint8)
    B = g.integers(0, 256, (h, nc * sb), dtype=np.uint8)
    A[h // 2:, :sb] = 0
    col = lambda M, c: (M[:, c * sb:(c + 1) * sb].astype(np.uint32) * (256 ** np.arange(sb))).sum(1)
    C = oracle.polymul_rows(r, A, B, 5)
    D = oracle.degree_rows(r, A)
    M = oracle.convert_rows(r, A.copy(), True)
    N = oracle.convert_rows(r, M.copy(), False)
    assert (N == A).all()
    for c in range(nc):
        assert (col(C, c) == oracle.polymul(r, col(A, c), col(B, c), 5)).all()
        assert D[c] == oracle.degree(col(A, c))
        assert (col(M, c) == oracle.to_monomial(r, col(A, c))).all()
