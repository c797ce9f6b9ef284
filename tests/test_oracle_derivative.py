"""Pins of the oracle's formal derivative (Sec. 4): three-way agreement of the
closed form (eq. D'_h(x)-2), the lower-multiplicative method (Sec. 4.2) and
term-by-term differentiation in the monomial basis, plus the paper's two
worked examples transcribed under tests/golden/."""
import os

import numpy as np
import pytest

from paper_1404_3458_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
BASIS8 = [0x1, 0x3, 0x7, 0xF0, 0x21, 0x44, 0x9C, 0x80]


def rand_syms(r, n, *kparts):
    return synth.uniform_int(synth.key(20, r, n, *kparts), n, 0, (1 << r) - 1).astype(np.uint32)


def _fixture(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line)
    return rows


@pytest.mark.parametrize("r,basis", [(8, None), (8, BASIS8), (16, None)])
def test_direct_equals_B_method(orc, r, basis):
    for lg in range(0, 9 if r == 8 else 10):
        h = 1 << lg
        d = rand_syms(r, h, lg)
        a = orc.deriv_direct(r, d, basis)
        b = orc.deriv_B(r, d, basis)
        assert (a == b).all(), h
        assert a[h - 1] == 0


@pytest.mark.parametrize("r,basis,hmax", [(8, None, 128), (8, BASIS8, 64), (16, None, 64)])
def test_derivative_matches_monomial_differentiation(orc, r, basis, hmax):
    h = 2
    while h <= hmax:
        d = rand_syms(r, h, 3)
        lhs = orc.to_monomial(r, orc.deriv_B(r, d, basis), basis)
        rhs = orc.monomial_derivative(r, orc.to_monomial(r, d, basis))
        assert (lhs == rhs).all(), h
        h *= 2


def test_h8_index_pattern_of_worked_example(orc):
    # With d = e_i, (Sigma d^d)/B_j is nonzero exactly when i is listed for j.
    pattern = {}
    for row in _fixture("deriv_h8_pattern.txt"):
        j, rest = row.split(":")
        pattern[int(j)] = {int(t) for t in rest.split()}
    assert sorted(pattern) == list(range(8))
    for r in (8, 16):
        B = orc.B_table(r, 8)
        for i in range(8):
            e = np.zeros(8, dtype=np.uint32)
            e[i] = 1
            out = orc.deriv_B(r, e, None)
            for j in range(8):
                expect = orc.mul(r, B[i], orc.inv(r, B[j])) if i in pattern[j] else 0
                assert out[j] == expect, (r, i, j)


def test_B_table_worked_example(orc):
    # Sec. 4.2: B_0 = 1, B_1 = W'_0, B_2 = W'_1, B_3 = W'_0 W'_1, ..., B_7 = W'_0 W'_1 W'_2
    for r in (8, 16):
        w = [orc.Wprime_norm(r, l) for l in range(3)]
        B = orc.B_table(r, 8)
        m = lambda *xs: __import__("functools").reduce(lambda a, b: orc.mul(r, a, b), xs, 1)
        assert list(B) == [1, w[0], w[1], m(w[0], w[1]), w[2], m(w[0], w[2]), m(w[1], w[2]),
                           m(w[0], w[1], w[2])]


def test_xprime13_worked_example(orc):
    terms = [tuple(int(t) for t in row.split()) for row in _fixture("xprime13.txt")]
    for r, basis in ((8, None), (8, BASIS8), (16, None)):
        e = np.zeros(16, dtype=np.uint32)
        e[13] = 1
        # X'_13 by monomial differentiation of X_13 ...
        lhs = orc.monomial_derivative(r, orc.to_monomial(r, e, basis))
        # ... equals sum W'_l X_index over the fixture's terms (monomial basis)
        rhs_x = np.zeros(16, dtype=np.uint32)
        for idx, l in terms:
            rhs_x[idx] = orc.Wprime_norm(r, l, basis)
        assert (lhs == orc.to_monomial(r, rhs_x, basis)).all()
        # and the closed form yields exactly those coefficients
        assert (orc.deriv_direct(r, e, basis) == rhs_x).all()


@pytest.mark.parametrize("r", [8, 16])
def test_derivative_rows(orc, r):
    h, ncols = 16, 5
    sym = r // 8
    data = synth.random_bytes(synth.key(21, r), h * ncols * sym).reshape(h, ncols * sym)
    out = orc.deriv_rows(r, data.copy())
    cols = data.astype(np.uint32) if r == 8 else data.view("<u2").astype(np.uint32)
    outc = out.astype(np.uint32) if r == 8 else out.view("<u2").astype(np.uint32)
    for c in range(ncols):
        assert (outc[:, c] == orc.deriv_direct(r, cols[:, c])).all()
