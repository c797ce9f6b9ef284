"""Pins of the oracle's subspace polynomials W_j (Sec. 2.2, Lemma 1), the
novel basis X_i (Sec. 2.3) and Lemma 3, checked against their defining
properties: vanishing set, degree, F2-linearity (monomials only at powers of
two), additivity, and a product recursion that does not appear in the oracle."""
import numpy as np
import pytest

from paper_1404_3458_amd import synth

BASIS8 = [0x1, 0x3, 0x7, 0xF0, 0x21, 0x44, 0x9C, 0x80]


@pytest.mark.parametrize("r,basis,jmax", [(8, None, 8), (8, BASIS8, 8), (16, None, 10)])
def test_W_vanishes_on_subspace_and_degree(orc, r, basis, jmax):
    for j in range(min(jmax, 7)):
        for i in range(1 << j):
            assert orc.W(r, j, orc.omega(r, i, basis), basis) == 0
        assert orc.W(r, j, orc.omega(r, 1 << j, basis), basis) != 0
        coef = orc.W_monomial(r, j, basis)
        assert len(coef) == (1 << j) + 1 and coef[-1] == 1      # monic, degree 2^j


@pytest.mark.parametrize("r,basis", [(8, None), (8, BASIS8), (16, None)])
def test_W_linearized_lemma1(orc, r, basis):
    jmax = 8 if r == 8 else 9
    for j in range(jmax):
        coef = orc.W_monomial(r, j, basis)
        powers = {1 << t for t in range(j + 1)}
        for deg, c in enumerate(coef):
            if deg not in powers:
                assert c == 0, (j, deg)
        # additivity W_j(x + y) = W_j(x) + W_j(y)
        xs = synth.uniform_int(synth.key(2, r, j), 40, 0, (1 << r) - 1)
        for x, y in xs.reshape(-1, 2):
            x, y = int(x), int(y)
            assert orc.W(r, j, x ^ y, basis) == orc.W(r, j, x, basis) ^ orc.W(r, j, y, basis)
            assert orc.poly_eval(r, coef, x) == orc.W(r, j, x, basis)


@pytest.mark.parametrize("r,basis", [(8, None), (8, BASIS8), (16, None)])
def test_W_recursion(orc, r, basis):
    # W_{j+1}(x) = W_j(x) W_j(x + v_j) = W_j(x) (W_j(x) + W_j(v_j)), which
    # follows from the definition and Lemma 1 but is not how the oracle computes W.
    for j in range(7):
        vj = orc.omega(r, 1 << j, basis)
        for x in synth.uniform_int(synth.key(3, r, j), 12, 0, (1 << r) - 1):
            x = int(x)
            wj = orc.W(r, j, x, basis)
            assert orc.W(r, j + 1, x, basis) == orc.mul(r, wj, wj ^ orc.W(r, j, vj, basis))


@pytest.mark.parametrize("r,basis", [(8, None), (8, BASIS8), (16, None)])
def test_lemma3_derivative_constant(orc, r, basis):
    # the x^1 coefficient of W_i equals prod_{j=1}^{2^i - 1} omega_j
    for i in range(8 if r == 8 else 9):
        coef = orc.W_monomial(r, i, basis)
        prod = 1
        for j in range(1, 1 << i):
            prod = orc.mul(r, prod, orc.omega(r, j, basis))
        assert coef[1] == prod


@pytest.mark.parametrize("r,basis", [(8, None), (8, BASIS8), (16, None)])
def test_X_degree_and_special_cases(orc, r, basis):
    pts = [int(x) for x in synth.uniform_int(synth.key(4, r), 6, 0, (1 << r) - 1)]
    for x in pts:
        assert orc.X(r, 0, x, basis) == 1
    for j in range(6):
        for x in pts:
            assert orc.X(r, 1 << j, x, basis) == orc.W_hat(r, j, x, basis)
    for i in list(range(40)) + [63, 100, 127]:
        coef = orc.X_monomial(r, i, basis)
        assert len(coef) == i + 1 and coef[i] != 0            # deg X_i = i
        for x in pts[:2]:
            assert orc.poly_eval(r, coef, x) == orc.X(r, i, x, basis)


def test_W_hat_normalisation(orc):
    for r in (8, 16):
        for j in range(7):
            assert orc.W_hat(r, j, orc.omega(r, 1 << j)) == 1
