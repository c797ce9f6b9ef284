"""Pins of the oracle's transform Psi_h^l (Sec. 3): the fast algorithm of
Sec. 3.2 against naive evaluation of the definition, the inverse of Sec. 3.3,
the exact operation counts of Sec. 3.4, the factor count of Sec. 3.5, and the
h = 1 and h = 2 closed forms."""
import numpy as np
import pytest

from paper_1404_3458_amd import synth

BASIS8 = [0x1, 0x3, 0x7, 0xF0, 0x21, 0x44, 0x9C, 0x80]


def rand_syms(r, n, *kparts):
    return synth.uniform_int(synth.key(10, r, n, *kparts), n, 0, (1 << r) - 1).astype(np.uint32)


@pytest.mark.parametrize("r,basis", [(8, None), (8, BASIS8), (16, None)])
def test_fft_equals_naive_evaluation(orc, r, basis):
    hmax = 128 if r == 8 else 64
    h = 1
    while h <= hmax:
        shifts = [0, h, 3 * h, 1, h // 2 + 1, (1 << r) - 1] if h > 1 else [0, 5]
        for l in shifts:
            l = int(l) % (1 << r)
            d = rand_syms(r, h, l)
            assert (orc.fft(r, d, l, basis) == orc.eval_naive(r, d, l, basis)).all(), (h, l)
        h *= 2


def test_fft_equals_naive_h256(orc):
    d = rand_syms(8, 256, 99)
    for l in (0, 37):
        assert (orc.fft(8, d, l) == orc.eval_naive(8, d, l)).all()


@pytest.mark.parametrize("r", [8, 16])
def test_inverse_roundtrip(orc, r):
    for lg in range(0, 11 if r == 16 else 9):
        h = 1 << lg
        for l in (0, h % (1 << r), 12345 % (1 << r)):
            d = rand_syms(r, h, lg, l)
            assert (orc.ifft(r, orc.fft(r, d, l), l) == d).all()
            assert (orc.fft(r, orc.ifft(r, d, l), l) == d).all()


@pytest.mark.parametrize("r", [8, 16])
def test_operation_counts(orc, r):
    # Sec. 3.4: A(h) = h lg h, M(h) = (h/2) lg h; with omega_l = 0,
    # A_0(h) = h lg h - h + 1 and M_0(h) = (h/2) lg h - h + 1.
    for lg in range(1, 9):
        h = 1 << lg
        d = rand_syms(r, h, 7)
        for inverse in (False, True):
            f = orc.ifft if inverse else orc.fft
            c = np.zeros(2, dtype=np.int64)
            f(r, d, 0, counts=c)
            assert c[0] == h * lg - h + 1 and c[1] == (h // 2) * lg - h + 1
            if h < (1 << r):
                c = np.zeros(2, dtype=np.int64)
                f(r, d, h, counts=c)          # no zero point when h divides l, l != 0
                assert c[0] == h * lg and c[1] == (h // 2) * lg


def test_factor_count(orc):
    # Sec. 3.5: an h-point transform needs h/2 + h/4 + ... + 1 = h - 1 factors
    for lg in range(0, 9):
        h = 1 << lg
        assert len(orc.factors(8, h, 3 % 256)) == h - 1


@pytest.mark.parametrize("r", [8, 16])
def test_h1_and_h2_closed_forms(orc, r):
    for l in (0, 1, 2, 7, (1 << r) - 1):
        d = rand_syms(r, 2, l)
        assert (orc.fft(r, d[:1], l) == d[:1]).all()
        s = orc.W_hat(r, 0, orc.omega(r, l))
        a = int(d[0]) ^ orc.mul(r, s, int(d[1]))
        b = int(d[0]) ^ orc.mul(r, s ^ 1, int(d[1]))
        assert list(orc.fft(r, d, l)) == [a, b]


@pytest.mark.parametrize("r", [8, 16])
def test_linearity(orc, r):
    h = 64
    a, b = rand_syms(r, h, 1), rand_syms(r, h, 2)
    for l in (0, 64, 5):
        assert (orc.fft(r, a ^ b, l) == orc.fft(r, a, l) ^ orc.fft(r, b, l)).all()


@pytest.mark.parametrize("r", [8, 16])
def test_rows_match_vector_transform(orc, r):
    h, ncols = 32, 9
    sym = r // 8
    data = synth.random_bytes(synth.key(11, r), h * ncols * sym).reshape(h, ncols * sym)
    if r == 8:
        cols = data.astype(np.uint32)
    else:
        cols = data.view("<u2").astype(np.uint32)
    for l in (0, 32, 3):
        out = orc.fft_rows(r, data.copy(), l)
        outc = out.astype(np.uint32) if r == 8 else out.view("<u2").astype(np.uint32)
        for c in range(ncols):
            assert (outc[:, c] == orc.fft(r, cols[:, c], l)).all()
        back = orc.ifft_rows(r, out, l)
        assert (back == data).all()
