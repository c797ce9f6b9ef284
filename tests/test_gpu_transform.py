"""GPU parity of the method tables, the multiply-by-constant, the transform
Psi_h^l and its inverse, and the formal derivative, against the oracle,
bit for bit, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
from paper_1404_3458_amd import rs, synth
from gpu_util import first_diff, rand_rows, to_dev, to_host

pytestmark = pytest.mark.gpu

BASIS8 = [0x1, 0x3, 0x7, 0xF0, 0x21, 0x44, 0x9C, 0x80]


def test_skew_table_matches_oracle_factors(codec16, codec8):
    for r, c in ((16, codec16), (8, codec8)):
        skew = c.table(rs.RS_TAB_SKEW)
        q = 1 << r
        assert len(skew) == q - 1
        # level i of the device table is the factor set of a 2^r-point transform at shift 0
        # restricted to level i; compare a few levels exhaustively and every level on samples
        f = oracle.factors(r, q if r == 8 else 1 << 12, 0)
        h = q if r == 8 else 1 << 12
        off_o = 0
        for i in range(int(np.log2(h))):
            nb = h >> (i + 1)
            off_d = q - (q >> i)
            assert (skew[off_d:off_d + nb] == f[off_o:off_o + nb]).all(), (r, i)
            off_o += nb


def test_B_table_matches_oracle(codec16, codec8):
    for r, c in ((16, codec16), (8, codec8)):
        B = c.table(rs.RS_TAB_B)
        Binv = c.table(rs.RS_TAB_BINV)
        h = 1 << (12 if r == 16 else 8)
        assert (B[:h] == oracle.B_table(r, h)).all()
        for j in synth.uniform_int(synth.key(40, r), 200, 0, (1 << r) - 1):
            assert oracle.mul(r, int(B[j]), int(Binv[j])) == 1


def test_log_exp_tables(codec8):
    lg = codec8.table(rs.RS_TAB_LOG)
    ex = codec8.table(rs.RS_TAB_EXP)
    for e in range(255):
        assert ex[e] == oracle.pow_(8, 2, e)
        assert lg[ex[e]] == e


@pytest.mark.parametrize("r", [16, 8])
def test_multiply_by_constant_exhaustive(r, codec16, codec8):
    # A 2-point transform at shift l maps (0, a) to (s a, (s + 1) a) with
    # s = W_0(omega_l) / W_0(omega_1) = l for the default basis: every symbol a
    # times every constant of GF(2^8), and times 0, 1, the largest element and
    # 60 seeded constants of GF(2^16).
    c = codec16 if r == 16 else codec8
    q = 1 << r
    sym = r // 8
    syms = np.arange(q, dtype=np.uint16 if r == 16 else np.uint8)
    data = np.zeros((2, q * sym), dtype=np.uint8)
    data[1] = syms.view(np.uint8)
    if r == 8:
        consts = list(range(q))
    else:
        consts = [0, 1, 2, q - 1] + [int(v) for v in synth.uniform_int(synth.key(41, r), 60, 0, q - 1)]
    for l in consts:
        d = to_dev(data)
        c.fft(2, l, d)
        got = to_host(d)
        exp = oracle.fft_rows(r, data.copy(), l)
        assert (got == exp).all(), (l, first_diff(got, exp))


def _check_xform(c, r, h, l, ncols, key, kind):
    sym = r // 8
    data = rand_rows(h, ncols * sym, 42, r, h, l, ncols, key)
    d = to_dev(data)
    if kind == "fft":
        c.fft(h, l, d)
        exp = oracle.fft_rows(r, data.copy(), l)
    elif kind == "ifft":
        c.ifft(h, l, d)
        exp = oracle.ifft_rows(r, data.copy(), l)
    else:
        c.derivative(h, d)
        exp = oracle.deriv_rows(r, data.copy())
    got = to_host(d)
    assert (got == exp).all(), (kind, r, h, l, ncols, first_diff(got, exp))


def _cols_for(h):
    if h <= 16:
        return [1, 3, 4, 5, 256, 517]
    if h <= 256:
        return [3, 4, 259, 1024 + 4]
    if h <= 4096:
        return [5, 260]
    return [3, 64]


@pytest.mark.parametrize("lg", list(range(0, 17)))
def test_fft_ifft_r16_every_size(codec16, lg):
    h = 1 << lg
    for ncols in _cols_for(h):
        shifts = {0, h % 65536, (3 * h) % 65536, 12345 % 65536 if h > 1 else 7}
        if h > 4096:
            shifts = {0, 12345}
        for l in sorted(shifts):
            _check_xform(codec16, 16, h, l, ncols, 1, "fft")
            _check_xform(codec16, 16, h, l, ncols, 2, "ifft")


@pytest.mark.parametrize("lg", list(range(0, 9)))
def test_fft_ifft_r8_every_size(codec8, lg):
    h = 1 << lg
    for ncols in _cols_for(h):
        for l in sorted({0, h % 256, 77}):
            _check_xform(codec8, 8, h, l, ncols, 3, "fft")
            _check_xform(codec8, 8, h, l, ncols, 4, "ifft")


@pytest.mark.parametrize("lg", list(range(0, 17)))
def test_derivative_r16_every_size(codec16, lg):
    h = 1 << lg
    for ncols in _cols_for(h)[:3]:
        _check_xform(codec16, 16, h, 0, ncols, 5, "deriv")


@pytest.mark.parametrize("lg", list(range(0, 9)))
def test_derivative_r8_every_size(codec8, lg):
    h = 1 << lg
    for ncols in _cols_for(h)[:3]:
        _check_xform(codec8, 8, h, 0, ncols, 6, "deriv")


def test_unaligned_rows(codec16):
    # rows of 3, 5 and 515 symbols (6, 10, 1030 bytes: not 8-byte multiples,
    # so full chunks start 2 mod 4 on every other row) in a buffer offset by
    # 2 bytes; and the derivative, which reads and writes the same rows
    for h, rb in ((16, 6), (64, 6), (512, 6), (16, 10), (256, 1030), (1024, 10)):
        data = rand_rows(h, rb, 43, h, rb)
        big = torch.zeros(h * rb + 2, dtype=torch.uint8, device="cuda")
        big[2:] = to_dev(data.reshape(-1))
        codec16.fft(h, 5, big.data_ptr() + 2, row_bytes=rb)
        got = to_host(big[2:]).reshape(h, rb)
        exp = oracle.fft_rows(16, data.copy(), 5)
        assert (got == exp).all(), (h, rb, first_diff(got, exp))
        big[2:] = to_dev(data.reshape(-1))
        codec16.derivative(h, big.data_ptr() + 2, row_bytes=rb)
        got = to_host(big[2:]).reshape(h, rb)
        exp = data.copy()
        oracle.deriv_rows(16, exp)
        assert (got == exp).all(), (h, rb, first_diff(got, exp))


def test_unaligned_rows_r8(codec8):
    # byte rows at every alignment: 4-symbol chunks starting 0, 1, 2, 3 mod 4
    for h, rb in ((16, 5), (64, 7), (256, 13), (128, 1027)):
        data = rand_rows(h, rb, 44, h, rb)
        big = torch.zeros(h * rb + 1, dtype=torch.uint8, device="cuda")
        big[1:] = to_dev(data.reshape(-1))
        codec8.ifft(h, 3, big.data_ptr() + 1, row_bytes=rb)
        got = to_host(big[1:]).reshape(h, rb)
        exp = oracle.ifft_rows(8, data.copy(), 3)
        assert (got == exp).all(), (h, rb, first_diff(got, exp))


def test_custom_basis():
    c = rs.Codec(8, BASIS8)
    try:
        for h in (8, 64, 256):
            data = rand_rows(h, 37, 44, h)
            d = to_dev(data)
            c.fft(h, 3, d)
            assert (to_host(d) == oracle.fft_rows(8, data.copy(), 3, BASIS8)).all(), h
            d = to_dev(data)
            c.derivative(h, d)
            exp = data.copy()
            oracle.deriv_rows(8, exp, BASIS8)
            assert (to_host(d) == exp).all(), h
    finally:
        c.close()


def test_bad_basis_and_field():
    with pytest.raises(rs.RSError) as e:
        rs.Codec(8, [1, 2, 3, 4, 8, 16, 32, 64])      # 3 = 1 + 2: dependent
    assert e.value.code == rs.RS_EBASIS
    with pytest.raises(rs.RSError) as e:
        rs.Codec(12)
    assert e.value.code == rs.RS_EFIELD
