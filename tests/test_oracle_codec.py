"""Pins of the oracle's codec (Sec. 5, Algorithms 1 and 2, appendix locator):
Algorithm 1 against Lagrange interpolation, Algorithm 2 against recovery from
every k-subset and against Lagrange decoding, the Walsh-Hadamard locator
against direct products at every length, and the shortening convention."""
import itertools

import numpy as np
import pytest

from paper_1404_3458_amd import synth

BASIS8 = [0x1, 0x3, 0x7, 0xF0, 0x21, 0x44, 0x9C, 0x80]


def stripe(r, rows, ncols, *kparts):
    sym = r // 8
    return synth.random_bytes(synth.key(30, r, rows, ncols, *kparts), rows * ncols * sym).reshape(rows, ncols * sym)


SHAPES8 = [(2, 1), (4, 2), (8, 4), (16, 8), (16, 4), (32, 8), (12, 8), (10, 3), (64, 48), (20, 16)]
SHAPES16 = [(4, 2), (16, 8), (64, 48), (24, 16), (40, 7)]


@pytest.mark.parametrize("r,basis,n,k", [(8, None, n, k) for n, k in SHAPES8] + [(8, BASIS8, 16, 8)]
                         + [(16, None, n, k) for n, k in SHAPES16])
def test_encode_equals_lagrange(orc, r, basis, n, k):
    msg = stripe(r, k, 3, n)
    a = orc.encode(r, n, k, msg, basis)
    b = orc.encode(r, n, k, msg, basis, lagrange=True)
    assert (a == b).all()


def test_mother_shapes(orc):
    # shortening reading: k' = pow2ceil(k), n' = pow2ceil(k' + n - k)
    assert orc.mother_shape(16, 64, 48) == (64, 128)
    assert orc.mother_shape(16, 256, 224) == (256, 512)
    assert orc.mother_shape(16, 65536, 32768) == (32768, 65536)
    assert orc.mother_shape(8, 16, 8) == (8, 16)
    with pytest.raises(ValueError):
        orc.mother_shape(8, 257, 200)        # mother length 512 > 2^8


@pytest.mark.parametrize("r", [8, 16])
def test_encode_linear_and_constant(orc, r):
    n, k = 32, 16
    a, b = stripe(r, k, 4, 1), stripe(r, k, 4, 2)
    pa, pb = orc.encode(r, n, k, a), orc.encode(r, n, k, b)
    assert (orc.encode(r, n, k, a ^ b) == pa ^ pb).all()
    const = np.tile(a[:1], (k, 1))          # every message symbol of a column equal
    assert (orc.encode(r, n, k, const) == np.tile(a[:1], (n - k, 1))).all()


def test_decode_every_k_subset_n16(orc):
    r, n, k = 8, 16, 8
    msg = stripe(r, k, 6, 7)
    cw = np.concatenate([msg, orc.encode(r, n, k, msg)])
    count = 0
    for keep in itertools.combinations(range(n), k):
        mask = np.ones(n, dtype=np.uint8)
        mask[list(keep)] = 0
        rx = cw.copy()
        rx[mask == 1] = 0x5A                 # garbage in erased rows
        assert (orc.decode(r, n, k, mask, rx) == cw).all()
        count += 1
    assert count == 12870


@pytest.mark.parametrize("r,n,k", [(8, 16, 8), (8, 12, 8), (8, 10, 3), (8, 64, 48), (16, 16, 8),
                                   (16, 64, 48), (16, 40, 7)])
def test_decode_random_patterns(orc, r, n, k):
    msg = stripe(r, k, 5, n, k)
    cw = np.concatenate([msg, orc.encode(r, n, k, msg)])
    for trial in range(12):
        e = int(synth.uniform_int(synth.key(31, n, k, trial), 1, 0, n - k)[0])
        mask = synth.erasure_mask(synth.key(32, n, k, trial), n, e)
        rx = cw.copy()
        rx[mask == 1] = 0
        out = orc.decode(r, n, k, mask, rx)
        assert (out == cw).all()
        assert (orc.decode(r, n, k, mask, rx, locator="direct") == cw).all()
        if n <= 64:
            assert (orc.decode(r, n, k, mask, rx, lagrange=True) == cw).all()


def test_decode_too_many_erasures(orc):
    r, n, k = 8, 16, 8
    msg = stripe(r, k, 2, 1)
    mask = np.zeros(n, dtype=np.uint8)
    mask[:9] = 1
    with pytest.raises(ValueError):
        orc.decode(r, n, k, mask, np.concatenate([msg, msg]))


@pytest.mark.parametrize("r", [8, 16])
def test_locator_fwht_equals_direct_every_length(orc, r):
    lgmax = 8 if r == 8 else 10
    for lg in range(0, lgmax + 1):
        N = 1 << lg
        for trial in range(3):
            e = int(synth.uniform_int(synth.key(33, r, N, trial), 1, 0, N)[0])
            er = synth.erasure_mask(synth.key(34, r, N, trial), N, e)
            logv = orc.locator_log_fwht(r, er)
            direct = orc.locator_direct(r, er)
            got = np.array([orc.pow_(r, 2, int(v)) for v in logv], dtype=np.uint32)
            assert (got == direct).all(), (N, e)


def test_locator_with_custom_basis(orc):
    r = 8
    er = synth.erasure_mask(synth.key(35), 64, 20)
    logv = orc.locator_log_fwht(r, er, BASIS8)
    direct = orc.locator_direct(r, er, BASIS8)
    assert all(orc.pow_(r, 2, int(v)) == int(d) for v, d in zip(logv, direct))


def test_fwht_involution_scale(orc):
    # H_N H_N = N I, modulo 2^r - 1
    for r in (8, 16):
        M = (1 << r) - 1
        v = synth.uniform_int(synth.key(36, r), 64, 0, M - 1).astype(np.uint32)
        w = orc.fwht_mod(r, orc.fwht_mod(r, v))
        assert (w.astype(np.int64) == (v.astype(np.int64) * 64) % M).all()


@pytest.mark.parametrize("r", [8, 16])
def test_decode_no_erasures_is_copy(orc, r):
    n, k = 16, 8
    msg = stripe(r, k, 3, 3)
    cw = np.concatenate([msg, orc.encode(r, n, k, msg)])
    assert (orc.decode(r, n, k, np.zeros(n, np.uint8), cw) == cw).all()


def test_decode_large_shape_fwht(orc):
    # larger mother code, one column: the FWHT locator path at N = 4096
    r, n, k = 16, 4096, 2048
    msg = stripe(r, k, 1, 9)
    cw = np.concatenate([msg, orc.encode(r, n, k, msg)])
    mask = synth.erasure_mask(synth.key(37), n, n - k)
    rx = cw.copy()
    rx[mask == 1] = 0
    assert (orc.decode(r, n, k, mask, rx) == cw).all()
