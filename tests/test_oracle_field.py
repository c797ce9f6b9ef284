"""Pins of the oracle's field GF(2^r) (Sec. 2.1) to facts that do not come from
the oracle itself: closed forms of the reduction, the group order, and the
field axioms checked exhaustively (r = 8) or on seeded samples (r = 16)."""
import numpy as np
import pytest

from paper_1404_3458_amd import synth


def test_reduction_closed_form(orc):
    # x^r reduced modulo the field polynomial is the polynomial minus x^r.
    assert orc.mul(8, 0x80, 0x02) == 0x11D ^ 0x100
    assert orc.mul(16, 0x8000, 0x02) == 0x1100B ^ 0x10000
    # x^(r+1) = x * (x^r mod P): one more shift, reduced again where needed.
    assert orc.mul(8, 0x80, 0x04) == 0x3A
    assert orc.mul(16, 0x8000, 0x04) == 0x2016


@pytest.mark.parametrize("r,primes", [(8, [3, 5, 17]), (16, [3, 5, 17, 257])])
def test_two_is_primitive(orc, r, primes):
    order = (1 << r) - 1
    assert orc.pow_(r, 2, order) == 1
    for p in primes:
        assert orc.pow_(r, 2, order // p) != 1


def test_gf256_axioms_exhaustive(orc):
    r = 8
    tab = np.array([[orc.mul(r, a, b) for b in range(256)] for a in range(256)], dtype=np.uint32)
    assert (tab == tab.T).all()                          # commutative
    assert (tab[1] == np.arange(256)).all()              # 1 is the identity
    assert (tab[0] == 0).all()
    # every nonzero row is a permutation (no zero divisors)
    for a in range(1, 256):
        assert len(set(tab[a].tolist())) == 256
    # distributivity over XOR, all a, b, c on a seeded sample of a
    rows = synth.uniform_int(synth.key(1, 1), 16, 0, 255)
    for a in rows:
        lhs = tab[a][np.bitwise_xor.outer(np.arange(256), np.arange(256))]
        rhs = tab[a][:, None] ^ tab[a][None, :]
        assert (lhs == rhs).all()
    # associativity on a sample
    trip = synth.uniform_int(synth.key(1, 2), 3 * 2000, 0, 255).reshape(-1, 3)
    for a, b, c in trip:
        assert tab[tab[a, b], c] == tab[a, tab[b, c]]


def test_gf256_frobenius_and_inverse(orc):
    for a in range(256):
        assert orc.pow_(8, a, 256) == a                  # x^(2^r) = x
        if a:
            assert orc.mul(8, a, orc.inv(8, a)) == 1


def test_gf65536_axioms_sampled(orc):
    r = 16
    v = synth.uniform_int(synth.key(1, 3), 3 * 3000, 0, 65535).reshape(-1, 3)
    for a, b, c in v:
        a, b, c = int(a), int(b), int(c)
        assert orc.mul(r, a, b) == orc.mul(r, b, a)
        assert orc.mul(r, a, b ^ c) == orc.mul(r, a, b) ^ orc.mul(r, a, c)
        assert orc.mul(r, orc.mul(r, a, b), c) == orc.mul(r, a, orc.mul(r, b, c))
        assert orc.pow_(r, a, 1 << 16) == a
        if a:
            assert orc.mul(r, a, orc.inv(r, a)) == 1


def test_gf65536_inverse_exhaustive(orc):
    r = 16
    seen = set()
    for a in range(1, 1 << 16):
        ia = orc.inv(r, a)
        assert orc.mul(r, a, ia) == 1
        seen.add(ia)
    assert len(seen) == (1 << 16) - 1


def test_omega_is_linear_in_index(orc):
    rng_basis = [0x1, 0x3, 0x7, 0xF0, 0x21, 0x44, 0x9C, 0x80]  # F2-independent over GF(2^8)
    for i in range(256):
        for j in (0, 1, 5, 77, 255):
            assert orc.omega(8, i ^ j, rng_basis) == orc.omega(8, i, rng_basis) ^ orc.omega(8, j, rng_basis)
    assert len({orc.omega(8, i, rng_basis) for i in range(256)}) == 256
    assert all(orc.omega(16, i) == i for i in (0, 1, 2, 3, 1000, 65535))
