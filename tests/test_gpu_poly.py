"""GPU parity of the polynomial operations of Sec. 6.1 (Table 1) through the C ABI: the
product by 2h-point transforms (nb_polymul), the degree (nb_degree) and the
conversion between the novel and the monomial basis (nb_to_monomial,
nb_from_monomial), bit for bit against the oracle on aligned and unaligned
rows, whole and ragged column tiles; plus the error paths."""
import numpy as np
import pytest
import torch

import oracle
from paper_1404_3458_amd import rs, synth
from gpu_util import first_diff, rand_rows, to_dev, to_host

pytestmark = pytest.mark.gpu

NCOLS = (260, 37)      # 8-byte-aligned rows with a whole and a ragged tile; rows of 74 bytes (r = 16)


def _codec(request, r):
    return request.getfixturevalue("codec%d" % r)


# products over 2h > 256 points: at shifts with no bit below 2h, two passes of
# up to 8 levels on LDS tiles (2^9: 5 + 4, 2^12: 6 + 6, 2^13: 7 + 6); at other
# shifts register-only passes of 4 or 5 levels (2^10: 5 + 5, 2^11: 4 + 4 + 3)
@pytest.mark.parametrize("r,h,l", [(16, 1, 0), (16, 2, 7), (16, 8, 16), (16, 64, 0), (16, 128, 300),
                                   (16, 256, 512), (16, 512, 1000), (16, 1024, 12345), (16, 2048, 0),
                                   (16, 4096, 8192), (8, 1, 0), (8, 4, 3), (8, 32, 64), (8, 128, 0)])
def test_polymul(request, r, h, l):
    c = _codec(request, r)
    sb = r // 8
    for i, nc in enumerate(NCOLS):
        a = rand_rows(h, nc * sb, 70, r, h, l, i)
        b = rand_rows(h, nc * sb, 71, r, h, l, i)
        if h > 2:
            a[h - 2:, :sb] = 0                        # a column of lower degree
        out = torch.full((2 * h, nc * sb), 0xA5, dtype=torch.uint8, device="cuda")
        c.polymul(h, l, to_dev(a), to_dev(b), out)
        got, exp = to_host(out), oracle.polymul_rows(r, a, b, l)
        assert (got == exp).all(), (r, h, l, nc, first_diff(got, exp))


def test_polymul_independent_of_shift(codec16):
    h, nc = 64, 100
    a, b = to_dev(rand_rows(h, 2 * nc, 72)), to_dev(rand_rows(h, 2 * nc, 73))
    outs = []
    for l in (0, 5, 128, 65535):
        o = torch.empty((2 * h, 2 * nc), dtype=torch.uint8, device="cuda")
        codec16.polymul(h, l, a, b, o)
        outs.append(to_host(o))
    assert all((o == outs[0]).all() for o in outs)


def test_polymul_errors(codec16, codec8):
    a = torch.zeros((4, 8), dtype=torch.uint8, device="cuda")
    big = torch.zeros((8, 8), dtype=torch.uint8, device="cuda")
    with pytest.raises(rs.RSError) as ei:
        codec16.polymul(4, 0, big[:4], a, big, row_bytes=8)        # out overlaps a
    assert ei.value.code == rs.RS_EINVAL
    with pytest.raises(rs.RSError) as ei:
        codec16.polymul(3, 0, a, a, big, row_bytes=8)
    assert ei.value.code == rs.RS_ESHAPE
    with pytest.raises(rs.RSError) as ei:
        codec8.polymul(256, 0, a, a, big, row_bytes=8)             # 2h > 2^8
    assert ei.value.code == rs.RS_ESHAPE
    with pytest.raises(rs.RSError) as ei:
        codec16.polymul(4, 1 << 16, a, a, big, row_bytes=8)
    assert ei.value.code == rs.RS_EINVAL
    with pytest.raises(rs.RSError) as ei:
        codec16.polymul(4, 0, a, a, big, row_bytes=7)
    assert ei.value.code == rs.RS_EALIGN
    codec16.polymul(4, 0, a, a, big, row_bytes=0)                   # no-op


@pytest.mark.parametrize("r,h", [(16, 1), (16, 7), (16, 256), (16, 4096), (8, 5), (8, 256)])
def test_degree(request, r, h):
    c = _codec(request, r)
    sb = r // 8
    g = np.random.default_rng(h)
    for i, nc in enumerate(NCOLS):
        d = rand_rows(h, nc * sb, 74, r, h, i)
        for col in range(nc):                       # random degrees, some zero columns
            top = int(g.integers(-1, h))
            d[top + 1:, col * sb:(col + 1) * sb] = 0
            if top >= 0 and not d[top, col * sb:(col + 1) * sb].any():
                d[top, col * sb] = 1
        deg = c.degree(h, to_dev(d))
        got, exp = to_host(deg), oracle.degree_rows(r, d)
        assert (got == exp).all(), (r, h, nc, first_diff(got, exp))


# levels up to 8 run in one block-tile launch; 512 rows add a ninth level of
# the one-level kernels in each direction
@pytest.mark.parametrize("r,h", [(16, 2), (16, 4), (16, 16), (16, 128), (16, 256), (16, 512), (8, 2), (8, 32),
                                 (8, 256)])
def test_conversion_matches_oracle(request, r, h):
    c = _codec(request, r)
    sb = r // 8
    for i, nc in enumerate(NCOLS):
        d = rand_rows(h, nc * sb, 75, r, h, i)
        t = to_dev(d)
        c.to_monomial(h, t)
        got, exp = to_host(t), oracle.convert_rows(r, d.copy(), True)
        assert (got == exp).all(), ("to", r, h, nc, first_diff(got, exp))
        m = rand_rows(h, nc * sb, 76, r, h, i)
        t = to_dev(m)
        c.from_monomial(h, t)
        got, exp = to_host(t), oracle.convert_rows(r, m.copy(), False)
        assert (got == exp).all(), ("from", r, h, nc, first_diff(got, exp))


def test_conversion_matches_oracle_4096(codec16):
    # the measured size: levels 1-8 in the block-tile kernels, 9-12 level by
    # level, on 4 columns (8-byte rows: vector accesses) against the oracle
    h, nc = 4096, 4
    d = rand_rows(h, 2 * nc, 80, h)
    t = to_dev(d)
    codec16.to_monomial(h, t)
    got, exp = to_host(t), oracle.convert_rows(16, d.copy(), True)
    assert (got == exp).all(), ("to", first_diff(got, exp))
    m = rand_rows(h, 2 * nc, 81, h)
    t = to_dev(m)
    codec16.from_monomial(h, t)
    got, exp = to_host(t), oracle.convert_rows(16, m.copy(), False)
    assert (got == exp).all(), ("from", first_diff(got, exp))


@pytest.mark.parametrize("h", [1024, 8192])
def test_conversion_round_trip_large(codec16, h):
    # sizes past the oracle's O(h^2) tables: the two conversions invert each
    # other, the monomial form has the same degree, and a product's monomial
    # form is checked on sampled columns against the oracle's schoolbook product
    nc = 37
    d = rand_rows(h, 2 * nc, 77, h)
    d[h // 2:, :2] = 0
    t = to_dev(d)
    codec16.to_monomial(h, t)
    mono = to_host(t)
    assert (to_host(codec16.degree(h, t)) == oracle.degree_rows(16, d)).all()
    codec16.from_monomial(h, t)
    assert (to_host(t) == d).all()
    hs = 64
    a, b = rand_rows(hs, 2 * nc, 78), rand_rows(hs, 2 * nc, 79)
    o = torch.empty((2 * hs, 2 * nc), dtype=torch.uint8, device="cuda")
    codec16.polymul(hs, 0, to_dev(a), to_dev(b), o)
    codec16.to_monomial(2 * hs, o)
    om = to_host(o)
    col = lambda M, c: M[:, 2 * c].astype(np.uint32) | (M[:, 2 * c + 1].astype(np.uint32) << 8)
    for cc in (0, 5, nc - 1):
        pm = oracle.poly_mul(16, oracle.to_monomial(16, col(a, cc)), oracle.to_monomial(16, col(b, cc)))
        assert (col(om, cc)[:2 * hs - 1] == pm).all() and col(om, cc)[-1] == 0
    assert mono.shape == d.shape



@pytest.mark.parametrize("r", [16, 8])
def test_product_of_constants_every_element(request, r):
    # h = 1: the product of two constant polynomials is the field product of
    # the constants, so a row holding every field element times a row of one
    # constant checks the point-by-point multiply against the oracle on all
    # of GF(2^r): for r = 16 the edge factors 0, 1, x, x^15, all ones, the
    # reduction word and one more, plus a row of random factors; for r = 8
    # every constant
    c = request.getfixturevalue("codec%d" % r)
    q = 1 << r
    dt = np.uint16 if r == 16 else np.uint8
    elems = np.arange(q, dtype=dt)
    if r == 16:
        rows_b = [np.full(q, v, dtype=dt) for v in (0, 1, 2, 0x8000, 0xFFFF, 0x100B, 0x1234)]
        rows_b.append(synth.uniform_int(synth.key(95, r), q, 0, q - 1).astype(dt))
    else:
        rows_b = [np.full(q, v, dtype=dt) for v in range(q)]
    a = torch.from_numpy(elems.view(np.uint8).reshape(1, -1).copy()).cuda()
    out = torch.empty((2, a.shape[1]), dtype=torch.uint8, device="cuda")
    for brow in rows_b:
        b = torch.from_numpy(brow.view(np.uint8).reshape(1, -1).copy()).cuda()
        c.polymul(1, 0, a, b, out)
        res = out.cpu().numpy()
        assert (res[1] == 0).all()
        got = res[0].view(dt)
        exp = np.array([oracle.mul(r, int(x), int(y)) for x, y in zip(elems, brow)], dtype=dt)
        assert (got == exp).all(), (r, int(brow[0]), int(np.argmax(got != exp)))
