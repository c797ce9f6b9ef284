"""GPU parity of every candidate schedule of the pass pipelines
(rs_schedule_set_parts, rs_schedule_set_tile): each split of a transform
over 2^N > 256 points into two, three or four parts of levels, and each
column tile, gives the oracle's parity and restores every erasure, for
aligned and unaligned rows; plus the error paths of the schedule calls, the
environment variable that sets schedules at rs_init, and the autotuner's
table."""
import math
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1404_3458_amd import rs, synth, tune
from gpu_util import first_diff, rand_rows, to_dev, to_host

pytestmark = pytest.mark.gpu

ENC_SHAPES = [(1024, 512), (2048, 1024), (4096, 2048), (8192, 4096), (16384, 8192)]   # N = lg k' = 9 .. 13
DEC_SHAPES = [(512, 256), (300, 200), (1024, 512), (2048, 1024), (4096, 2048), (8192, 4096),
              (5000, 4000)]                                                            # lg n' = 9 .. 13
# a whole and a ragged tile with 8-byte-aligned rows; unaligned rows (74-byte rows); rows of 124 symbols
# (248 bytes, aligned), which fill only half a wave and run the packed passes (as do the 74-byte rows)
NCOLS = (260, 37, 124)


def _cases(shapes, size_of):
    out = []
    for n, k in shapes:
        N = int(math.log2(size_of(*tune.mother(n, k))))
        out += [(n, k, N, t) for t in tune.candidates(N)]
    return out


@pytest.fixture(scope="module")
def cs():
    c = rs.Codec(16)
    yield c
    c.close()


def _stripes(n, k, key):
    if isinstance(key, tuple):
        key = sum(v << (4 * q) for q, v in enumerate(key))
    return [rand_rows(k, 2 * nc, 60, n, k, nc, key) for nc in NCOLS]


@pytest.mark.parametrize("n,k,N,T1", _cases(ENC_SHAPES, lambda np_, kp: kp))
def test_encode_every_split(cs, n, k, N, T1):
    cs.set_schedule(rs.RS_OP_ENCODE, N, T1)
    try:
        assert cs.get_schedule_parts(rs.RS_OP_ENCODE, N) == T1
        msgs = _stripes(n, k, T1)
        dm = [to_dev(m) for m in msgs]
        dp = [torch.zeros((n - k, m.shape[1]), dtype=torch.uint8, device="cuda") for m in msgs]
        cs.encode_batch([(n, k, dm[i], dp[i]) for i in range(len(msgs))])
        for i, m in enumerate(msgs):
            got, exp = to_host(dp[i]), oracle.encode(16, n, k, m)
            assert (got == exp).all(), (n, k, T1, NCOLS[i], first_diff(got, exp))
    finally:
        cs.set_schedule(rs.RS_OP_ENCODE, N, 0)


@pytest.mark.parametrize("n,k,N,T1", _cases(DEC_SHAPES, lambda np_, kp: np_))
def test_decode_every_split(cs, n, k, N, T1):
    cs.set_schedule(rs.RS_OP_DECODE, N, T1)
    try:
        assert cs.get_schedule_parts(rs.RS_OP_DECODE, N) == T1
        cws, masks, ds = [], [], []
        for i, m in enumerate(_stripes(n, k, 100 + sum(v << (4 * q) for q, v in enumerate(T1)))):
            cw = np.concatenate([m, oracle.encode(16, n, k, m)])
            mask = synth.erasure_mask(synth.key(61, n, k, len(T1), T1[0], i), n, [n - k, (n - k) // 2, 1][i])
            rx = cw.copy()
            rx[mask == 1] = 0x5A
            cws.append(cw)
            masks.append(mask)
            ds.append(to_dev(rx))
        cs.decode_batch([(n, k, masks[i], ds[i], ds[i]) for i in range(len(ds))])
        for i, cw in enumerate(cws):
            got = to_host(ds[i])
            assert (got == cw).all(), (n, k, T1, NCOLS[i], first_diff(got, cw))
    finally:
        cs.set_schedule(rs.RS_OP_DECODE, N, 0)


TILE_ENC = [(2048, 1024), (8192, 4096)]
TILE_DEC = [(300, 200), (4096, 2048), (5000, 4000)]


@pytest.mark.parametrize("cols", (128, 256))
@pytest.mark.parametrize("n,k,N,T1", _cases(TILE_ENC, lambda np_, kp: kp))
def test_encode_every_split_tile(cs, n, k, N, T1, cols):
    # 128: packed tiles for every row (260 columns: three tiles, the last of
    # one chunk); 256: 256-column tiles also for the narrow rows
    cs.set_schedule_tile(rs.RS_OP_ENCODE, N, cols)
    try:
        assert cs.get_schedule_tile(rs.RS_OP_ENCODE, N) == cols
        test_encode_every_split(cs, n, k, N, T1)
    finally:
        cs.set_schedule_tile(rs.RS_OP_ENCODE, N, 0)


@pytest.mark.parametrize("cols", (128, 256))
@pytest.mark.parametrize("n,k,N,T1", _cases(TILE_DEC, lambda np_, kp: np_))
def test_decode_every_split_tile(cs, n, k, N, T1, cols):
    cs.set_schedule_tile(rs.RS_OP_DECODE, N, cols)
    try:
        assert cs.get_schedule_tile(rs.RS_OP_DECODE, N) == cols
        test_decode_every_split(cs, n, k, N, T1)
    finally:
        cs.set_schedule_tile(rs.RS_OP_DECODE, N, 0)


def test_schedule_errors(cs, codec8):
    with pytest.raises(rs.RSError) as ei:
        cs.set_schedule(rs.RS_OP_DECODE, 12, 3)           # high part of 9 levels
    assert ei.value.code == rs.RS_EINVAL
    with pytest.raises(rs.RSError) as ei:
        cs.set_schedule(rs.RS_OP_DECODE, 12, 9)
    assert ei.value.code == rs.RS_EINVAL
    with pytest.raises(rs.RSError) as ei:
        cs.set_schedule(2, 12, 6)                          # no such operation
    assert ei.value.code == rs.RS_EINVAL
    with pytest.raises(rs.RSError) as ei:
        cs.set_schedule(rs.RS_OP_ENCODE, 8, 4)             # 256 points: one fused launch
    assert ei.value.code == rs.RS_ESHAPE
    with pytest.raises(rs.RSError) as ei:
        codec8.set_schedule(rs.RS_OP_ENCODE, 9, 5)         # GF(2^8) never exceeds 256 points
    assert ei.value.code == rs.RS_ESHAPE
    for N in range(9, 17):
        assert cs.get_schedule(rs.RS_OP_DECODE, N) == (N + 1) // 2
        assert cs.get_schedule_parts(rs.RS_OP_DECODE, N) == tune.default_split(N)
    for bad in ((4, 4, 3), (4, 4, 4, 4), (4, 4, 4, 1), (9, 3), (4, 4, 4, 4, 0)):
        with pytest.raises(rs.RSError) as ei:
            cs.set_schedule(rs.RS_OP_DECODE, 12, bad)
        assert ei.value.code == rs.RS_EINVAL, bad
    cs.set_schedule(rs.RS_OP_DECODE, 12, (4, 4, 4))
    assert cs.get_schedule_parts(rs.RS_OP_DECODE, 12) == (4, 4, 4) and cs.get_schedule(rs.RS_OP_DECODE, 12) == 4
    cs.set_schedule(rs.RS_OP_DECODE, 12, ())
    assert cs.get_schedule_parts(rs.RS_OP_DECODE, 12) == (6, 6)
    for N in range(9, 17):
        assert cs.get_schedule_tile(rs.RS_OP_ENCODE, N) == 0
    for args, code in (((rs.RS_OP_DECODE, 12, 64), rs.RS_EINVAL), ((2, 12, 128), rs.RS_EINVAL),
                       ((rs.RS_OP_DECODE, 8, 128), rs.RS_ESHAPE)):
        with pytest.raises(rs.RSError) as ei:
            cs.set_schedule_tile(*args)
        assert ei.value.code == code, args
    with pytest.raises(rs.RSError) as ei:
        codec8.set_schedule_tile(rs.RS_OP_DECODE, 9, 128)
    assert ei.value.code == rs.RS_ESHAPE


def test_schedule_environment():
    old = os.environ.get("RS_NB_SCHEDULE")
    try:
        os.environ["RS_NB_SCHEDULE"] = "dec:12:8,enc:11:4:128,dec:16:4/4/4/4:256"
        c = rs.Codec(16)
        assert c.get_schedule(rs.RS_OP_DECODE, 12) == 8
        assert c.get_schedule(rs.RS_OP_ENCODE, 11) == 4
        assert c.get_schedule(rs.RS_OP_DECODE, 11) == 6
        assert c.get_schedule_parts(rs.RS_OP_DECODE, 16) == (4, 4, 4, 4)
        assert (c.get_schedule_tile(rs.RS_OP_DECODE, 12), c.get_schedule_tile(rs.RS_OP_ENCODE, 11),
                c.get_schedule_tile(rs.RS_OP_DECODE, 16)) == (0, 128, 256)
        c.close()
        for bad in ("dec:12:3", "dec:12", "xyz:10:5", "enc:11:4;dec:12:6", "dec:12:4/4/3", "dec:12:4/",
                    "dec:12:6:64", "dec:12:6:"):
            os.environ["RS_NB_SCHEDULE"] = bad
            with pytest.raises(rs.RSError) as ei:
                rs.Codec(16)
            assert ei.value.code == rs.RS_EINVAL, bad
    finally:
        if old is None:
            os.environ.pop("RS_NB_SCHEDULE", None)
        else:
            os.environ["RS_NB_SCHEDULE"] = old


def test_autotuner_table(tmp_path):
    c = rs.Codec(16)
    try:
        tab = tune.tune(c, [(1024, 512), (16, 8)], row_bytes=(2048, 1026), target_bytes=4 << 20, warmup=1, reps=2)
        got = {(e["op"], e["N"]): e for e in tab["entries"]}
        assert set(got) == {("enc", 9), ("dec", 10)}
        for (op, N), e in got.items():
            assert tuple(e["parts"]) in tune.candidates(N)
            assert set(e["ms"]) == {tune.split_name(t) for t in tune.candidates(N)}
            assert c.get_schedule_parts(tune._OPS[op], N) == tuple(e["parts"])
            assert e["tile"] in tune.TILES and set(e["tile_ms"]) == {str(t) for t in tune.TILES}
            assert c.get_schedule_tile(tune._OPS[op], N) == e["tile"]
        path = str(tmp_path / "sched.json")
        tune.save(tab, path)
        c2 = rs.Codec(16)
        assert tune.load(path, c2) == tab
        for (op, N), e in got.items():
            assert c2.get_schedule_parts(tune._OPS[op], N) == tuple(e["parts"])
            assert c2.get_schedule_tile(tune._OPS[op], N) == e["tile"]
        c2.close()
    finally:
        c.close()


@pytest.mark.parametrize("parts,enc_parts", [((8, 8), (7, 8)), ((4, 4, 4, 4), (4, 4, 7)), ((4, 6, 6), (4, 5, 6)),
                                             ((6, 5, 5), (5, 5, 5))])
def test_largest_code_splits(cs, parts, enc_parts):
    # the (65536, 32768) code: decode over 2^16 points and encode over 2^15
    n, k, nc = 65536, 32768, 5
    N = 16
    cs.set_schedule(rs.RS_OP_DECODE, N, parts)
    cs.set_schedule(rs.RS_OP_ENCODE, 15, enc_parts)
    try:
        msg = rand_rows(k, 2 * nc, 62, len(parts))
        dm = to_dev(msg)
        dp = torch.zeros((n - k, 2 * nc), dtype=torch.uint8, device="cuda")
        cs.encode(n, k, dm, dp)
        par = to_host(dp)
        assert (par == oracle.encode(16, n, k, msg)).all(), enc_parts
        cw = np.concatenate([msg, par])
        mask = synth.erasure_mask(synth.key(63, len(parts), parts[0]), n, n - k)
        rx = cw.copy()
        rx[mask == 1] = 0
        d = to_dev(rx)
        cs.decode(n, k, mask, d)
        got = to_host(d)
        assert (got == cw).all(), (parts, first_diff(got, cw))
    finally:
        cs.set_schedule(rs.RS_OP_DECODE, N, 0)
        cs.set_schedule(rs.RS_OP_ENCODE, 15, 0)
