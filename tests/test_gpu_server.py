"""GPU tests of the serving loop (rs_server_*): results of requests served
in a concurrent, budget-limited mix equal the oracle's (Algorithm 1 parity
on every column, Algorithm 2 output equal to the codeword and to the
oracle's decoder on sampled columns) and the results of the same requests
run alone through the single-stripe calls, bit for bit; the admission
record never exceeds the budget except for a lone oversized request; bad
requests are refused at submit while the others complete; a request waits
for the stream that produced its input."""
import numpy as np
import pytest
import torch

import oracle
from paper_1404_3458_amd import rs, synth
from gpu_util import first_diff, rand_rows, to_dev, to_host

pytestmark = pytest.mark.gpu

SHAPES = [(16, 8), (64, 48), (256, 224), (256, 128), (1024, 512), (40, 7), (512, 256)]


def _requests(count, key):
    shapes = synth.uniform_int(synth.key(70, key), count, 0, len(SHAPES) - 1)
    sizes = synth.uniform_int(synth.key(71, key), count, 1, 700)
    ops = synth.uniform_float(synth.key(72, key), count)
    reqs = []
    for i in range(count):
        n, k = SHAPES[int(shapes[i])]
        rb = 2 * int(sizes[i])
        msg = rand_rows(k, rb, 73, key, i)
        if ops[i] < 0.7:
            reqs.append(("enc", n, k, msg, None))
        else:
            cw = np.concatenate([msg, oracle.encode(16, n, k, msg)])
            e = int(synth.uniform_int(synth.key(74, key, i), 1, 0, n - k)[0])
            mask = synth.erasure_mask(synth.key(75, key, i), n, e)
            reqs.append(("dec", n, k, cw, mask))
    return reqs


def _buffers(reqs):
    bufs = []
    for op, n, k, data, mask in reqs:
        if op == "enc":
            bufs.append((to_dev(data), torch.zeros((n - k, data.shape[1]), dtype=torch.uint8, device="cuda")))
        else:
            rx = data.copy()
            rx[mask == 1] = 0
            d = to_dev(rx)
            bufs.append((d, d))
    return bufs


@pytest.mark.parametrize("budget,max_batch,nstreams", [(1 << 20, 4, 3), (64 << 20, 64, 2), (1 << 14, 1, 1)])
def test_server_mix_equals_alone(codec16, budget, max_batch, nstreams):
    reqs = _requests(48, budget)
    alone = _buffers(reqs)
    for (op, n, k, data, mask), (src, dst) in zip(reqs, alone):
        if op == "enc":
            codec16.encode(n, k, src, dst)
        else:
            codec16.decode(n, k, mask, src)
    torch.cuda.synchronize()
    mixed = _buffers(reqs)
    torch.cuda.synchronize()                   # the server's streams do not wait for torch's
    srv = rs.Server(codec16, budget, max_batch=max_batch, nstreams=nstreams)
    try:
        for i, ((op, n, k, data, mask), (src, dst)) in enumerate(zip(reqs, mixed)):
            srv.submit(rs.RS_OP_ENCODE if op == "enc" else rs.RS_OP_DECODE, n, k, src, dst, mask=mask, tag=1000 + i)
        got = {}
        while len(got) < len(reqs):
            for tag, status, t in srv.poll(timeout_ms=2000):
                assert status == rs.RS_OK
                got[tag] = t
        assert sorted(got) == [1000 + i for i in range(len(reqs))]
        assert srv.pending() == 0
        stats = srv.stats()
    finally:
        srv.close()
    for i, ((op, n, k, data, mask), a, m) in enumerate(zip(reqs, alone, mixed)):
        ga, gm = to_host(a[1]), to_host(m[1])
        assert (ga == gm).all(), (i, op, n, k, first_diff(gm, ga))
        if op == "enc":
            exp = oracle.encode(16, n, k, data)                    # every column
            assert (gm == exp).all(), (i, n, k, first_diff(gm, exp))
        else:
            assert (gm == data).all(), (i, n, k)                   # the codeword is restored
            ncol = data.shape[1] // 2
            cols = sorted({0, ncol - 1} | set(int(c) for c in synth.uniform_int(synth.key(76, budget, i), 6, 0,
                                                                                 ncol - 1)))
            pick = lambda x: np.ascontiguousarray(x.reshape(n, ncol, 2)[:, cols, :].reshape(n, 2 * len(cols)))
            rx = pick(data).copy()
            rx[mask == 1] = 0
            exp = oracle.decode(16, n, k, mask, rx)
            assert (pick(gm) == exp).all(), (i, n, k, first_diff(pick(gm), exp))
    st = stats
    assert st["admitted"] == len(reqs) and st["inflight_bytes"] == 0 and st["retried"] == 0, st
    assert st["peak_shared_bytes"] <= budget, st
    if st["peak_bytes"] > budget:
        # only a request larger than the budget, admitted alone, goes above it
        assert st["oversize_admitted"] >= 1 and st["largest_oversize"] > budget, st
        assert st["peak_bytes"] == st["largest_oversize"], st
    else:
        assert st["oversize_admitted"] == 0, st


def test_server_rejects_bad_requests(codec16):
    srv = rs.Server(codec16, 1 << 20)
    try:
        d = torch.zeros((16, 8), dtype=torch.uint8, device="cuda")
        mask = np.ones(16, np.uint8)
        with pytest.raises(rs.RSError) as e:
            srv.submit(rs.RS_OP_DECODE, 16, 8, d, d, mask=mask)
        assert e.value.code == rs.RS_ETOOMANY
        with pytest.raises(rs.RSError) as e:             # n <= k, checked by the library
            srv.submit(rs.RS_OP_ENCODE, 8, 8, d[:8], d[8:], row_bytes=8)
        assert e.value.code == rs.RS_ESHAPE
        with pytest.raises(ValueError):                   # parity buffer of the wrong row count
            srv.submit(rs.RS_OP_ENCODE, 16, 8, d[:8], d[:4])
        assert srv.pending() == 0
    finally:
        srv.close()


def test_server_bad_request_in_a_mix(codec16):
    # a request the batched calls would refuse is refused at submit; the
    # requests around it are served and bit-exact against the oracle
    reqs = _requests(12, 5)
    bufs = _buffers(reqs)
    torch.cuda.synchronize()
    srv = rs.Server(codec16, 64 << 20, max_batch=16, nstreams=2)
    d = torch.zeros((16, 8), dtype=torch.uint8, device="cuda")
    bad = [
        (rs.RS_OP_ENCODE, 16, 8, d[:8], d[8:], None, dict(row_bytes=7), rs.RS_EALIGN),        # odd row length
        (rs.RS_OP_ENCODE, 65536 + 16, 8, d[:8], d[8:], None, dict(row_bytes=8), rs.RS_ESHAPE),  # n' > 2^16
        (rs.RS_OP_ENCODE, 16, 8, 0, d[8:], None, dict(row_bytes=8), rs.RS_EINVAL),           # null rows
        (rs.RS_OP_DECODE, 16, 8, d, d, np.ones(16, np.uint8), {}, rs.RS_ETOOMANY),
    ]
    try:
        served = 0
        for i, ((op, n, k, data, mask), (src, dst)) in enumerate(zip(reqs, bufs)):
            srv.submit(rs.RS_OP_ENCODE if op == "enc" else rs.RS_OP_DECODE, n, k, src, dst, mask=mask, tag=i)
            served += 1
            if i < len(bad):
                bop, bn, bk, bsrc, bdst, bmask, kw, code = bad[i]
                with pytest.raises(rs.RSError) as e:
                    srv.submit(bop, bn, bk, bsrc, bdst, mask=bmask, tag=900 + i, **kw)
                assert e.value.code == code, (i, e.value.code)
        got = {}
        while len(got) < served:
            for tag, status, t in srv.poll(timeout_ms=2000):
                got[tag] = status
        assert all(st == rs.RS_OK for st in got.values()), got
        assert sorted(got) == list(range(len(reqs)))
        assert srv.pending() == 0
    finally:
        srv.close()
    for (op, n, k, data, mask), (src, dst) in zip(reqs, bufs):
        g = to_host(dst)
        exp = oracle.encode(16, n, k, data) if op == "enc" else data
        assert (g == exp).all(), (op, n, k, first_diff(g, exp))


def test_server_waits_for_the_producer_stream(codec16):
    # the input is written on a side stream behind a long-running kernel;
    # the request names that stream and must not read the input before it
    n, k, rb = 256, 128, 4096
    msg = rand_rows(k, rb, 77, 1)
    host = torch.from_numpy(msg).pin_memory()
    src = torch.zeros((k, rb), dtype=torch.uint8, device="cuda")
    dst = torch.zeros((n - k, rb), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    srv = rs.Server(codec16, 64 << 20, max_batch=4, nstreams=2)
    try:
        with torch.cuda.stream(side):
            torch.cuda._sleep(50_000_000)             # about 20 ms of device time
            src.copy_(host, non_blocking=True)
            srv.submit(rs.RS_OP_ENCODE, n, k, src, dst, tag=7)   # after = the current (side) stream
        done = []
        while not done:
            done = srv.poll(timeout_ms=2000)
        assert done[0][0] == 7 and done[0][1] == rs.RS_OK
    finally:
        srv.close()
    side.synchronize()
    g = to_host(dst)
    exp = oracle.encode(16, n, k, msg)
    assert (g == exp).all(), first_diff(g, exp)
