"""GPU tests of the serving loop (rs_server_*): results of requests served
in a concurrent, budget-limited mix equal the results of the same requests
run alone through the single-stripe calls, bit for bit."""
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
    finally:
        srv.close()
    for i, ((op, n, k, data, mask), a, m) in enumerate(zip(reqs, alone, mixed)):
        ga, gm = to_host(a[1]), to_host(m[1])
        assert (ga == gm).all(), (i, op, n, k, first_diff(gm, ga))
        if op == "dec":
            assert (gm == data).all(), (i, n, k)          # the codeword is restored


def test_server_rejects_bad_requests(codec16):
    srv = rs.Server(codec16, 1 << 20)
    try:
        d = torch.zeros((16, 8), dtype=torch.uint8, device="cuda")
        mask = np.ones(16, np.uint8)
        with pytest.raises(rs.RSError) as e:
            srv.submit(rs.RS_OP_DECODE, 16, 8, d, d, mask=mask)
        assert e.value.code == rs.RS_ETOOMANY
        with pytest.raises(rs.RSError) as e:
            srv.submit(rs.RS_OP_ENCODE, 8, 8, d[:8], d[8:])
        assert e.value.code == rs.RS_ESHAPE
        assert srv.pending() == 0
    finally:
        srv.close()
