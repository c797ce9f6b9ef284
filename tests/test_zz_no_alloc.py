"""GPU test of rs_decode_static, the decode entry point that allocates
nothing: through the C ABI, its output equals rs_decode's (and the oracle's
codeword) bit for bit, on two calls in a row, the second on a smaller
input; mother codes over 256 points are refused."""
import numpy as np
import pytest
import torch

import oracle
from paper_1404_3458_amd import rs, synth
from gpu_util import first_diff, rand_rows, to_dev, to_host

pytestmark = pytest.mark.gpu


def _case(n, k, rb, e, key):
    msg = rand_rows(k, rb, 95, key)
    cw = np.concatenate([msg, oracle.encode(16, n, k, msg)])
    mask = synth.erasure_mask(synth.key(96, key), n, e)
    rx = cw.copy()
    rx[mask == 1] = 0
    return cw, rx, mask


@pytest.mark.parametrize("inplace", [True, False])
def test_decode_static_matches_decode(inplace):
    codec = rs.Codec(16)
    try:
        # a (256, 128) stripe with 128 erasures, then a smaller (64, 48) one
        # with a ragged row, on the same stream
        for n, k, rb, e, key in ((256, 128, 8192 + 6, 128, 1), (64, 48, 1030, 9, 2)):
            cw, rx, mask = _case(n, k, rb, e, key)
            a_in, b_in = to_dev(rx), to_dev(rx)
            a_out = a_in if inplace else torch.zeros_like(a_in)
            b_out = b_in if inplace else torch.zeros_like(b_in)
            codec.decode(n, k, mask, a_in, a_out)
            codec.decode_static(n, k, mask, b_in, b_out)
            ga, gb = to_host(a_out), to_host(b_out)
            assert (gb == ga).all(), (n, k, first_diff(gb, ga))
            assert (gb == cw).all(), (n, k, first_diff(gb, cw))
        # no erasures: a copy out of place, nothing in place
        cw, rx, mask = _case(16, 8, 64, 0, 3)
        src = to_dev(rx)
        dst = src if inplace else torch.zeros_like(src)
        codec.decode_static(16, 8, mask, src, dst)
        assert (to_host(dst) == cw).all()
        # mother codes over 256 points need the pass pipelines' scratch
        big = torch.zeros((512, 64), dtype=torch.uint8, device="cuda")
        with pytest.raises(rs.RSError) as ei:
            codec.decode_static(512, 256, np.zeros(512, np.uint8), big)
        assert ei.value.code == rs.RS_ESHAPE
    finally:
        codec.close()


def test_decode_static_in_a_graph():
    # captured once and replayed: the arena image travels in the captured
    # kernel's arguments, so each replay decodes its own erasure pattern
    codec = rs.Codec(16)
    try:
        n, k, rb, e = 256, 128, 4096, 100
        cw, rx, mask = _case(n, k, rb, e, 4)
        d = to_dev(rx)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                codec.decode_static(n, k, mask, d)
        for rep in range(3):
            d.copy_(to_dev(rx))
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            got = to_host(d)
            assert (got == cw).all(), (rep, first_diff(got, cw))
    finally:
        codec.close()
