"""GPU parity at the full sizes of the measured workloads, seeded and launched
as the benchmark launches them: the (16, 8) GF(2^8) batch element by element
against the oracle; the (256, 128) GF(2^16) batch on sampled columns against
the oracle and whole-codeword recovery; the 8192-stripe mixed batch through
autotuned plans replayed in HIP graphs, on sampled columns against the oracle
and recovery of every stripe (row and column sums of each stripe before
erasure and after decode, over its bytes as int64 words)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1404_3458_amd import rs, synth, tune
from gpu_util import first_diff, to_host

pytestmark = pytest.mark.gpu


def _fill(cws, cfg_id, k):
    for s in range(len(cws)):
        synth.fill_random_torch(synth.key(cfg_id, s, synth.DATA), cws[s][:k])


def test_c1_full_config(codec8):
    # 4096 stripes of (16, 8) over GF(2^8), 1-byte shards, 8 erasures each
    n, k, ns, S, e = 16, 8, 4096, 1, 8
    cw = torch.empty((ns, n, S), dtype=torch.uint8, device="cuda")
    _fill(cw, 1, k)
    masks = [synth.erasure_mask(synth.key(1, s, synth.ERASURE), n, e) for s in range(ns)]
    codec8.encode_batch([(n, k, cw[s, :k], cw[s, k:]) for s in range(ns)])
    host = to_host(cw)
    for s in range(ns):
        exp = oracle.encode(8, n, k, host[s, :k])
        assert (host[s, k:] == exp).all(), (s, first_diff(host[s, k:], exp))
    rx = host.copy()
    for s in range(ns):
        rx[s][masks[s] == 1] = 0xA5
    d = torch.from_numpy(rx).cuda()
    codec8.decode_batch([(n, k, masks[s], d[s], d[s]) for s in range(ns)])
    got = to_host(d)
    for s in range(ns):
        exp = oracle.decode(8, n, k, masks[s], rx[s])
        assert (got[s] == exp).all(), (s, first_diff(got[s], exp))


def test_c2_full_config(codec16):
    # 64 stripes of (256, 128) over GF(2^16), 64 KiB shards, 128 erasures each
    n, k, ns, S, e = 256, 128, 64, 65536, 128
    cw = torch.empty((ns, n, S), dtype=torch.uint8, device="cuda")
    _fill(cw, 2, k)
    masks = [synth.erasure_mask(synth.key(2, s, synth.ERASURE), n, e) for s in range(ns)]
    codec16.encode_batch([(n, k, cw[s, :k], cw[s, k:]) for s in range(ns)])
    torch.cuda.synchronize()
    ref = cw.clone()
    ncol = S // 2
    for s in range(ns):
        cw[s][torch.from_numpy(masks[s]).bool().cuda()] = 0
    rx_dev = cw.clone()
    codec16.decode_batch([(n, k, masks[s], cw[s], cw[s]) for s in range(ns)])
    torch.cuda.synchronize()
    assert torch.equal(cw, ref), "decode did not restore every codeword"
    for s in (0, 37, ns - 1):
        cols = sorted({0, 1, ncol - 1} | set(int(c) for c in synth.uniform_int(synth.key(2, s, 90), 24, 0, ncol - 1)))

        def sample(t):
            return np.ascontiguousarray(t[s].cpu().numpy().reshape(n, ncol, 2)[:, cols, :].reshape(n, 2 * len(cols)))

        full, rx = sample(ref), sample(rx_dev)
        exp = oracle.encode(16, n, k, full[:k])
        assert (full[k:] == exp).all(), (s, first_diff(full[k:], exp))
        dec = oracle.decode(16, n, k, masks[s], rx)
        assert (sample(cw) == dec).all(), (s, first_diff(sample(cw), dec))


def _sums(t, n, sb):
    # a stripe's n * sb bytes as int64 words in an (n / 8) x sb matrix (n is
    # a multiple of 8 in every class; sb need not be): its row and column sums
    w = t.reshape(-1).view(torch.int64).view(n // 8, sb)
    return w.sum(dim=1), w.sum(dim=0)


def test_c4_full_config():
    # 8192 stripes of the five classes, log-uniform shards of 1-64 KiB,
    # uniform erasure counts; autotuned schedules, plans replayed in graphs
    ns = 8192
    shapes = synth.mixed_stripes(4, ns)
    torch.cuda.empty_cache()
    codec = rs.Codec(16)
    try:
        offs, total = [], 0
        for n, k, sb, e in shapes:
            offs.append(total)
            total += (n * sb + 255) // 256 * 256
        buf = torch.empty(total, dtype=torch.uint8, device="cuda")
        cws = [buf[offs[s]:offs[s] + n * sb].view(n, sb) for s, (n, k, sb, e) in enumerate(shapes)]
        for s, (n, k, sb, e) in enumerate(shapes):
            synth.fill_random_torch(synth.key(4, s, synth.DATA), cws[s][:k])
        masks = [synth.erasure_mask(synth.key(4, s, synth.ERASURE), n, e) for s, (n, k, sb, e) in enumerate(shapes)]
        tune.tune(codec, [(n, k) for n, k, sb, e in shapes])
        pe = codec.plan_encode_batch([(n, k, cws[s][:k], cws[s][k:]) for s, (n, k, sb, e) in enumerate(shapes)])
        pd = codec.plan_decode_batch([(n, k, masks[s], cws[s], cws[s]) for s, (n, k, sb, e) in enumerate(shapes)])
        graphs = []
        for p_ in (pe, pd):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                p_.launch()
            graphs.append(g)
        graphs[0].replay()
        torch.cuda.synchronize()
        # parity of one stripe per class (the first with erasures) on sampled columns
        picks = {}
        for s, (n, k, sb, e) in enumerate(shapes):
            if e and (n, k) not in picks:
                picks[(n, k)] = s
        assert len(picks) == len(synth.MIXED_CLASSES)
        samples = {}
        for (n, k), s in picks.items():
            sb = shapes[s][2]
            cols = sorted({0, sb // 2 - 1} | set(int(c) for c in synth.uniform_int(synth.key(4, s, 90), 6, 0,
                                                                                      sb // 2 - 1)))
            full = np.ascontiguousarray(cws[s].cpu().numpy().reshape(n, sb // 2, 2)[:, cols, :]
                                        .reshape(n, 2 * len(cols)))
            exp = oracle.encode(16, n, k, full[:k])
            assert (full[k:] == exp).all(), ((n, k), s, first_diff(full[k:], exp))
            samples[s] = (cols, full)
        before = [_sums(cws[s], n, sb) for s, (n, k, sb, e) in enumerate(shapes)]
        for s, (n, k, sb, e) in enumerate(shapes):
            if e:
                cws[s][torch.from_numpy(masks[s]).bool().cuda()] = 0
        graphs[1].replay()
        torch.cuda.synchronize()
        for s, (n, k, sb, e) in enumerate(shapes):
            after = _sums(cws[s], n, sb)
            assert torch.equal(after[0], before[s][0]) and torch.equal(after[1], before[s][1]), \
                ("stripe not restored", s, shapes[s])
        # the oracle's decode of the sampled columns of each picked stripe
        for s, (cols, full) in samples.items():
            n, k, sb, e = shapes[s]
            rx = full.copy()
            rx[masks[s] == 1] = 0
            dec = oracle.decode(16, n, k, masks[s], rx)
            got = np.ascontiguousarray(cws[s].cpu().numpy().reshape(n, sb // 2, 2)[:, cols, :]
                                       .reshape(n, 2 * len(cols)))
            assert (got == dec).all(), (s, first_diff(got, dec))
        del graphs
        pe.close()
        pd.close()
        del cws, buf
    finally:
        codec.close()
        torch.cuda.empty_cache()
