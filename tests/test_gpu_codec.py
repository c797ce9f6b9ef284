"""GPU parity of Algorithm 1 (encode) and Algorithm 2 (erasure decode),
single-stripe and batched, against the oracle, bit for bit, through the C ABI;
plus the error paths of the boundary."""
import numpy as np
import pytest
import torch

import oracle
from paper_1404_3458_amd import rs, synth
from gpu_util import first_diff, rand_rows, to_dev, to_host

pytestmark = pytest.mark.gpu

SHAPES16 = [(4, 2), (16, 8), (64, 48), (256, 128), (256, 224), (40, 7), (1024, 512), (4096, 2048), (100, 32),
            (96, 32), (150, 40)]
# more than 256 points: 8-level pass pipelines (low / high level split 5+4 .. 7+6),
# shortened mother codes, and codes with several parity blocks
SHAPES16_WIDE = [(512, 256), (2048, 1024), (8192, 4096), (600, 500), (1000, 300), (2048, 512), (300, 200), (1024, 256),
                 (700, 200), (10000, 6000)]
SHAPES8 = [(2, 1), (16, 8), (12, 8), (10, 3), (64, 48), (256, 128), (200, 100)]


def _cols(n):
    return [1, 5, 259] if n <= 256 else [3, 260]


def _encode_check(c, r, n, k, ncols, key):
    sym = r // 8
    msg = rand_rows(k, ncols * sym, 50, r, n, k, ncols, key)
    dm = to_dev(msg)
    dp = torch.zeros((n - k, ncols * sym), dtype=torch.uint8, device="cuda")
    c.encode(n, k, dm, dp)
    got = to_host(dp)
    exp = oracle.encode(r, n, k, msg)
    assert (got == exp).all(), (r, n, k, ncols, first_diff(got, exp))
    return msg, exp


@pytest.mark.parametrize("n,k", SHAPES16 + SHAPES16_WIDE)
def test_encode_r16(codec16, n, k):
    for ncols in _cols(n):
        _encode_check(codec16, 16, n, k, ncols, 1)


@pytest.mark.parametrize("n,k", SHAPES8)
def test_encode_r8(codec8, n, k):
    for ncols in _cols(n):
        _encode_check(codec8, 8, n, k, ncols, 2)


def _decode_check(c, r, n, k, ncols, e, key, inplace):
    sym = r // 8
    msg = rand_rows(k, ncols * sym, 51, r, n, k, ncols, key)
    cw = np.concatenate([msg, oracle.encode(r, n, k, msg)])
    mask = synth.erasure_mask(synth.key(52, r, n, k, key), n, e)
    rx = cw.copy()
    rx[mask == 1] = 0xA5                       # garbage in erased rows
    ds = to_dev(rx)
    if inplace:
        c.decode(n, k, mask, ds)
        got = to_host(ds)
    else:
        do = torch.zeros_like(ds)
        c.decode(n, k, mask, ds, do)
        got = to_host(do)
        assert (to_host(ds) == rx).all()      # input untouched
    assert (got == cw).all(), (r, n, k, ncols, e, first_diff(got, cw))


@pytest.mark.parametrize("n,k", SHAPES16 + SHAPES16_WIDE)
def test_decode_r16(codec16, n, k):
    for ncols in _cols(n):
        for e, inplace in ((n - k, True), ((n - k) // 2, False), (1, True)):
            _decode_check(codec16, 16, n, k, ncols, e, ncols + e, inplace)


@pytest.mark.parametrize("n,k", SHAPES8)
def test_decode_r8(codec8, n, k):
    for ncols in _cols(n):
        for e, inplace in ((n - k, True), ((n - k) // 2, False), (0, False)):
            _decode_check(codec8, 8, n, k, ncols, e, ncols + e, inplace)


def test_decode_every_k_subset_n16_gpu(codec8):
    # all 12870 8-subsets of a (16, 8) code, one column each, as one batch
    import itertools

    n, k = 16, 8
    msg = rand_rows(k, 1, 53)
    cw = np.concatenate([msg, oracle.encode(8, n, k, msg)])
    pats = list(itertools.combinations(range(n), k))
    rx = np.tile(cw, (len(pats), 1, 1))
    masks = np.ones((len(pats), n), dtype=np.uint8)
    for i, keep in enumerate(pats):
        masks[i, list(keep)] = 0
    rx[masks == 1] = 0
    d = to_dev(rx)
    codec8.decode_batch([(n, k, masks[i], d[i], d[i]) for i in range(len(pats))])
    got = to_host(d)
    assert (got == cw[None]).all()


def test_c3_shape_encode_decode(codec16):
    # one (65536, 32768) codeword with 128 symbols per row (256-byte rows)
    n, k, ncols = 65536, 32768, 128
    msg, par = _encode_check(codec16, 16, n, k, ncols, 3)
    cw = np.concatenate([msg, par])
    mask = synth.erasure_mask(synth.key(54), n, n - k)
    rx = cw.copy()
    rx[mask == 1] = 0
    d = to_dev(rx)
    codec16.decode(n, k, mask, d)
    got = to_host(d)
    assert (got == cw).all(), first_diff(got, cw)


def test_batch_mixed_shapes(codec16):
    specs = [(16, 8, 1000), (64, 48, 514), (256, 224, 2050), (1024, 512, 300), (256, 128, 4096), (16, 8, 2),
             (4096, 2048, 72), (512, 256, 6), (1000, 300, 520), (1024, 512, 8)]
    msgs, pars, exps = [], [], []
    for i, (n, k, rb) in enumerate(specs):
        m = rand_rows(k, rb, 55, i)
        msgs.append(to_dev(m))
        pars.append(torch.zeros((n - k, rb), dtype=torch.uint8, device="cuda"))
        exps.append(oracle.encode(16, n, k, m))
    codec16.encode_batch([(n, k, msgs[i], pars[i]) for i, (n, k, _) in enumerate(specs)])
    for i in range(len(specs)):
        got = to_host(pars[i])
        assert (got == exps[i]).all(), (specs[i], first_diff(got, exps[i]))
    # decode all in one batch, half in place
    items, cws = [], []
    for i, (n, k, rb) in enumerate(specs):
        cw = np.concatenate([to_host(msgs[i]), exps[i]])
        e = int(synth.uniform_int(synth.key(56, i), 1, 0, n - k)[0])
        mask = synth.erasure_mask(synth.key(57, i), n, e)
        rx = cw.copy()
        rx[mask == 1] = 0
        ds = to_dev(rx)
        do = ds if i % 2 == 0 else torch.zeros_like(ds)
        items.append((n, k, mask, ds, do))
        cws.append(cw)
    codec16.decode_batch(items)
    for i, it in enumerate(items):
        got = to_host(it[4])
        assert (got == cws[i]).all(), (specs[i], first_diff(got, cws[i]))


def test_error_paths(codec16):
    d = torch.zeros((16, 8), dtype=torch.uint8, device="cuda")
    p = torch.zeros((8, 8), dtype=torch.uint8, device="cuda")
    with pytest.raises(rs.RSError) as e:
        codec16.encode(16, 16, d, d, row_bytes=8)
    assert e.value.code == rs.RS_ESHAPE
    with pytest.raises(rs.RSError) as e:
        codec16.encode(16, 8, d[:8], p, row_bytes=7)
    assert e.value.code == rs.RS_EALIGN
    with pytest.raises(rs.RSError) as e:
        codec16.encode(131072, 8, d[:8], p, row_bytes=8)
    assert e.value.code == rs.RS_ESHAPE
    mask = np.zeros(16, np.uint8)
    mask[:9] = 1
    with pytest.raises(rs.RSError) as e:
        codec16.decode(16, 8, mask, d)
    assert e.value.code == rs.RS_ETOOMANY
    with pytest.raises(rs.RSError) as e:
        codec16.fft(12, 0, d, row_bytes=8)
    assert e.value.code == rs.RS_ESHAPE
    assert codec16.raw_call("rs_encode", 16, 8, None, None, 8, None) == rs.RS_EINVAL
    # nothing was written by the rejected calls
    assert int(p.sum()) == 0 and int(d.sum()) == 0
    assert codec16.raw_call("rs_encode", 16, 8, None, None, 0, None) == rs.RS_OK   # empty rows: no-op


def test_corrupted_survivor_is_not_detected(codec16):
    # the decoder is erasure-only: a wrong surviving symbol silently yields a
    # wrong (but well-formed) result, as the paper's decoder has no check
    n, k = 16, 8
    msg = rand_rows(k, 8, 58)
    cw = np.concatenate([msg, oracle.encode(16, n, k, msg)])
    mask = np.zeros(n, np.uint8)
    mask[[1, 3, 9]] = 1
    rx = cw.copy()
    rx[0, 0] ^= 1
    d = to_dev(rx)
    codec16.decode(n, k, mask, d)
    got = to_host(d)
    assert not (got == cw).all()
    assert (got == oracle.decode(16, n, k, mask, rx)).all()


PLAN_SPECS = [(16, 8, 1000), (64, 48, 514), (256, 128, 4096), (256, 224, 2050), (1024, 512, 300), (512, 256, 6),
              (4096, 2048, 72), (1000, 300, 520)]


def _plan_buffers(specs, key):
    msgs, pars = [], []
    for i, (n, k, rb) in enumerate(specs):
        msgs.append(to_dev(rand_rows(k, rb, 60, key, i)))
        pars.append(torch.zeros((n - k, rb), dtype=torch.uint8, device="cuda"))
    return msgs, pars


def _refill(msgs, key):
    for i, m in enumerate(msgs):
        m.copy_(to_dev(rand_rows(m.shape[0], m.shape[1], 61, key, i)))


def _check_parity(specs, msgs, pars):
    for i, (n, k, rb) in enumerate(specs):
        exp = oracle.encode(16, n, k, to_host(msgs[i]))
        got = to_host(pars[i])
        assert (got == exp).all(), (specs[i], first_diff(got, exp))


def test_plan_encode_reuse_and_graph_replay(codec16):
    specs = PLAN_SPECS
    msgs, pars = _plan_buffers(specs, 1)
    plan = codec16.plan_encode_batch([(n, k, msgs[i], pars[i]) for i, (n, k, _) in enumerate(specs)])
    plan.launch()
    torch.cuda.synchronize()
    _check_parity(specs, msgs, pars)
    _refill(msgs, 2)                          # the plan reads the buffers' current contents
    plan.launch()
    torch.cuda.synchronize()
    _check_parity(specs, msgs, pars)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.launch()
    for rep in range(3):
        _refill(msgs, 10 + rep)               # eager work between replays
        for p_ in pars:
            p_.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _check_parity(specs, msgs, pars)
    plan.close()


def test_plan_decode_reuse_and_graph_replay(codec16):
    specs = PLAN_SPECS
    items, cws, rxs = [], [], []
    for i, (n, k, rb) in enumerate(specs):
        msg = rand_rows(k, rb, 62, i)
        cw = np.concatenate([msg, oracle.encode(16, n, k, msg)])
        e = [n - k, 0, 1, (n - k) // 2][i % 4]
        mask = synth.erasure_mask(synth.key(63, i), n, e)
        rx = cw.copy()
        rx[mask == 1] = 0x5A
        ds = to_dev(rx)
        do = ds if i % 2 == 0 else torch.zeros_like(ds)
        items.append((n, k, mask, ds, do))
        cws.append(cw)
        rxs.append(rx)
    plan = codec16.plan_decode_batch(items)

    def reset_and_check(run):
        for i, it in enumerate(items):
            it[3].copy_(to_dev(rxs[i]))
            if it[4] is not it[3]:
                it[4].zero_()
        torch.cuda.synchronize()
        run()
        torch.cuda.synchronize()
        for i, it in enumerate(items):
            got = to_host(it[4])
            assert (got == cws[i]).all(), (specs[i], first_diff(got, cws[i]))

    reset_and_check(plan.launch)
    reset_and_check(plan.launch)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.launch()
    for _ in range(3):
        reset_and_check(g.replay)
    plan.close()


@pytest.mark.parametrize("r,n,k,ns,ncols,inplace", [(16, 256, 128, 40, 16384 + 3, True), (16, 128, 64, 24, 16384, True),
                                                    (16, 64, 40, 30, 9000, True), (16, 256, 128, 40, 16384, True),
                                                    (16, 256, 200, 24, 8192, False), (16, 256, 128, 24, 8192, False),
                                                    (16, 200, 100, 21, 8192 + 5, False), (8, 256, 128, 24, 8192, True),
                                                    (8, 240, 120, 22, 8192 + 3, False)])
def test_decode_many_tiles(request, r, n, k, ns, ncols, inplace):
    # more tiles than workgroups resident on the device (for 2^8 points:
    # the streamed kernel, with runs of tiles that cross stripes), whole and
    # ragged tiles, aligned and unaligned rows, in place and out of place
    codec = request.getfixturevalue("codec%d" % r)
    sb = r // 8
    rb = sb * ncols
    cw = torch.empty((ns, n, rb), dtype=torch.uint8, device="cuda")
    for s in range(ns):
        synth.fill_random_torch(synth.key(80, n, s), cw[s, :k])
    codec.encode_batch([(n, k, cw[s, :k], cw[s, k:]) for s in range(ns)])
    torch.cuda.synchronize()
    cols = sorted({0, 1, ncols - 1} | set(int(c) for c in synth.uniform_int(synth.key(81, n), 12, 0, ncols - 1)))
    for s in (0, ns - 1):
        host = to_host(cw[s]).reshape(n, ncols, sb)[:, cols, :].reshape(n, sb * len(cols))
        assert (oracle.encode(r, n, k, np.ascontiguousarray(host[:k])) == host[k:]).all()
    ref = cw.clone()
    masks = []
    for s in range(ns):
        e = [n - k, (n - k) // 2, 1][s % 3]
        m = synth.erasure_mask(synth.key(82, n, s), n, e)
        cw[s][torch.from_numpy(m).bool().cuda()] = 0
        masks.append(m)
    rx = cw.clone()
    out = cw if inplace else torch.zeros_like(cw)
    codec.decode_batch([(n, k, masks[s], cw[s], out[s]) for s in range(ns)])
    torch.cuda.synchronize()
    for s in range(ns):
        assert torch.equal(out[s], ref[s]), s
        if not inplace:
            assert torch.equal(cw[s], rx[s]), s          # input untouched


@pytest.mark.parametrize("points", [256, 128])
def test_decode_persistent_mixed_stripes(codec16, points):
    # one decode launch of 2^8 or 2^7 points with more tiles than workgroup
    # slots over stripes of different shapes, widths (whole and ragged last
    # tiles) and erasure counts, in place and out of place in the same
    # batch: the workgroups' tile ranges cross stripes of every kind
    if points == 256:
        shapes = [(256, 128), (240, 120), (192, 96), (200, 128), (160, 64)]
        widths = [8192, 4100, 6000, 260]
    else:
        shapes = [(128, 64), (96, 48), (80, 40), (120, 64), (72, 16)]
        widths = [16384, 8196, 12000, 516]
    specs = [(shapes[i % 5], widths[i % 4]) for i in range(30)]
    cws, masks, refs, outs = [], [], [], []
    for i, ((n, k), ncols) in enumerate(specs):
        cw = torch.empty((n, 2 * ncols), dtype=torch.uint8, device="cuda")
        synth.fill_random_torch(synth.key(90, points, i), cw[:k])
        cws.append(cw)
    codec16.encode_batch([(n, k, cws[i][:k], cws[i][k:]) for i, ((n, k), _) in enumerate(specs)])
    torch.cuda.synchronize()
    for i in (0, 1, 7, 29):
        (n, k), ncols = specs[i]
        cols = sorted({0, ncols - 1} | set(int(c) for c in synth.uniform_int(synth.key(91, points, i), 6, 0, ncols - 1)))
        host = to_host(cws[i]).reshape(n, ncols, 2)[:, cols, :].reshape(n, 2 * len(cols))
        assert (oracle.encode(16, n, k, np.ascontiguousarray(host[:k])) == host[k:]).all(), specs[i]
    for i, ((n, k), ncols) in enumerate(specs):
        e = [n - k, (3 * (n - k)) // 4, n - k - 3][i % 3]
        m = synth.erasure_mask(synth.key(92, points, i), n, e)
        refs.append(cws[i].clone())
        cws[i][torch.from_numpy(m).bool().cuda()] = 0
        masks.append(m)
        outs.append(cws[i] if i % 2 == 0 else torch.zeros_like(cws[i]))
    rx = [c.clone() for c in cws]
    codec16.decode_batch([(n, k, masks[i], cws[i], outs[i]) for i, ((n, k), _) in enumerate(specs)])
    torch.cuda.synchronize()
    for i in range(len(specs)):
        assert torch.equal(outs[i], refs[i]), specs[i]
        if i % 2:
            assert torch.equal(cws[i], rx[i]), specs[i]       # input untouched


def test_plan_timestamps(codec16):
    # per-stripe completion stamps: every stripe a kernel works on is stamped
    # after the launch's start stamp and before the start of a later launch
    # on the same stream; stripes without kernel work keep 0; None stops them
    specs = PLAN_SPECS + [(64, 32, 0)]
    msgs, pars = _plan_buffers(specs, 3)
    enc = codec16.plan_encode_batch([(n, k, msgs[i], pars[i]) for i, (n, k, _) in enumerate(specs)])
    ts1 = torch.full((len(specs) + 1,), -1, dtype=torch.int64, device="cuda")
    ts2 = torch.full_like(ts1, -1)
    with pytest.raises(ValueError):                  # one entry short
        enc.set_timestamps(ts1[1:])
    khz = enc.set_timestamps(ts1)
    assert khz > 0
    enc.launch()
    enc.set_timestamps(ts2)
    enc.launch()
    torch.cuda.synchronize()
    _check_parity(specs, msgs, pars)
    a, b = ts1.cpu().numpy(), ts2.cpu().numpy()
    for t in (a, b):
        assert t[0] > 0
        for i, (n, k, rb) in enumerate(specs):
            if rb:
                assert t[1 + i] >= t[0], (specs[i], t)
            else:
                assert t[1 + i] == 0, (specs[i], t)
    assert b[0] >= a[1:].max()
    assert (b[1:] - b[0]).max() < 10 * khz * 1000      # under 10 s
    enc.set_timestamps(None)
    ts2.fill_(-1)
    enc.launch()
    torch.cuda.synchronize()
    assert (ts2.cpu().numpy() == -1).all()
    enc.close()

    items, cws, worked = [], [], []
    for i, (n, k, rb) in enumerate(specs):
        msg = rand_rows(k, rb, 64, i)
        cws.append(np.concatenate([msg, oracle.encode(16, n, k, msg)]))
        e = [n - k, 0, 1, 0][i % 4]
        mask = synth.erasure_mask(synth.key(65, i), n, e)
        rx = cws[i].copy()
        rx[mask == 1] = 0x33
        ds = to_dev(rx)
        do = ds if i % 4 != 3 else torch.zeros_like(ds)   # i % 4 == 3: no erasures, out of place
        items.append((n, k, mask, ds, do))
        worked.append(rb > 0 and e > 0)
    dec = codec16.plan_decode_batch(items)
    ts = torch.full((len(specs) + 1,), -1, dtype=torch.int64, device="cuda")
    dec.set_timestamps(ts)
    dec.launch()
    torch.cuda.synchronize()
    t = ts.cpu().numpy()
    for i, it in enumerate(items):
        got = to_host(it[4])
        assert (got == cws[i]).all(), (specs[i], first_diff(got, cws[i]))
        if worked[i]:
            assert t[1 + i] >= t[0] > 0, (specs[i], t)
        else:
            assert t[1 + i] == 0, (specs[i], t)
    dec.close()


@pytest.mark.parametrize("r,n,k", [(16, 16, 1), (16, 256, 1), (16, 300, 1), (16, 1024, 1), (16, 4096, 1),
                                   (16, 16, 15), (16, 256, 255), (16, 1000, 999), (8, 255, 1), (8, 2, 1),
                                   (8, 16, 15), (8, 128, 127)])
def test_degenerate_codes(request, r, n, k):
    # k = 1: the message polynomial is a constant, so every codeword row
    # repeats the message row; k = n - 1: one parity row.  Both recover from
    # every n - k erasures.
    c = request.getfixturevalue("codec%d" % r)
    msg, par = _encode_check(c, r, n, k, 131, 7)
    cw = np.concatenate([msg, par])
    if k == 1:
        assert (cw == msg[0][None, :]).all()
    for e in sorted({1, n - k}):
        mask = synth.erasure_mask(synth.key(71, r, n, k, e), n, e)
        rx = cw.copy()
        rx[mask == 1] = 0x3C
        d = to_dev(rx)
        c.decode(n, k, mask, d)
        got = to_host(d)
        assert (got == cw).all(), (r, n, k, e, first_diff(got, cw))


def test_mother_code_longer_than_the_field(codec8):
    # (256, 255) over GF(2^8) would need a 512-point mother code (k' = 256,
    # n' = pow2ceil(k' + 1)): refused before any work, like the oracle does
    msg = torch.zeros((255, 4), dtype=torch.uint8, device="cuda")
    par = torch.zeros((1, 4), dtype=torch.uint8, device="cuda")
    with pytest.raises(rs.RSError) as ei:
        codec8.encode(256, 255, msg, par)
    assert ei.value.code == rs.RS_ESHAPE


def test_empty_batches(codec16):
    # zero stripes, and stripes that all have empty rows, are no-ops through
    # the batched calls and the plans (whose stamps then only mark the start)
    assert codec16.encode_batch([]) == rs.RS_OK
    assert codec16.decode_batch([]) == rs.RS_OK
    assert codec16.raw_call("rs_encode_batch", None, 0, None) == rs.RS_OK
    assert codec16.raw_call("rs_encode_batch", None, -1, None) == rs.RS_EINVAL
    assert codec16.raw_call("rs_decode_batch", None, None, 1, None) == rs.RS_EINVAL
    e = torch.zeros((0,), dtype=torch.uint8, device="cuda")
    empties = [(16, 8, e, e, 0), (1024, 512, e, e, 0)]
    assert codec16.encode_batch(empties) == rs.RS_OK
    masks = [np.ones(16, np.uint8) * (np.arange(16) < 8), np.zeros(1024, np.uint8)]
    assert codec16.decode_batch([(n, k, masks[i], e, e, 0) for i, (n, k, _, _, _) in enumerate(empties)]) == rs.RS_OK
    for stripes in ([], empties):
        for pl in (codec16.plan_encode_batch(stripes), codec16.plan_decode_batch(
                [(n, k, masks[i], e, e, 0) for i, (n, k, _, _, _) in enumerate(stripes)])):
            ts = torch.full((len(stripes) + 1,), -1, dtype=torch.int64, device="cuda")
            pl.set_timestamps(ts)
            pl.launch()
            torch.cuda.synchronize()
            t = ts.cpu().numpy()
            assert t[0] > 0 and (t[1:] == 0).all(), t
            pl.close()
