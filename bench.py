#!/usr/bin/env python3
"""Benchmark of the novel-basis Reed-Solomon erasure codec on one MI355X.

A step is one pass of the whole hot path over one batch of synthetic stripes:
Algorithm 1 (encode every stripe), then Algorithm 2 (recover the erased rows
of every stripe, in place).  Default workload: GF(2^16) mod 0x1100B, the
(n, k) = (256, 128) code, 64 stripes of 64 KiB shards (512 MiB of message),
n - k = 128 uniformly drawn erasures per stripe.

Prints one JSON line.  `value` is message bytes per second of the whole step
(each message byte is encoded and then decoded once per step).  `roofline`
describes the dominant launch (the decode for the default workload), timed
with HIP events on the launch stream: its algorithmic HBM bytes (n * S per
stripe: survivors read and erased rows written, or message read and parity
written) over its average duration, against the 8 TB/s HBM peak and against a
device-to-device copy measured in the same run.  Beside it, `alu` gives the
same launch against the integer-ALU ceiling of this implementation's
multiply (the kernels are bound by its issue rate, not by HBM).
`cpu_baseline` times the CPU oracle on a bounded sample of the same workload
on this host's cores, and on one core.  The default line's detail also
carries the 8192-stripe mixed workload (batched plans in a HIP graph against
per-stripe calls, and per-stripe completion p50/p99), measured after the
default workload's buffers are released (--no-mixed skips it).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

CONFIGS = {
    "c2": dict(r=16, n=256, k=128, stripes=64, shard_bytes=65536, erasures=128,
               workload="GF(2^16) mod 0x1100B, (n,k)=(256,128), 64 stripes x 64 KiB shards, "
                        "encode + 128 erasures per stripe + decode"),
    "c1": dict(r=8, n=16, k=8, stripes=4096, shard_bytes=1, erasures=8,
               workload="GF(2^8) mod 0x11D, (n,k)=(16,8), 4096 stripes x 1 B shards, "
                        "encode + 8 erasures per stripe + decode"),
    "c3": dict(r=16, n=65536, k=32768, stripes=1, shard_bytes=256, erasures=32768, sets=64,
               workload="GF(2^16) mod 0x1100B, (n,k)=(65536,32768), 1 stripe x 256 B shards, "
                        "encode + 32768 erasures + decode; 64 codeword buffers (1 GiB) used in turn, "
                        "so that no step finds its data in the 256 MB last-level cache"),
    "c5": dict(r=16, stripes=5000, serving=True, budget=64 << 30, requests=5000, warm=500, encode_share=0.7,
               workload="GF(2^16) mod 0x1100B serving: Poisson arrivals, 70% encode / 30% decode requests, "
                        "(n,k) and shards as the mixed workload (5000 resident stripes), 64 GB admission budget; "
                        "saturated rate mu, then lambda = 0.5, 0.7, 0.9 mu with 5000 requests each after 500 warm-up"),
    "poly": dict(r=16, h=4096, cols=32768, poly="mul",
                 workload="GF(2^16) mod 0x1100B novel-basis product (Sec. 6.1, Table 1): two operands of h = 4096 "
                          "coefficients x 32768 columns, 8192-point transforms, point-by-point product, inverse"),
    "conv": dict(r=16, h=4096, cols=32768, poly="conv",
                 workload="GF(2^16) mod 0x1100B basis conversion novel -> monomial -> novel: h = 4096 "
                          "coefficients x 32768 columns"),
    "c4": dict(r=16, stripes=8192, mixed=True,
               workload="GF(2^16) mod 0x1100B, 8192 stripes, (n,k) uniform over (16,8) (64,48) (256,224) "
                        "(1024,512) (4096,2048), shards log-uniform 1-64 KiB, erasures uniform in [0,n-k]; "
                        "encode + decode, per-class batched plans replayed as one HIP graph (smallest class first) "
                        "vs per-stripe calls"),
}


def kernel_source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1404_3458_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(cfg_name):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (profiles/traffic_<cfg>.txt, "key: value" lines), or None when it
    was taken from different kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.txt" % cfg_name)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                key, val = line.split(":", 1)
                kv[key.strip()] = val.strip()
    if kv.get("kernel_source_hash") != kernel_source_hash():
        return None
    try:
        return int(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def pow2ceil(v):
    p = 1
    while p < v:
        p *= 2
    return p


def paper_mults_per_column(n, k, decode):
    """Multiplications of one codeword column by the paper's counts: an
    h-point transform takes (h/2) lg h, minus h - 1 at shift 0 (Sec. 3.4); the
    derivative h + h (Sec. 4.2); decode steps 2 and 6 one per stored row
    (Algorithm 2).  Shortened codes run on the mother code (n', k')."""
    kp = pow2ceil(k)
    npr = pow2ceil(kp + n - k)

    def m(h):
        return (h // 2) * (h.bit_length() - 1)

    def m0(h):
        return m(h) - (h - 1)

    if decode:
        return 2 * m0(npr) + 2 * npr + n
    return m0(kp) + (npr // kp - 1) * m(kp)


# Integer-ALU ceiling of the multiply-by-constant, from the chip's unit
# counts and clock: 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz = 78.6 T 32-bit
# lane operations per second for plain VALU operations (the rate behind the
# 157.3 TFLOP/s fp32 figure); v_perm_b32, and any VALU operation with a
# scalar-register operand, issue at half that rate (measured on this chip).
# One multiply-accumulate of 4 symbols by a wave-uniform constant costs, in
# full-rate slots: r = 16: 12 v_perm (24) + 6 three-input XOR + 10 selector
# shifts/masks = 40; r = 8: 3 v_perm (6) + 2 XOR + 5 selector ops = 13.
VALU_LANE_OPS_PER_S = 256 * 4 * 32 * 2.4e9
SLOTS_PER_4_MACS = {16: 40, 8: 13}


def mult_peak_per_s(r):
    return VALU_LANE_OPS_PER_S * 4 / SLOTS_PER_4_MACS[r]


def copy_gbps(nbytes=1 << 30, reps=10):
    """Device-to-device copy rate (bytes read + bytes written per second) of
    a plain torch copy of nbytes, timed with events: the practical HBM
    ceiling the roofline is also quoted against."""
    import numpy as np
    import torch

    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    dst.copy_(src)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in evs:
        a.record()
        dst.copy_(src)
        b.record()
    torch.cuda.synchronize()
    ms = float(np.median([a.elapsed_time(b) for a, b in evs]))
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def hbm_roofline(kernel, algo_bytes, launch_s, traffic, copy_rate, extra=None):
    """The roofline object of a launch: algorithmic bytes over its duration
    against the HBM peak, and against the measured copy rate."""
    achieved = algo_bytes / launch_s / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kernel,
            "algorithmic_bytes_per_launch": algo_bytes,
            "copy_GBps": round(copy_rate, 1) if copy_rate else None,
            "frac_of_copy": round(achieved / copy_rate, 4) if copy_rate else None}
    if extra:
        roof.update(extra)
    return roof


def alu_figures(mults, launch_s, r):
    peak = mult_peak_per_s(r)
    return {"alu": {"achieved_Tmul_s": round(mults / launch_s / 1e12, 4), "peak_Tmul_s": round(peak / 1e12, 4),
                    "frac": round(mults / launch_s / peak, 4), "mults_per_launch": mults,
                    "peak_basis": "this implementation's multiply: %d full-rate VALU slots per 4 symbols, "
                                  "78.6 T slots/s" % SLOTS_PER_4_MACS[r]}}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(cfg, sample_stripes, sample_cols, threads, target_s=12.0):
    """Oracle encode + decode of stripes of the workload restricted to
    `sample_cols` columns each, on `threads` host threads (column blocks): one
    stripe first, then as many more (up to the workload's count, at least
    `sample_stripes`) as fill about target_s seconds of wall time."""
    import concurrent.futures as cf

    import numpy as np

    import oracle
    from paper_1404_3458_amd import synth

    r, n, k, S = cfg["r"], cfg["n"], cfg["k"], cfg["shard_bytes"]
    sym = r // 8
    cols = min(sample_cols, S // sym)
    oracle.build()

    def blocks_of(s):
        msg = np.ascontiguousarray(synth.random_bytes(synth.key(cfg["id"], s, synth.DATA), k * S).reshape(k, S)
                                   [:, :cols * sym])
        mask = synth.erasure_mask(synth.key(cfg["id"], s, synth.ERASURE), n, cfg["erasures"])
        per = max(1, cols // threads)
        return [(msg[:, c0 * sym:min(cols, c0 + per) * sym].copy(), mask) for c0 in range(0, cols, per)]

    def work(item):
        msg, mask = item
        par = oracle.encode(r, n, k, msg)
        cw = np.concatenate([msg, par])
        rx = cw.copy()
        rx[mask == 1] = 0
        out = oracle.decode(r, n, k, mask, rx)
        assert (out == cw).all()
        return msg.nbytes

    def run(stripes):
        items = [b for s in stripes for b in blocks_of(s)]
        t0 = time.perf_counter()
        with cf.ThreadPoolExecutor(max_workers=threads) as ex:
            nb = sum(ex.map(work, items))
        return nb, time.perf_counter() - t0

    nbytes, dt = run([0])
    more = min(cfg["stripes"], max(sample_stripes, int(target_s / max(dt, 1e-3)))) - 1
    if more > 0:
        nb2, dt2 = run(range(1, 1 + more))
        nbytes, dt = nbytes + nb2, dt + dt2
    # one core: the first 1/threads of stripe 0's column blocks, one at a time
    items1 = blocks_of(0)[:1]
    t1 = time.perf_counter()
    nb1 = sum(work(it) for it in items1)
    dt1 = time.perf_counter() - t1
    return {"value": nbytes / dt / 1e9, "unit": "GB/s", "cores": threads, "kind": "oracle",
            "affinity_cores": len(os.sched_getaffinity(0)), "cpu_model": cpu_model(),
            "single_core_GBps": nb1 / dt1 / 1e9,
            "sample": "%d stripe(s) x %d columns of the same workload (%d B of message), encode + decode, "
                      "%.2f s wall on %d threads; single core: %d columns of one stripe, %.2f s"
                      % (1 + max(more, 0), cols, nbytes, dt, threads, items1[0][0].shape[1] // sym, dt1)}


def schedule_for(args, codec, shapes, target_bytes=256 << 20):
    """Pass-pipeline schedules for a workload, set in `codec`: a saved table
    (--schedule), the defaults (--no-tune), or the autotuner run on seeded
    batches of the workload's (n, k) classes with row lengths at the deciles
    of its shard lengths and about target_bytes of codeword per class (setup,
    outside every timed region)."""
    from paper_1404_3458_amd import tune

    t0 = time.perf_counter()
    if args.schedule:
        tab, src = tune.load(args.schedule, codec), "file " + os.path.basename(args.schedule)
    elif args.no_tune:
        return {"source": "default (T1 = ceil(N/2))"}
    else:
        sbs = sorted(sb for n, k, sb, e in shapes)
        rbs = tuple(sorted({sbs[int(q * (len(sbs) - 1))] for q in (0.1, 0.3, 0.5, 0.7, 0.9)}))
        tab = tune.tune(codec, sorted({(n, k) for n, k, sb, e in shapes}), row_bytes=rbs, target_bytes=target_bytes)
        src = "autotuned"
    return {"source": src, "setup_s": round(time.perf_counter() - t0, 2), "T1": tune.summary(tab),
            "candidate_ms": {"%s:%d" % (e["op"], e["N"]): e.get("ms") for e in tab["entries"]},
            "tile_ms": {"%s:%d" % (e["op"], e["N"]): e.get("tile_ms") for e in tab["entries"]}}


def conv_mults_per_column(h):
    """Constant multiplications of the two basis conversions of one column,
    as the kernels do them: level t of the way up, one per (output row, m)
    with a term; level t of the way down, one per quotient term plus the
    division, and one per remainder term."""
    L = h.bit_length() - 1
    up = down = 0
    for t in range(1, L + 1):
        hh, blocks = 1 << (t - 1), h >> t
        up += blocks * sum(1 for j in range(2 * hh) for m in range(t) if 0 <= j - (1 << m) < hh)
        q = sum(1 + sum(1 for m in range(t - 1) if (1 << m) > e) for e in range(hh))
        rem = sum(1 for j in range(hh) for m in range(t - 1) if (1 << m) <= j) if t > 1 else 0
        down += blocks * (q + rem)
    return up + down


def run_poly(args, cfg):
    """Polynomial operations of Sec. 6.1 (Table 1) on a fixed synthetic batch of columns:
    the product (nb_polymul) or the conversion round trip (nb_to_monomial then
    nb_from_monomial)."""
    import numpy as np
    import torch

    import oracle
    from paper_1404_3458_amd import rs, synth

    r, h, nc = cfg["r"], cfg["h"], cfg["cols"]
    sb = r // 8
    rb = nc * sb
    torch.cuda.set_device(0)
    codec = rs.Codec(r)
    stream = torch.cuda.current_stream()
    a = torch.empty((h, rb), dtype=torch.uint8, device="cuda")
    synth.fill_random_torch(synth.key(cfg["id"], 1, synth.DATA), a)
    mul = cfg["poly"] == "mul"
    if mul:
        b = torch.empty_like(a)
        synth.fill_random_torch(synth.key(cfg["id"], 2, synth.DATA), b)
        out = torch.empty((2 * h, rb), dtype=torch.uint8, device="cuda")

        def step():
            codec.polymul(h, 0, a, b, out)
    else:
        x = a.clone()

        def step():
            codec.to_monomial(h, x)
            codec.from_monomial(h, x)
    cols = [0, 1, nc // 3, nc - 1] if mul else [0, nc - 1]
    if not args.no_check:
        pick = lambda t: np.ascontiguousarray(
            t.cpu().numpy().reshape(t.shape[0], nc, sb)[:, cols, :].reshape(t.shape[0], len(cols) * sb))
        if mul:
            step()
            torch.cuda.synchronize()
            assert (pick(out) == oracle.polymul_rows(r, pick(a), pick(b), 0)).all(), "product differs from the oracle"
        else:
            codec.to_monomial(h, x)
            torch.cuda.synchronize()
            assert (pick(x) == oracle.convert_rows(r, pick(a), True)).all(), "monomial form differs from the oracle"
            codec.from_monomial(h, x)
            torch.cuda.synchronize()
            assert torch.equal(x, a), "conversion round trip"
    for _ in range(args.warmup):
        step()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1 in evs:
        e0.record(stream)
        step()
        e1.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / args.steps
    ms = np.array([e0.elapsed_time(e1) for e0, e1 in evs])
    t = float(ms.mean()) * 1e-3
    H = 2 * h
    if mul:
        per_col = 3 * ((H // 2) * (H.bit_length() - 1) - (H - 1)) + H      # Sec. 3.4 counts at shift 0
        nbytes = 2 * h * rb                                                 # operand coefficients
        algo_bytes = 2 * h * rb + H * rb
    else:
        per_col = conv_mults_per_column(h)
        nbytes = 2 * h * rb                                                 # two conversions of h rows
        algo_bytes = 4 * h * rb
    mults = per_col * nc
    cpu = None
    if not args.no_cpu:
        threads = min(16, len(os.sched_getaffinity(0)))
        sc = 256 if mul else 4
        sample = np.ascontiguousarray(a[:, :sc * sb].cpu().numpy())
        sample2 = np.ascontiguousarray(b[:, :sc * sb].cpu().numpy()) if mul else None
        t1 = time.perf_counter()
        if mul:
            import concurrent.futures as cf

            per = max(1, sc // threads)
            parts = [(c0, min(sc, c0 + per)) for c0 in range(0, sc, per)]
            with cf.ThreadPoolExecutor(max_workers=threads) as ex:
                list(ex.map(lambda p: oracle.polymul_rows(r, np.ascontiguousarray(sample[:, p[0] * sb:p[1] * sb]),
                                                          np.ascontiguousarray(sample2[:, p[0] * sb:p[1] * sb]), 0),
                            parts))
            used = threads
        else:
            m = oracle.convert_rows(r, sample.copy(), True)
            oracle.convert_rows(r, m, False)
            used = 1
        dt = time.perf_counter() - t1
        cpu = {"value": round(2 * h * sc * sb / dt / 1e9, 6), "unit": "GB/s", "cores": used, "kind": "oracle",
               "sample": "%d columns of the same operands (%s), %.2f s wall" %
                         (sc, "product by the oracle's transforms" if mul else
                          "the oracle's O(h^2) conversion both ways", dt)}
        cpu["ratio_gpu_over_cpu"] = round(nbytes / t / 1e9 / cpu["value"], 1)
    out = {
        "metric": "polynomial %s GB/s of operand coefficients" % ("product" if mul else "basis conversion"),
        "value": round(nbytes / t / 1e9, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(float(ms.mean()), 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u16" if r == 16 else "u8",
        "data": "synthetic (seeded splitmix64 bytes)",
        "config": {"workload": cfg["workload"], "field_bits": r, "h": h, "columns": nc,
                   "parallelism": "single GPU"},
        "roofline": hbm_roofline("whole call (all launches)", algo_bytes, t, None, copy_gbps(),
                                 alu_figures(mults, t, r)),
        "cpu_baseline": cpu,
        "detail": {"step_ms_p50": round(float(np.percentile(ms, 50)), 4),
                   "step_ms_p99": round(float(np.percentile(ms, 99)), 4), "wall_ms_per_step": round(wall, 4),
                   "mults_per_column": per_col},
    }
    print(json.dumps(out))
    codec.close()


def run_mixed(args, cfg):
    """The mixed-stripe workload: every stripe encoded and then decoded in
    place per step, as one encode plan and one decode plan per (n, k) class
    replayed in one HIP graph, the classes in order of size (each class's
    encode, then its decode, so that a stripe of a small class completes
    early); also timed as one encode and one decode plan over all stripes, as
    batched calls and as per-stripe calls, overall and per class."""
    import numpy as np
    import torch

    from paper_1404_3458_amd import rs, synth

    ns = args.stripes or cfg["stripes"]
    shapes = synth.mixed_stripes(cfg["id"], ns)
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    offs, total = [], 0
    for n, k, sb, e in shapes:
        offs.append(total)
        total += (n * sb + 255) // 256 * 256
    buf = torch.empty(total, dtype=torch.uint8, device=dev)
    cws = [buf[offs[s]:offs[s] + n * sb].view(n, sb) for s, (n, k, sb, e) in enumerate(shapes)]
    for s, (n, k, sb, e) in enumerate(shapes):
        synth.fill_random_torch(synth.key(cfg["id"], s, synth.DATA), cws[s][:k])
    masks = [synth.erasure_mask(synth.key(cfg["id"], s, synth.ERASURE), n, e) for s, (n, k, sb, e) in
             enumerate(shapes)]
    codec = rs.Codec(16)
    sched = schedule_for(args, codec, shapes)
    stream = torch.cuda.current_stream()
    enc_list = [(n, k, cws[s][:k], cws[s][k:]) for s, (n, k, sb, e) in enumerate(shapes)]
    dec_list = [(n, k, masks[s], cws[s], cws[s]) for s, (n, k, sb, e) in enumerate(shapes)]
    enc_b, dec_b = codec.prepare_encode_batch(enc_list), codec.prepare_decode_batch(dec_list)
    msg_bytes = sum(k * sb for n, k, sb, e in shapes)
    cw_bytes = sum(n * sb for n, k, sb, e in shapes)

    codec.encode_batch(enc_b)
    torch.cuda.synchronize()
    if not args.no_check:
        # recovery of zeroed erasures on a sample of stripes of every class,
        # and parity against the oracle on sampled columns of one per class
        import oracle

        sample = []
        for c in synth.MIXED_CLASSES:
            sample += [s for s, sh in enumerate(shapes) if sh[:2] == c][:3]
        ref = {s: cws[s].clone() for s in sample}
        for s, (n, k, sb, e) in enumerate(shapes):
            if e:
                cws[s][torch.from_numpy(masks[s]).bool().to(dev)] = 0
        codec.decode_batch(dec_b)
        torch.cuda.synchronize()
        for s in sample:
            assert torch.equal(cws[s], ref[s]), ("decode did not restore stripe", s, shapes[s])
        for c in synth.MIXED_CLASSES:
            s = next(t for t, sh in enumerate(shapes) if sh[:2] == c)
            n, k, sb, e = shapes[s]
            cols = list(range(0, sb // 2, max(1, sb // 2 // 8)))[:8]
            host = cws[s].cpu().numpy().reshape(n, sb // 2, 2)[:, cols, :].reshape(n, len(cols) * 2)
            assert (oracle.encode(16, n, k, np.ascontiguousarray(host[:k])) == host[k:]).all(), ("parity", c)
        del ref

    def timed(fn, reps):
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for a, b in evs:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / reps
        return wall, np.array([a.elapsed_time(b) for a, b in evs])

    def graph_of(plans):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for p_ in plans:
                p_.launch()
        return g

    classes = [c for c in synth.MIXED_CLASSES if any(sh[:2] == c for sh in shapes)]
    cidx = {c: [s for s, sh in enumerate(shapes) if sh[:2] == c] for c in classes}
    cplans = {c: (codec.plan_encode_batch([enc_list[s] for s in cidx[c]]),
                  codec.plan_decode_batch([dec_list[s] for s in cidx[c]])) for c in classes}
    # the measured configuration: per-class plans, smallest class first
    g = graph_of([p_ for c in classes for p_ in cplans[c]])
    for _ in range(args.warmup):
        g.replay()
    wall_g, ev_g = timed(g.replay, args.steps)
    # the same work as one encode and one decode plan over all stripes
    pe, pd = codec.plan_encode_batch(enc_b), codec.plan_decode_batch(dec_b)
    g1 = graph_of([pe, pd])
    g1.replay()
    wall_g1, ev_g1 = timed(g1.replay, max(2, args.steps // 2))
    del g1
    # per-stripe completion within a step, from device stamps written as the
    # last workgroup on each stripe finishes (eager launches of the same
    # per-class plans in the same order; the graph was captured without
    # stamps), relative to the start of the first launch: a stripe is done
    # when its decode is, or its encode when its decode has no work (no
    # erasures)
    stamps = {c: (torch.zeros(len(cidx[c]) + 1, dtype=torch.int64, device=dev),
                  torch.zeros(len(cidx[c]) + 1, dtype=torch.int64, device=dev)) for c in classes}
    khz = None
    for c in classes:
        khz = cplans[c][0].set_timestamps(stamps[c][0])
        cplans[c][1].set_timestamps(stamps[c][1])
    done = []
    for _ in range(3):
        for c in classes:
            cplans[c][0].launch()
            cplans[c][1].launch()
        torch.cuda.synchronize()
        t0 = int(stamps[classes[0]][0][0].item())
        fin = np.zeros(ns)
        for c in classes:
            te, td = stamps[c][0].cpu().numpy(), stamps[c][1].cpu().numpy()
            fin[cidx[c]] = np.where(td[1:] > 0, td[1:], te[1:])
        done.append((fin - t0) / khz)
    for c in classes:
        cplans[c][0].set_timestamps(None)
        cplans[c][1].set_timestamps(None)
    done = np.stack(done)
    # batched calls (planned on every call)
    for _ in range(max(1, args.warmup // 2)):
        codec.encode_batch(enc_b)
        codec.decode_batch(dec_b)
    wall_b, ev_b = timed(lambda: (codec.encode_batch(enc_b), codec.decode_batch(dec_b)), max(2, args.steps // 2))

    def per_stripe(idx):
        for s in idx:
            n, k, sb, e = shapes[s]
            codec.encode(n, k, cws[s][:k], cws[s][k:])
        for s in idx:
            n, k, sb, e = shapes[s]
            codec.decode(n, k, masks[s], cws[s])

    per_class = {}
    wall_ps_total = 0.0
    for c in classes:
        idx = cidx[c]
        cb = sum(shapes[s][1] * shapes[s][2] for s in idx)
        gc = graph_of(list(cplans[c]))
        gc.replay()
        wall_c, _ = timed(gc.replay, 3)
        per_stripe(idx)
        wall_p, _ = timed(lambda: per_stripe(idx), 1)
        wall_ps_total += wall_p
        per_class["%d,%d" % c] = {"stripes": len(idx), "msg_GB": round(cb / 1e9, 3),
                                  "done_ms_p50": round(float(np.percentile(done[:, idx], 50)), 3),
                                  "done_ms_p99": round(float(np.percentile(done[:, idx], 99)), 3),
                                  "graph_ms": round(wall_c, 3), "per_stripe_ms": round(wall_p, 3),
                                  "graph_msg_GBps": round(cb / wall_c / 1e6, 1),
                                  "per_stripe_msg_GBps": round(cb / wall_p / 1e6, 1),
                                  "factor": round(wall_p / wall_c, 2)}
        del gc
    value = msg_bytes / (wall_g * 1e-3) / 1e9
    hbm = 2 * cw_bytes / (wall_g * 1e-3) / 1e9        # encode n*S + decode n*S per stripe
    mults = sum(sb // 2 * (paper_mults_per_column(n, k, False) + paper_mults_per_column(n, k, True))
                for n, k, sb, e in shapes)
    out = {
        "metric": "RS encode/decode GB/s of message data (% HBM peak); batched vs per-stripe; p99",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall_g, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16",
        "data": "synthetic (seeded splitmix64 bytes, shapes and erasure subsets)",
        "config": {"workload": cfg["workload"], "field_bits": 16, "stripes": ns,
                   "message_GB": round(msg_bytes / 1e9, 2), "codeword_GB": round(cw_bytes / 1e9, 2),
                   "parallelism": "single GPU"},
        "roofline": hbm_roofline("whole step (encode and decode plans of every class, in order)", 2 * cw_bytes,
                                 wall_g * 1e-3, None, None, alu_figures(mults, wall_g * 1e-3, 16)),
        "cpu_baseline": None,
        "detail": {
            "graph_step_ms_p50": round(float(np.percentile(ev_g, 50)), 3),
            "graph_step_ms_p99": round(float(np.percentile(ev_g, 99)), 3),
            "stripe_done_ms_p50": round(float(np.percentile(done, 50)), 3),
            "stripe_done_ms_p99": round(float(np.percentile(done, 99)), 3),
            "stripe_done_ms_max": round(float(done.max()), 3),
            "one_plan_graph_step_ms": round(wall_g1, 3),
            "one_plan_graph_step_ms_p99": round(float(np.percentile(ev_g1, 99)), 3),
            "batched_call_step_ms": round(wall_b, 3),
            "batched_call_step_ms_p99": round(float(np.percentile(ev_b, 99)), 3),
            "per_stripe_step_ms": round(wall_ps_total, 3),
            "graph_over_per_stripe": round(wall_ps_total / wall_g, 2),
            "batched_calls_over_per_stripe": round(wall_ps_total / wall_b, 2),
            "per_class": per_class,
            "schedule": sched,
        },
    }
    pe.close()
    pd.close()
    for c in classes:
        cplans[c][0].close()
        cplans[c][1].close()
    codec.close()
    return out


def mixed_summary(out):
    """The figures of a mixed-workload line that the default line carries."""
    d = out["detail"]
    return {"workload": out["config"]["workload"], "steps": out["steps"], "msg_GBps": out["value"],
            "ms_per_step": out["ms_per_step"], "hbm_frac": out["roofline"]["frac"],
            "one_plan_graph_step_ms": d["one_plan_graph_step_ms"],
            "batched_graph_over_per_stripe": d["graph_over_per_stripe"],
            "batched_calls_over_per_stripe": d["batched_calls_over_per_stripe"],
            "per_stripe_step_ms": d["per_stripe_step_ms"],
            "stripe_done_ms_p50": d["stripe_done_ms_p50"], "stripe_done_ms_p99": d["stripe_done_ms_p99"],
            "per_class": {c: {key: v[key] for key in ("stripes", "factor", "done_ms_p50", "done_ms_p99",
                                                      "graph_msg_GBps")}
                          for c, v in d["per_class"].items()}}


def run_serving(args, cfg):
    """Continuous-batching server under Poisson arrivals: first the saturated
    rate mu (all requests queued at once), then lambda = 0.5, 0.7 and 0.9 mu.
    Latency is completion (event observed by the server) minus the request's
    scheduled arrival time."""
    import numpy as np
    import torch

    from paper_1404_3458_amd import rs, synth

    pool_n = args.stripes or cfg["stripes"]
    shapes = synth.mixed_stripes(cfg["id"], pool_n)
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    offs, total = [], 0
    for n, k, sb, e in shapes:
        offs.append(total)
        total += (n * sb + 255) // 256 * 256
    buf = torch.empty(total, dtype=torch.uint8, device=dev)
    cws = [buf[offs[s]:offs[s] + n * sb].view(n, sb) for s, (n, k, sb, e) in enumerate(shapes)]
    for s, (n, k, sb, e) in enumerate(shapes):
        synth.fill_random_torch(synth.key(cfg["id"], s, synth.DATA), cws[s][:k])
    masks = [synth.erasure_mask(synth.key(cfg["id"], s, synth.ERASURE), n, e) for s, (n, k, sb, e) in
             enumerate(shapes)]
    codec = rs.Codec(16)
    sched = schedule_for(args, codec, shapes)
    codec.encode_batch([(n, k, cws[s][:k], cws[s][k:]) for s, (n, k, sb, e) in enumerate(shapes)])
    torch.cuda.synchronize()
    srv = rs.Server(codec, cfg["budget"], max_batch=512, nstreams=3)
    share = cfg["encode_share"]

    def op_of(i):
        return rs.RS_OP_ENCODE if synth.uniform_float(synth.key(cfg["id"], i, 77), 1)[0] < share else rs.RS_OP_DECODE

    ops_cache = {}

    def submit(i, tag):
        s = i % pool_n
        n, k, sb, e = shapes[s]
        op = ops_cache.setdefault(i, op_of(i))
        # the payloads were written and synchronized before serving began, so
        # requests need not wait for a producer stream (after=False)
        if op == rs.RS_OP_ENCODE:
            srv.submit(op, n, k, cws[s][:k], cws[s][k:], tag=tag, after=False)
        else:
            srv.submit(op, n, k, cws[s], cws[s], mask=masks[s], tag=tag, after=False)
        return k * sb

    def run(first, count, arrivals_ns):
        """Submit requests first..first+count-1 at t0 + arrivals_ns[j]; return
        (latencies ns, message bytes, span ns)."""
        done = {}
        msg = 0
        t0 = time.monotonic_ns() + 2_000_000
        for j in range(count):
            target = t0 + int(arrivals_ns[j])
            while time.monotonic_ns() < target:
                for tag, st, t in srv.poll(0):
                    done[tag] = (st, t)
            msg += submit(first + j, j)
            for tag, st, t in srv.poll(0):
                done[tag] = (st, t)
        while len(done) < count:
            for tag, st, t in srv.poll(1000):
                done[tag] = (st, t)
        assert all(st == rs.RS_OK for st, _ in done.values())
        lat = np.array([done[j][1] - (t0 + int(arrivals_ns[j])) for j in range(count)], dtype=np.float64)
        span = max(t for _, t in done.values()) - (t0 + int(arrivals_ns[0]))
        return lat, msg, span

    # saturated rate: everything queued at once
    nsat = min(3000, 3 * pool_n)
    run(0, 200, np.zeros(200))
    lat, msg, span = run(200, nsat, np.zeros(nsat))
    mu = nsat / (span * 1e-9)
    sat = {"requests": nsat, "req_per_s": round(mu, 1), "msg_GBps": round(msg / span, 2),
           "p50_ms": round(float(np.percentile(lat, 50)) / 1e6, 3),
           "p99_ms": round(float(np.percentile(lat, 99)) / 1e6, 3)}
    loads = {}
    first = 200 + nsat
    nreq, warm = cfg["requests"], cfg["warm"]
    for frac in (0.5, 0.7, 0.9):
        lam = frac * mu
        gaps = -np.log(1.0 - synth.uniform_float(synth.key(cfg["id"], int(frac * 10), synth.ARRIVAL), warm + nreq))
        arr = np.cumsum(gaps / lam) * 1e9
        arr -= arr[0]
        lat, msg, span = run(first, warm + nreq, arr)
        first += warm + nreq
        lm = lat[warm:]
        msg_meas = sum(shapes[(first - nreq + j) % pool_n][1] * shapes[(first - nreq + j) % pool_n][2]
                       for j in range(nreq))
        span_meas = (arr[-1] - arr[warm]) * 1e-9
        loads["%.1f" % frac] = {"lambda_req_per_s": round(lam, 1), "requests": nreq,
                                "p50_ms": round(float(np.percentile(lm, 50)) / 1e6, 3),
                                "p99_ms": round(float(np.percentile(lm, 99)) / 1e6, 3),
                                "msg_GBps": round(msg_meas / max(span_meas, 1e-9) / 1e9, 2)}
    srv.close()
    out = {
        "metric": "RS encode/decode GB/s of message data (% HBM peak); batched vs per-stripe; p99",
        "value": sat["msg_GBps"],
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": nsat,
        "warmup": 200,
        "ms_per_step": round(1e3 / mu, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16",
        "data": "synthetic (seeded splitmix64 bytes, shapes, erasures and arrivals)",
        "config": {"workload": cfg["workload"], "field_bits": 16, "resident_stripes": pool_n,
                   "budget_GB": cfg["budget"] / 1e9, "streams": 3, "max_batch": 512,
                   "parallelism": "single GPU"},
        "roofline": None,
        "cpu_baseline": None,
        "detail": {"saturated": sat, "poisson": loads, "schedule": sched,
                   "note": "step = one request at the saturated rate; latency = completion - scheduled arrival"},
    }
    print(json.dumps(out))
    codec.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c2", choices=sorted(CONFIGS))
    ap.add_argument("--cpu-stripes", type=int, default=2)
    ap.add_argument("--cpu-cols", type=int, default=32768)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-per-stripe", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-mixed", action="store_true",
                    help="default workload: skip the mixed-workload block of the detail")
    ap.add_argument("--stripes", type=int, default=0, help="mixed workload: stripe count (default 8192)")
    ap.add_argument("--schedule", default="", help="mixed workloads: schedule table (JSON) instead of autotuning")
    ap.add_argument("--no-tune", action="store_true", help="mixed workloads: default schedules")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy --steps times (the reference "
                         "kernel that scales the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (no collectives or sharding); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1404_3458_amd import rs, synth

    if args.copy_calibration:
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1)
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": 1 << 30, "launches": args.steps}))
        return

    cfg = dict(CONFIGS[args.config])
    cfg["id"] = {"c1": 1, "c2": 2, "c3": 3, "c4": 4, "c5": 5, "poly": 6, "conv": 7}[args.config]
    if cfg.get("poly"):
        return run_poly(args, cfg)
    if cfg.get("mixed"):
        print(json.dumps(run_mixed(args, cfg)))
        return
    if cfg.get("serving"):
        return run_serving(args, cfg)
    r, n, k, S, ns, e = cfg["r"], cfg["n"], cfg["k"], cfg["shard_bytes"], cfg["stripes"], cfg["erasures"]
    sets = cfg.get("sets", 1)
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    codec = rs.Codec(r)
    stream = torch.cuda.current_stream()
    # codes over more than 256 points run pass pipelines: tune their splits
    kp_ = pow2ceil(k)
    sched = schedule_for(args, codec, [(n, k, S, e)], target_bytes=ns * n * S) \
        if r == 16 and pow2ceil(kp_ + n - k) > 256 else None

    # Codeword buffers: stripe s rows 0..k-1 are its message, k..n-1 its
    # parity.  A workload smaller than the last-level cache keeps `sets`
    # copies (same erasure patterns, distinct data) and step i uses copy
    # i mod sets, so every step reads data that has left the cache.
    cws = torch.empty((sets, ns, n, S), dtype=torch.uint8, device=dev)
    for j in range(sets):
        for s in range(ns):
            synth.fill_random_torch(synth.key(cfg["id"], s, synth.DATA, *((j,) if j else ())), cws[j, s, :k])
    cw = cws[0]
    masks = [synth.erasure_mask(synth.key(cfg["id"], s, synth.ERASURE), n, e) for s in range(ns)]
    enc_sets = [codec.prepare_encode_batch([(n, k, cws[j, s, :k], cws[j, s, k:]) for s in range(ns)])
                for j in range(sets)]
    dec_sets = [codec.prepare_decode_batch([(n, k, masks[s], cws[j, s], cws[j, s]) for s in range(ns)])
                for j in range(sets)]
    enc_items, dec_items = enc_sets[0], dec_sets[0]
    for j in range(1, sets):
        codec.encode_batch(enc_sets[j])

    # Parity check on a column sample before timing (the oracle, one column
    # block of two stripes), and recovery of explicitly zeroed erasures.
    if not args.no_check:
        import oracle

        codec.encode_batch(enc_items)
        torch.cuda.synchronize()
        ref = cw.clone()
        for s in range(ns):
            cw[s][torch.from_numpy(masks[s]).bool().to(dev)] = 0
        codec.decode_batch(dec_items)
        torch.cuda.synchronize()
        assert torch.equal(cw, ref), "decode did not restore the codeword"
        sym = r // 8
        for s in sorted({0, ns - 1}):
            cols = sorted({0, 1, 2, 3, S // sym - 1, S // sym - 4} | set(
                int(c) for c in synth.uniform_int(synth.key(cfg["id"], s, 77), 24, 0, S // sym - 1)))
            cols = [c for c in cols if 0 <= c < S // sym]
            host = cw[s].cpu().numpy().reshape(n, S // sym, sym)[:, cols, :].reshape(n, len(cols) * sym)
            par = oracle.encode(r, n, k, np.ascontiguousarray(host[:k]))
            assert (par == host[k:]).all(), "parity differs from the oracle on sampled columns"
        del ref

    for i in range(args.warmup):
        codec.encode_batch(enc_sets[i % sets])
        codec.decode_batch(dec_sets[i % sets])
    torch.cuda.synchronize()

    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    host_ms = np.zeros((args.steps, 2))
    t0 = time.perf_counter()
    for i in range(args.steps):
        j = (args.warmup + i) % sets
        ev[i][0].record(stream)
        h0 = time.perf_counter()
        codec.encode_batch(enc_sets[j])
        h1 = time.perf_counter()
        ev[i][1].record(stream)
        codec.decode_batch(dec_sets[j])
        h2 = time.perf_counter()
        ev[i][2].record(stream)
        host_ms[i] = ((h1 - h0) * 1e3, (h2 - h1) * 1e3)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    enc_ms = np.array([ev[i][0].elapsed_time(ev[i][1]) for i in range(args.steps)])
    dec_ms = np.array([ev[i][1].elapsed_time(ev[i][2]) for i in range(args.steps)])
    step_ms = enc_ms + dec_ms
    ms_per_step = wall * 1e3 / args.steps

    msg_bytes = ns * k * S
    algo_bytes = ns * n * S               # per encode launch and per decode launch
    value = msg_bytes / (ms_per_step * 1e-3) / 1e9
    enc_gbs = msg_bytes / (enc_ms.mean() * 1e-3) / 1e9
    dec_gbs = msg_bytes / (dec_ms.mean() * 1e-3) / 1e9
    # The dominant launch (larger median) is the roofline kernel; its
    # achieved rate uses the mean event-timed duration over the timed steps.
    dom = "decode" if np.median(dec_ms) >= np.median(enc_ms) else "encode"
    dom_ms = float((dec_ms if dom == "decode" else enc_ms).mean())
    cols = S // (r // 8)
    mults = ns * cols * paper_mults_per_column(n, k, dom == "decode")
    lg = int(np.log2(pow2ceil(k) if dom == "encode" else pow2ceil(pow2ceil(k) + n - k)))
    copy_rate = copy_gbps()
    # GF(2^16) decodes of 128 or 256 points over 8-byte-aligned rows run the
    # persistent decode kernel when there are more tiles than workgroup slots
    # (one per CU for 256 points, two for 128, on 256 CUs)
    slots = 256 if lg == 8 else 512
    persist = dom == "decode" and r == 16 and lg in (7, 8) and S % 8 == 0 and ns * -(-cols // 256) > slots
    kname = "k_dec_persist" if persist else ("k_tiled" if 4 < lg <= 8 else ("k_small" if lg <= 4 else "multi-pass"))
    roof = hbm_roofline("%s launch (%s, L=%d)" % (dom, kname, lg),
                        algo_bytes, dom_ms * 1e-3, traffic_from_profiles(args.config), copy_rate,
                        alu_figures(mults, dom_ms * 1e-3, r))

    extra = {
        "encode_ms": round(float(enc_ms.mean()), 4), "decode_ms": round(float(dec_ms.mean()), 4),
        "encode_msg_GBps": round(enc_gbs, 1), "decode_msg_GBps": round(dec_gbs, 1),
        "encode_hbm_frac": round(algo_bytes / (enc_ms.mean() * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "decode_hbm_frac": round(algo_bytes / (dec_ms.mean() * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "step_ms_p50": round(float(np.percentile(step_ms, 50)), 4),
        "step_ms_p99": round(float(np.percentile(step_ms, 99)), 4),
        "step_ms_max": round(float(step_ms.max()), 4),
        "slowest_step": int(step_ms.argmax()),
        "host_call_ms_max": [round(float(host_ms[:, 0].max()), 3), round(float(host_ms[:, 1].max()), 3)],
        "host_call_ms_p50": [round(float(np.median(host_ms[:, 0])), 3), round(float(np.median(host_ms[:, 1])), 3)],
        "msg_over_hbm_peak": round(value / HBM_PEAK_GBS, 4),
    }
    if sched is not None:
        extra["schedule"] = sched

    # The same step as two reusable plans replayed in a HIP graph: what a
    # caller that repeats a batch pays once its host planning is done (with
    # several buffer sets, one graph runs the step on every set in turn).
    plans = [(codec.plan_encode_batch(enc_sets[j]), codec.plan_decode_batch(dec_sets[j])) for j in range(sets)]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for pe, pd in plans:
            pe.launch()
            pd.launch()
    for _ in range(max(1, args.warmup // sets)):
        g.replay()
    greps = max(2, args.steps // sets)
    gev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(greps)]
    torch.cuda.synchronize()
    for e0, e1 in gev:
        e0.record(stream)
        g.replay()
        e1.record(stream)
    torch.cuda.synchronize()
    gms = np.array([e0.elapsed_time(e1) for e0, e1 in gev]) / sets
    extra["graph_ms_per_step_p50"] = round(float(np.percentile(gms, 50)), 4)
    extra["graph_ms_per_step_p99"] = round(float(np.percentile(gms, 99)), 4)
    extra["graph_msg_GBps"] = round(msg_bytes / (float(gms.mean()) * 1e-3) / 1e9, 2)
    del g
    for pe, pd in plans:
        pe.close()
        pd.close()

    if not args.no_per_stripe and ns > 1:
        # the same work as per-stripe launches (one call per stripe and direction)
        reps = max(2, args.steps // 4)
        for s in range(ns):
            codec.encode(n, k, cw[s, :k], cw[s, k:])
            codec.decode(n, k, masks[s], cw[s])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(reps):
            for s in range(ns):
                codec.encode(n, k, cw[s, :k], cw[s, k:])
            for s in range(ns):
                codec.decode(n, k, masks[s], cw[s])
        torch.cuda.synchronize()
        ps_ms = (time.perf_counter() - t1) * 1e3 / reps
        extra["per_stripe_ms_per_step"] = round(ps_ms, 3)
        extra["batched_over_per_stripe"] = round(ps_ms / ms_per_step, 3)

    if args.config == "c2" and not args.no_mixed:
        # the batched-vs-per-stripe figures of the 8192-stripe mixed workload
        # (its own line with --config c4): measured after this workload's
        # buffers are released
        del cws, cw, enc_sets, dec_sets, enc_items, dec_items
        torch.cuda.empty_cache()
        margs = argparse.Namespace(**vars(args))
        margs.steps, margs.warmup, margs.stripes = 3, 1, 0
        mcfg = dict(CONFIGS["c4"])
        mcfg["id"] = 4
        extra["mixed"] = mixed_summary(run_mixed(margs, mcfg))

    cpu = None
    if not args.no_cpu:
        threads = min(16, len(os.sched_getaffinity(0)))
        cpu = cpu_baseline(cfg, min(args.cpu_stripes, ns), args.cpu_cols, threads)
        cpu["ratio_gpu_over_cpu"] = round(value / cpu["value"], 1)

    out = {
        "metric": "RS encode/decode GB/s of message data (% HBM peak); batched vs per-stripe; p99",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16" if r == 16 else "u8",
        "data": "synthetic (seeded splitmix64 bytes, uniform erasure subsets)",
        "config": {"workload": cfg["workload"], "field_bits": r, "n": n, "k": k, "stripes": ns,
                   "shard_bytes": S, "erasures_per_stripe": e, "buffer_sets": sets, "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "detail": extra,
    }
    print(json.dumps(out))
    codec.close()


if __name__ == "__main__":
    main()
