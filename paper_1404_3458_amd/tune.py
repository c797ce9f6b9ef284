"""Autotuner of the pass-pipeline schedules (rs_schedule_set in include/rs.h).

A code whose transforms exceed 256 points runs each transform over 2^N
points as 2 to 4 parts of consecutive levels, each applied by passes over
groups of rows that differ only in that part's index bits (the low part:
groups of consecutive rows); every split into parts of 4..8 levels computes
the same result (level i only pairs rows j and j + 2^i, Sec. 3.2), but the
kernels of different group sizes use the device differently (workgroup
size, LDS per workgroup, resident workgroups per CU, arithmetic per byte
moved), and more parts mean more passes over the rows.  For every
(operation, N) class of a workload the tuner times each candidate split on
a seeded synthetic batch of that class through a reusable plan and keeps
the fastest, then times that split with the other column tiles
(rs_schedule_set_tile: 256-column tiles, or packed 128-column tiles in
which each wave's halves hold two sets of rows) and keeps the fastest
tile.  The result is a versioned JSON table that apply() or load() puts
into a context.
"""
from __future__ import annotations

import json
import math
import time

from . import rs, synth

VERSION = 3
FUSED_MAX_L = 8
TILES = (0, 128, 256)      # rs_schedule_set_tile: default, packed everywhere, 256-column only
_OPS = {"enc": rs.RS_OP_ENCODE, "dec": rs.RS_OP_DECODE}


def pow2ceil(v: int) -> int:
    return 1 << max(0, (v - 1).bit_length())


def mother(n: int, k: int):
    """(n', k') of the shortened code (the layout of include/rs.h)."""
    kp = pow2ceil(k)
    return pow2ceil(kp + n - k), kp


def candidates(N: int):
    """Candidate splits (level counts, low part first) of a transform over
    2^N points: every two-part split, the three-part splits with at most 6
    levels per part, and four parts of 4 levels."""
    out = [(t, N - t) for t in range(4, 9) if 4 <= N - t <= 8]
    out += [(a, b, N - a - b) for a in range(4, 7) for b in range(4, 7) if 4 <= N - a - b <= 6]
    if N == 16:
        out.append((4, 4, 4, 4))
    return out


def default_split(N: int):
    return ((N + 1) // 2, N // 2)


def split_name(parts):
    return "/".join(str(p) for p in parts)


def classes(shapes):
    """{("enc"|"dec", N): [(n, k), ...]} for the (n, k) shapes whose
    transforms run as pass pipelines (GF(2^16), more than 256 points)."""
    out = {}
    for n, k in sorted(set(shapes)):
        np_, kp = mother(n, k)
        for op, size in (("enc", kp), ("dec", np_)):
            N = int(math.log2(size))
            if N > FUSED_MAX_L:
                out.setdefault((op, N), []).append((n, k))
    return out


def _time_plan(plan, stream, warmup, reps):
    import torch

    for _ in range(warmup):
        plan.launch(stream)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in evs:
        a.record(stream)
        plan.launch(stream)
        b.record(stream)
    torch.cuda.synchronize()
    ts = sorted(a.elapsed_time(b) for a, b in evs)
    return ts[len(ts) // 2]


def tune(codec, shapes, row_bytes=(1024, 4096, 16384, 65536), target_bytes=256 << 20, warmup=2, reps=5,
         seed_id=0x7E, log=None):
    """Time every split of every pass-pipeline class of `shapes` ((n, k)
    pairs) on a synthetic batch of about target_bytes of codeword per class
    (stripes of each shape, row lengths cycling through row_bytes), set the
    fastest in `codec` and return the table."""
    import torch

    stream = torch.cuda.current_stream()
    table = {"version": VERSION, "device": torch.cuda.get_device_name(), "field_bits": codec.r,
             "row_bytes": list(row_bytes), "target_bytes": int(target_bytes), "entries": []}
    for (op, N), shp in sorted(classes(shapes).items(), key=lambda kv: (kv[0][1], kv[0][0])):
        # one batch of the class: stripes of each shape in turn
        stripes, total, s = [], 0, 0
        while total < target_bytes or not stripes:
            n, k = shp[s % len(shp)]
            sb = row_bytes[s % len(row_bytes)]
            stripes.append((n, k, sb, s))
            total += n * sb
            s += 1
        bufs = []
        for n, k, sb, i in stripes:
            cw = torch.empty((n, sb), dtype=torch.uint8, device="cuda")
            synth.fill_random_torch(synth.key(seed_id, N, i, synth.DATA), cw[:k])
            bufs.append(cw)
        enc = codec.prepare_encode_batch([(n, k, bufs[j][:k], bufs[j][k:]) for j, (n, k, sb, i) in enumerate(stripes)])
        codec.encode_batch(enc)
        if op == "dec":
            masks = [synth.erasure_mask(synth.key(seed_id, N, i, synth.ERASURE), n, (n - k + 1) // 2)
                     for n, k, sb, i in stripes]
            batch = codec.prepare_decode_batch([(n, k, masks[j], bufs[j], bufs[j])
                                                for j, (n, k, sb, i) in enumerate(stripes)])
        else:
            batch = enc
        torch.cuda.synchronize()
        def timed():
            plan = codec.plan_decode_batch(batch) if op == "dec" else codec.plan_encode_batch(batch)
            t = _time_plan(plan, stream, warmup, reps)
            plan.close()
            return t

        ms = {}
        codec.set_schedule_tile(_OPS[op], N, 0)
        for parts in candidates(N):
            codec.set_schedule(_OPS[op], N, parts)
            ms[parts] = timed()
        best = min(ms, key=lambda t: (ms[t], len(t), t))
        codec.set_schedule(_OPS[op], N, best)
        tms = {0: ms[best]}
        for cols in TILES[1:]:
            codec.set_schedule_tile(_OPS[op], N, cols)
            tms[cols] = timed()
        tile = min(tms, key=lambda c: (tms[c], c))
        codec.set_schedule_tile(_OPS[op], N, tile)
        entry = {"op": op, "N": N, "parts": list(best), "tile": tile, "default": list(default_split(N)),
                 "shapes": [list(x) for x in shp], "stripes": len(stripes), "codeword_bytes": total,
                 "ms": {split_name(t): round(v, 4) for t, v in sorted(ms.items())},
                 "tile_ms": {str(c): round(v, 4) for c, v in sorted(tms.items())}}
        table["entries"].append(entry)
        if log:
            log(entry)
        del bufs, enc, batch
    return table


def apply(codec, table):
    """Set every entry of a table in `codec` (tables of version 2 have no
    column tiles: those stay at the default)."""
    if table.get("version") not in (2, VERSION):
        raise ValueError("schedule table version %r, expected %d" % (table.get("version"), VERSION))
    for e in table["entries"]:
        codec.set_schedule(_OPS[e["op"]], int(e["N"]), tuple(int(p) for p in e["parts"]))
        codec.set_schedule_tile(_OPS[e["op"]], int(e["N"]), int(e.get("tile", 0)))


def save(table, path):
    with open(path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)


def load(path, codec=None):
    with open(path) as f:
        table = json.load(f)
    if codec is not None:
        apply(codec, table)
    return table


def summary(table):
    """{"dec:12": "4/4/4", "enc:15": "7/8 t128", ...} of a table, for
    reports (a non-default column tile after the split)."""
    return {"%s:%d" % (e["op"], e["N"]): split_name(e["parts"]) + (" t%d" % e["tile"] if e.get("tile") else "")
            for e in table["entries"]}


if __name__ == "__main__":
    import argparse

    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", required=True, help="JSON file to write")
    ap.add_argument("--shapes", default="256,224;1024,512;4096,2048",
                    help="(n,k) pairs separated by ';'")
    ap.add_argument("--target-mib", type=int, default=256)
    a = ap.parse_args()
    shp = [tuple(int(v) for v in p.split(",")) for p in a.shapes.split(";") if p]
    t0 = time.perf_counter()
    c = rs.Codec(16)
    tab = tune(c, shp, target_bytes=a.target_mib << 20, log=lambda e: print(json.dumps(e), flush=True))
    save(tab, a.out)
    print("tuned %d classes in %.1f s -> %s" % (len(tab["entries"]), time.perf_counter() - t0, a.out))
