"""Write the expected full-size results of two measured workloads as SHA-256
digests, computed by the CPU oracle alone (Algorithm 1 for the parity rows,
Algorithm 2 with the appendix's locator for the decoded codeword) on the
seeded inputs the GPU tests and the benchmark generate:

  * the 64 stripes of the (256, 128) GF(2^16) workload with 64 KiB shards
    and 128 erasures each: every stripe;
  * a seeded 1 % (82 stripes) of the 8192-stripe mixed workload: every
    column of each picked stripe.

Output: ``fullsize.json`` beside this script.  Each entry holds the digest of
the oracle's n - k parity rows (row-major bytes) and of the n rows the
oracle's decoder returns for the codeword with the erased rows zeroed.  The
script calls nothing but ``oracle`` and the seeded generators; run it from
the repository root with ``python3 tests/golden/make_fullsize.py`` (about
70 CPU-minutes, about 9 minutes on 8 cores).
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1404_3458_amd import synth  # noqa: E402

C2 = dict(cfg=2, n=256, k=128, stripes=64, shard_bytes=65536, erasures=128)
C4_STRIPES = 8192
C4_SUBSET = 82            # 1 % of the mixed batch
C4_SUBSET_KEY = (4, 92)   # synth key of the subset draw
ABOUT = ("SHA-256 digests of the oracle's results (Algorithm 1 parity rows, Algorithm 2 decoded rows) on the seeded "
         "full-size inputs: every stripe of the (256, 128) x 64 KiB workload and a seeded 1 % of the mixed "
         "workload; written by make_fullsize.py, which calls only the oracle and the seeded generators")


def c4_subset():
    """The picked stripes of the mixed workload: the first 82 distinct values
    of a seeded uniform draw over the stripe indices."""
    v = synth.uniform_int(synth.key(*C4_SUBSET_KEY), 1000, 0, C4_STRIPES - 1)
    pick = []
    for x in v:
        if int(x) not in pick:
            pick.append(int(x))
        if len(pick) == C4_SUBSET:
            break
    return sorted(pick)


def _blocks(ncols, parts):
    per = max(1, -(-ncols // parts))
    return [(c0, min(ncols, c0 + per)) for c0 in range(0, ncols, per)]


def oracle_stripe(ex, n, k, msg, mask):
    """Oracle parity and decoded codeword of one GF(2^16) stripe, columns
    split over the pool (every column is an independent codeword)."""
    ncols = msg.shape[1] // 2
    blocks = _blocks(ncols, 4 * (os.cpu_count() or 1))
    par = np.zeros((n - k, msg.shape[1]), dtype=np.uint8)

    def enc(b):
        c0, c1 = b
        par[:, 2 * c0:2 * c1] = oracle.encode(16, n, k, np.ascontiguousarray(msg[:, 2 * c0:2 * c1]))

    list(ex.map(enc, blocks))
    rx = np.concatenate([msg, par])
    rx[mask == 1] = 0
    out = np.zeros_like(rx)

    def dec(b):
        c0, c1 = b
        out[:, 2 * c0:2 * c1] = oracle.decode(16, n, k, mask, np.ascontiguousarray(rx[:, 2 * c0:2 * c1]))

    list(ex.map(dec, blocks))
    return par, out


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def main():
    oracle.build()
    res = {"about": ABOUT, "c2": [], "c4": []}
    t0 = time.time()
    with cf.ThreadPoolExecutor(max_workers=os.cpu_count() or 1) as ex:
        n, k, S = C2["n"], C2["k"], C2["shard_bytes"]
        for s in range(C2["stripes"]):
            msg = synth.random_bytes(synth.key(C2["cfg"], s, synth.DATA), k * S).reshape(k, S)
            mask = synth.erasure_mask(synth.key(C2["cfg"], s, synth.ERASURE), n, C2["erasures"])
            par, out = oracle_stripe(ex, n, k, msg, mask)
            res["c2"].append({"stripe": s, "parity_sha256": digest(par), "decoded_sha256": digest(out)})
            print("c2 stripe %d  %.0f s" % (s, time.time() - t0), flush=True)
        shapes = synth.mixed_stripes(4, C4_STRIPES)
        for s in c4_subset():
            n, k, sb, e = shapes[s]
            msg = synth.random_bytes(synth.key(4, s, synth.DATA), k * sb).reshape(k, sb)
            mask = synth.erasure_mask(synth.key(4, s, synth.ERASURE), n, e)
            par, out = oracle_stripe(ex, n, k, msg, mask)
            res["c4"].append({"stripe": s, "n": n, "k": k, "shard_bytes": sb, "erasures": e,
                              "parity_sha256": digest(par), "decoded_sha256": digest(out)})
            print("c4 stripe %d (%d, %d) x %d B  %.0f s" % (s, n, k, sb, time.time() - t0), flush=True)
    with open(os.path.join(HERE, "fullsize.json"), "w") as f:
        json.dump(res, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
