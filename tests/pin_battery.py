"""A compact battery of the oracle's pins (definitions, closed forms,
invariants, brute force), run as one function so that the same checks can be
pointed at deliberately broken builds of the oracle (test_oracle_mutants.py).
Returns the names of the checks that fail."""
import itertools

import numpy as np

import oracle
from paper_1404_3458_amd import synth


def _syms(r, n, *parts):
    return synth.uniform_int(synth.key(90, r, n, *parts), n, 0, (1 << r) - 1).astype(np.uint32)


def _check(fails, name, fn):
    try:
        if not fn():
            fails.append(name)
    except Exception:                      # a crash or a rejected call is a failed pin too
        fails.append(name)


def run():
    fails = []
    primes = {8: (3, 5, 17), 16: (3, 5, 17, 257)}

    def alpha_order():
        for r in (8, 16):
            m = (1 << r) - 1
            if oracle.pow_(r, 2, m) != 1:
                return False
            if any(oracle.pow_(r, 2, m // q) == 1 for q in primes[r]):
                return False
        return True

    def inverse_and_distributive():
        for r in (8, 16):
            a, b, c = (_syms(r, 64, t) for t in range(3))
            for x, y, z in zip(a, b, c):
                x, y, z = int(x), int(y), int(z)
                if x and oracle.mul(r, x, oracle.inv(r, x)) != 1:
                    return False
                if oracle.mul(r, x, y ^ z) != oracle.mul(r, x, y) ^ oracle.mul(r, x, z):
                    return False
        return True

    def transform_equals_naive():
        for r, hs in ((8, (2, 4, 16, 64)), (16, (8, 32))):
            for h in hs:
                for l in {0, h, 5 % (1 << r)}:
                    d = _syms(r, h, l)
                    if not (oracle.fft(r, d, l) == oracle.eval_naive(r, d, l)).all():
                        return False
        return True

    def round_trip():
        for r, h, l in ((8, 64, 3), (16, 128, 256), (16, 16, 0)):
            d = _syms(r, h, 7)
            if not (oracle.ifft(r, oracle.fft(r, d, l), l) == d).all():
                return False
            if not (oracle.fft(r, oracle.ifft(r, d, l), l) == d).all():
                return False
        return True

    def op_counts():
        for r, h in ((8, 32), (16, 64)):
            lg = h.bit_length() - 1
            for l, zero in ((0, h - 1), (h, 0)):
                c = np.zeros(2, dtype=np.int64)
                oracle.fft(r, _syms(r, h, 8), l, counts=c)
                if list(c) != [h * lg - zero, h // 2 * lg - zero]:
                    return False
        return True

    def derivative_three_ways():
        for r, h in ((8, 32), (16, 16)):
            d = _syms(r, h, 9)
            a, b = oracle.deriv_direct(r, d), oracle.deriv_B(r, d)
            if not (a == b).all():
                return False
            lhs = oracle.to_monomial(r, b)
            rhs = oracle.monomial_derivative(r, oracle.to_monomial(r, d))
            if not (lhs == rhs).all():
                return False
        return True

    def encode_equals_lagrange():
        for r, n, k, cols in ((8, 16, 8, 3), (8, 12, 5, 2), (16, 8, 4, 2), (8, 40, 9, 1)):
            sym = r // 8
            msg = synth.random_bytes(synth.key(91, r, n, k), k * cols * sym).reshape(k, cols * sym)
            if not (oracle.encode(r, n, k, msg) == oracle.encode(r, n, k, msg, lagrange=True)).all():
                return False
        return True

    def decode_every_pattern():
        r, n, k = 8, 8, 4
        msg = synth.random_bytes(synth.key(92), k * 2).reshape(k, 2)
        cw = np.concatenate([msg, oracle.encode(r, n, k, msg)])
        for er in itertools.combinations(range(n), n - k):
            mask = np.zeros(n, np.uint8)
            mask[list(er)] = 1
            rx = cw.copy()
            rx[mask == 1] = 0
            if not (oracle.decode(r, n, k, mask, rx) == cw).all():
                return False
        return True

    def decode_shortened():
        for r, n, k in ((8, 12, 5), (16, 20, 7)):
            sym = r // 8
            msg = synth.random_bytes(synth.key(93, r, n), k * 3 * sym).reshape(k, 3 * sym)
            cw = np.concatenate([msg, oracle.encode(r, n, k, msg)])
            mask = synth.erasure_mask(synth.key(94, r, n), n, n - k)
            rx = cw.copy()
            rx[mask == 1] = 0
            if not (oracle.decode(r, n, k, mask, rx) == cw).all():
                return False
        return True

    def locator_fwht_equals_direct():
        for r, N in ((8, 16), (8, 64), (16, 32)):
            er = (synth.uniform_float(synth.key(95, r, N), N) < 0.4).astype(np.uint8)
            lg = oracle.locator_log_fwht(r, er)
            direct = oracle.locator_direct(r, er)
            if not all(oracle.pow_(r, 2, int(lg[j])) == int(direct[j]) for j in range(N)):
                return False
        return True

    def polymul_is_the_product():
        # values at 2h points of another coset, by naive evaluation of the basis
        for r, h, l in ((8, 8, 3), (16, 16, 100)):
            a, b = _syms(r, h, 1), _syms(r, h, 2)
            c = oracle.polymul(r, a, b, l)
            z = np.zeros(h, dtype=np.uint32)
            shift = (1 << r) - 2 * h
            va = oracle.eval_naive(r, np.concatenate([a, z]), shift)
            vb = oracle.eval_naive(r, np.concatenate([b, z]), shift)
            vc = oracle.eval_naive(r, c, shift)
            if not all(int(vc[j]) == oracle.mul(r, int(va[j]), int(vb[j])) for j in range(2 * h)):
                return False
        return True

    def conversion_and_degree():
        for r, h in ((8, 32), (16, 16)):
            d = _syms(r, h, 3)
            d[h - 3:] = 0
            m = oracle.to_monomial(r, d)
            if not (oracle.from_monomial(r, m) == d).all():
                return False
            if oracle.degree(d) != int(np.nonzero(m)[0][-1]):
                return False
            e = np.zeros(h, dtype=np.uint32)
            e[h - 1] = 1
            x = np.zeros(h, dtype=np.uint32)
            x[:h] = oracle.X_monomial(r, h - 1)
            if not (oracle.from_monomial(r, x) == e).all():
                return False
        return True

    for name, fn in (("alpha_order", alpha_order), ("inverse_and_distributive", inverse_and_distributive),
                     ("transform_equals_naive", transform_equals_naive), ("round_trip", round_trip),
                     ("op_counts", op_counts), ("derivative_three_ways", derivative_three_ways),
                     ("encode_equals_lagrange", encode_equals_lagrange),
                     ("decode_every_pattern", decode_every_pattern), ("decode_shortened", decode_shortened),
                     ("locator_fwht_equals_direct", locator_fwht_equals_direct),
                     ("polymul_is_the_product", polymul_is_the_product),
                     ("conversion_and_degree", conversion_and_degree)):
        _check(fails, name, fn)
    return fails
