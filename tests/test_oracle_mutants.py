"""The pins reject broken oracles: each mutant below plants one plausible
mistake (a dropped term, a wrong operand, a wrong level or index, a missing
normalisation) in a copy of oracle/nb_oracle.c, built on the CPU; the pin
battery (tests/pin_battery.py) must pass on the real oracle and fail on every
mutant.  Each mutant runs in its own process with NB_ORACLE_LIB pointing at
its build."""
import json
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "nb_oracle.c")

# (name, text in nb_oracle.c, replacement)
MUTANTS = [
    ("field polynomial (not primitive)", "return r == 8 ? 0x11Du", "return r == 8 ? 0x11Bu"),
    ("reduction misses the last step", "for (int t = 2 * r - 2; t >= r; t--)", "for (int t = 2 * r - 2; t > r; t--)"),
    ("factor not normalised (W for W-hat)",
     "f[off + c / step] = orc_What(r, basis, i, orc_omega(r, basis, (uint32_t)c) ^ wl);",
     "f[off + c / step] = orc_W(r, basis, i, orc_omega(r, basis, (uint32_t)c) ^ wl);"),
    ("factor of the wrong block",
     "f[off + c / step] = orc_What(r, basis, i, orc_omega(r, basis, (uint32_t)c) ^ wl);",
     "f[off + c / step] = orc_What(r, basis, i, orc_omega(r, basis, (uint32_t)c + 1u) ^ wl);"),
    ("forward butterfly adds the old a",
     "b ^= a;                                  /* eq. Deltajimcoplusloplusi2 */",
     "b ^= x[c + m];"),
    ("inverse butterfly drops b += a",
     "b ^= a;                                  /* eq. Deltaj22imiomegacomegal */",
     ";"),
    ("derivative drops the l = 0 partner",
     "            if (!((j >> l) & 1))\n                acc ^= dd[j + (1 << l)];",
     "            if (!((j >> l) & 1) && l > 0)\n                acc ^= dd[j + (1 << l)];"),
    ("derivative scales by B instead of 1/B",
     "out[j] = orc_mul(r, acc, orc_inv(r, B[j]));", "out[j] = orc_mul(r, acc, B[j]);"),
    ("locator without the 1/N normalisation",
     "uint64_t ninv = ((uint64_t)1 << (r - ilog2(N))) % M;", "uint64_t ninv = 1;"),
    ("product without the zero padding of b",
     "memcpy(tb, b, sizeof(uint32_t) * (size_t)h);", "memcpy(tb, b, sizeof(uint32_t) * (size_t)h); tb[h] = b[0];"),
    ("product transformed back forward", "    ifft_core(r, basis, H, l, f, out, NULL);\n    free(f); free(tb);",
     "    fft_core(r, basis, H, l, f, out, NULL);\n    free(f); free(tb);"),
    ("conversion divides by the wrong leading coefficient",
     "d[j] = orc_mul(r, work[j], orc_inv(r, xj[j]));", "d[j] = orc_mul(r, work[j], orc_inv(r, xj[0] ? xj[0] : 1));"),
    ("decode divides by Pi' squared",
     "cst[p] = orc_inv(r, cst[p]);              /* divisor of step 6 */",
     "cst[p] = orc_inv(r, orc_mul(r, cst[p], cst[p]));"),
]


def _battery(env):
    """Names of the failing checks; a process that crashes (a broken oracle
    may index its tables out of range) counts as every check failing."""
    code = "import sys, json; sys.path.insert(0, %r); sys.path.insert(0, %r); import pin_battery; " \
           "print(json.dumps(pin_battery.run()))" % (HERE, ROOT)
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
    if out.returncode != 0:
        return ["process exited with %d" % out.returncode]
    return json.loads(out.stdout.strip().splitlines()[-1])


def test_battery_passes_on_the_oracle():
    env = dict(os.environ)
    env.pop("NB_ORACLE_LIB", None)
    assert _battery(env) == []


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_battery_rejects_mutant(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, "anchor not found once: %r" % old
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fvisibility=hidden", "-o", str(lib),
                    str(path)], check=True)
    env = dict(os.environ)
    env["NB_ORACLE_LIB"] = str(lib)
    fails = _battery(env)
    assert fails, "no pin caught the mutant: " + name
