"""The C-ABI library loads on a machine without a GPU and exports every
function that include/rs.h declares (no compute call is made here)."""
import ctypes
import os

from paper_1404_3458_amd import build, rs


def _lib_path():
    if not os.path.exists(rs.LIB_PATH):
        build.build()
    return rs.LIB_PATH


def test_header_declares_the_boundary():
    names = rs.header_functions()
    for fn in ("rs_init", "rs_free", "rs_encode", "rs_decode", "nb_fft", "nb_ifft", "nb_derivative",
               "rs_encode_batch", "rs_decode_batch", "rs_sync", "rs_get_table", "rs_strerror"):
        assert fn in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib_path())
    for name in rs.header_functions():
        assert hasattr(lib, name), name


def test_strerror_without_device():
    rs.load()
    assert rs.strerror(rs.RS_ETOOMANY) == "more erasures than parity symbols"
    assert rs.strerror(12345) == "unknown error"


def test_library_does_not_link_the_oracle():
    import subprocess

    out = subprocess.run(["nm", "-D", _lib_path()], capture_output=True, text=True).stdout
    assert "orc_" not in out


def test_plan_timestamps_argument_checks():
    # the binding refuses a timestamp array the device could write past
    # (host memory, too short, wrong type) before any library call
    import pytest
    import torch

    pl = rs.Plan(None, ctypes.c_void_p(), 3)
    for bad in (torch.zeros(4, dtype=torch.int64), torch.zeros(4, dtype=torch.int32), [0, 0, 0, 0]):
        with pytest.raises(ValueError):
            pl.set_timestamps(bad)


def _run(code):
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    return subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=120)


def test_missing_library_fails_loudly():
    # no fallback: without the HIP library every codec entry point raises
    out = _run("from paper_1404_3458_amd import rs\n"
               "rs.LIB_PATH = '/nonexistent/librs_nb.so'\n"
               "try:\n"
               "    rs.Codec(16)\n"
               "except RuntimeError as e:\n"
               "    print('raised:', e)\n")
    assert out.returncode == 0, out.stderr
    assert "raised: librs_nb.so is not built" in out.stdout


def test_package_does_not_import_the_oracle():
    out = _run("import sys\n"
               "import paper_1404_3458_amd\n"
               "from paper_1404_3458_amd import rs, synth, tune, build\n"
               "print(sorted(m for m in sys.modules if m == 'oracle' or m.startswith('oracle.')))\n")
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "[]"
