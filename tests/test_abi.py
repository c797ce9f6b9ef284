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
