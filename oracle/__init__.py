"""CPU oracle for the novel-basis transform and the Reed-Solomon erasure codec.

TEST INFRASTRUCTURE ONLY: this package may be imported by ``tests/``, by
``__graft_entry__.smoke()`` and by the CPU-baseline leg of ``bench.py``, and by
nothing else.  It wraps ``nb_oracle.c`` (plain C, bitwise carry-less field
multiplication) through ctypes and shares no code with the GPU library.

Every function mirrors a C entry point of ``nb_oracle.c``; the comments there
cite the section, equation or algorithm of Lin-Chung-Han (arXiv:1404.3458)
each one follows.  Arrays are numpy arrays; stripes are ``uint8`` arrays of
shape ``(rows, row_bytes)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nb_oracle.c")
_LIB = os.path.join(_HERE, "libnb_oracle.so")
_lock = threading.Lock()
_lib = None
# Test infrastructure: a prebuilt variant of the library to load instead
# (used to check that the pins reject deliberately broken oracles).
_LIB_OVERRIDE = os.environ.get("NB_ORACLE_LIB")

ERR_TOOMANY = -2


def build(force: bool = False) -> str:
    """Compile nb_oracle.c into libnb_oracle.so with gcc (plain -O2)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fvisibility=hidden",
               "-Wall", "-Wextra", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if _LIB_OVERRIDE:
                lib = ctypes.CDLL(_LIB_OVERRIDE)
            else:
                build()
                lib = ctypes.CDLL(_LIB)
            u32, i32, sz = ctypes.c_uint32, ctypes.c_int, ctypes.c_size_t
            p = ctypes.c_void_p
            sig = {
                "orc_field_poly": (u32, [i32]),
                "orc_mul": (u32, [i32, u32, u32]),
                "orc_pow": (u32, [i32, u32, ctypes.c_uint64]),
                "orc_inv": (u32, [i32, u32]),
                "orc_omega": (u32, [i32, p, u32]),
                "orc_W": (u32, [i32, p, i32, u32]),
                "orc_What": (u32, [i32, p, i32, u32]),
                "orc_X": (u32, [i32, p, u32, u32]),
                "orc_poly_eval": (u32, [i32, i32, p, u32]),
                "orc_W_monomial": (i32, [i32, p, i32, p]),
                "orc_X_monomial": (i32, [i32, p, u32, p]),
                "orc_to_monomial": (i32, [i32, p, i32, p, p]),
                "orc_monomial_derivative": (i32, [i32, i32, p, p]),
                "orc_eval_naive": (i32, [i32, p, i32, u32, p, p]),
                "orc_fft_vec": (i32, [i32, p, i32, u32, p, p]),
                "orc_ifft_vec": (i32, [i32, p, i32, u32, p, p]),
                "orc_factors": (i32, [i32, p, i32, u32, p]),
                "orc_Wprime_norm": (u32, [i32, p, i32]),
                "orc_deriv_direct_vec": (i32, [i32, p, i32, p, p]),
                "orc_deriv_B_vec": (i32, [i32, p, i32, p, p]),
                "orc_B_table": (i32, [i32, p, i32, p]),
                "orc_fft_rows": (i32, [i32, p, i32, u32, p, sz, sz]),
                "orc_ifft_rows": (i32, [i32, p, i32, u32, p, sz, sz]),
                "orc_deriv_rows": (i32, [i32, p, i32, p, sz, sz]),
                "orc_mother_shape": (i32, [i32, i32, i32, p, p]),
                "orc_encode": (i32, [i32, p, i32, i32, p, p, sz, sz]),
                "orc_encode_lagrange": (i32, [i32, p, i32, i32, p, p, sz, sz]),
                "orc_fwht_mod": (i32, [i32, i32, p]),
                "orc_locator_fwht": (i32, [i32, p, i32, p, p]),
                "orc_locator_direct": (i32, [i32, p, i32, p, p]),
                "orc_decode": (i32, [i32, p, i32, i32, p, p, p, sz, sz, i32]),
                "orc_decode_lagrange": (i32, [i32, p, i32, i32, p, p, p, sz, sz]),
                "orc_poly_mul": (i32, [i32, i32, p, i32, p, p]),
                "orc_from_monomial": (i32, [i32, p, i32, p, p]),
                "orc_degree": (i32, [i32, p]),
                "orc_polymul_fft": (i32, [i32, p, i32, u32, p, p, p]),
                "orc_polymul_rows": (i32, [i32, p, i32, u32, p, p, p, sz, sz]),
                "orc_degree_rows": (i32, [i32, i32, p, sz, sz, p]),
                "orc_convert_rows": (i32, [i32, p, i32, i32, p, sz, sz]),
            }
            for name, (res, args) in sig.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _basis(basis):
    if basis is None:
        return None
    return np.ascontiguousarray(np.asarray(basis, dtype=np.uint32))


def _u32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint32))


def _check(rc, what):
    if rc != 0:
        raise ValueError("%s failed (%d)" % (what, rc))


# ---------------------------------------------------------------- field
def field_poly(r):
    return _load().orc_field_poly(r)


def mul(r, a, b):
    return _load().orc_mul(r, a, b)


def pow_(r, a, e):
    return _load().orc_pow(r, a, e)


def inv(r, a):
    return _load().orc_inv(r, a)


def omega(r, i, basis=None):
    b = _basis(basis)
    return _load().orc_omega(r, _ptr(b), i)


# ---------------------------------------------------------------- basis
def W(r, j, x, basis=None):
    b = _basis(basis)
    return _load().orc_W(r, _ptr(b), j, x)


def W_hat(r, j, x, basis=None):
    b = _basis(basis)
    return _load().orc_What(r, _ptr(b), j, x)


def X(r, i, x, basis=None):
    b = _basis(basis)
    return _load().orc_X(r, _ptr(b), i, x)


def poly_eval(r, coef, x):
    c = _u32(coef)
    return _load().orc_poly_eval(r, len(c), _ptr(c), x)


def W_monomial(r, j, basis=None):
    b = _basis(basis)
    out = np.zeros((1 << j) + 1, dtype=np.uint32)
    _check(_load().orc_W_monomial(r, _ptr(b), j, _ptr(out)), "W_monomial")
    return out


def X_monomial(r, i, basis=None):
    b = _basis(basis)
    out = np.zeros(i + 1, dtype=np.uint32)
    _check(_load().orc_X_monomial(r, _ptr(b), i, _ptr(out)), "X_monomial")
    return out


def to_monomial(r, d, basis=None):
    b = _basis(basis)
    d = _u32(d)
    out = np.zeros(len(d), dtype=np.uint32)
    _check(_load().orc_to_monomial(r, _ptr(b), len(d), _ptr(d), _ptr(out)), "to_monomial")
    return out


def monomial_derivative(r, mono):
    m = _u32(mono)
    out = np.zeros(len(m), dtype=np.uint32)
    _check(_load().orc_monomial_derivative(r, len(m), _ptr(m), _ptr(out)), "monomial_derivative")
    return out


# ---------------------------------------------------------------- transforms
def eval_naive(r, d, l=0, basis=None):
    b = _basis(basis)
    d = _u32(d)
    out = np.zeros(len(d), dtype=np.uint32)
    _check(_load().orc_eval_naive(r, _ptr(b), len(d), l, _ptr(d), _ptr(out)), "eval_naive")
    return out


def fft(r, d, l=0, basis=None, counts=None):
    """Algorithmic forward transform of one vector; counts -> [adds, mults]."""
    b = _basis(basis)
    x = _u32(d).copy()
    cnt = np.zeros(2, dtype=np.int64)
    _check(_load().orc_fft_vec(r, _ptr(b), len(x), l, _ptr(x), _ptr(cnt)), "fft")
    if counts is not None:
        counts[:] = cnt
    return x


def ifft(r, d, l=0, basis=None, counts=None):
    b = _basis(basis)
    x = _u32(d).copy()
    cnt = np.zeros(2, dtype=np.int64)
    _check(_load().orc_ifft_vec(r, _ptr(b), len(x), l, _ptr(x), _ptr(cnt)), "ifft")
    if counts is not None:
        counts[:] = cnt
    return x


def factors(r, h, l=0, basis=None):
    b = _basis(basis)
    out = np.zeros(max(h - 1, 1), dtype=np.uint32)
    _check(_load().orc_factors(r, _ptr(b), h, l, _ptr(out)), "factors")
    return out[: h - 1]


def Wprime_norm(r, l, basis=None):
    b = _basis(basis)
    return _load().orc_Wprime_norm(r, _ptr(b), l)


def deriv_direct(r, d, basis=None):
    b = _basis(basis)
    d = _u32(d)
    out = np.zeros(len(d), dtype=np.uint32)
    _check(_load().orc_deriv_direct_vec(r, _ptr(b), len(d), _ptr(d), _ptr(out)), "deriv_direct")
    return out


def deriv_B(r, d, basis=None):
    b = _basis(basis)
    d = _u32(d)
    out = np.zeros(len(d), dtype=np.uint32)
    _check(_load().orc_deriv_B_vec(r, _ptr(b), len(d), _ptr(d), _ptr(out)), "deriv_B")
    return out


def B_table(r, h, basis=None):
    b = _basis(basis)
    out = np.zeros(h, dtype=np.uint32)
    _check(_load().orc_B_table(r, _ptr(b), h, _ptr(out)), "B_table")
    return out


# ---------------------------------------------------------------- stripes
def _rows(a):
    assert a.dtype == np.uint8 and a.ndim == 2 and a.flags["C_CONTIGUOUS"]
    return a


def fft_rows(r, data, l=0, basis=None, ncols=None):
    """In-place transform of every column of ``data`` (h rows x row_bytes)."""
    b = _basis(basis)
    d = _rows(data)
    nc = d.shape[1] // (r // 8) if ncols is None else ncols
    _check(_load().orc_fft_rows(r, _ptr(b), d.shape[0], l, _ptr(d), d.strides[0], nc), "fft_rows")
    return d


def ifft_rows(r, data, l=0, basis=None, ncols=None):
    b = _basis(basis)
    d = _rows(data)
    nc = d.shape[1] // (r // 8) if ncols is None else ncols
    _check(_load().orc_ifft_rows(r, _ptr(b), d.shape[0], l, _ptr(d), d.strides[0], nc), "ifft_rows")
    return d


def deriv_rows(r, data, basis=None):
    b = _basis(basis)
    d = _rows(data)
    nc = d.shape[1] // (r // 8)
    _check(_load().orc_deriv_rows(r, _ptr(b), d.shape[0], _ptr(d), d.strides[0], nc), "deriv_rows")
    return d


def mother_shape(r, n, k):
    kp, np_ = ctypes.c_int(), ctypes.c_int()
    rc = _load().orc_mother_shape(r, n, k, ctypes.byref(kp), ctypes.byref(np_))
    _check(rc, "mother_shape")
    return kp.value, np_.value


def encode(r, n, k, msg, basis=None, lagrange=False):
    """Parity rows (n-k, row_bytes) of the systematic codeword (Algorithm 1)."""
    b = _basis(basis)
    m = _rows(msg)
    assert m.shape[0] == k
    par = np.zeros((n - k, m.shape[1]), dtype=np.uint8)
    fn = _load().orc_encode_lagrange if lagrange else _load().orc_encode
    _check(fn(r, _ptr(b), n, k, _ptr(m), _ptr(par), m.strides[0], m.shape[1] // (r // 8)), "encode")
    return par


def encode_into(r, n, k, msg, parity, basis=None):
    """Column-range friendly encode: msg/parity may be column slices of larger
    row-major arrays (rows keep their stride)."""
    b = _basis(basis)
    assert msg.dtype == np.uint8 and parity.dtype == np.uint8
    assert msg.strides[1] == 1 and parity.strides[0] == msg.strides[0]
    rc = _load().orc_encode(r, _ptr(b), n, k, msg.ctypes.data_as(ctypes.c_void_p),
                            parity.ctypes.data_as(ctypes.c_void_p), msg.strides[0],
                            msg.shape[1] // (r // 8))
    _check(rc, "encode")


def decode(r, n, k, mask, shards, basis=None, locator="fwht", lagrange=False):
    """All n rows of the codeword from ``shards`` (erased rows ignored)."""
    b = _basis(basis)
    s = _rows(shards)
    mk = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
    assert s.shape[0] == n and mk.shape == (n,)
    out = np.zeros_like(s)
    if lagrange:
        rc = _load().orc_decode_lagrange(r, _ptr(b), n, k, _ptr(mk), _ptr(s), _ptr(out),
                                         s.strides[0], s.shape[1] // (r // 8))
    else:
        rc = _load().orc_decode(r, _ptr(b), n, k, _ptr(mk), _ptr(s), _ptr(out), s.strides[0],
                                s.shape[1] // (r // 8), 0 if locator == "fwht" else 1)
    if rc == ERR_TOOMANY:
        raise ValueError("too many erasures")
    _check(rc, "decode")
    return out


def decode_into(r, n, k, mask, shards, out, basis=None):
    b = _basis(basis)
    mk = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
    assert shards.strides[1] == 1 and out.strides[0] == shards.strides[0]
    rc = _load().orc_decode(r, _ptr(b), n, k, _ptr(mk), shards.ctypes.data_as(ctypes.c_void_p),
                            out.ctypes.data_as(ctypes.c_void_p), shards.strides[0],
                            shards.shape[1] // (r // 8), 0)
    _check(rc, "decode")


# ---------------------------------------------------------------- locator
def fwht_mod(r, v):
    x = _u32(v).copy()
    _check(_load().orc_fwht_mod(r, len(x), _ptr(x)), "fwht_mod")
    return x


def locator_log_fwht(r, erased, basis=None):
    b = _basis(basis)
    e = np.ascontiguousarray(np.asarray(erased, dtype=np.uint8))
    out = np.zeros(len(e), dtype=np.uint32)
    _check(_load().orc_locator_fwht(r, _ptr(b), len(e), _ptr(e), _ptr(out)), "locator_fwht")
    return out


def locator_direct(r, erased, basis=None):
    b = _basis(basis)
    e = np.ascontiguousarray(np.asarray(erased, dtype=np.uint8))
    out = np.zeros(len(e), dtype=np.uint32)
    _check(_load().orc_locator_direct(r, _ptr(b), len(e), _ptr(e), _ptr(out)), "locator_direct")
    return out


# ---------------------------------------------------------------- polynomial operations (Sec. 6.1, Table 1)
def poly_mul(r, a, b):
    """Monomial-basis product (schoolbook)."""
    a, b = _u32(a), _u32(b)
    out = np.zeros(len(a) + len(b) - 1, dtype=np.uint32)
    _check(_load().orc_poly_mul(r, len(a), _ptr(a), len(b), _ptr(b), _ptr(out)), "poly_mul")
    return out


def from_monomial(r, mono, basis=None):
    """Novel-basis coefficients of a polynomial given in the monomial basis."""
    b = _basis(basis)
    m = _u32(mono)
    out = np.zeros(len(m), dtype=np.uint32)
    _check(_load().orc_from_monomial(r, _ptr(b), len(m), _ptr(m), _ptr(out)), "from_monomial")
    return out


def degree(d):
    d = _u32(d)
    return _load().orc_degree(len(d), _ptr(d))


def polymul(r, a, b, l=0, basis=None):
    """Sec. 6.1 (Table 1) product of two novel-basis polynomials of h coefficients: 2h coefficients."""
    bs = _basis(basis)
    a, b = _u32(a), _u32(b)
    assert len(a) == len(b)
    out = np.zeros(2 * len(a), dtype=np.uint32)
    _check(_load().orc_polymul_fft(r, _ptr(bs), len(a), l, _ptr(a), _ptr(b), _ptr(out)), "polymul")
    return out


def polymul_rows(r, a, b, l=0, basis=None, ncols=None):
    """Column-wise polymul of row-major stripes a, b (h rows): 2h rows."""
    bs = _basis(basis)
    a, b = _rows(a), _rows(b)
    assert a.shape == b.shape
    out = np.zeros((2 * a.shape[0], a.shape[1]), dtype=np.uint8)
    nc = a.shape[1] // (r // 8) if ncols is None else ncols
    _check(_load().orc_polymul_rows(r, _ptr(bs), a.shape[0], l, _ptr(a), _ptr(b), _ptr(out), a.strides[0], nc),
           "polymul_rows")
    return out


def degree_rows(r, data, ncols=None):
    d = _rows(data)
    nc = d.shape[1] // (r // 8) if ncols is None else ncols
    out = np.zeros(nc, dtype=np.int32)
    _check(_load().orc_degree_rows(r, d.shape[0], _ptr(d), d.strides[0], nc, _ptr(out)), "degree_rows")
    return out


def convert_rows(r, data, to_monomial, basis=None, ncols=None):
    """In place, column by column: novel -> monomial basis (to_monomial) or back."""
    bs = _basis(basis)
    d = _rows(data)
    nc = d.shape[1] // (r // 8) if ncols is None else ncols
    _check(_load().orc_convert_rows(r, _ptr(bs), d.shape[0], 1 if to_monomial else 0, _ptr(d), d.strides[0], nc),
           "convert_rows")
    return d
