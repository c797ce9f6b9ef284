"""ctypes binding of librs_nb.so (the C ABI of include/rs.h).

Argument marshalling only: every step of the codec runs in the HIP library.
Device buffers are torch tensors (uint8, CUDA/HIP device, C-contiguous) or
raw integer device addresses; streams default to torch's current stream.
The library is loaded from the package directory; if it has not been built
the first call raises, and nothing falls back to another implementation.
"""
from __future__ import annotations

import ctypes
import os
import re
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librs_nb.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "rs.h")

RS_OK, RS_EINVAL, RS_EFIELD, RS_EBASIS, RS_ESHAPE, RS_ETOOMANY, RS_EALIGN, RS_ENOMEM, RS_EDEVICE = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
RS_TAB_SKEW, RS_TAB_B, RS_TAB_BINV, RS_TAB_LOG, RS_TAB_EXP = range(5)

_lib = None


class RSError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__("%s: %s (%d)" % (what, strerror(code) if _lib else "error", code))


class StripeDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("k", ctypes.c_int32), ("row_bytes", ctypes.c_uint64),
                ("in_", ctypes.c_void_p), ("out", ctypes.c_void_p)]


class PreparedBatch:
    """Descriptor array (and concatenated masks) of a batch call, kept alive
    together with the pointers handed to the library."""

    def __init__(self, arr, masks, count):
        self.arr = arr
        self.masks = masks
        self.count = count
        self.desc_ptr = ctypes.cast(arr, ctypes.c_void_p)
        self.mask_ptr = masks.ctypes.data_as(ctypes.c_void_p) if masks is not None else None


class Plan:
    """An rs_plan: launch() queues the planned batch on a stream (capturable
    in a HIP graph); close() frees it."""

    def __init__(self, codec, handle, count):
        self._codec = codec          # keeps the context alive
        self._h = handle
        self.count = count           # stripes of the batch

    def launch(self, stream=None):
        return _check(load().rs_plan_launch(self._h, _stream(stream)), "rs_plan_launch")

    def set_timestamps(self, ts=None):
        """Stamp completion times into ts (int64 device tensor of count + 1,
        None stops); returns the counter's rate in kHz."""
        if ts is not None:
            import torch

            if not isinstance(ts, torch.Tensor) or not ts.is_cuda or ts.dtype not in (torch.int64, torch.uint64) \
                    or not ts.is_contiguous() or ts.numel() < self.count + 1:
                raise ValueError("timestamps: a contiguous int64 device tensor of at least %d elements"
                                 % (self.count + 1))
        khz = ctypes.c_int()
        _check(load().rs_plan_set_timestamps(self._h, _ptr(ts), ctypes.byref(khz)), "rs_plan_set_timestamps")
        self._ts = ts
        return khz.value

    def close(self):
        if self._h:
            load().rs_plan_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


RS_OP_ENCODE, RS_OP_DECODE = 0, 1


class Request(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("desc", StripeDesc), ("mask", ctypes.c_void_p), ("tag", ctypes.c_uint64),
                ("after", ctypes.c_void_p)]


class ServerStats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_uint64) for name in (
        "budget", "inflight_bytes", "peak_bytes", "peak_shared_bytes", "oversize_admitted", "largest_oversize",
        "admitted", "batches", "retried")]


class Completion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32), ("t_done_ns", ctypes.c_int64)]


class Server:
    """An rs_server: continuous batching of encode/decode requests with FIFO
    admission by a device-memory budget, over `nstreams` streams.
    Completion times are time.monotonic_ns() values."""

    def __init__(self, codec, budget_bytes, max_batch=256, nstreams=2):
        self._codec = codec
        self._h = ctypes.c_void_p()
        _check(load().rs_server_create(codec._ctx, int(budget_bytes), max_batch, nstreams, ctypes.byref(self._h)),
               "rs_server_create")
        self._buf = (Completion * 4096)()
        self._live = {}              # tag -> [(src, dst)] of requests not yet returned by poll

    def submit(self, op, n, k, src, dst, mask=None, tag=0, row_bytes=None, after=None):
        """op RS_OP_ENCODE: src = k message rows, dst = n - k parity rows;
        RS_OP_DECODE: src = n shards, dst = n output rows (may be src).
        The request runs after the work queued so far on `after` (default:
        torch's current stream; False: no ordering).  src and dst are kept
        referenced until poll() returns the request's completion."""
        enc = op == RS_OP_ENCODE
        if row_bytes is None:
            row_bytes = _rows(src, k if enc else n)[1]
            if _rows(dst, n - k if enc else n)[1] != row_bytes:
                raise ValueError("dst rows differ in length from src rows")
        if after is False:
            after_ptr = None
        else:
            after_ptr = _stream(after)
        req = Request(op, StripeDesc(n, k, row_bytes, _ptr(src), _ptr(dst)), None, tag, after_ptr)
        mk = None
        if op == RS_OP_DECODE:
            mk = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
            if mk.shape != (n,):
                raise ValueError("mask must hold n bytes")
            req.mask = mk.ctypes.data_as(ctypes.c_void_p)
        rc = _check(load().rs_server_submit(self._h, ctypes.cast(ctypes.pointer(req), ctypes.c_void_p)),
                    "rs_server_submit")
        self._live.setdefault(tag, []).append((src, dst))
        return rc

    def poll(self, timeout_ms=0):
        """List of (tag, status, t_done_ns) of completed requests."""
        n = load().rs_server_poll(self._h, ctypes.cast(self._buf, ctypes.c_void_p), len(self._buf), int(timeout_ms))
        if n < 0:
            raise RSError(n, "rs_server_poll")
        out = [(self._buf[i].tag, self._buf[i].status, self._buf[i].t_done_ns) for i in range(n)]
        for tag, _, _ in out:
            held = self._live.get(tag)
            if held:
                held.pop(0)
                if not held:
                    del self._live[tag]
        return out

    def stats(self):
        """The server's admission record (rs_server_get_stats) as a dict."""
        st = ServerStats()
        _check(load().rs_server_get_stats(self._h, ctypes.byref(st)), "rs_server_get_stats")
        return {name: int(getattr(st, name)) for name, _ in ServerStats._fields_}

    def pending(self):
        return load().rs_server_pending(self._h)

    def close(self):
        if self._h:
            load().rs_server_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def load():
    """Load librs_nb.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("librs_nb.so is not built (run python -m paper_1404_3458_amd.build)")
        lib = ctypes.CDLL(LIB_PATH)
        vp, i32, u32, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32, ctypes.c_size_t
        sig = {
            "rs_init": (i32, [i32, vp, ctypes.POINTER(vp)]),
            "rs_free": (None, [vp]),
            "rs_encode": (i32, [vp, i32, i32, vp, vp, sz, vp]),
            "rs_decode": (i32, [vp, i32, i32, vp, vp, vp, sz, vp]),
            "rs_decode_static": (i32, [vp, i32, i32, vp, vp, vp, sz, vp]),
            "nb_fft": (i32, [vp, i32, u32, vp, sz, vp]),
            "nb_ifft": (i32, [vp, i32, u32, vp, sz, vp]),
            "nb_derivative": (i32, [vp, i32, vp, sz, vp]),
            "nb_polymul": (i32, [vp, i32, u32, vp, vp, vp, sz, vp]),
            "nb_degree": (i32, [vp, i32, vp, sz, vp, vp]),
            "nb_to_monomial": (i32, [vp, i32, vp, sz, vp]),
            "nb_from_monomial": (i32, [vp, i32, vp, sz, vp]),
            "rs_encode_batch": (i32, [vp, vp, i32, vp]),
            "rs_decode_batch": (i32, [vp, vp, vp, i32, vp]),
            "rs_plan_encode_batch": (i32, [vp, vp, i32, ctypes.POINTER(vp)]),
            "rs_plan_decode_batch": (i32, [vp, vp, vp, i32, ctypes.POINTER(vp)]),
            "rs_plan_launch": (i32, [vp, vp]),
            "rs_plan_set_timestamps": (i32, [vp, vp, ctypes.POINTER(i32)]),
            "rs_plan_free": (None, [vp]),
            "rs_server_create": (i32, [vp, sz, i32, i32, ctypes.POINTER(vp)]),
            "rs_server_submit": (i32, [vp, vp]),
            "rs_server_poll": (i32, [vp, vp, i32, i32]),
            "rs_server_pending": (i32, [vp]),
            "rs_server_get_stats": (i32, [vp, vp]),
            "rs_server_free": (None, [vp]),
            "rs_schedule_set": (i32, [vp, i32, i32, i32]),
            "rs_schedule_get": (i32, [vp, i32, i32, ctypes.POINTER(i32)]),
            "rs_schedule_set_parts": (i32, [vp, i32, i32, vp, i32]),
            "rs_schedule_get_parts": (i32, [vp, i32, i32, vp, ctypes.POINTER(i32)]),
            "rs_schedule_set_tile": (i32, [vp, i32, i32, i32]),
            "rs_schedule_get_tile": (i32, [vp, i32, i32, ctypes.POINTER(i32)]),
            "rs_sync": (i32, [vp, vp]),
            "rs_get_table": (i32, [vp, i32, vp, sz]),
            "rs_strerror": (ctypes.c_char_p, [i32]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def header_functions():
    """Names of the functions include/rs.h declares."""
    txt = open(HEADER_PATH).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b((?:rs|nb)_[a-z_]+)\s*\(", txt)))


def strerror(code):
    return load().rs_strerror(code).decode()


def _check(rc, what):
    if rc != RS_OK:
        raise RSError(rc, what)
    return rc


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _rows(t, nrows=None):
    """(rows, row_bytes) of a contiguous uint8 tensor; raw ints pass through."""
    import torch

    if not isinstance(t, torch.Tensor) or t.dtype != torch.uint8 or not t.is_contiguous():
        raise ValueError("expected a contiguous uint8 tensor")
    if nrows is not None and (t.dim() != 2 or t.shape[0] != nrows):
        raise ValueError("expected %d rows, got shape %s" % (nrows, tuple(t.shape)))
    return t.shape[0], (t.shape[1] if t.dim() == 2 else 0)


class Codec:
    """One rs_ctx: field GF(2^r) with a basis, tables resident on the current device."""

    def __init__(self, r=16, basis=None):
        lib = load()
        self.r = r
        self._ctx = ctypes.c_void_p()
        self._plans = weakref.WeakSet()
        b = None
        if basis is not None:
            self._basis = np.ascontiguousarray(np.asarray(basis, dtype=np.uint32))
            b = self._basis.ctypes.data_as(ctypes.c_void_p)
        _check(lib.rs_init(r, b, ctypes.byref(self._ctx)), "rs_init")

    def close(self):
        """Free the context (and any plan still open on it first)."""
        for pl in list(self._plans):
            pl.close()
        if self._ctx:
            load().rs_free(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ codec
    def encode(self, n, k, msg, parity, row_bytes=None, stream=None):
        if row_bytes is None:
            _, row_bytes = _rows(msg, k)
            _rows(parity, n - k)
        return _check(load().rs_encode(self._ctx, n, k, _ptr(msg), _ptr(parity), row_bytes, _stream(stream)),
                      "rs_encode")

    def decode(self, n, k, mask, shards, out=None, row_bytes=None, stream=None):
        mk = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
        assert mk.shape == (n,)
        if out is None:
            out = shards
        if row_bytes is None:
            _, row_bytes = _rows(shards, n)
            _rows(out, n)
        return _check(load().rs_decode(self._ctx, n, k, mk.ctypes.data_as(ctypes.c_void_p), _ptr(shards),
                                       _ptr(out), row_bytes, _stream(stream)), "rs_decode")

    def decode_static(self, n, k, mask, shards, out=None, row_bytes=None, stream=None):
        """rs_decode_static: decode with no allocation (mother codes of at most
        256 points; calls that overlap on one GPU race)."""
        mk = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
        if mk.shape != (n,):
            raise ValueError("mask must hold n bytes")
        if out is None:
            out = shards
        if row_bytes is None:
            _, row_bytes = _rows(shards, n)
            _rows(out, n)
        return _check(load().rs_decode_static(self._ctx, n, k, mk.ctypes.data_as(ctypes.c_void_p), _ptr(shards),
                                              _ptr(out), row_bytes, _stream(stream)), "rs_decode_static")

    def prepare_encode_batch(self, stripes):
        """Marshal a list of (n, k, msg, parity[, row_bytes]) once, for
        repeated encode_batch calls on the same buffers."""
        arr = (StripeDesc * len(stripes))()
        for i, s in enumerate(stripes):
            n, k, msg, par = s[:4]
            rb = s[4] if len(s) > 4 else _rows(msg, k)[1]
            arr[i] = StripeDesc(n, k, rb, _ptr(msg), _ptr(par))
        return PreparedBatch(arr, None, len(stripes))

    def prepare_decode_batch(self, stripes):
        """Marshal a list of (n, k, mask, shards, out[, row_bytes]) once."""
        arr = (StripeDesc * len(stripes))()
        masks = []
        for i, s in enumerate(stripes):
            n, k, mask, sh, out = s[:5]
            rb = s[5] if len(s) > 5 else _rows(sh, n)[1]
            arr[i] = StripeDesc(n, k, rb, _ptr(sh), _ptr(out if out is not None else sh))
            masks.append(np.asarray(mask, dtype=np.uint8).reshape(-1))
        allm = np.ascontiguousarray(np.concatenate(masks) if masks else np.zeros(0, np.uint8))
        return PreparedBatch(arr, allm, len(stripes))

    def encode_batch(self, stripes, stream=None):
        """stripes: list of (n, k, msg, parity[, row_bytes]) or a prepared batch."""
        b = stripes if isinstance(stripes, PreparedBatch) else self.prepare_encode_batch(stripes)
        return _check(load().rs_encode_batch(self._ctx, b.desc_ptr, b.count, _stream(stream)), "rs_encode_batch")

    def decode_batch(self, stripes, stream=None):
        """stripes: list of (n, k, mask, shards, out[, row_bytes]) or a prepared batch."""
        b = stripes if isinstance(stripes, PreparedBatch) else self.prepare_decode_batch(stripes)
        return _check(load().rs_decode_batch(self._ctx, b.desc_ptr, b.mask_ptr, b.count, _stream(stream)),
                      "rs_decode_batch")

    def plan_encode_batch(self, stripes):
        """A reusable plan of encode_batch(stripes) (rs_plan_encode_batch)."""
        b = stripes if isinstance(stripes, PreparedBatch) else self.prepare_encode_batch(stripes)
        h = ctypes.c_void_p()
        _check(load().rs_plan_encode_batch(self._ctx, b.desc_ptr, b.count, ctypes.byref(h)), "rs_plan_encode_batch")
        pl = Plan(self, h, b.count)
        self._plans.add(pl)
        return pl

    def plan_decode_batch(self, stripes):
        """A reusable plan of decode_batch(stripes) (rs_plan_decode_batch)."""
        b = stripes if isinstance(stripes, PreparedBatch) else self.prepare_decode_batch(stripes)
        h = ctypes.c_void_p()
        _check(load().rs_plan_decode_batch(self._ctx, b.desc_ptr, b.mask_ptr, b.count, ctypes.byref(h)),
               "rs_plan_decode_batch")
        pl = Plan(self, h, b.count)
        self._plans.add(pl)
        return pl

    # ------------------------------------------------------------ transforms
    def fft(self, h, l, data, row_bytes=None, stream=None):
        if row_bytes is None:
            _, row_bytes = _rows(data, h)
        return _check(load().nb_fft(self._ctx, h, l, _ptr(data), row_bytes, _stream(stream)), "nb_fft")

    def ifft(self, h, l, data, row_bytes=None, stream=None):
        if row_bytes is None:
            _, row_bytes = _rows(data, h)
        return _check(load().nb_ifft(self._ctx, h, l, _ptr(data), row_bytes, _stream(stream)), "nb_ifft")

    def derivative(self, h, data, row_bytes=None, stream=None):
        if row_bytes is None:
            _, row_bytes = _rows(data, h)
        return _check(load().nb_derivative(self._ctx, h, _ptr(data), row_bytes, _stream(stream)),
                      "nb_derivative")

    # ------------------------------------------------------------ polynomial operations (Sec. 6.1, Table 1)
    def polymul(self, h, l, a, b, out, row_bytes=None, stream=None):
        """out (2h rows) = product of the novel-basis polynomials in a and b (h rows each)."""
        if row_bytes is None:
            _, row_bytes = _rows(a, h)
            _rows(b, h)
            _rows(out, 2 * h)
        return _check(load().nb_polymul(self._ctx, h, l, _ptr(a), _ptr(b), _ptr(out), row_bytes, _stream(stream)),
                      "nb_polymul")

    def degree(self, h, data, deg=None, row_bytes=None, stream=None):
        """int32 tensor of the column degrees (-1 for zero columns)."""
        import torch

        if row_bytes is None:
            _, row_bytes = _rows(data, h)
        if deg is None:
            deg = torch.empty(row_bytes // (self.r // 8), dtype=torch.int32, device=data.device)
        _check(load().nb_degree(self._ctx, h, _ptr(data), row_bytes, _ptr(deg), _stream(stream)), "nb_degree")
        return deg

    def to_monomial(self, h, data, row_bytes=None, stream=None):
        if row_bytes is None:
            _, row_bytes = _rows(data, h)
        return _check(load().nb_to_monomial(self._ctx, h, _ptr(data), row_bytes, _stream(stream)), "nb_to_monomial")

    def from_monomial(self, h, data, row_bytes=None, stream=None):
        if row_bytes is None:
            _, row_bytes = _rows(data, h)
        return _check(load().nb_from_monomial(self._ctx, h, _ptr(data), row_bytes, _stream(stream)),
                      "nb_from_monomial")

    # ------------------------------------------------------------ schedules
    def set_schedule(self, op, N, split):
        """Pass-pipeline schedule for transforms over 2^N points (op
        RS_OP_ENCODE: N = lg k'; RS_OP_DECODE: N = lg n'): an int is the low
        part's level count (0 = default), a sequence the parts' counts, low first."""
        if isinstance(split, int):
            return _check(load().rs_schedule_set(self._ctx, op, N, split), "rs_schedule_set")
        arr = (ctypes.c_int * max(1, len(split)))(*split)
        return _check(load().rs_schedule_set_parts(self._ctx, op, N, arr, len(split)), "rs_schedule_set_parts")

    def get_schedule(self, op, N):
        """The low part's level count in effect."""
        t = ctypes.c_int()
        _check(load().rs_schedule_get(self._ctx, op, N, ctypes.byref(t)), "rs_schedule_get")
        return t.value

    def get_schedule_parts(self, op, N):
        arr, m = (ctypes.c_int * 4)(), ctypes.c_int()
        _check(load().rs_schedule_get_parts(self._ctx, op, N, arr, ctypes.byref(m)), "rs_schedule_get_parts")
        return tuple(arr[:m.value])

    def set_schedule_tile(self, op, N, cols):
        """Column tiles of the pass pipelines over 2^N points: 0 (default),
        128 (packed tiles for every row) or 256 (256-column tiles only)."""
        return _check(load().rs_schedule_set_tile(self._ctx, op, N, cols), "rs_schedule_set_tile")

    def get_schedule_tile(self, op, N):
        t = ctypes.c_int()
        _check(load().rs_schedule_get_tile(self._ctx, op, N, ctypes.byref(t)), "rs_schedule_get_tile")
        return t.value

    # ------------------------------------------------------------ misc
    def sync(self, stream=None):
        return _check(load().rs_sync(self._ctx, _stream(stream)), "rs_sync")

    def table(self, which):
        q = 1 << self.r
        out = np.zeros(q, dtype=np.uint32)
        n = load().rs_get_table(self._ctx, which, out.ctypes.data_as(ctypes.c_void_p), q)
        if n < 0:
            raise RSError(n, "rs_get_table")
        return out[:n]

    def raw_call(self, name, *args):
        """Call a C-ABI function with this context first and return its code
        (error-path tests)."""
        return getattr(load(), name)(self._ctx, *args)
