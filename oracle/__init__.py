"""Jiffy CPU oracle -- TEST INFRASTRUCTURE ONLY.

ctypes binding of ``liborc.so`` (plain C99, built by ``oracle/build.py``).
Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package; the GPU library never does.  Inputs
and outputs are numpy arrays on the host.
"""
import ctypes
import os

import numpy as np

from . import build as _build

MAX_ATTRS = 8
OK, E_INVALID, E_CAPACITY, E_CORRUPT = 0, -1, -2, -3
MODE_AUTO, MODE_I_ONLY, MODE_P_ONLY, MODE_BRUTE = 0, 1, 2, 3

_DT = {1: np.uint8, 2: np.uint16, 4: np.uint32}


class Layout(ctypes.Structure):
    _fields_ = [
        ("height", ctypes.c_uint32),
        ("width", ctypes.c_uint32),
        ("n_attrs", ctypes.c_uint32),
        ("width_bytes", ctypes.c_uint8 * MAX_ATTRS),
        ("precision", ctypes.c_uint32 * MAX_ATTRS),
    ]


class Options(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_uint32), ("trial_rows", ctypes.c_uint32)]


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle status {code}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        u32, u64, sz = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t
        vp, up = ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32)
        L.orc_quantize.restype, L.orc_quantize.argtypes = u64, [u64, u32]
        L.orc_dequantize.restype, L.orc_dequantize.argtypes = u64, [u64, u32, ctypes.c_uint]
        L.orc_zigzag.restype, L.orc_zigzag.argtypes = u32, [u32, ctypes.c_uint]
        L.orc_unzigzag.restype, L.orc_unzigzag.argtypes = u32, [u32, ctypes.c_uint]
        L.orc_pfor_choose.restype = u32
        L.orc_pfor_choose.argtypes = [vp, ctypes.POINTER(ctypes.c_uint), ctypes.POINTER(ctypes.c_uint),
                                      ctypes.POINTER(ctypes.c_uint)]
        L.orc_pfor_cost.restype, L.orc_pfor_cost.argtypes = u64, [vp, sz]
        L.orc_pfor_encode.restype, L.orc_pfor_encode.argtypes = sz, [vp, u32, vp, sz]
        L.orc_pfor_decode.restype = ctypes.c_int
        L.orc_pfor_decode.argtypes = [vp, sz, ctypes.c_uint, u32, vp, ctypes.POINTER(sz)]
        L.orc_frame.restype, L.orc_frame.argtypes = sz, [vp, sz, vp, sz]
        L.orc_unframe.restype, L.orc_unframe.argtypes = ctypes.c_int, [vp, sz, vp, sz]
        L.orc_trial_rows.restype, L.orc_trial_rows.argtypes = ctypes.c_uint, [u32, u32, up]
        L.orc_encode_bound.restype = sz
        L.orc_encode_bound.argtypes = [ctypes.POINTER(Layout), u32]
        L.orc_encode.restype = ctypes.c_int
        L.orc_encode.argtypes = [ctypes.POINTER(Layout), ctypes.POINTER(Options), u32, vp, vp, vp, sz,
                                 ctypes.POINTER(sz), vp]
        L.orc_peek.restype = ctypes.c_int
        L.orc_peek.argtypes = [vp, sz, ctypes.POINTER(Layout), ctypes.POINTER(u32)]
        L.orc_decode.restype = ctypes.c_int
        L.orc_decode.argtypes = [vp, sz, vp]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def make_layout(height, width, widths, precisions=None):
    lay = Layout()
    lay.height, lay.width, lay.n_attrs = height, width, len(widths)
    precisions = precisions or [1] * len(widths)
    for i, (w, p) in enumerate(zip(widths, precisions)):
        lay.width_bytes[i] = w
        lay.precision[i] = p
    return lay


# ---- single steps --------------------------------------------------------
def quantize(x, p):
    return lib().orc_quantize(int(x), int(p))


def dequantize(q, p, bits):
    return lib().orc_dequantize(int(q), int(p), int(bits))


def zigzag(d, bits):
    return lib().orc_zigzag(int(d), int(bits))


def unzigzag(z, bits):
    return lib().orc_unzigzag(int(z), int(bits))


def pfor_choose(frame):
    f = np.ascontiguousarray(frame, dtype=np.uint32)
    assert f.shape == (128,)
    b, n, B = ctypes.c_uint(), ctypes.c_uint(), ctypes.c_uint()
    cost = lib().orc_pfor_choose(_ptr(f), ctypes.byref(b), ctypes.byref(n), ctypes.byref(B))
    return b.value, n.value, B.value, cost


def pfor_cost(z):
    z = np.ascontiguousarray(z, dtype=np.uint32)
    return lib().orc_pfor_cost(_ptr(z), z.size)


def pfor_encode(z):
    z = np.ascontiguousarray(z, dtype=np.uint32)
    n = lib().orc_pfor_encode(_ptr(z), z.size, None, 0)
    out = np.zeros(max(n, 1), np.uint8)
    lib().orc_pfor_encode(_ptr(z), z.size, _ptr(out), out.size)
    return out[:n].tobytes()


def pfor_decode(data, bits, n):
    buf = np.frombuffer(bytes(data) + b"\0", np.uint8)
    z = np.zeros(max(n, 1), np.uint32)
    used = ctypes.c_size_t()
    rc = lib().orc_pfor_decode(_ptr(buf), len(data), bits, n, _ptr(z), ctypes.byref(used))
    if rc:
        raise OracleError(rc)
    return z[:n], used.value


def frame(content):
    c = np.frombuffer(bytes(content) + b"\0", np.uint8)
    n = lib().orc_frame(_ptr(c), len(content), None, 0)
    out = np.zeros(n, np.uint8)
    lib().orc_frame(_ptr(c), len(content), _ptr(out), n)
    return out.tobytes()


def unframe(data, n):
    buf = np.frombuffer(bytes(data) + b"\0", np.uint8)
    out = np.zeros(max(n, 1), np.uint8)
    rc = lib().orc_unframe(_ptr(buf), len(data), _ptr(out), n)
    if rc:
        raise OracleError(rc)
    return out[:n].tobytes()


def trial_rows(height, k=4):
    rows = (ctypes.c_uint32 * max(k, 1))()
    cnt = lib().orc_trial_rows(height, k, rows)
    return list(rows[:cnt])


# ---- whole codec ---------------------------------------------------------
def encode_bound(layout, n_scans):
    return lib().orc_encode_bound(ctypes.byref(layout), n_scans)


def encode(planes, precisions=None, mode=MODE_AUTO, trial_rows=0, prev=None):
    """planes: list of [T, H, W] uint8/uint16/uint32 arrays (one per attribute).
    prev: optional list of [H, W] arrays the first scan may predict from.
    Returns (stream bytes, modes [T, A] uint8)."""
    planes = [np.ascontiguousarray(p) for p in planes]
    T, H, W = planes[0].shape
    widths = [p.dtype.itemsize for p in planes]
    lay = make_layout(H, W, widths, precisions)
    opt = Options(mode, trial_rows)
    arr = (ctypes.c_void_p * len(planes))(*[p.ctypes.data for p in planes])
    parr = None
    if prev is not None:
        prev = [np.ascontiguousarray(p, dtype=planes[i].dtype) for i, p in enumerate(prev)]
        parr = (ctypes.c_void_p * len(prev))(*[p.ctypes.data for p in prev])
    cap = encode_bound(lay, T)
    out = np.zeros(cap, np.uint8)
    modes = np.zeros((max(T, 1), len(planes)), np.uint8)
    n = ctypes.c_size_t()
    rc = lib().orc_encode(ctypes.byref(lay), ctypes.byref(opt), T, ctypes.cast(arr, ctypes.c_void_p),
                          ctypes.cast(parr, ctypes.c_void_p) if parr is not None else None,
                          _ptr(out), cap, ctypes.byref(n), _ptr(modes))
    if rc:
        raise OracleError(rc)
    return out[: n.value].tobytes(), modes[:T]


def peek(data):
    buf = np.frombuffer(bytes(data) + b"\0", np.uint8)
    lay, T = Layout(), ctypes.c_uint32()
    rc = lib().orc_peek(_ptr(buf), len(data), ctypes.byref(lay), ctypes.byref(T))
    if rc:
        raise OracleError(rc)
    return lay, T.value


def decode(data):
    """Returns the list of decoded [T, H, W] planes."""
    lay, T = peek(data)
    planes = [np.zeros((T, lay.height, lay.width), _DT[lay.width_bytes[a]]) for a in range(lay.n_attrs)]
    buf = np.frombuffer(bytes(data) + b"\0", np.uint8)
    arr = (ctypes.c_void_p * len(planes))(*[p.ctypes.data for p in planes])
    rc = lib().orc_decode(_ptr(buf), len(data), ctypes.cast(arr, ctypes.c_void_p))
    if rc:
        raise OracleError(rc)
    return planes
