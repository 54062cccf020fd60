"""Python binding of libjiffy.so (the C ABI of include/jiffy.h).

Argument marshalling only: every step of encoding and decoding runs in the
library's HIP kernels.  Tensors are PyTorch device tensors (device memory
and the current HIP stream); results the C ABI returns on the host (lengths,
modes) come back as Python / numpy values.  There is no fallback: without
the built library every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libjiffy.so")
MAX_ATTRS = 8

OK, E_INVALID, E_CAPACITY, E_CORRUPT, E_DEVICE, E_SHAPE, E_SCRATCH = 0, -1, -2, -3, -4, -5, -6
MODE_AUTO, MODE_I_ONLY, MODE_P_ONLY, MODE_BRUTE = 0, 1, 2, 3

SYMBOLS = ("jiffy_encode_bound", "jiffy_encode", "jiffy_encode_noalloc", "jiffy_peek", "jiffy_decode", "jiffy_decode_layout",
           "jiffy_status_string",
           "jiffy_stream_create", "jiffy_stream_state_bytes", "jiffy_stream_create_at",
           "jiffy_batch_encode_step", "jiffy_stream_reset", "jiffy_stream_destroy",
           "jiffy_step_workspace_bytes", "jiffy_step_create", "jiffy_step_submit", "jiffy_step_finish",
           "jiffy_step_destroy",
           "jiffy_batch_create", "jiffy_batch_run", "jiffy_batch_destroy",
           "jiffy_set_tuning", "jiffy_get_tuning", "jiffy_ablate", "jiffy_standardize",
           "jiffy_encode_many", "jiffy_decode_many",
           "jiffy_profile_enable", "jiffy_profile_read")


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


class Tuning(ctypes.Structure):
    _fields_ = [("fused", ctypes.c_uint32), ("wgs_per_cu", ctypes.c_uint32)]


class Grid(ctypes.Structure):
    _fields_ = [
        ("height", ctypes.c_uint32),
        ("width", ctypes.c_uint32),
        ("range_bytes", ctypes.c_uint32),
        ("n_attrs", ctypes.c_uint32),
        ("attr_bytes", ctypes.c_uint8 * MAX_ATTRS),
        ("elev_lo", ctypes.c_double),
        ("elev_hi", ctypes.c_double),
        ("range_unit", ctypes.c_double),
    ]


class JiffyError(RuntimeError):
    def __init__(self, code, what=""):
        msg = lib().jiffy_status_string(code).decode() if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")
        self.code = code


_lib = None


def lib():
    """Loads libjiffy.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2209_08196_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz, u32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint32
        L.jiffy_encode_bound.restype = sz
        L.jiffy_encode_bound.argtypes = [ctypes.POINTER(Layout), u32]
        L.jiffy_encode.restype = ctypes.c_int
        L.jiffy_encode.argtypes = [ctypes.POINTER(Layout), ctypes.POINTER(Options), u32, vp, vp, sz,
                                   ctypes.POINTER(sz), vp, vp]
        L.jiffy_encode_noalloc.restype = ctypes.c_int
        L.jiffy_encode_noalloc.argtypes = L.jiffy_encode.argtypes
        L.jiffy_peek.restype = ctypes.c_int
        L.jiffy_peek.argtypes = [vp, sz, ctypes.POINTER(Layout), ctypes.POINTER(u32)]
        L.jiffy_decode.restype = ctypes.c_int
        L.jiffy_decode.argtypes = [vp, sz, vp, vp]
        L.jiffy_decode_layout.restype = ctypes.c_int
        L.jiffy_decode_layout.argtypes = [ctypes.POINTER(Layout), u32, vp, sz, vp, vp]
        L.jiffy_status_string.restype = ctypes.c_char_p
        L.jiffy_status_string.argtypes = [ctypes.c_int]
        L.jiffy_stream_create.restype = ctypes.c_int
        L.jiffy_stream_create.argtypes = [ctypes.POINTER(Layout), ctypes.POINTER(Options), ctypes.POINTER(vp)]
        L.jiffy_stream_state_bytes.restype = sz
        L.jiffy_stream_state_bytes.argtypes = [ctypes.POINTER(Layout)]
        L.jiffy_stream_create_at.restype = ctypes.c_int
        L.jiffy_stream_create_at.argtypes = [ctypes.POINTER(Layout), ctypes.POINTER(Options), vp, sz,
                                             ctypes.POINTER(vp)]
        L.jiffy_step_workspace_bytes.restype = sz
        L.jiffy_step_workspace_bytes.argtypes = [u32, ctypes.c_uint64]
        L.jiffy_step_create.restype = ctypes.c_int
        L.jiffy_step_create.argtypes = [u32, ctypes.c_uint64, ctypes.POINTER(vp)]
        L.jiffy_step_submit.restype = ctypes.c_int
        L.jiffy_step_submit.argtypes = [vp, vp, u32, vp, vp, sz, vp]
        L.jiffy_step_finish.restype = ctypes.c_int
        L.jiffy_step_finish.argtypes = [vp, vp, vp]
        L.jiffy_step_destroy.restype = None
        L.jiffy_step_destroy.argtypes = [vp]
        L.jiffy_batch_encode_step.restype = ctypes.c_int
        L.jiffy_batch_encode_step.argtypes = [vp, u32, vp, vp, vp, vp, vp, vp]
        L.jiffy_stream_reset.restype = ctypes.c_int
        L.jiffy_stream_reset.argtypes = [vp]
        L.jiffy_stream_destroy.restype = None
        L.jiffy_stream_destroy.argtypes = [vp]
        L.jiffy_batch_create.restype = ctypes.c_int
        L.jiffy_batch_create.argtypes = [vp, u32, vp, vp, vp, ctypes.POINTER(vp)]
        L.jiffy_batch_run.restype = ctypes.c_int
        L.jiffy_batch_run.argtypes = [vp, vp, vp, vp, vp]
        L.jiffy_batch_destroy.restype = None
        L.jiffy_batch_destroy.argtypes = [vp]
        L.jiffy_set_tuning.restype = ctypes.c_int
        L.jiffy_set_tuning.argtypes = [ctypes.POINTER(Tuning)]
        L.jiffy_get_tuning.restype = ctypes.c_int
        L.jiffy_get_tuning.argtypes = [ctypes.POINTER(Tuning), ctypes.POINTER(u32)]
        L.jiffy_encode_many.restype = ctypes.c_int
        L.jiffy_encode_many.argtypes = [ctypes.POINTER(Layout), ctypes.POINTER(Options), u32, u32, vp, vp, vp, vp, vp,
                                        vp]
        L.jiffy_decode_many.restype = ctypes.c_int
        L.jiffy_decode_many.argtypes = [ctypes.POINTER(Layout), u32, u32, vp, vp, vp, vp]
        L.jiffy_ablate.restype = ctypes.c_int
        L.jiffy_ablate.argtypes = [ctypes.POINTER(Layout), u32, vp, vp, vp]
        L.jiffy_standardize.restype = ctypes.c_int
        L.jiffy_standardize.argtypes = [ctypes.POINTER(Grid), u32, u32, vp, vp, vp, vp, vp]
        L.jiffy_profile_enable.restype = ctypes.c_int
        L.jiffy_profile_enable.argtypes = [ctypes.c_int]
        L.jiffy_profile_read.restype = ctypes.c_int
        L.jiffy_profile_read.argtypes = [u32, vp, vp, vp]
        _lib = L
    return _lib


def set_tuning(fused=0, wgs_per_cu=0):
    """The encoders' launch configuration from now on (jiffy_set_tuning)."""
    rc = lib().jiffy_set_tuning(ctypes.byref(Tuning(int(fused), int(wgs_per_cu))))
    if rc:
        raise JiffyError(rc, "jiffy_set_tuning")


def get_tuning():
    """-> (current tuning dict, workgroups of the fused kernel per compute unit)."""
    t, m = Tuning(), ctypes.c_uint32()
    rc = lib().jiffy_get_tuning(ctypes.byref(t), ctypes.byref(m))
    if rc:
        raise JiffyError(rc, "jiffy_get_tuning")
    return {"fused": t.fused, "wgs_per_cu": t.wgs_per_cu}, m.value


def profile_enable(on: bool = True):
    lib().jiffy_profile_enable(1 if on else 0)


def profile_read():
    """-> {kernel name: (total ms, launches)} since profile_enable(True)."""
    n = lib().jiffy_profile_read(0, None, None, None)
    names = ctypes.create_string_buffer(32 * max(n, 1))
    ms = (ctypes.c_double * max(n, 1))()
    cnt = (ctypes.c_uint32 * max(n, 1))()
    n = lib().jiffy_profile_read(n, names, ms, cnt)
    out = {}
    for k in range(n):
        nm = names.raw[32 * k:32 * k + 32].split(b"\0", 1)[0].decode()
        out[nm] = (ms[k], cnt[k])
    return out


def _stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def make_layout(height, width, widths, precisions=None):
    lay = Layout()
    lay.height, lay.width, lay.n_attrs = int(height), int(width), len(widths)
    precisions = precisions if precisions is not None else [1] * len(widths)
    for i, (w, p) in enumerate(zip(widths, precisions)):
        lay.width_bytes[i] = int(w)
        lay.precision[i] = int(p)
    return lay


def encode_bound(layout: Layout, n_scans: int) -> int:
    return lib().jiffy_encode_bound(ctypes.byref(layout), n_scans)


_SAMPLE_DTYPES = None


def _sample_dtypes():
    global _SAMPLE_DTYPES
    if _SAMPLE_DTYPES is None:
        import torch
        _SAMPLE_DTYPES = (torch.uint8, torch.int16, torch.int32, torch.uint16, torch.uint32)
    return _SAMPLE_DTYPES


def _check_tensor(t, numel, width_bytes, what):
    """A contiguous device tensor of `numel` samples of `width_bytes` bytes
    (the C ABI reads or writes exactly that many bytes through its pointer)."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{what}: expected a torch tensor, got {type(t).__name__}")
    if t.device.type != "cuda":
        raise ValueError(f"{what}: must be a device tensor (got {t.device})")
    if not t.is_contiguous():
        raise ValueError(f"{what}: must be contiguous")
    if t.dtype not in _sample_dtypes():
        raise ValueError(f"{what}: unsupported dtype {t.dtype}")
    if t.element_size() != width_bytes:
        raise ValueError(f"{what}: {t.element_size()}-byte samples where the layout has {width_bytes}")
    if t.numel() != numel:
        raise ValueError(f"{what}: {t.numel()} samples where {numel} are needed")


def _check_bytes_out(t, what):
    """A contiguous device uint8 tensor (an output byte buffer)."""
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.uint8 \
            or not t.is_contiguous() or t.dim() != 1:
        raise ValueError(f"{what}: must be a contiguous 1-D device uint8 tensor")


def _check_planes(planes):
    import torch
    if not planes or len(planes) > MAX_ATTRS:
        raise ValueError(f"between 1 and {MAX_ATTRS} attribute planes are needed")
    if not isinstance(planes[0], torch.Tensor) or planes[0].dim() != 3:
        raise ValueError("planes must be [T, H, W] tensors")
    T, H, W = planes[0].shape
    for a, p in enumerate(planes):
        if not isinstance(p, torch.Tensor) or tuple(p.shape) != (T, H, W):
            raise ValueError("planes must be contiguous device tensors of one [T, H, W] shape")
        _check_tensor(p, T * H * W, p.element_size(), f"plane {a}")
    return T, H, W


def _check_outs(layout, T, outs):
    """Decode outputs: one device tensor per attribute of T*H*W samples of
    the attribute's width."""
    if outs is None or len(outs) != layout.n_attrs:
        raise ValueError(f"{layout.n_attrs} output planes are needed")
    n = T * layout.height * layout.width
    for a, o in enumerate(outs):
        _check_tensor(o, n, layout.width_bytes[a], f"output plane {a}")


def _check_scan(stream, tensors, what):
    """One scan of a stream: a device tensor of H*W samples per attribute."""
    lay = stream.layout
    if tensors is None or len(tensors) != lay.n_attrs:
        raise ValueError(f"{what}: {lay.n_attrs} attribute tensors are needed")
    for a, t in enumerate(tensors):
        _check_tensor(t, lay.height * lay.width, lay.width_bytes[a], f"{what}, attribute {a}")


def encode(planes, precisions=None, mode=MODE_AUTO, trial_rows=0, out=None, stream=None, noalloc=False):
    """planes: list of contiguous device tensors [T, H, W] (uint8, uint16 /
    int16 or uint32 / int32 storage).  Returns (stream tensor uint8 [n],
    modes ndarray [T, A] uint8).  noalloc=True calls jiffy_encode_noalloc
    (the library's fixed scratch instead of its own allocations; `out` must
    then be given, so that nothing is allocated here either)."""
    import torch
    if noalloc and out is None:
        raise ValueError("encode(noalloc=True) needs an output buffer")
    T, H, W = _check_planes(planes)
    widths = [p.element_size() for p in planes]
    lay = make_layout(H, W, widths, precisions)
    opt = Options(mode, trial_rows)
    if out is None:
        out = torch.empty(encode_bound(lay, T), dtype=torch.uint8, device=planes[0].device)
    _check_bytes_out(out, "out")
    arr = (ctypes.c_void_p * len(planes))(*[p.data_ptr() for p in planes])
    n = ctypes.c_size_t()
    modes = np.zeros((max(T, 1), len(planes)), np.uint8)
    fn = lib().jiffy_encode_noalloc if noalloc else lib().jiffy_encode
    rc = fn(ctypes.byref(lay), ctypes.byref(opt), T, ctypes.cast(arr, ctypes.c_void_p),
            ctypes.c_void_p(out.data_ptr()), out.numel(), ctypes.byref(n),
            modes.ctypes.data_as(ctypes.c_void_p), _stream_handle(stream))
    if rc:
        raise JiffyError(rc, "jiffy_encode_noalloc" if noalloc else "jiffy_encode")
    return out[: n.value], modes[:T]


ABL_SIZES = 5
ABL_NAMES = ("pfor", "delta_pfor", "delta_zigzag_pfor", "rl_mask_i", "rl_mask_p")


def ablate(planes, precisions=None, stream=None):
    """Record sizes under the ablated codecs and the run-length mask codec
    (jiffy_ablate).  planes: as encode.  Returns uint64 [T, A, 5] in the
    order of ABL_NAMES."""
    T, H, W = _check_planes(planes)
    widths = [p.element_size() for p in planes]
    lay = make_layout(H, W, widths, precisions)
    arr = (ctypes.c_void_p * len(planes))(*[p.data_ptr() for p in planes])
    out = np.zeros((max(T, 1), len(planes), ABL_SIZES), np.uint64)
    rc = lib().jiffy_ablate(ctypes.byref(lay), T, ctypes.cast(arr, ctypes.c_void_p),
                            out.ctypes.data_as(ctypes.c_void_p), _stream_handle(stream))
    if rc:
        raise JiffyError(rc, "jiffy_ablate")
    return out[:T]


_WIDTH_DTYPE = None


def standardize(xyz, height, width, elev_lo, elev_hi, range_unit=0.001, range_bytes=4, attrs=(), outs=None,
                stream=None):
    """Cartesian points to range and attribute images (jiffy_standardize).
    xyz: contiguous device float32 tensor [S, N, 3] (or [N, 3]: one scan);
    attrs: device tensors [S, N] (or [N]) of 1-, 2- or 4-byte integers.
    Returns (range tensor [S, H, W], list of attribute tensors [S, H, W]);
    16- and 32-bit images are int16 / int32 storage of unsigned values."""
    import torch
    global _WIDTH_DTYPE
    if _WIDTH_DTYPE is None:
        _WIDTH_DTYPE = {1: torch.uint8, 2: torch.int16, 4: torch.int32}
    if not isinstance(xyz, torch.Tensor) or xyz.device.type != "cuda" or xyz.dtype != torch.float32 \
            or not xyz.is_contiguous() or xyz.dim() not in (2, 3) or xyz.shape[-1] != 3:
        raise ValueError("xyz: must be a contiguous device float32 tensor [S, N, 3] or [N, 3]")
    single = xyz.dim() == 2
    S, N = (1, xyz.shape[0]) if single else (xyz.shape[0], xyz.shape[1])
    if len(attrs) > MAX_ATTRS:
        raise ValueError(f"at most {MAX_ATTRS} attributes")
    for a, t in enumerate(attrs):
        _check_tensor(t, S * N, t.element_size() if isinstance(t, torch.Tensor) else 0, f"attribute {a}")
    if range_bytes not in (1, 2, 4):
        raise ValueError("range_bytes must be 1, 2 or 4")
    g = Grid()
    g.height, g.width, g.range_bytes, g.n_attrs = height, width, range_bytes, len(attrs)
    for a, t in enumerate(attrs):
        g.attr_bytes[a] = t.element_size()
    g.elev_lo, g.elev_hi, g.range_unit = elev_lo, elev_hi, range_unit
    if outs is None:
        rng = torch.empty((S, height, width), dtype=_WIDTH_DTYPE[range_bytes], device=xyz.device)
        aout = [torch.empty((S, height, width), dtype=_WIDTH_DTYPE[t.element_size()], device=xyz.device)
                for t in attrs]
    else:
        rng, aout = outs[0], list(outs[1])
        _check_tensor(rng, S * height * width, range_bytes, "range image")
        if len(aout) != len(attrs):
            raise ValueError("one output image per attribute is needed")
        for a, (o, t) in enumerate(zip(aout, attrs)):
            _check_tensor(o, S * height * width, t.element_size(), f"attribute image {a}")
    ain = (ctypes.c_void_p * max(1, len(attrs)))(*[t.data_ptr() for t in attrs])
    aon = (ctypes.c_void_p * max(1, len(attrs)))(*[o.data_ptr() for o in aout])
    rc = lib().jiffy_standardize(ctypes.byref(g), S, N, ctypes.c_void_p(xyz.data_ptr()),
                                 ctypes.cast(ain, ctypes.c_void_p), ctypes.c_void_p(rng.data_ptr()),
                                 ctypes.cast(aon, ctypes.c_void_p), _stream_handle(stream))
    if rc:
        raise JiffyError(rc, "jiffy_standardize")
    if single:
        return rng[0], [o[0] for o in aout]
    return rng, aout


def peek(data: bytes):
    buf = np.frombuffer(bytes(data), np.uint8)
    lay, T = Layout(), ctypes.c_uint32()
    rc = lib().jiffy_peek(buf.ctypes.data_as(ctypes.c_void_p), len(data), ctypes.byref(lay), ctypes.byref(T))
    if rc:
        raise JiffyError(rc, "jiffy_peek")
    return lay, T.value


_TORCH_DT = {1: "uint8", 2: "int16", 4: "int32"}


def _peek_device(stream_bytes):
    """Layout and scan count of a device stream: copies the header and the
    record-length table (the whole stream only when it has no table)."""
    n = stream_bytes.numel()
    head = stream_bytes[: min(n, 20)].cpu().numpy().tobytes()
    if len(head) < 20:
        raise JiffyError(E_CORRUPT, "jiffy_peek")
    A = int.from_bytes(head[6:8], "little")
    T = int.from_bytes(head[16:20], "little")
    if T == 0:
        return peek(stream_bytes.cpu().numpy().tobytes())
    need = min(n, 20 + 8 * A + 4 * T * A)
    blob = np.zeros(need, np.uint8)
    blob[:need] = stream_bytes[:need].cpu().numpy()
    # jiffy_peek reads only the header and the table when the table is present
    lay, T2 = Layout(), ctypes.c_uint32()
    rc = lib().jiffy_peek(blob.ctypes.data_as(ctypes.c_void_p), n, ctypes.byref(lay), ctypes.byref(T2))
    if rc:
        raise JiffyError(rc, "jiffy_peek")
    return lay, T2.value


def decode(stream_bytes, layout: Layout = None, n_scans: int = None, outs=None, stream=None):
    """stream_bytes: device uint8 tensor holding a whole stream.  layout /
    n_scans come from jiffy_peek of its header when not given; when given
    (n_scans >= 1) the stream is decoded by jiffy_decode_layout, which checks
    them on the device.  Returns the list of decoded [T, H, W] device tensors
    (int16 / int32 storage for 16 / 32-bit attributes)."""
    import torch
    known = layout is not None and n_scans is not None and n_scans >= 1
    if not known:
        layout, n_scans = _peek_device(stream_bytes)
    dev = stream_bytes.device
    if outs is None:
        outs = [torch.empty((n_scans, layout.height, layout.width), dtype=getattr(torch, _TORCH_DT[layout.width_bytes[a]]),
                            device=dev) for a in range(layout.n_attrs)]
    _check_bytes_out(stream_bytes, "stream_bytes")
    _check_outs(layout, n_scans, outs)
    arr = (ctypes.c_void_p * len(outs))(*[o.data_ptr() for o in outs])
    if known:
        rc = lib().jiffy_decode_layout(ctypes.byref(layout), n_scans, ctypes.c_void_p(stream_bytes.data_ptr()),
                                       stream_bytes.numel(), ctypes.cast(arr, ctypes.c_void_p), _stream_handle(stream))
    else:
        rc = lib().jiffy_decode(ctypes.c_void_p(stream_bytes.data_ptr()), stream_bytes.numel(),
                                ctypes.cast(arr, ctypes.c_void_p), _stream_handle(stream))
    if rc:
        raise JiffyError(rc, "jiffy_decode_layout" if known else "jiffy_decode")
    return outs


class Encoder:
    """jiffy_encode of fixed planes into a fixed output buffer, prepared once:
    the tensors are checked and the call's arguments built at construction,
    so a call is one foreign-function call (the library also reuses its plan
    for repeated arguments).  The tensors must stay alive and keep their
    storage; their contents are read afresh on every call.  The stream is
    the one given, else the current stream at construction."""

    def __init__(self, planes, precisions=None, mode=MODE_AUTO, trial_rows=0, out=None, stream=None):
        import torch
        T, H, W = _check_planes(planes)
        self.planes = list(planes)
        self.layout = make_layout(H, W, [p.element_size() for p in planes], precisions)
        self._opt = Options(mode, trial_rows)
        self.T = T
        if out is None:
            out = torch.empty(encode_bound(self.layout, T), dtype=torch.uint8, device=planes[0].device)
        _check_bytes_out(out, "out")
        self.out = out
        self._arr = (ctypes.c_void_p * len(planes))(*[p.data_ptr() for p in planes])
        self._n = ctypes.c_size_t()
        self._modes = np.zeros((max(T, 1), len(planes)), np.uint8)
        self._args = (ctypes.byref(self.layout), ctypes.byref(self._opt), T, ctypes.cast(self._arr, ctypes.c_void_p),
                      ctypes.c_void_p(out.data_ptr()), out.numel(), ctypes.byref(self._n),
                      self._modes.ctypes.data_as(ctypes.c_void_p), _stream_handle(stream))

    def __call__(self):
        """Returns (stream tensor uint8 [n], modes ndarray [T, A]), as encode()."""
        rc = lib().jiffy_encode(*self._args)
        if rc:
            raise JiffyError(rc, "jiffy_encode")
        return self.out[: self._n.value], self._modes[: self.T]


class Decoder:
    """jiffy_decode_layout of streams of one layout and scan count into fixed
    output planes, prepared once (as Encoder)."""

    def __init__(self, layout: Layout, n_scans: int, outs, stream=None):
        if n_scans < 1:
            raise ValueError("n_scans must be at least 1")
        _check_outs(layout, n_scans, outs)
        self.layout, self.T, self.outs = layout, n_scans, list(outs)
        self._arr = (ctypes.c_void_p * len(outs))(*[o.data_ptr() for o in outs])
        self._stream = _stream_handle(stream)

    def __call__(self, stream_bytes):
        """Decodes the device stream tensor into the output planes; returns them."""
        _check_bytes_out(stream_bytes, "stream_bytes")
        rc = lib().jiffy_decode_layout(ctypes.byref(self.layout), self.T, ctypes.c_void_p(stream_bytes.data_ptr()),
                                       stream_bytes.numel(), ctypes.cast(self._arr, ctypes.c_void_p), self._stream)
        if rc:
            raise JiffyError(rc, "jiffy_decode_layout")
        return self.outs


class EncoderMany:
    """jiffy_encode_many of fixed planes of several streams (one layout, one
    scan count) into fixed outputs, prepared once (as Encoder): every
    stream's records share each kernel launch; each output equals that
    stream's jiffy_encode."""

    def __init__(self, streams, precisions=None, mode=MODE_AUTO, trial_rows=0, outs=None, stream=None):
        import torch
        if not streams:
            raise ValueError("at least one stream is needed")
        shape = _check_planes(streams[0])
        widths = [p.element_size() for p in streams[0]]
        for i, planes in enumerate(streams):
            if _check_planes(planes) != shape or [p.element_size() for p in planes] != widths:
                raise ValueError(f"stream {i}: every stream needs the same shape and sample widths")
        T, H, W = shape
        self.streams = [list(p) for p in streams]
        self.layout = make_layout(H, W, widths, precisions)
        self._opt = Options(mode, trial_rows)
        self.T, n = T, len(streams)
        if outs is None:
            bound = encode_bound(self.layout, T)
            outs = [torch.empty(bound, dtype=torch.uint8, device=streams[0][0].device) for _ in range(n)]
        if len(outs) != n:
            raise ValueError("one output buffer per stream is needed")
        for i, o in enumerate(outs):
            _check_bytes_out(o, f"out {i}")
        self.outs = list(outs)
        A = len(widths)
        self._rows = [(ctypes.c_void_p * A)(*[p.data_ptr() for p in planes]) for planes in streams]
        self._planes = (ctypes.c_void_p * n)(*[ctypes.cast(r, ctypes.c_void_p) for r in self._rows])
        self._outs = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
        self._caps = (ctypes.c_size_t * n)(*[o.numel() for o in outs])
        self._lens = (ctypes.c_size_t * n)()
        self._modes = np.zeros((n, T, A), np.uint8)
        self._args = (ctypes.byref(self.layout), ctypes.byref(self._opt), n, T,
                      ctypes.cast(self._planes, ctypes.c_void_p), ctypes.cast(self._outs, ctypes.c_void_p),
                      ctypes.cast(self._caps, ctypes.c_void_p), ctypes.cast(self._lens, ctypes.c_void_p),
                      self._modes.ctypes.data_as(ctypes.c_void_p), _stream_handle(stream))

    def __call__(self):
        """Returns (list of stream tensors, modes ndarray [n, T, A])."""
        rc = lib().jiffy_encode_many(*self._args)
        if rc:
            raise JiffyError(rc, "jiffy_encode_many")
        return [o[: self._lens[i]] for i, o in enumerate(self.outs)], self._modes

    @property
    def lengths(self):
        return list(self._lens)


class DecoderMany:
    """jiffy_decode_many of streams of one layout and scan count into fixed
    output planes, prepared once for fixed stream buffers."""

    def __init__(self, layout: Layout, n_scans: int, ins, outs, stream=None):
        if n_scans < 1:
            raise ValueError("n_scans must be at least 1")
        if not ins or len(ins) != len(outs):
            raise ValueError("one list of output planes per stream is needed")
        for i, (b, o) in enumerate(zip(ins, outs)):
            _check_bytes_out(b, f"stream {i}")
            _check_outs(layout, n_scans, o)
        n = len(ins)
        self.layout, self.T, self.ins, self.outs = layout, n_scans, list(ins), [list(o) for o in outs]
        A = layout.n_attrs
        self._rows = [(ctypes.c_void_p * A)(*[p.data_ptr() for p in o]) for o in outs]
        self._planes = (ctypes.c_void_p * n)(*[ctypes.cast(r, ctypes.c_void_p) for r in self._rows])
        self._ins = (ctypes.c_void_p * n)(*[b.data_ptr() for b in ins])
        self._lens = (ctypes.c_size_t * n)(*[b.numel() for b in ins])
        self._stream = _stream_handle(stream)

    def __call__(self, lengths=None):
        """Decodes every stream (its first lengths[s] bytes, else the whole
        buffer) into the output planes; returns them."""
        if lengths is not None:
            for s, n in enumerate(lengths):
                if not 0 < n <= self.ins[s].numel():
                    raise ValueError(f"stream {s}: length {n} outside its buffer")
                self._lens[s] = n
        rc = lib().jiffy_decode_many(ctypes.byref(self.layout), len(self.ins), self.T,
                                     ctypes.cast(self._ins, ctypes.c_void_p), ctypes.cast(self._lens, ctypes.c_void_p),
                                     ctypes.cast(self._planes, ctypes.c_void_p), self._stream)
        if rc:
            raise JiffyError(rc, "jiffy_decode_many")
        return self.outs


def stream_state_bytes(height, width, widths):
    """Device bytes of a stream's resident state (jiffy_stream_state_bytes)."""
    lay = make_layout(height, width, widths)
    return lib().jiffy_stream_state_bytes(ctypes.byref(lay))


class Stream:
    """A sensor stream whose previous quantized scan stays resident on the
    device (jiffy_stream).  With `state` (a device uint8 tensor of at least
    stream_state_bytes() bytes, 256-byte aligned) the state lives in that
    caller-owned memory (jiffy_stream_create_at), which must outlive the
    stream."""

    def __init__(self, height, width, widths, precisions=None, mode=MODE_AUTO, trial_rows=0, state=None):
        self.layout = make_layout(height, width, widths, precisions)
        self.widths = list(widths)
        opt = Options(mode, trial_rows)
        h = ctypes.c_void_p()
        if state is None:
            rc = lib().jiffy_stream_create(ctypes.byref(self.layout), ctypes.byref(opt), ctypes.byref(h))
        else:
            _check_bytes_out(state, "state")
            rc = lib().jiffy_stream_create_at(ctypes.byref(self.layout), ctypes.byref(opt),
                                              ctypes.c_void_p(state.data_ptr()), state.numel(), ctypes.byref(h))
        if rc:
            raise JiffyError(rc, "jiffy_stream_create" if state is None else "jiffy_stream_create_at")
        self.state = state
        self.handle = h
        self.key = (int(height), int(width), tuple(int(w) for w in widths))  # what a PreparedScan must match

    def record_bound(self):
        lay = self.layout
        return encode_bound(lay, 1) - (20 + 8 * lay.n_attrs + 4 * lay.n_attrs)

    def reset(self):
        rc = lib().jiffy_stream_reset(self.handle)
        if rc:
            raise JiffyError(rc, "jiffy_stream_reset")

    def close(self):
        if self.handle:
            lib().jiffy_stream_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _check_batch(streams, scans, outs):
    if len(scans) != len(streams) or len(outs) != len(streams):
        raise ValueError("one scan and one output buffer per stream are needed")
    for i, (s, sc, o) in enumerate(zip(streams, scans, outs)):
        if not getattr(s, "handle", None):
            raise ValueError(f"stream {i} is closed")
        _check_any_scan(s, sc, f"stream {i}")
        _check_bytes_out(o, f"output of stream {i}")


def _check_any_scan(s, sc, what):
    """A scan given as tensors (checked now) or as a PreparedScan (checked
    when it was prepared, for this stream's layout)."""
    if isinstance(sc, PreparedScan):
        if sc.key != _stream_key(s):
            raise ValueError(f"{what}: the prepared scan was checked for another layout")
    else:
        _check_scan(s, sc, what)


def _scan_ptrs(scans):
    return [(ctypes.c_void_p * len(sc.ptrs))(*sc.ptrs) if isinstance(sc, PreparedScan)
            else (ctypes.c_void_p * len(sc))(*[t.data_ptr() for t in sc]) for sc in scans]


def _batch_args(streams, scans, outs):
    _check_batch(streams, scans, outs)
    n = len(streams)
    sh = (ctypes.c_void_p * n)(*[s.handle.value for s in streams])
    inner = _scan_ptrs(scans)
    planes = (ctypes.c_void_p * n)(*[ctypes.cast(x, ctypes.c_void_p).value for x in inner])
    dout = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
    caps = (ctypes.c_size_t * n)(*[o.numel() for o in outs])
    return sh, inner, planes, dout, caps


def _split_modes(streams, mbuf):
    modes = np.zeros((len(streams), max(s.layout.n_attrs for s in streams)), np.uint8)
    k = 0
    for i, s in enumerate(streams):
        a = s.layout.n_attrs
        modes[i, :a] = mbuf[k:k + a]
        k += a
    return modes


class Batch:
    """A fixed set of streams encoded together, one HIP graph launch per step
    (jiffy_batch).  inputs[i][a]: the device tensor ([H, W]) holding stream
    i's next scan of attribute a (run() may name others); outs[i]: the device
    uint8 tensor receiving stream i's records, fixed for the batch's life.
    The tensors must stay alive while the batch reads or writes them."""

    def __init__(self, streams, inputs, outs):
        self.streams, self.inputs, self.outs = list(streams), inputs, outs
        sh, self._inner, planes, dout, caps = _batch_args(self.streams, inputs, outs)
        h = ctypes.c_void_p()
        rc = lib().jiffy_batch_create(ctypes.cast(sh, ctypes.c_void_p), len(self.streams),
                                      ctypes.cast(planes, ctypes.c_void_p), ctypes.cast(dout, ctypes.c_void_p),
                                      ctypes.cast(caps, ctypes.c_void_p), ctypes.byref(h))
        if rc:
            raise JiffyError(rc, "jiffy_batch_create")
        self.handle = h
        self._lens = (ctypes.c_size_t * len(self.streams))()
        self._mbuf = np.zeros(sum(s.layout.n_attrs for s in self.streams), np.uint8)

    def run(self, scans=None, stream=None):
        """One step; scans[i][a] (optional) names this step's input tensors,
        else the inputs given last are read.  Returns (lengths list, modes
        ndarray [n, A])."""
        planes = None
        if scans is not None:
            if len(scans) != len(self.streams):
                raise ValueError("one scan per stream is needed")
            for i, (s, sc) in enumerate(zip(self.streams, scans)):
                _check_any_scan(s, sc, f"stream {i}")
            self._inner = _scan_ptrs(scans)
            planes = (ctypes.c_void_p * len(self.streams))(*[ctypes.cast(x, ctypes.c_void_p).value
                                                             for x in self._inner])
            self.inputs = scans
        rc = lib().jiffy_batch_run(self.handle, ctypes.cast(planes, ctypes.c_void_p) if planes is not None else None,
                                   ctypes.cast(self._lens, ctypes.c_void_p),
                                   self._mbuf.ctypes.data_as(ctypes.c_void_p), _stream_handle(stream))
        if rc:
            raise JiffyError(rc, "jiffy_batch_run")
        return list(self._lens), _split_modes(self.streams, self._mbuf)

    def close(self):
        if self.handle:
            lib().jiffy_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_encode_step(streams, scans, outs, stream=None):
    """streams: list of Stream; scans[i]: list of [H, W] device tensors (one
    per attribute); outs[i]: device uint8 tensors.  Returns (lengths list,
    modes ndarray [n, A])."""
    n = len(streams)
    if n == 0:
        return [], np.zeros((0, 0), np.uint8)
    sh, _inner, planes, dout, caps = _batch_args(streams, scans, outs)
    lens = (ctypes.c_size_t * n)()
    mbuf = np.zeros(sum(s.layout.n_attrs for s in streams), np.uint8)
    rc = lib().jiffy_batch_encode_step(ctypes.cast(sh, ctypes.c_void_p), n, ctypes.cast(planes, ctypes.c_void_p),
                                       ctypes.cast(dout, ctypes.c_void_p), ctypes.cast(caps, ctypes.c_void_p),
                                       ctypes.cast(lens, ctypes.c_void_p), mbuf.ctypes.data_as(ctypes.c_void_p),
                                       _stream_handle(stream))
    if rc:
        raise JiffyError(rc, "jiffy_batch_encode_step")
    return list(lens), _split_modes(streams, mbuf)


class PreparedScan:
    """One scan's attribute tensors, checked once against a layout (sample
    count, width, device, contiguity) so that repeated submissions pass
    their pointers without checking again.  Holds the tensors alive."""
    __slots__ = ("tensors", "ptrs", "key")

    def __init__(self, height, width, widths, tensors):
        lay = make_layout(height, width, widths)
        if tensors is None or len(tensors) != lay.n_attrs:
            raise ValueError(f"{lay.n_attrs} attribute tensors are needed")
        for a, t in enumerate(tensors):
            _check_tensor(t, height * width, widths[a], f"attribute {a}")
        self.tensors = list(tensors)
        self.ptrs = tuple(t.data_ptr() for t in tensors)
        self.key = (int(height), int(width), tuple(int(w) for w in widths))


def _stream_key(s):
    return s.key


def step_workspace_bytes(max_records, max_samples):
    """Device bytes a Step of these limits holds (jiffy_step_workspace_bytes)."""
    return lib().jiffy_step_workspace_bytes(int(max_records), int(max_samples))


class Step:
    """An asynchronous batch step (jiffy_step): a workspace sized once for
    batches of at most max_records records and max_samples samples.
    submit() enqueues one scan of each stream and returns at once; finish()
    waits and returns (lengths, modes).  The records of all streams land
    packed in `out`, stream after stream."""

    def __init__(self, max_records, max_samples):
        h = ctypes.c_void_p()
        rc = lib().jiffy_step_create(int(max_records), int(max_samples), ctypes.byref(h))
        if rc:
            raise JiffyError(rc, "jiffy_step_create")
        self.handle = h
        self.max_records = int(max_records)
        self._lens = (ctypes.c_size_t * 1)()
        self._modes = np.zeros(1, np.uint8)
        self._streams = []
        self._keep = None

    def submit(self, streams, scans, out, stream=None):
        n = len(streams)
        if n == 0 or len(scans) != n:
            raise ValueError("one scan per stream is needed")
        for i, (s, sc) in enumerate(zip(streams, scans)):
            if not getattr(s, "handle", None):
                raise ValueError(f"stream {i} is closed")
            _check_any_scan(s, sc, f"stream {i}")
        _check_bytes_out(out, "out")
        sh = (ctypes.c_void_p * n)(*[s.handle.value for s in streams])
        inner = _scan_ptrs(scans)
        planes = (ctypes.c_void_p * n)(*[ctypes.cast(x, ctypes.c_void_p).value for x in inner])
        rc = lib().jiffy_step_submit(self.handle, ctypes.cast(sh, ctypes.c_void_p), n,
                                     ctypes.cast(planes, ctypes.c_void_p), ctypes.c_void_p(out.data_ptr()),
                                     out.numel(), _stream_handle(stream))
        if rc:
            raise JiffyError(rc, "jiffy_step_submit")
        self._streams = list(streams)
        self._keep = (sh, inner, planes, scans, out)  # alive until the step is finished
        self._lens = (ctypes.c_size_t * n)()
        self._modes = np.zeros(sum(s.layout.n_attrs for s in streams), np.uint8)

    def finish(self):
        """-> (lengths list, modes ndarray [n, A]) of the submitted step."""
        rc = lib().jiffy_step_finish(self.handle, ctypes.cast(self._lens, ctypes.c_void_p),
                                     self._modes.ctypes.data_as(ctypes.c_void_p))
        self._keep = None
        if rc:
            raise JiffyError(rc, "jiffy_step_finish")
        return list(self._lens), _split_modes(self._streams, self._modes)

    def close(self):
        if self.handle:
            lib().jiffy_step_destroy(self.handle)
            self.handle = None
            self._keep = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
