"""The C-ABI library loads and exports every function include/jiffy.h
declares; its host-only entry points (bound, header parse, status strings)
agree with the oracle.  CPU only: no device call is made."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2209_08196_amd import jiffy, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "jiffy.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(jiffy_[a-z_]+)\s*\(", src)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(jiffy.LIB_PATH):
        pytest.fail("libjiffy.so is not built (run __graft_entry__.build())")
    return jiffy.lib()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert set(names) == set(jiffy.SYMBOLS)
    for n in names:
        assert hasattr(lib, n), n
        assert ctypes.cast(getattr(lib, n), ctypes.c_void_p).value


def test_every_launched_kernel_is_in_the_code_object(lib):
    """Each kernel name the host side registers has a kernel descriptor
    (`.kd`) in the gfx950 code object built into the library.  A kernel
    whose parameters carry an address-space qualifier gets a different
    mangled name in the device compilation, and launching it aborts."""
    blob = open(jiffy.LIB_PATH, "rb").read()
    names = set(re.findall(rb"_ZN5jiffy\d+k_\w+", blob))
    kds = {n for n in names if (n + b".kd") in blob}
    assert kds, "no kernel descriptors found"
    missing = sorted(n.decode() for n in names - kds if not n.endswith(b"_kd"))
    assert not missing, missing


def test_status_strings(lib):
    for code in (0, -1, -2, -3, -4, -5, -6):
        s = lib.jiffy_status_string(code)
        assert s and s != b"unknown status"
    assert lib.jiffy_status_string(7) == b"unknown status"


def test_encode_bound_matches_oracle_bound(lib):
    rng = np.random.default_rng(0)
    for _ in range(50):
        H, W = int(rng.integers(1, 300)), int(rng.integers(1, 5000))
        widths = list(rng.choice([1, 2, 4], size=int(rng.integers(1, 9))))
        precs = [int(p) for p in rng.integers(1, 100, len(widths))]
        T = int(rng.integers(0, 50))
        lay_g = jiffy.make_layout(H, W, widths, precs)
        lay_o = oracle.make_layout(H, W, widths, precs)
        assert jiffy.encode_bound(lay_g, T) == oracle.encode_bound(lay_o, T)
    bad = jiffy.make_layout(4, 4, [3])
    assert jiffy.encode_bound(bad, 1) == 0


def test_peek_agrees_with_oracle(lib):
    g = synth.stream(2, 0)
    planes = [p[:, :16, :64] for p in g.scans(0, 3)]
    s, _ = oracle.encode(planes)
    lay, T = jiffy.peek(s)
    lo, To = oracle.peek(s)
    assert T == To == 3
    assert (lay.height, lay.width, lay.n_attrs) == (lo.height, lo.width, lo.n_attrs)
    assert list(lay.width_bytes[:5]) == list(lo.width_bytes[:5])
    assert list(lay.precision[:5]) == list(lo.precision[:5])
    for cut in (0, 10, 27, len(s) - 1):
        with pytest.raises(jiffy.JiffyError):
            jiffy.peek(s[:cut])
    with pytest.raises(jiffy.JiffyError):
        jiffy.peek(b"XFY1" + s[4:])


def test_oversized_records_are_rejected_on_the_host(lib):
    """Record lengths, section sizes and offsets are 32-bit stream fields:
    a layout whose worst-case record reaches 4 GiB is invalid.  Checked
    before any device call (the pointers are never used)."""
    big = jiffy.make_layout(16384, 65535, [4])      # 2^30 samples of 4 bytes: a record can pass 4 GiB
    assert jiffy.encode_bound(big, 1) == 0
    n = ctypes.c_size_t()
    arr = (ctypes.c_void_p * 1)(0x1000)
    rc = lib.jiffy_encode(ctypes.byref(big), None, 1, ctypes.cast(arr, ctypes.c_void_p), ctypes.c_void_p(0x1000),
                          1 << 40, ctypes.byref(n), None, None)
    assert rc == jiffy.E_INVALID
    h = ctypes.c_void_p()
    assert lib.jiffy_stream_create(ctypes.byref(big), None, ctypes.byref(h)) == jiffy.E_INVALID
    ok = jiffy.make_layout(32768, 65535, [1])       # 1-byte samples: every record stays below 4 GiB
    assert 0 < jiffy.encode_bound(ok, 1) < (1 << 32) + 4096


def test_binding_rejects_bad_tensors_before_any_call():
    """The binding checks tensors on the host before it calls the library:
    host tensors, wrong ranks and mismatched shapes raise ValueError."""
    import torch
    cpu = torch.zeros((2, 4, 8), dtype=torch.int32)
    with pytest.raises(ValueError):
        jiffy.encode([cpu])
    with pytest.raises(ValueError):
        jiffy.Encoder([cpu])
    with pytest.raises(ValueError):
        jiffy.encode([])
    with pytest.raises(ValueError):
        jiffy.encode([torch.zeros((4, 8), dtype=torch.int32)])
    lay = jiffy.make_layout(4, 8, [4, 2])
    with pytest.raises(ValueError):
        jiffy.Decoder(lay, 2, [cpu])                 # one plane for two attributes
    with pytest.raises(ValueError):
        jiffy.Decoder(lay, 2, [cpu, torch.zeros((2, 4, 8), dtype=torch.int16)])  # host tensors


def test_noalloc_refuses_calls_beyond_its_scratch(lib):
    """jiffy_encode_noalloc works in a fixed 64 MiB device array: a call that
    needs more (here 32 scans of 128x4096 32-bit samples, about 168 MB of
    workspace) returns JIFFY_E_SCRATCH with a zero length before any device
    call (the pointers are never used)."""
    lay = jiffy.make_layout(128, 4096, [4])
    n = ctypes.c_size_t(123)
    arr = (ctypes.c_void_p * 1)(0x1000)
    rc = lib.jiffy_encode_noalloc(ctypes.byref(lay), None, 32, ctypes.cast(arr, ctypes.c_void_p),
                                  ctypes.c_void_p(0x1000), 1 << 40, ctypes.byref(n), None, None)
    assert rc == jiffy.E_SCRATCH and n.value == 0
    assert lib.jiffy_status_string(rc) != b"unknown status"
