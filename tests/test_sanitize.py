"""AddressSanitizer and UndefinedBehaviorSanitizer builds, on the CPU.

The oracle (``oracle/jiffy_oracle.c``) is built with gcc under both
sanitizers together with ``oracle/sanitize_main.c``, which round-trips
seeded sequences in every mode and decodes every truncation and many byte
flips of small streams.  The library's host code (the C ABI's argument and
layout checks, worst-case sizes, header parsing, step limits) is built with
hipcc, the sanitizers on the host side only, and driven by
``tests/sanitize_host_main.c``; no GPU is needed.  Either run aborts on the
first finding."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, **kw):
    return subprocess.run(cmd, capture_output=True, text=True, **kw)


def _gcc_has_sanitizers(tmp):
    src = os.path.join(tmp, "probe.c")
    open(src, "w").write("int main(void) { return 0; }\n")
    r = _run(["gcc", "-fsanitize=address,undefined", src, "-o", os.path.join(tmp, "probe")])
    return r.returncode == 0


def test_oracle_under_sanitizers(tmp_path):
    if not shutil.which("gcc") or not _gcc_has_sanitizers(str(tmp_path)):
        pytest.skip("gcc with sanitizer runtimes is not available")
    exe = str(tmp_path / "orc_san")
    r = _run(["gcc", "-O1", "-g", "-std=c99", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
              "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "oracle"),
              os.path.join(ROOT, "oracle", "jiffy_oracle.c"), os.path.join(ROOT, "oracle", "sanitize_main.c"),
              "-o", exe])
    assert r.returncode == 0, r.stderr[-3000:]
    r = _run([exe], env=SAN_ENV, timeout=600)
    assert r.returncode == 0, (r.stdout + r.stderr)[-5000:]
    assert "no finding" in r.stdout


def test_host_abi_under_sanitizers(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc is not available")
    csrc = os.path.join(ROOT, "paper_2209_08196_amd", "csrc")
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    jobs, objs = [], []
    for name in ("jiffy_encode", "jiffy_decode", "jiffy_standardize", "jiffy_api"):
        obj = str(tmp_path / (name + ".o"))
        objs.append(obj)
        jobs.append(subprocess.Popen([HIPCC] + flags + ["-c", os.path.join(csrc, name + ".hip"), "-o", obj],
                                     stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
    main = str(tmp_path / "main.o")
    r = _run([HIPCC] + flags + ["-x", "hip", "-c", os.path.join(ROOT, "tests", "sanitize_host_main.c"), "-o", main])
    assert r.returncode == 0, r.stderr[-3000:]
    for j in jobs:
        _, err = j.communicate(timeout=900)
        assert j.returncode == 0, err[-3000:]
    exe = str(tmp_path / "host_san")
    r = _run([HIPCC, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
              "-fsanitize=undefined", main] + objs + ["-o", exe])
    assert r.returncode == 0, r.stderr[-3000:]
    r = _run([exe], env=SAN_ENV, timeout=600)
    assert r.returncode == 0, (r.stdout + r.stderr)[-5000:]
    assert "no finding" in r.stdout
