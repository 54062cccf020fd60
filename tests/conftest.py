import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) device and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def load_golden(name):
    """Reads a tests/golden/*.txt fixture: `key = hex...` entries whose hex
    may continue on indented lines; '#' starts a comment."""
    out, key = {}, None
    with open(os.path.join(HERE, "golden", name)) as f:
        for raw in f:
            line = raw.split("#", 1)[0].rstrip()
            if not line:
                continue
            if "=" in line and not line.startswith((" ", "\t")):
                key, val = (s.strip() for s in line.split("=", 1))
                out[key] = val
            elif key is not None:
                out[key] += " " + line.strip()
    return out


def hexbytes(s):
    return bytes.fromhex("".join(s.split()))


@pytest.fixture
def golden():
    return load_golden
