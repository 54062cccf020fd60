"""GPU: the precision sweep (Sec. IV-G, Fig. 4) -- P = 1, 2, 4 ... 64 mm on
range scans -- gives streams byte-identical to the oracle's, and the GPU
decode is within floor(P/2) of the input at every in-range sample."""
import numpy as np
import pytest

import oracle
from gpu_util import banner, to_dev, to_host
from paper_2209_08196_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def J():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2209_08196_amd import jiffy
    jiffy.lib()
    return jiffy


@pytest.mark.parametrize("P", [1, 2, 4, 8, 16, 32, 64])
def test_precision_sweep(J, P):
    g = synth.stream(2, 0)
    x = g.scans(0, 4)[0][:, :64, :1024]
    banner("precision", P)
    ref, mref = oracle.encode([x], [P])
    s, m = J.encode([to_dev(x)], [P])
    assert np.array_equal(m, mref)
    assert s.cpu().numpy().tobytes() == ref
    y = to_host(J.decode(s)[0], 4).astype(np.int64)
    nz = x != 0
    assert np.abs(y - x.astype(np.int64))[nz].max() <= P // 2
    assert (y[~nz] == 0).all()
