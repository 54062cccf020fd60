"""GPU: the binding rejects device tensors that do not match the layout
(wrong sample width, wrong sample count, non-contiguous, wrong output dtype,
too few attribute tensors) with ValueError before it calls the library, so
no kernel ever reads or writes past a tensor.  No kernel is launched by the
rejected calls."""
import pytest

from gpu_util import banner

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def J():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2209_08196_amd import jiffy
    jiffy.lib()
    return jiffy


def test_encode_and_decode_argument_checks(J):
    import torch
    banner("binding checks: encode / decode")
    x = torch.zeros((2, 4, 64), dtype=torch.int32, device="cuda")
    with pytest.raises(ValueError):
        J.encode([x, torch.zeros((2, 4, 32), dtype=torch.int16, device="cuda")])  # shapes differ
    with pytest.raises(ValueError):
        J.encode([x.transpose(1, 2)])                                            # not contiguous
    with pytest.raises(ValueError):
        J.encode([x], out=torch.empty(64, dtype=torch.int32, device="cuda"))     # output not bytes
    with pytest.raises(ValueError):
        J.encode([x.float()])                                                    # not integer samples
    lay = J.make_layout(4, 64, [4])
    s, _ = J.encode([x])
    with pytest.raises(ValueError):
        J.decode(s, lay, 2, outs=[torch.empty((2, 4, 64), dtype=torch.int16, device="cuda")])  # narrower
    with pytest.raises(ValueError):
        J.decode(s, lay, 2, outs=[torch.empty((1, 4, 64), dtype=torch.int32, device="cuda")])  # too short
    with pytest.raises(ValueError):
        J.Decoder(lay, 2, [torch.empty((2, 4, 63), dtype=torch.int32, device="cuda")])
    with pytest.raises(ValueError):
        J.Decoder(lay, 2, [torch.empty((2, 4, 64), dtype=torch.int32, device="cuda")])(s.to(torch.int8))


def test_batch_argument_checks(J):
    import torch
    banner("binding checks: batches")
    s = J.Stream(4, 64, [4, 2])
    out = torch.empty(s.record_bound(), dtype=torch.uint8, device="cuda")
    good = [torch.zeros((4, 64), dtype=torch.int32, device="cuda"), torch.zeros((4, 64), dtype=torch.int16,
                                                                                device="cuda")]
    try:
        with pytest.raises(ValueError):
            J.batch_encode_step([s], [good[:1]], [out])                       # one attribute missing
        with pytest.raises(ValueError):
            J.batch_encode_step([s], [[good[0], good[0]]], [out])             # 4-byte samples for a 2-byte one
        with pytest.raises(ValueError):
            J.batch_encode_step([s], [[good[0][:2], good[1]]], [out])         # half a scan
        with pytest.raises(ValueError):
            J.batch_encode_step([s], [good], [torch.empty(64, dtype=torch.int32, device="cuda")])  # not bytes
        with pytest.raises(ValueError):
            J.batch_encode_step([s], [good, good], [out])                     # more scans than streams
        with pytest.raises(ValueError):
            J.Batch([s], [good[:1]], [out])
        b = J.Batch([s], [good], [out])
        try:
            with pytest.raises(ValueError):
                b.run([[good[1], good[1]]])
            lens, _ = b.run([good])                                           # the checked call still works
            assert lens[0] > 0
        finally:
            b.close()
    finally:
        s.close()
