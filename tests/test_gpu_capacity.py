"""Output buffers smaller than the compressed stream, through the C ABI.

A field whose payload does not fit its buffer reports SZNB_ENOSPC and the
batch completes: every block of that field still takes part in the offset
scan over its field, it only stores nothing past the buffer.  Fields of the
same batch with room are unaffected and equal the oracle's streams, and a
buffer of exactly the stream's size is enough.
"""
import numpy as np
import pytest

import oracle
from paper_1711_03888_amd import datagen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1711_03888_amd import sznb  # noqa: E402


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda()


@pytest.mark.parametrize("policy", [sznb.PRED_LV, sznb.PRED_BESTFIT])
def test_payload_overflow_reports_enospc(policy):
    rng = np.random.default_rng(5)
    noise = rng.random(1 << 22).astype(np.float32)  # 1024 blocks, about 13 bits a value
    other = datagen.cosmology(1 << 18, seed=3)["vx"]
    mode = policy | sznb.EB_REL
    caps = [sznb.compress_min_capacity(noise.size, mode), sznb.compress_bound(other.size, mode)]
    print("overflow policy %d caps %s" % (policy, caps), flush=True)
    c = sznb.compress_batch_async([_dev(noise), _dev(other)], 1e-4, mode, caps=caps)
    first, st = sznb.read_status(c.ws, 2)
    assert st == [sznb.ENOSPC, sznb.OK] and first == sznb.ENOSPC
    assert bytes(c.streams()[1].cpu().numpy()) == oracle.compress(other, 1e-4, mode)
    # the same workspace serves the next call with room for both
    c2 = sznb.compress_batch_async([_dev(noise), _dev(other)], 1e-4, mode, ws=c.ws)
    assert sznb.read_status(c2.ws, 2)[1] == [sznb.OK, sznb.OK]
    assert bytes(c2.streams()[0].cpu().numpy()) == oracle.compress(noise, 1e-4, mode)


def test_exact_capacity():
    # the minimum capacity holds three codebooks at their largest, so the
    # field is one whose stream is well beyond it
    x = np.random.default_rng(8).random((1 << 20) + 77).astype(np.float32)
    mode = sznb.PRED_BESTFIT | sznb.EB_REL
    ref = oracle.compress(x, 1e-4, mode)
    assert len(ref) - 1 >= sznb.compress_min_capacity(x.size, mode)
    c = sznb.compress_batch_async([_dev(x)], 1e-4, mode, caps=[len(ref)])
    assert sznb.read_status(c.ws, 1)[1] == [sznb.OK]
    assert bytes(c.streams()[0].cpu().numpy()) == ref
    c = sznb.compress_batch_async([_dev(x)], 1e-4, mode, caps=[len(ref) - 1])
    assert sznb.read_status(c.ws, 1)[1] == [sznb.ENOSPC]
