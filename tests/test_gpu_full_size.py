"""Parity at the full size of the cosmology workload the bench times.

2^26 particles x 6 float32 fields, best-fit policy, 4096-value blocks, the
six fields in one batched call, as in the bench: at eb_rel 1e-4 every stream
equals the oracle's byte for byte; at eb_rel 1e-3 every decoded value equals
the oracle's lattice point of the input, fl32(fma(p, step, mn)) (the codes
are lossless on the lattice), and the error bound holds everywhere.
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

_SNAP = {}


def _snapshot():
    if "snap" not in _SNAP:
        print("generating 2^26 particles", flush=True)
        _SNAP["snap"] = datagen.cosmology(1 << 26, seed=2)
    return _SNAP["snap"]


def _gpu(fields, eb):
    mode = sznb.PRED_BESTFIT | sznb.EB_REL | sznb.BLOCK_LOG2(12)
    dev = [torch.from_numpy(np.ascontiguousarray(f, np.float32)).cuda() for f in fields]
    streams = sznb.compress_batch(dev, eb, mode)
    ys = sznb.decompress_batch(streams, [f.size for f in fields])
    return mode, streams, ys


def test_full_size_streams_equal_oracle():
    snap = _snapshot()
    names = list(datagen.FIELD_NAMES)
    fields = [snap[k] for k in names]
    mode, streams, ys = _gpu(fields, 1e-4)
    for name, x, s, y in zip(names, fields, streams, ys):
        print("eb 1e-4 field %s: oracle compress" % name, flush=True)
        ref = oracle.compress(x, 1e-4, mode)
        assert bytes(s.cpu().numpy()) == ref, name
        h = oracle.header(ref)
        p = oracle.lattice(x, 1e-4)
        want = oracle.reconstruct_array(p, h["step"], h["mn"])
        assert np.array_equal(y.cpu().numpy().view(np.uint32), want.view(np.uint32)), name


def test_full_size_lattice_reconstruction_eb1e3():
    snap = _snapshot()
    names = list(datagen.FIELD_NAMES)
    fields = [snap[k] for k in names]
    _, streams, ys = _gpu(fields, 1e-3)
    for name, x, s, y in zip(names, fields, streams, ys):
        print("eb 1e-3 field %s: lattice check" % name, flush=True)
        h = oracle.header(bytes(s[:128].cpu().numpy()))
        pr = oracle.params(x, 1e-3)
        assert h["step"] == pr["step"] and h["mn"] == pr["mn"]
        want = oracle.reconstruct_array(oracle.lattice(x, 1e-3), pr["step"], pr["mn"])
        got = y.cpu().numpy()
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), name
        assert np.abs(got.astype(np.float64) - x.astype(np.float64)).max() <= pr["eb_abs"], name
