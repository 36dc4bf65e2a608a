"""Plans, HIP-graph replay, launch width and the autotuner.

The bar: a plan's eager launch and every graph replay give the same stream
bytes as the oracle for the inputs current at that launch (inputs are
changed in place between replays, with the program's own eager work and
synchronisations in between); the persistent-grid width never changes bytes;
the autotuner returns a legal configuration and honours its cache.
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


def _fields():
    snap = datagen.cosmology(1 << 16, seed=41)
    return [datagen.random_walk(70000, seed=5), snap["xx"], snap["vz"], datagen.random_walk(4096 * 3 + 17, seed=6)]


EBS = [1e-3, 1e-4, 1e-4, 1e-5]


def _ref(xs, mode):
    return [oracle.compress(x, e, mode) for x, e in zip(xs, EBS)]


def test_plan_launch_and_graph_replays():
    mode = sznb.PRED_BESTFIT | sznb.EB_REL
    xs = _fields()
    dev = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in xs]
    plan = sznb.CompressPlan(dev, EBS, mode)
    plan.launch()
    torch.cuda.synchronize()
    assert [bytes(s.cpu().numpy()) for s in plan.streams()] == _ref(xs, mode)
    side = torch.cuda.Stream()
    plan.capture(side)
    for rep in range(3):
        print("replay %d" % rep, flush=True)
        # eager work of the program between replays: change the inputs
        with torch.no_grad():
            for t in dev:
                t.mul_(1.0 + 0.001 * (rep + 1)).add_(0.5)
        torch.cuda.synchronize()
        cur = [t.cpu().numpy() for t in dev]
        side.wait_stream(torch.cuda.current_stream())
        plan.launch(side)
        side.synchronize()
        first, st = sznb.read_status(plan.ws, len(dev))
        assert first == sznb.OK, st
        assert [bytes(s.cpu().numpy()) for s in plan.streams()] == _ref(cur, mode)
        # the streams decode through the ordinary path
        y = sznb.decompress(plan.streams()[1].clone())
        assert y.numel() == dev[1].numel()
    plan.close()


def test_workgroups_per_cu_does_not_change_bytes():
    mode = sznb.PRED_LV | sznb.EB_REL
    xs = _fields()
    dev = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in xs]
    out = []
    try:
        for wg in (1, 2, 16):
            sznb.set_workgroups_per_cu(wg)
            out.append([bytes(s.cpu().numpy()) for s in sznb.compress_batch(dev, EBS, mode)])
    finally:
        sznb.set_workgroups_per_cu(8)
    assert out[0] == out[1] == out[2] == _ref(xs, mode)


def test_autotune_and_cache(tmp_path):
    xs = _fields()
    dev = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in xs]
    cache = tmp_path / "tune.txt"
    mode, wg = sznb.autotune(dev, EBS, sznb.PRED_BESTFIT | sznb.EB_REL, cache)
    assert mode & 3 == sznb.PRED_BESTFIT and mode & sznb.EB_REL
    assert 10 <= (mode >> 8) & 15 <= 14 and wg in (2, 4, 8, 16)
    assert cache.read_text().count("\n") == 1
    assert sznb.autotune(dev, EBS, sznb.PRED_BESTFIT | sznb.EB_REL, cache) == (mode, wg)
    assert cache.read_text().count("\n") == 1  # answered from the cache
    # the tuned configuration compresses to the oracle's bytes with that block size
    sznb.set_workgroups_per_cu(wg)
    try:
        got = [bytes(s.cpu().numpy()) for s in sznb.compress_batch(dev, EBS, mode)]
    finally:
        sznb.set_workgroups_per_cu(8)
    assert got == _ref(xs, mode)


def test_decompress_plan_graph_replays():
    mode = sznb.PRED_BESTFIT | sznb.EB_REL
    xs = _fields()
    dev = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in xs]
    cplan = sznb.CompressPlan(dev, EBS, mode)
    cplan.launch()
    torch.cuda.synchronize()
    streams = cplan.streams()
    # decode buffers sized for the largest stream a replay may hold
    bufs = [torch.zeros(c, dtype=torch.uint8, device="cuda") for c in cplan.caps]
    for b, s in zip(bufs, streams):
        b[:s.numel()].copy_(s)
    dplan = sznb.DecompressPlan(bufs, [x.size for x in xs])
    dplan.launch()
    torch.cuda.synchronize()
    for y, s in zip(dplan.outs, streams):
        assert np.array_equal(y.cpu().numpy().view(np.uint32), oracle.decompress(bytes(s.cpu().numpy())).view(np.uint32))
    side = torch.cuda.Stream()
    dplan.capture(side)
    for rep in range(3):
        print("decode replay %d" % rep, flush=True)
        with torch.no_grad():
            for t in dev:
                t.mul_(0.999).add_(0.25)
        torch.cuda.synchronize()
        cplan.launch()
        torch.cuda.synchronize()
        new = cplan.streams()
        for b, s in zip(bufs, new):
            b.zero_()
            b[:s.numel()].copy_(s)
        torch.cuda.synchronize()
        side.wait_stream(torch.cuda.current_stream())
        dplan.launch(side)
        side.synchronize()
        first, st = sznb.read_status(dplan.ws, len(dev))
        assert first == sznb.OK, st
        for y, s in zip(dplan.outs, new):
            ref = oracle.decompress(bytes(s.cpu().numpy()))
            assert np.array_equal(y.cpu().numpy().view(np.uint32), ref.view(np.uint32))
    dplan.close()
    cplan.close()
