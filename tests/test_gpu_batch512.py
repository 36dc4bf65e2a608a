"""The 512-field uneven batch that bench.py times, through the same path:
autotuned block size and grid width, one compression plan captured into a
HIP graph and replayed.  A fixed sample of the streams (the eight smallest
and the two largest fields) must equal the oracle's byte for byte and decode
within the bound; every field must report success."""
import numpy as np
import pytest

import oracle
from paper_1711_03888_amd import datagen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1711_03888_amd import sznb  # noqa: E402


def test_batch512_sample_equals_oracle():
    print("batch512: generating", flush=True)
    walk = datagen.random_walk(1 << 28, seed=7)
    cosmo = datagen.cosmology(1 << 26, seed=2)
    specs, host = datagen.batch_from_sources(walk, cosmo)
    del walk
    fields = [torch.from_numpy(h).cuda() for h in host]
    ebs = [sp["eb_rel"] for sp in specs]
    print("batch512: %d fields, %.2f GB; autotune" % (len(fields), 4e-9 * sum(h.size for h in host)), flush=True)
    mode, wg = sznb.autotune(fields, ebs, sznb.PRED_BESTFIT | sznb.EB_REL)
    print("batch512: mode %#x wg %d" % (mode, wg), flush=True)
    sznb.set_workgroups_per_cu(wg)
    try:
        plan = sznb.CompressPlan(fields, ebs, mode)
        side = torch.cuda.Stream()
        plan.capture(side)
        for _ in range(2):
            plan.launch(side)
        side.synchronize()
        first, st = sznb.read_status(plan.ws, len(fields))
        assert first == sznb.OK, st
        streams = plan.streams()
        sizes = [h.size for h in host]
        order = np.argsort(sizes, kind="stable")
        sample = list(order[:8]) + list(order[-2:])
        for i in sample:
            print("batch512: field %d n=%d eb_rel=%g" % (i, sizes[i], ebs[i]), flush=True)
            ref = oracle.compress(host[i], ebs[i], mode)
            got = bytes(streams[i].cpu().numpy())
            assert got == ref, "field %d differs from the oracle" % i
            y = sznb.decompress(streams[i], sizes[i]).cpu().numpy()
            eb_abs = oracle.header(ref)["eb_abs"]
            assert np.abs(host[i].astype(np.float64) - y).max() <= eb_abs
        plan.close()
    finally:
        sznb.set_workgroups_per_cu(8)
