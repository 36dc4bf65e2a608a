"""The configurations of the rate-distortion and ablation sweeps
(paper_1711_03888_amd/sweep.py) against the oracle, on samples: every
bound of the sweep on a slice of each cosmology field with each policy, and
every MD mode of the segment, ignored-digit and rate-distortion sweeps on a
small FCC snapshot; streams and containers byte for byte."""
import numpy as np
import pytest

import oracle
from oracle import md
from paper_1711_03888_amd import datagen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1711_03888_amd import sweep, sznb  # noqa: E402

_COSMO = {}


def _cosmo():
    if not _COSMO:
        snap = datagen.cosmology(1 << 20, seed=2, n_halos=max(1, int(20000 * (1 << 20) / float(1 << 26))))
        _COSMO.update({k: np.ascontiguousarray(v[:1 << 16]) for k, v in snap.items()})
    return _COSMO


@pytest.mark.parametrize("eb", sweep.EBS)
@pytest.mark.parametrize("policy", list(sweep.POLICIES.values()))
def test_sweep_bounds_cosmology(eb, policy):
    mode = policy | sznb.EB_REL
    for name, x in _cosmo().items():
        print("sweep cosmology %s policy %d eb %g" % (name, policy, eb), flush=True)
        s = sznb.compress(torch.from_numpy(x).cuda(), eb, mode)
        assert bytes(s.cpu().numpy()) == oracle.compress(x, eb, mode), name


_FCC = datagen.md_lattice(cells=(16, 16, 36), seed=3)
MD_POINTS = ([sznb.md_mode(sznb.MD_TRADEOFF, sl, 0) for sl in range(10, 15)]
             + [sznb.md_mode(sznb.MD_TRADEOFF, 14, k) for k in (0, 2, 4, 6, 8)])


@pytest.mark.parametrize("mode", MD_POINTS)
def test_sweep_md_segments_and_digits(mode):
    fields = list(_FCC.values())
    print("sweep md mode %#x" % mode, flush=True)
    ref, rperm = md.compress_md(fields, 1e-4, mode)
    blob, perm = sznb.md_compress([torch.from_numpy(f).cuda() for f in fields], 1e-4, mode, want_perm=True)
    assert bytes(blob.cpu().numpy()) == ref
    assert np.array_equal(perm.cpu().numpy().astype(np.int64), rperm)


@pytest.mark.parametrize("eb", sweep.EBS)
@pytest.mark.parametrize("kind", list(sweep.MD_KINDS.values()))
def test_sweep_md_kinds_across_bounds(eb, kind):
    fields = list(_FCC.values())
    print("sweep md kind %d eb %g" % (kind, eb), flush=True)
    ref, _ = md.compress_md(fields, eb, kind)
    blob, _ = sznb.md_compress([torch.from_numpy(f).cuda() for f in fields], eb, kind)
    assert bytes(blob.cpu().numpy()) == ref
