"""GPU MD modes vs the CPU oracle, through the C ABI.

The bar: container bytes identical to the oracle's (R-index keys, partial
radix order, CPC2000 key code, SZ-LV streams of the reordered fields), the
same permutation, decompressed floats bit-identical to the oracle's.
"""
import numpy as np
import pytest

from oracle import md
from paper_1711_03888_amd import datagen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1711_03888_amd import sznb  # noqa: E402


def _run(fields, eb, mode, label):
    print("md %s mode=%d nf=%d n=%d eb=%g" % (label, mode, len(fields), fields[0].size, eb), flush=True)
    ref, rperm = md.compress_md(fields, eb, mode)
    dev = [torch.from_numpy(np.ascontiguousarray(f)).cuda() for f in fields]
    blob, perm = sznb.md_compress(dev, eb, mode, want_perm=True)
    got = bytes(blob.cpu().numpy())
    if got != ref:
        diff = next((i for i in range(min(len(got), len(ref))) if got[i] != ref[i]), None)
        raise AssertionError("%s: container mismatch, len %d vs %d, first diff at byte %s"
                             % (label, len(got), len(ref), diff))
    assert np.array_equal(perm.cpu().numpy().astype(np.int64), rperm), label
    outs = sznb.md_decompress(blob, len(fields), fields[0].size)
    yref = md.decompress_md(ref)
    for y, r in zip(outs, yref):
        assert np.array_equal(y.cpu().numpy().view(np.uint32), r.view(np.uint32)), label


@pytest.mark.parametrize("mode", [sznb.MD_SPEED, sznb.MD_TRADEOFF, sznb.MD_COMPRESSION])
@pytest.mark.parametrize("velocities", [False, True])
def test_md_lattice_modes(mode, velocities):
    # 36864 atoms: two full segments and a ragged one
    snap = datagen.md_lattice(cells=(16, 16, 36), seed=3, velocities=velocities)
    _run(list(snap.values()), 1e-4, mode, "lattice")


def test_cpc_rice_parameter_outside_the_mean_window():
    # Pairs of particles 1e-3 apart, the pairs spread over the box: the
    # sorted keys alternate tiny and huge deltas, so the cheapest Rice
    # parameter lies far from the deltas' mean bit length and the device
    # costs every parameter (the window's lower bounds do not exclude them)
    rng = np.random.default_rng(3)
    c = rng.uniform(0, 100, size=(3 * 16384 // 2, 3)).astype(np.float32)
    p = np.repeat(c, 2, axis=0)
    p[1::2] += np.float32(1e-3)
    _run([np.ascontiguousarray(p[:, i]) for i in range(3)], 1e-6, sznb.MD_COMPRESSION, "rice fallback")


@pytest.mark.parametrize("mode", [sznb.MD_TRADEOFF, sznb.MD_COMPRESSION])
@pytest.mark.parametrize("eb", [1e-2, 1e-5])
def test_md_error_bounds(mode, eb):
    snap = datagen.md_lattice(cells=(8, 16, 20), seed=5)
    _run(list(snap.values()), eb, mode, "eb")


@pytest.mark.parametrize("n", [1, 2, 777, 16384, 16385])
def test_md_small_and_edge_sizes(n):
    snap = datagen.md_lattice(cells=(16, 16, 16), seed=6, velocities=True)
    fields = [np.ascontiguousarray(v[:n]) for v in snap.values()]
    for mode in (sznb.MD_TRADEOFF, sznb.MD_COMPRESSION):
        _run(fields, 1e-4, mode, "n=%d" % n)


def test_md_fully_shuffled():
    snap = datagen.md_lattice(cells=(16, 16, 16), seed=7, shuffle_frac=1.0, velocities=True)
    for mode in (sznb.MD_SPEED, sznb.MD_TRADEOFF, sznb.MD_COMPRESSION):
        _run(list(snap.values()), 1e-4, mode, "shuffled")


def test_md_bound_too_small_is_an_error():
    snap = datagen.md_lattice(cells=(8, 8, 8), seed=3)
    dev = [torch.from_numpy(v).cuda() for v in snap.values()]
    with pytest.raises(sznb.SznbError) as e:
        sznb.md_compress(dev, 1e-7, sznb.MD_COMPRESSION)
    assert e.value.code == sznb.EEBTOOSMALL
    import oracle
    with pytest.raises((ValueError, oracle.OracleError)):
        md.compress_md(list(snap.values()), 1e-7, md.COMPRESSION)


def test_md_corrupt_container_is_rejected():
    snap = datagen.md_lattice(cells=(8, 8, 40), seed=3)
    dev = [torch.from_numpy(v).cuda() for v in snap.values()]
    blob, _ = sznb.md_compress(dev, 1e-4, sznb.MD_COMPRESSION)
    n = snap["xx"].size
    bad = blob.clone()
    bad[0] ^= 1
    with pytest.raises(sznb.SznbError):
        sznb.md_decompress(bad, 3, n)
    # a coordinate stream whose segment bit count overruns the stream
    bad = blob.clone()
    bad[96 + 104:96 + 108] = torch.tensor([255, 255, 255, 127], dtype=torch.uint8, device=bad.device)
    with pytest.raises(sznb.SznbError):
        sznb.md_decompress(bad, 3, n)
    outs = sznb.md_decompress(blob, 3, n)  # the good container still decodes
    assert outs[0].numel() == n


@pytest.mark.parametrize("mode", [sznb.MD_CPC2000, sznb.md_mode(sznb.MD_TRADEOFF, 12, 0, sznb.MD_KEY_VEL),
                                  sznb.md_mode(sznb.MD_TRADEOFF, 12, 0, sznb.MD_KEY_ALL),
                                  sznb.md_mode(sznb.MD_TRADEOFF, 10, 4), sznb.md_mode(sznb.MD_TRADEOFF, 13, 2),
                                  sznb.md_mode(sznb.MD_COMPRESSION, 11), sznb.md_mode(sznb.MD_CPC2000, 12)])
def test_md_variants(mode):
    # segment sizes, ignored digits, velocity and six-field keys, CPC2000
    # velocities: two full 16384-particle segments and a ragged one
    snap = datagen.md_lattice(cells=(16, 16, 36), seed=4, velocities=True)
    _run(list(snap.values()), 1e-4, mode, "variant %#x" % mode)


@pytest.mark.parametrize("mode", [sznb.md_mode(sznb.MD_TRADEOFF, 12, 0, sznb.MD_KEY_COORD),
                                  sznb.md_mode(sznb.MD_TRADEOFF, 12, 0, sznb.MD_KEY_VEL),
                                  sznb.md_mode(sznb.MD_TRADEOFF, 12, 0, sznb.MD_KEY_ALL), sznb.MD_CPC2000])
def test_cosmology_rindex_variants(mode):
    # the cosmology R-index studies (Table 6: segments of 4096) on a
    # 2^16-particle snapshot
    snap = datagen.cosmology(1 << 16, seed=9)
    _run([snap[k] for k in datagen.FIELD_NAMES], 1e-4, mode, "cosmology %#x" % mode)


def test_md_velocity_keys_need_six_fields():
    snap = datagen.md_lattice(cells=(8, 8, 8), seed=3)
    dev = [torch.from_numpy(v).cuda() for v in snap.values()]
    for bad in (sznb.md_mode(sznb.MD_TRADEOFF, key=sznb.MD_KEY_VEL), sznb.md_mode(sznb.MD_COMPRESSION, key=1),
                sznb.md_mode(sznb.MD_SPEED, 12), sznb.md_mode(sznb.MD_TRADEOFF, 9), 4):
        with pytest.raises(sznb.SznbError) as e:
            sznb.md_compress(dev, 1e-4, bad)
        assert e.value.code == sznb.EINVAL


@pytest.mark.parametrize("mode", [sznb.MD_SPEED, sznb.MD_TRADEOFF, sznb.MD_COMPRESSION, sznb.MD_CPC2000])
def test_md_full_size(mode):
    # the benched FCC snapshot: 2^21 atoms, 128 segments of 16384
    snap = datagen.md_lattice()
    _run(list(snap.values()), 1e-4, mode, "full")
