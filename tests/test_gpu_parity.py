"""GPU path vs the CPU oracle, through the C ABI.

The bar: stream bytes identical to the oracle's (codes, predictor choices,
Huffman codebooks, bit packing), reconstructed floats bit-identical to the
oracle's decompression, and |x - x~| <= eb_abs on every element.
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


def _gpu_roundtrip(x, eb, mode):
    xt = torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda()
    s = sznb.compress(xt, eb, mode)
    y = sznb.decompress(s, x.size)
    return bytes(s.cpu().numpy()), y.cpu().numpy()


def _check(x, eb, mode, label=""):
    ref = oracle.compress(x, eb, mode)
    got, y = _gpu_roundtrip(x, eb, mode)
    if got != ref:
        h1, h2 = oracle.header(ref), oracle.header(got) if len(got) >= 128 else {}
        diff = next((i for i in range(min(len(got), len(ref))) if got[i] != ref[i]), None)
        raise AssertionError("%s stream mismatch: len %d vs %d, first diff at byte %s\nref %s\ngpu %s"
                             % (label, len(got), len(ref), diff, h1, h2))
    yref = oracle.decompress(ref)
    assert np.array_equal(y.view(np.uint32), yref.view(np.uint32)), label
    if x.size:
        eb_abs = oracle.header(ref)["eb_abs"]
        assert np.abs(x.astype(np.float64) - y.astype(np.float64)).max() <= eb_abs, label
    return ref


POLICIES = [sznb.PRED_LV, sznb.PRED_LCF, sznb.PRED_BESTFIT]


def _three_predictor_field():
    """A fast sine (QCF wins), a random walk (LV) and a slower sine (LCF at
    eb_rel 1e-4), with ragged ends."""
    t = np.arange(3 * 4096 + 1500, dtype=np.float64)
    return np.concatenate([(1000 * np.sin(t / 20.0)).astype(np.float32), datagen.random_walk(2 * 4096, seed=21),
                           (1000 * np.sin(np.arange(2 * 4096 + 333) / 100.0)).astype(np.float32)])


@pytest.mark.parametrize("eb_rel", [1e-4, 1e-5])
def test_all_three_predictors(eb_rel):
    x = _three_predictor_field()
    preds, _ = oracle.select(oracle.lattice(x, eb_rel), 4096)
    assert 0 in preds and 2 in preds
    print("three predictors eb=%g choices %s" % (eb_rel, preds.tolist()), flush=True)
    _check(x, eb_rel, sznb.PRED_BESTFIT | sznb.EB_REL, "three predictors")


@pytest.mark.parametrize("policy", POLICIES)
@pytest.mark.parametrize("eb_rel", [1e-3, 1e-4])
def test_walk_ragged(policy, eb_rel):
    print("walk ragged policy=%d eb=%g" % (policy, eb_rel), flush=True)
    x = datagen.random_walk(3 * 4096 + 777, seed=11)
    _check(x, eb_rel, policy | sznb.EB_REL, "walk")


@pytest.mark.parametrize("policy", POLICIES)
def test_cosmology_fields(policy):
    snap = datagen.cosmology(1 << 16, seed=5)
    for name, x in snap.items():
        print("cosmo %s policy=%d" % (name, policy), flush=True)
        _check(x, 1e-4, policy | sznb.EB_REL, name)


def test_md_lattice_bestfit_mixes_predictors():
    md = datagen.md_lattice(cells=(8, 8, 32), seed=3)
    for name, x in md.items():
        print("md %s" % name, flush=True)
        ref = _check(x, 1e-3, sznb.PRED_BESTFIT | sznb.EB_REL, name)
        h = oracle.header(ref)
        if name == "zz":
            pred = np.frombuffer(ref, np.uint8, count=h["nblocks"], offset=h["off_pred"])
            assert (pred == 1).any()


@pytest.mark.parametrize("log2s", [10, 11, 13, 14])
@pytest.mark.parametrize("policy", [sznb.PRED_LV, sznb.PRED_BESTFIT])
def test_block_sizes(log2s, policy):
    print("block 2^%d policy=%d" % (log2s, policy), flush=True)
    x = datagen.random_walk(5 * (1 << log2s) + 123, seed=log2s)
    _check(x, 1e-4, policy | sznb.EB_REL | sznb.BLOCK_LOG2(log2s), "S=2^%d" % log2s)


@pytest.mark.parametrize("n", [1, 5, 1000, 4096, 4097])
def test_small_sizes(n):
    print("small n=%d" % n, flush=True)
    x = np.random.default_rng(n).normal(0, 1, n).astype(np.float32)
    _check(x, 1e-3, sznb.PRED_BESTFIT | sznb.EB_REL, "n=%d" % n)


def test_empty_and_constant():
    print("empty/const", flush=True)
    ref = oracle.compress(np.zeros(0, np.float32), 1e-4, sznb.EB_REL)
    xt = torch.zeros(0, dtype=torch.float32, device="cuda")
    s = sznb.compress(xt, 1e-4, sznb.EB_REL)
    assert bytes(s.cpu().numpy()) == ref
    assert sznb.decompress(s, 0).numel() == 0
    x = np.full(5000, -2.5, np.float32)
    _check(x, 1e-4, sznb.PRED_BESTFIT | sznb.EB_REL, "const")
    _check(x, 0.1, sznb.PRED_LV, "const-abs")


def test_escapes_and_absolute_bound():
    print("escapes", flush=True)
    rng = np.random.default_rng(9)
    x = np.cumsum(rng.normal(0, 1, 20000)).astype(np.float32)
    x[5000] += 3e4
    x[12345] -= 5e4
    for policy in POLICIES:
        # absolute bound well above 2 ulp of the largest magnitude (~5e4)
        ref = _check(x, 0.05, policy, "escapes abs")
        h = oracle.header(ref)
        nesc = np.frombuffer(ref, np.uint16, count=h["nblocks"], offset=h["off_nesc"])
        assert nesc.sum() > 0


def test_negative_zero_and_negative_values():
    print("signs", flush=True)
    x = np.array([-0.0, 0.0, -1.5, 2.25, -0.0] * 2000, np.float32)
    _check(x, 1e-3, sznb.PRED_BESTFIT | sznb.EB_REL, "signs")


def test_device_errors():
    print("device errors", flush=True)
    x = np.linspace(0, 1, 9000).astype(np.float32)
    x[77] = np.nan
    with pytest.raises(sznb.SznbError) as e:
        sznb.compress(torch.from_numpy(x).cuda(), 1e-3, sznb.EB_REL)
    assert e.value.code == sznb.ENONFINITE
    y = np.linspace(1000, 1008, 9000).astype(np.float32)
    with pytest.raises(sznb.SznbError) as e:
        sznb.compress(torch.from_numpy(y).cuda(), 1e-7, sznb.EB_REL)
    assert e.value.code == sznb.EEBTOOSMALL
    with pytest.raises(sznb.SznbError) as e:
        sznb.compress(torch.from_numpy(y).cuda(), -1.0, sznb.EB_REL)
    assert e.value.code == sznb.EINVAL


def test_corrupt_streams_rejected():
    print("corrupt", flush=True)
    x = datagen.random_walk(50000, seed=2)
    s = oracle.compress(x, 1e-4, sznb.PRED_BESTFIT | sznb.EB_REL)
    good = torch.from_numpy(np.frombuffer(s, np.uint8).copy()).cuda()
    y = sznb.decompress(good, x.size).cpu().numpy()
    assert np.array_equal(y, oracle.decompress(s))
    bad = good.clone()
    bad[0] ^= 0xFF
    with pytest.raises(sznb.SznbError) as e:
        sznb.decompress(bad, x.size)
    assert e.value.code == sznb.ECORRUPT
    with pytest.raises(sznb.SznbError):
        sznb.decompress(good[: good.numel() - 8].clone(), x.size)
    bad = good.clone()
    h = oracle.header(s)
    bad[h["off_cwords"]] = 0xFF
    bad[h["off_cwords"] + 1] = 0xFF
    with pytest.raises(sznb.SznbError):
        sznb.decompress(bad, x.size)
    # a wrong skip-table entry breaks the chain of range entry points
    bad = good.clone()
    bad[h["off_payload"] + 3] ^= 0x10
    with pytest.raises(sznb.SznbError) as e:
        sznb.decompress(bad, x.size)
    assert e.value.code == sznb.ECORRUPT
    with pytest.raises(oracle.OracleError):
        oracle.decompress(bytes(bad.cpu().numpy()))


def test_batch_equals_single():
    print("batch", flush=True)
    xs = [datagen.random_walk(70000, seed=1), datagen.cosmology(1 << 15, seed=4)["vx"],
          datagen.random_walk(4096, seed=3), np.full(3000, 1.0, np.float32)]
    modes = [sznb.PRED_LV | sznb.EB_REL, sznb.PRED_BESTFIT | sznb.EB_REL, sznb.PRED_LCF, sznb.PRED_BESTFIT]
    ebs = [1e-4, 1e-3, 0.01, 1e-3]
    ts = [torch.from_numpy(x).cuda() for x in xs]
    streams = sznb.compress_batch(ts, ebs, modes)
    for x, e, m, s in zip(xs, ebs, modes, streams):
        assert bytes(s.cpu().numpy()) == oracle.compress(x, e, m)
    outs = sznb.decompress_batch(streams, [x.size for x in xs])
    for x, e, m, y in zip(xs, ebs, modes, outs):
        assert np.array_equal(y.cpu().numpy(), oracle.decompress(oracle.compress(x, e, m)))


def test_stream_alignment():
    """Streams start at 8-byte aligned addresses (the decoder reads the block
    table in 8-byte words): a stream at any other offset is refused with
    EINVAL, one at offset 8 of a buffer decodes like the oracle, alone and in
    a batch (block counts that are and are not multiples of 8, one predictor
    and three)."""
    print("alignment", flush=True)
    xs = [_three_predictor_field(), datagen.random_walk(4096 * 9 + 5, seed=11),
          datagen.cosmology(1 << 15, seed=12)["xx"], datagen.random_walk(4096 * 16, seed=13)]
    modes = [sznb.PRED_BESTFIT | sznb.EB_REL, sznb.PRED_LV | sznb.EB_REL, sznb.PRED_BESTFIT | sznb.EB_REL,
             sznb.PRED_LCF | sznb.EB_REL]
    refs = [oracle.compress(x, 1e-4, m) for x, m in zip(xs, modes)]
    want = [oracle.decompress(r) for r in refs]
    for off in range(9):
        print("offset %d" % off, flush=True)
        views = []
        for r in refs:
            buf = torch.zeros(len(r) + 8, dtype=torch.uint8, device="cuda")
            buf[off:off + len(r)] = torch.frombuffer(bytearray(r), dtype=torch.uint8).cuda()
            views.append(buf[off:off + len(r)])
        if views[0].data_ptr() % 8:
            with pytest.raises(sznb.SznbError) as e:
                sznb.decompress(views[0], xs[0].size)
            assert e.value.code == sznb.EINVAL
            continue
        for v, x, w in zip(views, xs, want):
            assert np.array_equal(sznb.decompress(v, x.size).cpu().numpy().view(np.uint32), w.view(np.uint32)), off
        outs = sznb.decompress_batch(views, [x.size for x in xs])
        for o, w in zip(outs, want):
            assert np.array_equal(o.cpu().numpy().view(np.uint32), w.view(np.uint32)), off


def test_decompress_many_small_streams():
    """More (stream, predictor) groups than decode workgroups: 700 streams of
    1 to 9 blocks (ragged ends, three policies, some constant) in one batch,
    so the decoder has pieces without a workgroup of their own and every
    workgroup moves between groups; every output equals the oracle's."""
    print("many streams", flush=True)
    rng = np.random.default_rng(33)
    xs, modes, ebs = [], [], []
    for i in range(700):
        n = int(rng.integers(1, 9)) * 4096 + int(rng.integers(0, 4096))
        x = np.full(n, 2.5, np.float32) if i % 97 == 0 else datagen.random_walk(n, seed=1000 + i)
        xs.append(x)
        modes.append([sznb.PRED_LV, sznb.PRED_LCF, sznb.PRED_BESTFIT][i % 3] | sznb.EB_REL)
        ebs.append([1e-3, 1e-4, 3e-4][i % 3])
    streams = sznb.compress_batch([torch.from_numpy(x).cuda() for x in xs], ebs, modes)
    refs = [oracle.compress(x, e, m) for x, e, m in zip(xs, ebs, modes)]
    for i, (s_, r) in enumerate(zip(streams, refs)):
        assert bytes(s_.cpu().numpy()) == r, i
    outs = sznb.decompress_batch(streams, [x.size for x in xs])
    for i, (o, r) in enumerate(zip(outs, refs)):
        assert np.array_equal(o.cpu().numpy().view(np.uint32), oracle.decompress(r).view(np.uint32)), i


def test_workspace_reuse_two_calls():
    print("reuse", flush=True)
    x1 = datagen.random_walk(100000, seed=7)
    x2 = datagen.random_walk(30000, seed=8)
    ws = sznb.workspace(sznb.compress_workspace_bytes([x1.size], [sznb.PRED_BESTFIT | sznb.EB_REL]))
    for x in (x1, x2, x1):
        s = sznb.compress(torch.from_numpy(x).cuda(), 1e-4, sznb.PRED_BESTFIT | sznb.EB_REL, ws=ws)
        assert bytes(s.cpu().numpy()) == oracle.compress(x, 1e-4, sznb.PRED_BESTFIT | sznb.EB_REL)


def test_config1_full_bitexact():
    print("config1 full", flush=True)
    x = datagen.random_walk()
    _check(x, 1e-4, sznb.PRED_LV | sznb.EB_REL, "config1")


def test_histogram_counter_wraps():
    # 2^27 values of a piecewise-constant field: every quantization workgroup
    # sees far more than 65535 zero residuals, so its 16-bit LDS counters wrap
    # and carry into the global histogram; the stream must still equal the
    # oracle's byte for byte
    n = 1 << 27
    print("wraps n=%d" % n, flush=True)
    x = (np.arange(n, dtype=np.int64) // 3000000).astype(np.float32)
    x[::7919] += np.float32(0.25)
    ref = oracle.compress(x, 1e-3, sznb.PRED_LV | sznb.EB_REL)
    got, y = _gpu_roundtrip(x, 1e-3, sznb.PRED_LV | sznb.EB_REL)
    assert got == ref
    assert np.abs(y.astype(np.float64) - x).max() <= oracle.header(ref)["eb_abs"]


def test_histogram_neighbour_counters_both_wrap():
    # Residuals 0 and +1 in equal measure: codes 32768 and 32769 share one
    # 32-bit word of the LDS window, and with one quantization workgroup per
    # CU every workgroup visit covers 2^26 / 256 = 262144 values, so both
    # counters of the word pass the 0x8000 hand-over point several times in
    # the same visit.  Each block restarts at 0 (its first value is stored
    # as the anchor), so the values stay small integers.
    n, S = 1 << 26, 4096
    print("neighbour wraps n=%d" % n, flush=True)
    rng = np.random.default_rng(77)
    steps = rng.integers(0, 2, size=(n // S, S), dtype=np.int32)
    steps[:, 0] = 0
    x = np.cumsum(steps, axis=1, dtype=np.int32).astype(np.float32).ravel()
    del steps
    mode = sznb.PRED_LV
    ref = oracle.compress(x, 0.5, mode)
    q = oracle.lattice(x, 0.5, eb_rel=False)
    r = oracle.residuals(q, S, 0)
    assert (r == 0).sum() > n // 3 and (r == 1).sum() > n // 3
    sznb.set_workgroups_per_cu(1)
    try:
        got, y = _gpu_roundtrip(x, 0.5, mode)
    finally:
        sznb.set_workgroups_per_cu(8)
    assert got == ref
    assert np.abs(y.astype(np.float64) - x).max() <= 0.5


def _unlimited_huffman_depth(w):
    """Depth of the deepest leaf of a Huffman tree without a length limit
    (heap merge of the two lightest nodes)."""
    import heapq
    h = [(int(v), i, 0) for i, v in enumerate(w)]
    heapq.heapify(h)
    nxt = len(h)
    while len(h) > 1:
        a, b = heapq.heappop(h), heapq.heappop(h)
        heapq.heappush(h, (a[0] + b[0], nxt, max(a[2], b[2]) + 1))
        nxt += 1
    return h[0][2]


_DEEP = {}


def _deep_field():
    # x coordinates of a 2^24-particle snapshot: at eb_rel 1e-4 the LV code
    # is deeper than 24 bits until the weights are halved once
    if "x" not in _DEEP:
        n = 1 << 24
        snap = datagen.cosmology(n, seed=3, n_halos=max(1, int(20000 * n / float(1 << 26))))
        x = snap["xx"]
        q = oracle.lattice(x, 1e-4)
        r = oracle.residuals(q, 4096, 0)
        h = np.bincount(np.where(np.abs(r) < 32768, r + 32768, 0), minlength=65536)
        w = h[h > 0].astype(np.int64)
        depths = [_unlimited_huffman_depth(w)]
        while depths[-1] > 24:
            w = (w + 1) // 2
            depths.append(_unlimited_huffman_depth(w))
        _DEEP["x"], _DEEP["depths"] = x, depths
        _DEEP["ref"] = oracle.compress(x, 1e-4, sznb.PRED_LV | sznb.EB_REL)
    return _DEEP["x"], _DEEP["depths"], _DEEP["ref"]


@pytest.mark.parametrize("nextra", [0, 7, 10])
def test_huffman_length_limit_variants(nextra):
    # one field: four workgroups per (field, predictor) pair, starting from
    # 0..3 halvings; eight fields: two; eleven fields: one per pair, which
    # halves in turn.  The code must be the one the sequential rule picks.
    x, depths, ref = _deep_field()
    print("length limit, %d extra fields, depths %s" % (nextra, depths), flush=True)
    assert depths[0] > 24 and len(depths) == 2
    mode = sznb.PRED_LV | sznb.EB_REL
    fields = [x] + [datagen.random_walk(5000 + 701 * i, seed=60 + i) for i in range(nextra)]
    outs = sznb.compress_batch([torch.from_numpy(np.ascontiguousarray(f)).cuda() for f in fields], 1e-4, mode)
    assert bytes(outs[0].cpu().numpy()) == ref
    for f, o in zip(fields[1:], outs[1:]):
        assert bytes(o.cpu().numpy()) == oracle.compress(f, 1e-4, mode)
