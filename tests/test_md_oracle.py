"""Pins of the MD-mode oracle (R-index, partial radix sort, CPC2000 key code).

Each pin checks the oracle against something other than itself: bit strings
built character by character for the R-index, a literal 3-bit-digit LSD radix
sort for PRX (Sec. 5.2), brute-force Rice parameter search, a hand-worked
Rice example, lossless key round trips and the error bound of every mode.

`tests/oracle_mutations.py` plants one plausible mistake at a time in a copy
of the oracle (a dropped term, a wrong sign, index or tie rule) and checks
that one of these pins fails for each.
"""
import numpy as np
import pytest

import oracle
from oracle import md
from paper_1711_03888_amd import datagen


def _small_md(cells=(8, 8, 16), seed=3, velocities=False):
    return datagen.md_lattice(cells=cells, seed=seed, velocities=velocities)


def test_rindex_matches_bit_strings():
    # key = for each bit j from the top: x_j y_j z_j, read as one binary number
    snap = _small_md()
    coords = [snap["xx"], snap["yy"], snap["zz"]]
    key, B = md.rindex_keys(coords, 1e-3)
    ps = [oracle.lattice(c, 1e-3) for c in coords]
    for i in range(0, key.size, 97):
        s = "".join(format(int(ps[0][i]), "0%db" % B)[j] + format(int(ps[1][i]), "0%db" % B)[j]
                    + format(int(ps[2][i]), "0%db" % B)[j] for j in range(B))
        assert int(s, 2) == int(key[i])


def test_rindex_bits_per_coordinate():
    snap = _small_md()
    coords = [snap["xx"], snap["yy"], snap["zz"]]
    _, B = md.rindex_keys(coords, 1e-3)
    top = max(int(oracle.params(c, 1e-3)["P"]) for c in coords)
    assert 2 ** (B - 1) <= top < 2 ** B


def test_deinterleave_inverts_rindex():
    snap = _small_md()
    coords = [snap["xx"], snap["yy"], snap["zz"]]
    key, B = md.rindex_keys(coords, 1e-4)
    back = md.deinterleave(key, B)
    for c in range(3):
        assert np.array_equal(back[c], oracle.lattice(coords[c], 1e-4).astype(np.int64))


def _lsd_radix_3bit(keys, k, ndigits):
    """The paper's partial radix sort written out: buckets on 3-bit digits
    from digit k upward, each pass stable."""
    order = list(range(len(keys)))
    for d in range(k, ndigits):
        buckets = [[] for _ in range(8)]
        for i in order:
            buckets[(int(keys[i]) >> (3 * d)) & 7].append(i)
        order = [i for b in buckets for i in b]
    return order


@pytest.mark.parametrize("k", [0, 2, 6])
def test_prx_is_lsd_radix_from_digit_k(k):
    rng = np.random.default_rng(7)
    n = md.SEG + 3001  # two segments, the second ragged
    keys = rng.integers(0, 1 << 30, size=n).astype(np.uint64)
    keys[:500] = keys[:500] & np.uint64(0x3f)  # many ties below digit 2
    perm = md.segment_order(keys, k)
    for s in range(0, n, md.SEG):
        seg = keys[s:s + md.SEG]
        want = [s + i for i in _lsd_radix_3bit(seg, k, 10)]
        assert perm[s:s + md.SEG].tolist() == want


def test_prx_order_properties():
    snap = _small_md(cells=(16, 16, 32))
    coords = [snap["xx"], snap["yy"], snap["zz"]]
    key, _ = md.rindex_keys(coords, 1e-4)
    for k in (0, 6):
        perm = md.segment_order(key, k)
        assert np.array_equal(np.sort(perm), np.arange(key.size))  # a bijection
        for s in range(0, key.size, md.SEG):
            seg = perm[s:s + md.SEG]
            assert seg.min() == s and seg.max() < s + md.SEG  # stays in its segment
            top = key[seg] >> np.uint64(3 * k)
            assert np.all(np.diff(top.astype(np.int64)) >= 0)


def test_rice_parameter_brute_force():
    rng = np.random.default_rng(9)
    for scale in (1, 40, 5000, 1 << 20):
        d = rng.geometric(1.0 / scale, size=300).astype(np.uint64) - np.uint64(1)
        kb = 39
        costs = []
        for r in range(kb + 1):
            c = 0
            for v in d.tolist():
                q = v >> r
                c += 32 + kb if q >= 32 else q + 1 + r
            costs.append(c)
        assert md.rice_parameter(d, kb) == costs.index(min(costs))


def test_cpc_hand_example():
    # keys 5 6 8 8 13 in 6-bit keys: deltas 1 2 0 5; Rice costs r=0: 12,
    # r=1: 11, r=2: 13 -> r = 1.  Bits: 000101 | 000001 | 0 1 | 10 0 | 0 0 | 110 1
    words, nbits = md.cpc_encode_segment(np.array([5, 6, 8, 8, 13], np.uint64), 6)
    bits = "000101" + "000001" + "01" + "100" + "00" + "1101"
    assert nbits == len(bits) == 23
    assert words.tolist() == [int(bits + "0" * 9, 2)]
    back = md.cpc_decode_segment(words, 5, 6)
    assert back.tolist() == [5, 6, 8, 8, 13]


def test_cpc_escape_round_trip():
    keys = np.array([0, 1, 2, 3, 1 << 40, (1 << 40) + 1, (1 << 44) - 1], np.uint64)
    words, nbits = md.cpc_encode_segment(keys, 45)
    r = md.rice_parameter(np.diff(keys), 45)
    assert r == 0
    # first key + parameter + three 1-deltas + escape + 1-delta + escape
    assert nbits == 45 + 6 + 3 * 2 + (32 + 45) + 2 + (32 + 45)
    assert md.cpc_decode_segment(words, keys.size, 45).tolist() == keys.tolist()


@pytest.mark.parametrize("nzero,r", [(58, 1), (59, 0)])
def test_rice_escape_against_stop_bits(nzero, r):
    # nzero zero deltas and one delta of 33 in 45-bit keys.  r = 0: the 33
    # escapes (32 ones + 45 raw bits) and each zero costs its stop bit:
    # nzero + 77.  r = 1: 33 -> quotient 16, 16 + 1 + 1 = 18 bits, each zero
    # 2 bits: 2 nzero + 18.  58 zeros: 135 vs 134 -> r = 1; 59 zeros: 136 vs
    # 136, a tie -> the smaller r = 0.
    keys = np.concatenate([np.zeros(nzero + 1, np.uint64), np.uint64([33])])
    assert md.rice_parameter(np.diff(keys), 45) == r
    words, nbits = md.cpc_encode_segment(keys, 45)
    assert nbits == 45 + 6 + (nzero + 77 if r == 0 else 2 * nzero + 18)
    assert md.cpc_decode_segment(words, keys.size, 45).tolist() == keys.tolist()


@pytest.mark.parametrize("mode", [md.SPEED, md.TRADEOFF, md.COMPRESSION])
@pytest.mark.parametrize("velocities", [False, True])
def test_md_modes_error_bound_and_order(mode, velocities):
    snap = _small_md(cells=(16, 16, 20), velocities=velocities)
    names = list(snap)
    fields = [snap[k] for k in names]
    n = fields[0].size
    eb = 1e-4
    blob, perm = md.compress_md(fields, eb, mode)
    out = md.decompress_md(blob)
    assert len(out) == len(fields)
    if mode == md.SPEED:
        assert np.array_equal(perm, np.arange(n))
    for f, y in zip(fields, out):
        eb_abs = oracle.params(f, eb)["eb_abs"]
        assert np.abs(f[perm].astype(np.float64) - y.astype(np.float64)).max() <= eb_abs


def test_cpc_coordinates_are_lattice_points():
    snap = _small_md(cells=(16, 16, 20))
    fields = [snap["xx"], snap["yy"], snap["zz"]]
    blob, perm = md.compress_md(fields, 1e-4, md.COMPRESSION)
    out = md.decompress_md(blob)
    for c in range(3):
        pr = oracle.params(fields[c], 1e-4)
        p = oracle.lattice(fields[c][perm], 1e-4)
        assert np.array_equal(out[c].view(np.uint32),
                              oracle.reconstruct_array(p, pr["step"], pr["mn"]).view(np.uint32))


def test_container_layout():
    import struct
    snap = _small_md(cells=(8, 8, 8), velocities=True)
    fields = list(snap.values())
    blob, _ = md.compress_md(fields, 1e-3, md.COMPRESSION)
    magic, ver, mode, nf, n, seg, k, total, *offs = struct.unpack_from("<4sHBBQIIQ6Q", blob, 0)
    assert struct.unpack_from("<I", blob, 80)[0] == md.KEY_COORD
    assert (magic, ver, mode, nf, n, seg, k, total) == (b"SZMD", 1, 2, 6, fields[0].size, md.SEG, 0, len(blob))
    assert offs[0] == md.MD_HDR and all(o % 8 == 0 for o in offs[:4]) and offs[4:] == [0, 0]
    assert blob[offs[0]:offs[0] + 4] == b"SZCP"
    assert all(blob[o:o + 4] == b"SZNB" for o in offs[1:4])


def test_cpc_entry_points_start_codes():
    # every stored entry point is where the code of key SUB c begins: an
    # independent bit reader started there decodes the right delta
    rng = np.random.default_rng(12)
    keys = np.cumsum(rng.geometric(1 / 3000.0, size=1000)).astype(np.uint64)
    kb = 40
    words, nbits, ent = md.cpc_encode_segment(keys, kb, with_entries=True)
    bits = "".join(format(int(w), "032b") for w in words)[:nbits]
    r = int(bits[kb:kb + 6], 2)
    assert list(ent[:1]) == [0] and len(ent) == -(-1000 // md.SUB)
    for c in range(1, len(ent)):
        p = int(ent[c])
        q = 0
        while q < md.CPC_ESC_Q and bits[p] == "1":
            q += 1
            p += 1
        if q == md.CPC_ESC_Q:
            d = int(bits[p:p + kb], 2)
        else:
            d = (q << r) | (int(bits[p + 1:p + 1 + r], 2) if r else 0)
        assert d == int(keys[md.SUB * c] - keys[md.SUB * c - 1])


# ---- velocity keys, six-field keys, segment sizes and CPC2000 velocities

def test_mode_word():
    assert md.parse_mode(md.TRADEOFF) == (md.TRADEOFF, 16384, 6, md.KEY_COORD)
    assert md.parse_mode(md.COMPRESSION) == (md.COMPRESSION, 16384, 0, md.KEY_COORD)
    m = md.mode(md.TRADEOFF, seg_log2=12, ignored=0, key=md.KEY_ALL)
    assert md.parse_mode(m) == (md.TRADEOFF, 4096, 0, md.KEY_ALL)
    for bad in (7, md.mode(md.TRADEOFF, seg_log2=9), 1 << 18):
        with pytest.raises(ValueError):
            md.parse_mode(bad)


def test_rindex6_matches_bit_strings():
    # each of the six lattice indices cut to its D leading bits, then
    # for each bit j from the top: xx_j yy_j zz_j vx_j vy_j vz_j
    snap = _small_md(velocities=True)
    fields = list(snap.values())
    key, D = md.rindex_keys6(fields, 1e-4)
    widths = [int(oracle.params(f, 1e-4)["P"]).bit_length() for f in fields]
    assert D == min(max(widths), 10) and min(widths) > 10  # the cut is exercised
    ps = [oracle.lattice(f, 1e-4) for f in fields]
    for i in range(0, key.size, 89):
        bs = [format(int(p[i]), "0%db" % w)[:D].rjust(D, "0") for p, w in zip(ps, widths)]
        s = "".join(b[j] for j in range(D) for b in bs)
        assert int(s, 2) == int(key[i]), i


def _lsd_radix(keys, k, ndigits, digit):
    order = list(range(len(keys)))
    for d in range(k, ndigits):
        buckets = [[] for _ in range(1 << digit)]
        for i in order:
            buckets[(int(keys[i]) >> (digit * d)) & ((1 << digit) - 1)].append(i)
        order = [i for b in buckets for i in b]
    return order


@pytest.mark.parametrize("seg,k,digit", [(1024, 0, 3), (4096, 2, 6), (2048, 3, 3)])
def test_prx_segments_and_six_bit_digits(seg, k, digit):
    rng = np.random.default_rng(17)
    n = 2 * seg + 777
    keys = rng.integers(0, 1 << 36, size=n).astype(np.uint64)
    keys[:300] &= np.uint64(0xfff)
    perm = md.segment_order(keys, k, seg, digit)
    for s in range(0, n, seg):
        want = [s + i for i in _lsd_radix(keys[s:s + seg], k, 36 // digit, digit)]
        assert perm[s:s + seg].tolist() == want


def test_cpv_hand_example():
    # values 7 5 9 5 in 4-bit values: minimum 5, offsets 2 0 4 0; Rice costs
    # r=0: 3+1+5+1 = 10, r=1: 3+2+4+2 = 11, r=2: 3+3+4+3 = 13 -> r = 0.
    # Bits: 0101 | 000000 | 110 | 0 | 11110 | 0; value 0 starts at bit 10
    words, nbits, ent = md.cpv_encode_segment(np.array([7, 5, 9, 5], np.uint64), 4)
    bits = "0101" + "000000" + "110" + "0" + "11110" + "0"
    assert nbits == len(bits) == 20
    assert words.tolist() == [int(bits + "0" * 12, 2)]
    assert ent.tolist() == [10]
    assert md.cpv_decode_segment(words, 4, 4).tolist() == [7, 5, 9, 5]


def test_cpv_escape_and_entries():
    rng = np.random.default_rng(5)
    vals = rng.integers(0, 3000, size=700).astype(np.uint64)
    vals[[10, 400]] = [1 << 20, (1 << 21) - 1]  # far above the rest: escaped
    words, nbits, ent = md.cpv_encode_segment(vals, 21)
    assert md.cpv_decode_segment(words, vals.size, 21).tolist() == vals.tolist()
    bits = "".join(format(int(w), "032b") for w in words)
    r = int(bits[21:27], 2)
    mn = int(vals.min())
    for c, e in enumerate(ent.tolist()):  # an independent reader started at each entry point
        p, q = e, 0
        while q < md.CPC_ESC_Q and bits[p] == "1":
            q += 1
            p += 1
        d = int(bits[p:p + 21], 2) if q == md.CPC_ESC_Q else (q << r) | (int(bits[p + 1:p + 1 + r], 2) if r else 0)
        assert mn + d == int(vals[md.SUB * c])


@pytest.mark.parametrize("m", [md.CPC2000, md.mode(md.TRADEOFF, 12, 0, md.KEY_VEL),
                               md.mode(md.TRADEOFF, 12, 0, md.KEY_ALL), md.mode(md.TRADEOFF, 10, 4),
                               md.mode(md.COMPRESSION, 11)])
def test_md_variants_error_bound(m):
    snap = _small_md(cells=(16, 16, 20), velocities=True)
    fields = list(snap.values())
    blob, perm = md.compress_md(fields, 1e-4, m)
    out = md.decompress_md(blob)
    assert np.array_equal(np.sort(perm), np.arange(fields[0].size))
    kind, seg, _, _ = md.parse_mode(m)
    for s in range(0, perm.size, seg):
        assert perm[s:s + seg].min() >= s and perm[s:s + seg].max() < s + seg
    for f, y in zip(fields, out):
        eb_abs = oracle.params(f, 1e-4)["eb_abs"]
        assert np.abs(f[perm].astype(np.float64) - y.astype(np.float64)).max() <= eb_abs
    if kind == md.CPC2000:  # velocities come back on their own lattice
        for f, y in zip(fields[3:], out[3:]):
            pr = oracle.params(f, 1e-4)
            want = oracle.reconstruct_array(oracle.lattice(f[perm], 1e-4), pr["step"], pr["mn"])
            assert np.array_equal(y.view(np.uint32), want.view(np.uint32))
