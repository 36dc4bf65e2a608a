"""Oracle of the molecular-dynamics modes (test infrastructure only).

The paper's three modes for MD snapshots (Sec. 5.2 and Sec. 6):

* best_speed       = SZ-LV on every field in stored order;
* best_tradeoff    = SZ-LV-PRX: reorder the particles by a partial radix
  sort of their R-index within fixed index segments, then SZ-LV;
* best_compression = SZ-CPC2000: CPC2000 coding of the sorted coordinate
  keys, SZ-LV on the velocities reordered the same way.

R-index (Sec. 5.2, after CPC2000 in Sec. 2): the coordinates are turned into
integers by the error bound and their binary digits interleaved.  Partial
radix sort (Sec. 5.2): LSD radix on 3-bit digits that skips the k least
significant digits, i.e. a stable sort by key >> 3k.  Sorting reorders every
array the same way and no index is stored (Sec. 5.2).

Readings where the paper is silent:
* integers = the compressor's own lattice index of each coordinate field
  (range, bound and guard exactly as in sznb_oracle.c), so decoding a key
  gives back lattice points within the bound;
* B = max over the three coordinates of bitlen(P_c) bits per coordinate, at
  most 21 (a 63-bit key); digit j of the key holds (x_j, y_j, z_j), x highest;
* segments are index ranges of 16384 particles (Tables 4 and 5);
* the coordinate stream also stores, for every 64 keys of a segment, the
  bit offset where their code starts, so that a decoder can start at each
  of them (the entry for key 0 of the segment is 0);
* velocity-based R-index (Sec. 5.3, Table 6): the same interleave built from
  vx, vy, vz; coordinate & velocity-based R-index: the six lattice indices,
  each cut to its D = min(max bit length, 10) most significant bits, one bit
  of each per 6-bit digit (xx highest, then yy, zz, vx, vy, vz), a 6D-bit
  key; the partial radix sort then ignores k whole digits (3 or 6 bits);
* CPC2000's velocities (Sec. 2 step 1 and 4; Sec. 5.2: integer velocities
  coded by the adaptive variable-length code with status bits): each
  velocity field's own lattice indices in R-index order, per segment the
  minimum raw (Bv = bit length of the field's lattice span), a Rice
  parameter chosen as for the keys, and every value minus the minimum
  Rice-coded (escape to Bv raw bits); entry points every 64 values;
* CPC2000's "adaptive variable-length encoding with status bits" (Sec. 2,
  Sec. 5.2) is read as Rice coding of the key deltas of each sorted segment:
  parameter r = argmin_r sum(floor(d / 2^r) + 1 + r) (ties to the smaller r),
  a delta coded as floor(d / 2^r) one-bits, a zero, then the r low bits; a
  quotient of 32 or more is coded as 32 one-bits followed by the raw delta in
  3B bits.  PARITY UNPINNED against the paper: its exact variable-length code
  is not given; the tests pin the code by lossless round trip and by
  independent decoding.
"""
from __future__ import annotations

import struct

import numpy as np

from . import EB_REL, LV, compress, decompress, lattice, params, reconstruct_array

SEG = 16384
SUB = 64  # keys per decoder entry point
SPEED, TRADEOFF, COMPRESSION, CPC2000 = 0, 1, 2, 3
KEY_COORD, KEY_VEL, KEY_ALL = 0, 1, 2
PRX_IGNORED = 6  # Table 5: segment 16384, six ignored 3-bit digits
CPC_ESC_Q = 32
KEY6_BITS = 10   # bits per field of a six-field key


def mode(kind, seg_log2=None, ignored=None, key=KEY_COORD):
    """MD mode word: kind (0..3), segment size 2^seg_log2 (10..14, default
    14), ignored digits k (default 6 for best_tradeoff, else 0), key fields."""
    m = kind
    if seg_log2 is not None:
        m |= seg_log2 << 8
    if ignored is not None:
        m |= (ignored + 1) << 12
    return m | (key << 16)


def parse_mode(md_mode):
    """(kind, segment size, ignored digits, key fields) of a mode word."""
    kind = md_mode & 0xFF
    sl = (md_mode >> 8) & 15
    kf = (md_mode >> 12) & 15
    key = (md_mode >> 16) & 3
    k = kf - 1 if kf else (PRX_IGNORED if kind == TRADEOFF else 0)
    if kind > CPC2000 or key > KEY_ALL or (sl and not 10 <= sl <= 14) or md_mode >> 18:
        raise ValueError("bad MD mode")
    return kind, 1 << (sl or 14), k, key


def bits_per_coord(coords, eb_rel):
    ps = [params(c, eb_rel)["P"] for c in coords]
    B = max(int(P).bit_length() for P in ps)
    return max(B, 1)


def rindex_keys(coords, eb_rel):
    """Interleaved lattice keys of the particles (first field's bit highest
    in each 3-bit digit)."""
    B = bits_per_coord(coords, eb_rel)
    if B > 21:
        raise ValueError("lattice too fine for a 63-bit key")
    ps = [lattice(c, eb_rel).astype(np.uint64) for c in coords]
    key = np.zeros(ps[0].size, np.uint64)
    for j in range(B):
        for c in range(3):
            bit = (ps[c] >> np.uint64(j)) & np.uint64(1)
            key |= bit << np.uint64(3 * j + (2 - c))
    return key, B


def rindex_keys6(fields, eb_rel):
    """Six-field key: each lattice index cut to its D most significant bits,
    D = min(widest bit length, 10); digit j holds bit j of each, xx highest."""
    widths = [max(int(params(f, eb_rel)["P"]).bit_length(), 1) for f in fields]
    D = min(max(widths), KEY6_BITS)
    ps = [lattice(f, eb_rel).astype(np.uint64) >> np.uint64(max(0, w - D)) for f, w in zip(fields, widths)]
    key = np.zeros(ps[0].size, np.uint64)
    for j in range(D):
        for c in range(6):
            bit = (ps[c] >> np.uint64(j)) & np.uint64(1)
            key |= bit << np.uint64(6 * j + (5 - c))
    return key, D


def deinterleave(key, B):
    out = [np.zeros(key.size, np.int64) for _ in range(3)]
    for j in range(B):
        for c in range(3):
            out[c] |= ((key >> np.uint64(3 * j + (2 - c))) & np.uint64(1)).astype(np.int64) << j
    return out


def segment_order(key, k, seg=SEG, digit=3):
    """Stable sort of each segment by key >> (digit k) (LSD radix from
    digit k)."""
    n = key.size
    perm = np.empty(n, np.int64)
    sk = key >> np.uint64(digit * k)
    for s in range(0, n, seg):
        perm[s:s + seg] = s + np.argsort(sk[s:s + seg], kind="stable")
    return perm


# ----------------------------------------------------------- CPC2000 keys

def rice_parameter(deltas, keybits):
    best, best_cost = 0, None
    for r in range(0, keybits + 1):
        q = deltas >> np.uint64(r)
        esc = q >= CPC_ESC_Q
        cost = int(np.where(esc, CPC_ESC_Q + keybits, q.astype(np.int64) + 1 + r).sum())
        if best_cost is None or cost < best_cost:
            best, best_cost = r, cost
    return best


def pack_fields(values, nbits):
    """MSB-first concatenation of (value, width) fields into u32 words."""
    values = np.asarray(values, np.uint64)
    nbits = np.asarray(nbits, np.int64)
    total = int(nbits.sum())
    idx = np.repeat(np.arange(values.size), nbits)
    start = np.concatenate([[0], np.cumsum(nbits)[:-1]])
    within = np.arange(total) - np.repeat(start, nbits)
    shift = (np.repeat(nbits, nbits) - 1 - within).astype(np.uint64)
    bits = ((values[idx] >> shift) & np.uint64(1)).astype(np.uint8)
    bits = np.concatenate([bits, np.zeros(-total % 32, np.uint8)])
    words = np.packbits(bits).view(">u4").astype(np.uint32)
    return words, total


def cpc_encode_segment(keys_sorted, keybits, with_entries=False):
    """First key raw, 6-bit Rice parameter, then the Rice-coded deltas;
    optionally also the bit offset of key 0, SUB, 2 SUB, ... of the segment."""
    d = np.diff(keys_sorted.astype(np.uint64))
    r = rice_parameter(d, keybits) if d.size else 0
    q = (d >> np.uint64(r)).astype(np.int64)
    esc = q >= CPC_ESC_Q
    qq = np.where(esc, 0, q)
    # per delta: unary part (q ones then a zero, or 32 ones), then r low bits
    # or the raw delta
    unary_v = np.where(esc, np.uint64((1 << CPC_ESC_Q) - 1), (np.uint64(1) << (qq + 1).astype(np.uint64)) - np.uint64(2))
    unary_n = np.where(esc, CPC_ESC_Q, qq + 1)
    tail_v = np.where(esc, d, d & np.uint64((1 << r) - 1))
    tail_n = np.where(esc, keybits, r)
    vals = np.empty(2 + 2 * d.size, np.uint64)
    lens = np.empty(2 + 2 * d.size, np.int64)
    vals[0], lens[0] = np.uint64(keys_sorted[0]), keybits
    vals[1], lens[1] = np.uint64(r), 6
    vals[2::2], lens[2::2] = unary_v, unary_n
    vals[3::2], lens[3::2] = tail_v, tail_n
    words, total = pack_fields(vals, lens)
    if not with_entries:
        return words, total
    # bit offset where key i starts: key 0 at 0, key i >= 1 after the first
    # key, the parameter and deltas 1 .. i - 1
    per_key = np.concatenate([[keybits + 6], unary_n + tail_n]).astype(np.int64)
    starts = np.concatenate([[0], np.cumsum(per_key)[:-1]])
    return words, total, starts[::SUB].astype(np.uint32)


def cpc_decode_segment(words, count, keybits):
    bits = np.unpackbits(words.astype(">u4").view(np.uint8))
    pos = 0

    def take(nb):
        nonlocal pos
        v = 0
        for _ in range(nb):
            v = (v << 1) | int(bits[pos])
            pos += 1
        return v

    keys = [take(keybits)]
    r = take(6)
    for _ in range(count - 1):
        q = 0
        while q < CPC_ESC_Q and bits[pos] == 1:
            q += 1
            pos += 1
        if q == CPC_ESC_Q:
            d = take(keybits)
        else:
            pos += 1  # the terminating zero
            d = (q << r) | take(r)
        keys.append(keys[-1] + d)
    return np.array(keys, np.uint64)


def cpv_encode_segment(vals, vbits):
    """CPC2000 velocity code of one segment: the minimum raw (vbits), the
    6-bit Rice parameter, then every value minus the minimum Rice-coded.
    Returns (words, bits, entry points of values 0, SUB, 2 SUB, ...)."""
    vals = np.asarray(vals, np.uint64)
    mn = vals.min()
    d = vals - mn
    r = rice_parameter(d, vbits)
    q = (d >> np.uint64(r)).astype(np.int64)
    esc = q >= CPC_ESC_Q
    qq = np.where(esc, 0, q)
    unary_v = np.where(esc, np.uint64((1 << CPC_ESC_Q) - 1), (np.uint64(1) << (qq + 1).astype(np.uint64)) - np.uint64(2))
    unary_n = np.where(esc, CPC_ESC_Q, qq + 1)
    tail_v = np.where(esc, d, d & np.uint64((1 << r) - 1))
    tail_n = np.where(esc, vbits, r)
    vals_ = np.empty(2 + 2 * d.size, np.uint64)
    lens = np.empty(2 + 2 * d.size, np.int64)
    vals_[0], lens[0] = mn, vbits
    vals_[1], lens[1] = np.uint64(r), 6
    vals_[2::2], lens[2::2] = unary_v, unary_n
    vals_[3::2], lens[3::2] = tail_v, tail_n
    words, total = pack_fields(vals_, lens)
    per = (unary_n + tail_n).astype(np.int64)
    starts = vbits + 6 + np.concatenate([[0], np.cumsum(per)[:-1]])
    return words, total, starts[::SUB].astype(np.uint32)


def cpv_decode_segment(words, count, vbits):
    """Inverse of cpv_encode_segment, read bit by bit."""
    bits = np.unpackbits(words.astype(">u4").view(np.uint8))
    pos = 0

    def take(nb):
        nonlocal pos
        v = 0
        for _ in range(nb):
            v = (v << 1) | int(bits[pos])
            pos += 1
        return v

    mn = take(vbits)
    r = take(6)
    out = []
    for _ in range(count):
        q = 0
        while q < CPC_ESC_Q and bits[pos] == 1:
            q += 1
            pos += 1
        if q == CPC_ESC_Q:
            d = take(vbits)
        else:
            pos += 1
            d = (q << r) | take(r)
        out.append(mn + d)
    return np.array(out, np.uint64)


# --------------------------------------------------------------- container

MD_MAGIC = b"SZMD"
MD_HDR = 96


CP_FMT = "<4sHBBQIII6f3d3d"


CV_FMT = "<4sHBBQIIIffdd"


def _tables(seg_bits, entries):
    tab = np.array(seg_bits, np.uint32).tobytes()
    tab += b"\0" * (-len(tab) % 8)
    ent = np.concatenate(entries).astype("<u4").tobytes()
    ent += b"\0" * (-len(ent) % 8)
    return tab + ent


def _coord_stream(coords, eb_rel, perm_keys, B, seg):
    """CPC2000 coordinate stream: header, per-segment bit counts, entry
    points, payload."""
    n = perm_keys.size
    keybits = 3 * B
    nseg = (n + seg - 1) // seg
    pr = [params(c, eb_rel) for c in coords]
    seg_words, seg_bits, entries = [], [], []
    for s in range(nseg):
        w, nb, ent = cpc_encode_segment(perm_keys[s * seg:(s + 1) * seg], keybits, with_entries=True)
        seg_words.append(w)
        seg_bits.append(nb)
        entries.append(ent)
    head = struct.pack(CP_FMT, b"SZCP", 2, B, 0, n, nseg, seg, keybits,
                       pr[0]["mn"], pr[0]["mx"], pr[1]["mn"], pr[1]["mx"], pr[2]["mn"], pr[2]["mx"],
                       pr[0]["eb_abs"], pr[1]["eb_abs"], pr[2]["eb_abs"],
                       pr[0]["step"], pr[1]["step"], pr[2]["step"])
    head += b"\0" * (-len(head) % 8)
    body = b"".join(w.astype("<u4").tobytes() for w in seg_words)
    return head + _tables(seg_bits, entries) + body


def _vel_stream(v, eb_rel, perm, seg):
    """CPC2000 velocity stream of one field: header, per-segment bit counts,
    entry points, payload."""
    n = v.size
    pr = params(v, eb_rel)
    vbits = max(int(pr["P"]).bit_length(), 1)
    p = lattice(v, eb_rel).astype(np.uint64)[perm]
    nseg = (n + seg - 1) // seg
    seg_words, seg_bits, entries = [], [], []
    for s in range(nseg):
        w, nb, ent = cpv_encode_segment(p[s * seg:(s + 1) * seg], vbits)
        seg_words.append(w)
        seg_bits.append(nb)
        entries.append(ent)
    head = struct.pack(CV_FMT, b"SZCV", 1, vbits, 0, n, nseg, seg, vbits, pr["mn"], pr["mx"], pr["eb_abs"],
                       pr["step"])
    head += b"\0" * (-len(head) % 8)
    body = b"".join(w.astype("<u4").tobytes() for w in seg_words)
    return head + _tables(seg_bits, entries) + body


def compress_md(fields, eb_rel, md_mode):
    """fields: 3 coordinate arrays, optionally followed by 3 velocity arrays.
    Returns (container bytes, permutation applied to the particles)."""
    fields = [np.ascontiguousarray(f, np.float32) for f in fields]
    nf = len(fields)
    n = fields[0].size
    if nf not in (3, 6) or any(f.size != n for f in fields):
        raise ValueError("3 or 6 equal-length fields")
    kind, seg, k, keysrc = parse_mode(md_mode)
    if keysrc != KEY_COORD and (nf != 6 or kind not in (SPEED, TRADEOFF)):
        raise ValueError("velocity keys need six fields and SZ-LV sub-streams")
    if kind == SPEED and (keysrc or k or seg != SEG):
        raise ValueError("best_speed takes no reordering parameters")
    mode_lv = LV | EB_REL
    if kind == SPEED:
        perm = np.arange(n)
    else:
        if keysrc == KEY_ALL:
            key, B = rindex_keys6(fields, eb_rel)
            digit = 6
        else:
            key, B = rindex_keys(fields[:3] if keysrc == KEY_COORD else fields[3:], eb_rel)
            digit = 3
        if digit * k >= 64:
            raise ValueError("too many ignored digits")
        perm = segment_order(key, k, seg, digit)
    subs = []
    if kind in (COMPRESSION, CPC2000):
        subs.append(_coord_stream(fields[:3], eb_rel, key[perm], B, seg))
        for f in fields[3:]:
            subs.append(compress(f[perm], eb_rel, mode_lv) if kind == COMPRESSION else _vel_stream(f, eb_rel, perm, seg))
    else:
        for f in fields:
            subs.append(compress(f[perm], eb_rel, mode_lv))
    offs, o = [], MD_HDR
    for sb in subs:
        offs.append(o)
        o += len(sb) + (-len(sb) % 8)
    offs += [0] * (6 - len(offs))
    head = struct.pack("<4sHBBQIIQ6QI", MD_MAGIC, 1, kind, nf, n, seg, k, o, *offs, keysrc)
    head += b"\0" * (MD_HDR - len(head))
    body = b"".join(sb + b"\0" * (-len(sb) % 8) for sb in subs)
    return head + body, perm


def decompress_md(blob):
    magic, ver, kind, nf, n, seg, k, total, *rest = struct.unpack_from("<4sHBBQIIQ6QI", blob, 0)
    offs = rest[:6]
    assert magic == MD_MAGIC and ver == 1
    out = []
    nsub = nf if kind not in (COMPRESSION, CPC2000) else nf - 2
    ends = [offs[i + 1] if i + 1 < nsub else total for i in range(nsub)]
    subs = [blob[offs[i]:ends[i]] for i in range(nsub)]
    if kind in (COMPRESSION, CPC2000):
        out += decode_coord_stream(subs[0])
        for sb in subs[1:]:
            out.append(decompress(sb) if kind == COMPRESSION else decode_vel_stream(sb))
    else:
        for sb in subs:
            out.append(decompress(sb))
    return out


def _read_tables(sb, hlen, n, nseg, seg):
    seg_bits = np.frombuffer(sb, np.uint32, count=nseg, offset=hlen)
    o = hlen + 4 * nseg
    o += -o % 8
    counts = [min(seg, n - s * seg) for s in range(nseg)]
    nent = sum(-(-c // SUB) for c in counts)
    entries = np.frombuffer(sb, "<u4", count=nent, offset=o)
    o += 4 * nent
    o += -o % 8
    return seg_bits, counts, entries, o


def decode_coord_stream(sb):
    vals = struct.unpack_from(CP_FMT, sb, 0)
    magic, ver, B, _, n, nseg, seg, keybits = vals[:8]
    mnmx = vals[8:14]
    steps = vals[17:20]
    assert magic == b"SZCP" and ver == 2
    hlen = struct.calcsize(CP_FMT)
    hlen += -hlen % 8
    seg_bits, counts, entries, o = _read_tables(sb, hlen, n, nseg, seg)
    keys = []
    e0 = 0
    for s in range(nseg):
        nw = (int(seg_bits[s]) + 31) // 32
        words = np.frombuffer(sb, "<u4", count=nw, offset=o)
        o += 4 * nw
        cnt = counts[s]
        seg_keys = cpc_decode_segment(words, cnt, keybits)
        # the entry points are where the code of every SUB-th key starts
        _, _, ent = cpc_encode_segment(seg_keys, keybits, with_entries=True)
        assert np.array_equal(ent, entries[e0:e0 + ent.size])
        e0 += ent.size
        keys.append(seg_keys)
    key = np.concatenate(keys)
    ps = deinterleave(key, B)
    # reconstruction x~ = fl32(fma(p, step, mn)) per coordinate
    return [reconstruct_array(ps[c], steps[c], mnmx[2 * c]) for c in range(3)]


def decode_vel_stream(sb):
    magic, ver, vbits, _, n, nseg, seg, vb2, mn, mx, eb_abs, step = struct.unpack_from(CV_FMT, sb, 0)
    assert magic == b"SZCV" and ver == 1 and vb2 == vbits
    hlen = struct.calcsize(CV_FMT)
    hlen += -hlen % 8
    seg_bits, counts, entries, o = _read_tables(sb, hlen, n, nseg, seg)
    ps = []
    e0 = 0
    for s in range(nseg):
        nw = (int(seg_bits[s]) + 31) // 32
        words = np.frombuffer(sb, "<u4", count=nw, offset=o)
        o += 4 * nw
        v = cpv_decode_segment(words, counts[s], vbits)
        _, nb, ent = cpv_encode_segment(v, vbits)
        assert nb == seg_bits[s] and np.array_equal(ent, entries[e0:e0 + ent.size])
        e0 += ent.size
        ps.append(v)
    p = np.concatenate(ps).astype(np.int64)
    return reconstruct_array(p, step, mn)
