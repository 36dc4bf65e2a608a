"""Rate-distortion and ablation sweeps of the paper's analyses, run on the
GPU path over the synthetic snapshots.

    python -m paper_1711_03888_amd.sweep [--particles N] [--atoms-cells I J K]
                                          [--json PATH] [--reps R]

Sections (each point: ratio, bit-rate 32 / ratio, PSNR = -20 log10(NRMSE),
max error / eb_abs, compress and decompress GB/s of original bytes):

* ``rate_distortion`` -- Sec. 6, Fig. 9: the cosmology snapshot with SZ-LV,
  SZ-LCF and the per-block best fit, and the FCC snapshot in the four MD
  kinds (best_speed = SZ-LV, best_tradeoff = SZ-LV-PRX, best_compression =
  SZ-CPC2000, CPC2000), at eb_rel 1e-2 .. 1e-6;
* ``lcf_vs_lv`` -- Sec. 5.1, Table 3 and Fig. 4: SZ-LCF against SZ-LV per
  field (ratio, NRMSE) at eb_rel 1e-4 on both snapshots;
* ``rx_segments`` -- Sec. 5.2, Table 4: FCC particles fully sorted by
  R-index inside segments of 1K .. 16K, then SZ-LV;
* ``prx_digits`` -- Sec. 5.2, Table 5: segments of 16384, 0, 2, 4, 6, 8
  least significant 3-bit digits ignored;
* ``rindex_variants`` -- Sec. 5.3, Table 6: the cosmology snapshot with
  coordinate-, velocity- and coordinate-and-velocity-based R-index sorting
  (segments of 4096) against SZ-LV and CPC2000, per field and overall.

Every point checks the bound on every value; the byte-exactness of these
configurations against the oracle is covered by the GPU tests.  Error
statistics are computed with torch on the GPU (analysis, not the
compression path).
"""
from __future__ import annotations

import argparse
import json
import math
import struct
import sys

import numpy as np
import torch

from . import datagen, sznb

EBS = (1e-2, 1e-3, 1e-4, 1e-5, 1e-6)
POLICIES = {"SZ-LV": sznb.PRED_LV, "SZ-LCF": sznb.PRED_LCF, "best-fit": sznb.PRED_BESTFIT}
MD_KINDS = {"best_speed (SZ-LV)": sznb.MD_SPEED, "best_tradeoff (SZ-LV-PRX)": sznb.MD_TRADEOFF,
            "best_compression (SZ-CPC2000)": sznb.MD_COMPRESSION, "CPC2000": sznb.MD_CPC2000}


def _timed(fn, reps):
    """Average milliseconds of fn() over reps launches (one warm-up)."""
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def _errors(x, y, eb_abs):
    """(NRMSE, max error / eb_abs) of one field; raises if the bound fails."""
    xd, yd = x.double(), y.double()
    e = (xd - yd).abs()
    emax = e.max().item()
    if emax > eb_abs:
        raise SystemExit("error bound violated: %g > %g" % (emax, eb_abs))
    R = (xd.max() - xd.min()).item()
    nrmse = math.sqrt((e * e).mean().item()) / R if R > 0 else 0.0
    return nrmse, emax / eb_abs


def _psnr(nrmse):
    return math.inf if nrmse == 0 else -20.0 * math.log10(nrmse)


def _eb_abs(stream):
    return sznb.stream_info(bytes(stream[:sznb.HEADER_BYTES].cpu().numpy()))["eb_abs"]


def sz_point(fields, names, eb, policy, reps):
    """Batched SZ compression of the fields (value-range-relative bound)."""
    dev = fields[0].device
    n = fields[0].numel()
    mode = policy | sznb.EB_REL
    caps = [sznb.compress_bound(n, mode)] * len(fields)
    outs = [torch.empty(c, dtype=torch.uint8, device=dev) for c in caps]
    lens = torch.zeros(len(fields), dtype=torch.int64, device=dev)
    ws = sznb.workspace(sznb.compress_workspace_bytes([n] * len(fields), [mode] * len(fields)), dev)
    wsd = sznb.workspace(sznb.decompress_workspace_bytes([n] * len(fields)), dev)
    rec = [torch.empty(n, dtype=torch.float32, device=dev) for _ in fields]
    c_ms = _timed(lambda: sznb.compress_batch_async(fields, eb, mode, caps=caps, ws=ws, outs=outs, lens=lens), reps)
    first, st = sznb.read_status(ws, len(fields))
    if first != sznb.OK:
        raise SystemExit("compression failed at eb %g: %s" % (eb, st))
    d_ms = _timed(lambda: sznb.decompress_batch_async(outs, [n] * len(fields), outs=rec, ws=wsd), reps)
    first, st = sznb.read_status(wsd, len(fields))
    if first != sznb.OK:
        raise SystemExit("decompression failed at eb %g: %s" % (eb, st))
    sizes = [int(v) for v in lens.cpu()]
    per = {}
    for name, x, y, s, size in zip(names, fields, rec, outs, sizes):
        nr, em = _errors(x, y, _eb_abs(s))
        per[name] = {"ratio": round(4.0 * n / size, 3), "nrmse": float("%.4g" % nr), "psnr": round(_psnr(nr), 2),
                     "max_err_over_eb": round(em, 4)}
    raw = 4.0 * n * len(fields)
    ratio = raw / sum(sizes)
    return {"ratio": round(ratio, 3), "bit_rate": round(32.0 / ratio, 3),
            "psnr_mean": round(float(np.mean([p["psnr"] for p in per.values()])), 2),
            "compress_GBps": round(raw / (c_ms * 1e-3) / 1e9, 1), "decompress_GBps": round(raw / (d_ms * 1e-3) / 1e9, 1),
            "fields": per}


def _md_sub_sizes(blob, nf):
    """Byte size of each sub-stream of an MD container (host parse of the
    96-byte header)."""
    h = bytes(blob[:sznb.MD_HEADER_BYTES].cpu().numpy())
    kind, hnf = h[6], h[7]
    total = struct.unpack_from("<Q", h, 24)[0]
    offs = struct.unpack_from("<6Q", h, 32)
    nsub = hnf - 2 if kind >= 2 else hnf
    return [(offs[i + 1] if i + 1 < nsub else total) - offs[i] for i in range(nsub)], kind


def md_point(fields, names, eb, mode, reps):
    """One MD container: per-field and overall ratio (a CPC coordinate
    stream counts for the three coordinates together), errors against the
    reordered input, GB/s."""
    dev = fields[0].device
    nf, n = len(fields), fields[0].numel()
    ws = sznb.workspace(sznb.md_workspace_bytes(nf, n), dev)
    out = torch.empty(sznb.md_bound(nf, n), dtype=torch.uint8, device=dev)
    olen = torch.zeros(1, dtype=torch.int64, device=dev)
    perm = torch.empty(n, dtype=torch.int32, device=dev)
    rec = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(nf)]
    c_ms = _timed(lambda: sznb.md_compress_async(fields, eb, mode, ws=ws, out=out, olen=olen, perm=perm), reps)
    first, _ = sznb.read_status(ws, 1)
    if first != sznb.OK:
        raise SystemExit("MD compression %#x failed at eb %g: %d" % (mode, eb, first))
    blob = out[:int(olen.item())]
    d_ms = _timed(lambda: sznb.md_decompress_async(blob, nf, n, ws=ws, outs=rec), reps)
    first, _ = sznb.read_status(ws, 1)
    if first != sznb.OK:
        raise SystemExit("MD decompression %#x failed at eb %g: %d" % (mode, eb, first))
    sizes, kind = _md_sub_sizes(blob, nf)
    p = perm.long()
    per = {}
    for f, (name, x, y) in enumerate(zip(names, fields, rec)):
        xp = x[p]
        R = (xp.double().max() - xp.double().min()).item()
        nr, em = _errors(xp, y, eb * R)
        if kind >= 2:
            size = sizes[0] / 3.0 if f < 3 else sizes[f - 2]
        else:
            size = sizes[f]
        per[name] = {"ratio": round(4.0 * n / size, 3), "nrmse": float("%.4g" % nr), "psnr": round(_psnr(nr), 2),
                     "max_err_over_eb": round(em, 4)}
    raw = 4.0 * n * nf
    ratio = raw / blob.numel()
    return {"ratio": round(ratio, 3), "bit_rate": round(32.0 / ratio, 3),
            "psnr_mean": round(float(np.mean([q["psnr"] for q in per.values()])), 2),
            "compress_GBps": round(raw / (c_ms * 1e-3) / 1e9, 2), "decompress_GBps": round(raw / (d_ms * 1e-3) / 1e9, 2),
            "fields": per}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--particles", type=int, default=1 << 26, help="cosmology snapshot size")
    ap.add_argument("--atoms-cells", type=int, nargs=3, default=(64, 64, 128), help="FCC cells (4 atoms each)")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--json", default=None)
    ap.add_argument("--sections", default="rate_distortion,lcf_vs_lv,rx_segments,prx_digits,rindex_variants")
    args = ap.parse_args(argv)
    sections = set(args.sections.split(","))
    dev = torch.device("cuda:0")
    cosmo_np = datagen.cosmology(args.particles, seed=2)
    names6 = list(datagen.FIELD_NAMES)
    cosmo = [torch.from_numpy(cosmo_np[k]).to(dev) for k in names6]
    fcc_np = datagen.md_lattice(cells=tuple(args.atoms_cells), seed=3, velocities=True)
    fcc6 = [torch.from_numpy(fcc_np[k]).to(dev) for k in names6]
    fcc3 = fcc6[:3]
    res = {"workloads": {"cosmology": "%d particles x 6 float32 fields (halos + background, 8^3 cell order)"
                                      % args.particles,
                         "fcc": "%d atoms, FCC lattice, 3 coordinates (+ 3 N(0,1) velocity components where noted)"
                                % fcc3[0].numel()}}
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    if "rate_distortion" in sections:
        rd = {"cosmology": {}, "fcc": {}}
        for eb in EBS:
            for pname, pol in POLICIES.items():
                log("rate-distortion cosmology %s eb %g" % (pname, eb))
                rd["cosmology"].setdefault(pname, {})["%g" % eb] = sz_point(cosmo, names6, eb, pol, args.reps)
            for kname, kind in MD_KINDS.items():
                log("rate-distortion fcc %s eb %g" % (kname, eb))
                try:
                    rd["fcc"].setdefault(kname, {})["%g" % eb] = md_point(fcc3, names6[:3], eb, kind, args.reps)
                except SystemExit as e:  # a bound too fine for the 63-bit key
                    rd["fcc"].setdefault(kname, {})["%g" % eb] = {"refused": str(e)}
        res["rate_distortion"] = rd
    if "lcf_vs_lv" in sections:
        lv = {}
        for wname, fields, names in (("cosmology", cosmo, names6), ("fcc", fcc3, names6[:3])):
            for pname in ("SZ-LV", "SZ-LCF"):
                log("lcf vs lv %s %s" % (wname, pname))
                lv.setdefault(wname, {})[pname] = sz_point(fields, names, 1e-4, POLICIES[pname], args.reps)
        res["lcf_vs_lv"] = lv
    if "rx_segments" in sections:
        rx = {"SZ-LV (no sorting)": md_point(fcc3, names6[:3], 1e-4, sznb.MD_SPEED, args.reps)}
        for sl in range(10, 15):
            log("rx segment %d" % (1 << sl))
            rx["RX segment %d" % (1 << sl)] = md_point(fcc3, names6[:3], 1e-4, sznb.md_mode(sznb.MD_TRADEOFF, sl, 0),
                                                       args.reps)
        res["rx_segments"] = rx
    if "prx_digits" in sections:
        prx = {}
        for k in (0, 2, 4, 6, 8):
            log("prx ignored digits %d" % k)
            prx["ignored %d" % k] = md_point(fcc3, names6[:3], 1e-4, sznb.md_mode(sznb.MD_TRADEOFF, 14, k), args.reps)
        res["prx_digits"] = prx
    if "rindex_variants" in sections:
        rv = {"SZ-LV": md_point(cosmo, names6, 1e-4, sznb.MD_SPEED, args.reps),
              "CPC2000": md_point(cosmo, names6, 1e-4, sznb.MD_CPC2000, args.reps)}
        for label, key in (("SZ-LV + coordinate R-index", sznb.MD_KEY_COORD),
                           ("SZ-LV + velocity R-index", sznb.MD_KEY_VEL),
                           ("SZ-LV + coordinate & velocity R-index", sznb.MD_KEY_ALL)):
            log("rindex variant %s" % label)
            rv[label] = md_point(cosmo, names6, 1e-4, sznb.md_mode(sznb.MD_TRADEOFF, 12, 0, key), args.reps)
        res["rindex_variants"] = rv
    text = json.dumps(res)
    if args.json:
        with open(args.json, "w") as f:
            f.write(text)
    print(text)


if __name__ == "__main__":
    main()
