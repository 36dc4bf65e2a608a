#!/usr/bin/env python3
"""Benchmark: compress + decompress throughput of a cosmology-like snapshot.

Workload: 2^26 particles x 6 float32 fields (xx yy zz vx vy vz, 1.5 GiB),
20k Poisson halos with Gaussian offsets plus a 30% uniform background in 8^3
spatial-cell order, velocities = halo bulk + thermal; bound eb = 1e-4 x value
range per field; best-fit LV / LCF / QCF predictor per 4096-value block;
one canonical Huffman code per predictor.  Inputs are resident in HBM before
timing starts.

A step compresses the six fields in one batched launch sequence and
decompresses them in another.  `value` is original bytes over the time of a
step (compress + decompress).  The dominant kernel's HBM roofline fraction is
its algorithmic bytes per launch over its average launch duration, measured
with HIP events on the launch stream inside the timed region.  The CPU
oracle is timed on a bounded sample of the same fields on one host core.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "compress+decompress GB/s and ratio at eb=1e-4·range vs oracle; % HBM peak"
PROFILES = os.path.join(ROOT, "profiles")


def algorithmic_bytes(kernel, n_total, comp_bytes):
    """Bytes the method must move per launch of each kernel (see design notes)."""
    return {
        "k_range": 4 * n_total,               # read every value
        "k_quant": 4 * n_total,               # read every value
        "k_pack": 4 * n_total + comp_bytes,   # read every value, write the stream
        "d_decode": comp_bytes + 4 * n_total,  # read the stream, write every value
    }.get(kernel)


def measured_traffic(kernel, tag):
    """HBM bytes per launch of `kernel` from the committed counter passes of
    this workload, or None when they were taken on other library sources."""
    path = os.path.join(PROFILES, "traffic_%s.json" % tag)
    if not os.path.exists(path):
        return None
    from paper_1711_03888_amd.profile_summary import source_hash
    with open(path) as f:
        t = json.load(f)
    if t.get("source_sha256") != source_hash():
        return None
    # the traces name template kernels with their arguments (k_pack<16>)
    keys = [k for k in t.get("kernels", {}) if k == kernel or k.startswith(kernel + "<")]
    if len(keys) != 1:
        return None
    return round(t["kernels"][keys[0]]["bytes"])


def md_modes(dev, eb, reps):
    """The MD modes on the 2M-atom FCC snapshot: GB/s, ratio and HBM
    fraction (enqueued back to back, no host waits inside the timing)."""
    import torch

    from paper_1711_03888_amd import datagen, sznb
    snap = datagen.md_lattice()
    fields = [torch.from_numpy(v).to(dev) for v in snap.values()]
    n = fields[0].numel()
    ws = sznb.workspace(sznb.md_workspace_bytes(3, n), dev)
    out = torch.empty(sznb.md_bound(3, n), dtype=torch.uint8, device=dev)
    outs = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(3)]
    olen = torch.zeros(1, dtype=torch.int64, device=dev)
    res = {}
    for mode, name in ((0, "best_speed"), (1, "best_tradeoff"), (2, "best_compression"), (3, "cpc2000")):
        blob, _ = sznb.md_compress(fields, eb, mode, ws=ws, out=out)
        sznb.md_decompress(blob, 3, n, ws=ws, outs=outs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            sznb.md_compress_async(fields, eb, mode, ws=ws, out=out, olen=olen)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        first, _ = sznb.read_status(ws, 1)
        assert first == sznb.OK and int(olen.item()) == blob.numel(), (name, first)
        for _ in range(reps):
            sznb.md_decompress_async(blob, 3, n, ws=ws, outs=outs)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        first, _ = sznb.read_status(ws, 1)
        assert first == sznb.OK, (name, first)
        c_s, d_s = (t1 - t0) / reps, (t2 - t1) / reps
        # algorithmic bytes: read the fields, write the container; a reordering
        # also reads every field and the key fields once more and writes the
        # reordered fields
        cb = 12.0 * n + blob.numel() + (36.0 * n if mode else 0.0)
        db = 12.0 * n + blob.numel()
        res[name] = {"ratio": round(12.0 * n / blob.numel(), 4),
                     "compress_GBps": round(12.0 * n / c_s / 1e9, 2),
                     "decompress_GBps": round(12.0 * n / d_s / 1e9, 2),
                     "compress_hbm_frac": round(cb / c_s / 1e9 / HBM_PEAK_GBPS, 5),
                     "decompress_hbm_frac": round(db / d_s / 1e9 / HBM_PEAK_GBPS, 5)}
    res["workload"] = "FCC lattice %d atoms x 3 float32 coordinates, eb_rel %g" % (n, eb)
    return res


def learned_section(fields, eb, block_log2, steps, bestfit_ms, bestfit_quant_ms, bestfit_ratio):
    """The learned policy on the same snapshot: compress GB/s, ratio, fallback
    rate, and the quantization kernel's time next to the exhaustive trial's."""
    import torch

    from paper_1711_03888_amd import selector, sznb
    params, tau, rec = selector.load(selector.SELECTORS["nbody"])
    sznb.set_selector(params, tau)
    dev = fields[0].device
    n = fields[0].numel()
    mode = sznb.PRED_LEARNED | sznb.EB_REL | sznb.BLOCK_LOG2(block_log2)
    caps = [sznb.compress_bound(n, mode)] * len(fields)
    outs = [torch.empty(c, dtype=torch.uint8, device=dev) for c in caps]
    lens = torch.zeros(len(fields), dtype=torch.int64, device=dev)
    ws = sznb.workspace(sznb.compress_workspace_bytes([n] * len(fields), [mode] * len(fields)), dev)
    run = lambda: sznb.compress_batch_async(fields, eb, mode, caps=caps, ws=ws, outs=outs, lens=lens)
    run()
    torch.cuda.synchronize()
    sznb.profile(True)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        run()
    b.record()
    torch.cuda.synchronize()
    sznb.profile(False)
    kern = sznb.profile_summary()
    ms = a.elapsed_time(b) / steps
    first, st = sznb.read_status(ws, len(fields))
    if first != sznb.OK:
        raise SystemExit("learned compression failed: %s" % st)
    sizes = [int(v) for v in lens.cpu()]
    fb = sznb.compress_fallbacks(ws, len(fields))
    nblocks = len(fields) * -(-n // (1 << block_log2))
    recon = sznb.decompress_batch([o[:m] for o, m in zip(outs, sizes)], [n] * len(fields))
    for x, y, o in zip(fields, recon, outs):
        eb_abs = sznb.stream_info(bytes(o[:128].cpu().numpy()))["eb_abs"]
        assert (x.double() - y.double()).abs().max().item() <= eb_abs
    ratio = 4.0 * n * len(fields) / sum(sizes)
    qms = kern["k_quant"][0] / kern["k_quant"][1]
    return {"compress_GBps": round(4.0 * n * len(fields) / (ms * 1e-3) / 1e9, 2), "ratio": round(ratio, 4),
            "ratio_vs_exhaustive": round(ratio / bestfit_ratio, 5),
            "speedup_vs_exhaustive": round(bestfit_ms / ms, 3),
            "k_quant_ms": round(qms, 4), "k_quant_ms_exhaustive": round(bestfit_quant_ms, 4),
            "fallback_rate": round(sum(fb) / nblocks, 5), "tau": tau,
            "training": {k: rec.get(k) for k in ("blocks", "label_histogram", "heldout_accuracy", "data")}}


def _gbps(nbytes, ms):
    return round(nbytes / (ms * 1e-3) / 1e9, 2)


def single_call_latency(dev, f0, mode):
    """One eager compression and one eager decompression of one field (host
    call to stream completion), median of 21."""
    import torch

    from paper_1711_03888_amd import sznb
    n = f0.numel()
    cap = sznb.compress_bound(n, mode)
    o1 = torch.empty(cap, dtype=torch.uint8, device=dev)
    l1 = torch.zeros(1, dtype=torch.int64, device=dev)
    ws1 = sznb.workspace(sznb.compress_workspace_bytes([n], [mode]), dev)
    wsd1 = sznb.workspace(sznb.decompress_workspace_bytes([n]), dev)
    r1 = torch.empty(n, dtype=torch.float32, device=dev)

    def eager_c():
        sznb.compress_batch_async([f0], 1e-4, mode, caps=[cap], ws=ws1, outs=[o1], lens=l1)
        torch.cuda.synchronize()
    eager_c()
    s1 = o1[:int(l1.item())]

    def eager_d():
        sznb.decompress_batch_async([s1], [n], outs=[r1], ws=wsd1)
        torch.cuda.synchronize()
    eager_d()
    lat_c = _median_time(eager_c, 21) * 1e3
    lat_d = _median_time(eager_d, 21) * 1e3
    one = 4.0 * n
    return {"compress_ms": round(lat_c, 4), "decompress_ms": round(lat_d, 4),
            "compress_GBps": _gbps(one, lat_c), "decompress_GBps": _gbps(one, lat_d),
            "compress_hbm_frac": round((one + s1.numel()) / (lat_c * 1e-3) / 1e9 / HBM_PEAK_GBPS, 5),
            "decompress_hbm_frac": round((one + s1.numel()) / (lat_d * 1e-3) / 1e9 / HBM_PEAK_GBPS, 5)}


def planned_section(fields, eb, mode, recon, steps, sizes):
    """The same step through plans: the field table and the stream headers
    are prepared once (the decompression plan reads the block and codebook
    sizes at creation), so a step enqueues kernels only, with no header
    read-back between compression and decompression.  Every kernel still
    runs on the step's data; the streams must equal the ordinary path's."""
    import torch

    from paper_1711_03888_amd import sznb
    cp = sznb.CompressPlan(fields, eb, mode)
    cp.launch()
    dp = sznb.DecompressPlan(cp.outs, [f.numel() for f in fields], outs=recon)
    for _ in range(2):
        cp.launch()
        dp.launch()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        ev[i][0].record()
        cp.launch()
        ev[i][1].record()
        dp.launch()
        ev[i][2].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for ws, nf in ((cp.ws, len(fields)), (dp.ws, len(fields))):
        first, st = sznb.read_status(ws, nf)
        if first != sznb.OK:
            raise SystemExit("planned step failed: %s" % st)
    assert [int(v) for v in cp.lens.cpu()] == sizes
    raw = 4.0 * sum(f.numel() for f in fields)
    c_ms = sum(a.elapsed_time(b) for a, b, _ in ev) / steps
    d_ms = sum(b.elapsed_time(c) for _, b, c in ev) / steps
    cp.close()
    dp.close()
    return {"GBps": round(raw / (wall / steps) / 1e9, 2), "ms_per_step": round(wall * 1e3 / steps, 3),
            "compress_GBps": _gbps(raw, c_ms), "decompress_GBps": _gbps(raw, d_ms)}


def config1_steady(dev, walk, reps, single_call=True):
    """256 distinct random-walk fields of 2^20 values (1 GiB), LV, one
    graph-captured batched compression and one graph-captured batched
    decompression; HBM fraction of each on algorithmic bytes."""
    import torch

    from paper_1711_03888_amd import sznb
    from paper_1711_03888_amd import datagen
    n, nf = 1 << 20, 256
    fields = [torch.from_numpy(f).to(dev) for f in datagen.steady_fields(walk, n, nf)]
    mode = sznb.PRED_LV | sznb.EB_REL
    # single-call latency: one eager compression and one eager decompression
    # of one field, from the host call to the stream's completion
    single = single_call_latency(dev, fields[0], mode) if single_call else None
    plan = sznb.CompressPlan(fields, 1e-4, mode)
    side = torch.cuda.Stream()
    # one eager launch under the library's event profiler: per-kernel times
    plan.launch(side)
    side.synchronize()
    sznb.profile(True)
    plan.launch(side)
    side.synchronize()
    sznb.profile(False)
    kern_c = {k: round(v[0], 4) for k, v in sznb.profile_summary().items()}
    plan.capture(side)
    plan.launch(side)
    side.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(side)
    for _ in range(reps):
        plan.launch(side)
    b.record(side)
    side.synchronize()
    c_ms = a.elapsed_time(b) / reps
    first, st = sznb.read_status(plan.ws, nf)
    assert first == sznb.OK, st
    streams = plan.streams()
    comp = sum(s.numel() for s in streams)
    dplan = sznb.DecompressPlan(streams, [n] * nf)
    recon = dplan.outs
    dplan.launch(side)
    side.synchronize()
    sznb.profile(True)
    dplan.launch(side)
    side.synchronize()
    sznb.profile(False)
    kern_d = {k: round(v[0], 4) for k, v in sznb.profile_summary().items()}
    dplan.capture(side)
    a.record(side)
    for _ in range(reps):
        dplan.launch(side)
    b.record(side)
    side.synchronize()
    d_ms = a.elapsed_time(b) / reps
    first, st = sznb.read_status(dplan.ws, nf)
    assert first == sznb.OK, st
    for x, y, o in zip(fields[:4], recon[:4], streams[:4]):
        eb_abs = sznb.stream_info(bytes(o[:128].cpu().numpy()))["eb_abs"]
        assert (x.double() - y.double()).abs().max().item() <= eb_abs
    raw = 4.0 * n * nf
    plan.close()
    dplan.close()
    return {"workload": "256 random-walk fields x 2^20 float32 (1 GiB), LV, eb_rel 1e-4",
            "ratio": round(raw / comp, 3),
            "compress_GBps": _gbps(raw, c_ms), "decompress_GBps": _gbps(raw, d_ms),
            "compress_hbm_frac": round((raw + comp) / (c_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
            "decompress_hbm_frac": round((raw + comp) / (d_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
            "compress_ms": round(c_ms, 4), "decompress_ms": round(d_ms, 4),
            "kernels_ms": {"compress": kern_c, "decompress": kern_d},
            "single_call": single}


def batched_512(dev, walk, cosmo, reps):
    """512 uneven fields (sizes log-uniform in [64K, 16M], eb per field from
    {1e-3, 1e-4, 1e-5}): even fields are slices of a long random walk, odd
    fields slices of the cosmology snapshot; best-fit; autotuned block size
    and grid width; one graph-captured launch against per-field launches."""
    import torch

    from paper_1711_03888_amd import datagen, sznb
    specs, host = datagen.batch_from_sources(walk, cosmo)
    fields = [torch.from_numpy(h).to(dev) for h in host]
    ebs = [sp["eb_rel"] for sp in specs]
    del host
    raw = 4.0 * sum(f.numel() for f in fields)
    policy = sznb.PRED_BESTFIT | sznb.EB_REL
    t0 = time.perf_counter()
    mode, wg = sznb.autotune(fields, ebs, policy)
    tune_s = time.perf_counter() - t0
    sznb.set_workgroups_per_cu(wg)
    try:
        plan = sznb.CompressPlan(fields, ebs, mode)
        side = torch.cuda.Stream()
        plan.capture(side)
        plan.launch(side)
        side.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(side)
        for _ in range(reps):
            plan.launch(side)
        b.record(side)
        side.synchronize()
        g_ms = a.elapsed_time(b) / reps
        first, st = sznb.read_status(plan.ws, len(fields))
        assert first == sznb.OK, st
        comp = sum(s.numel() for s in plan.streams())
        plan.close()
        # the same fields, one compression call (launch sequence) per field
        caps = [sznb.compress_bound(f.numel(), mode) for f in fields]
        outs = [torch.empty(c, dtype=torch.uint8, device=dev) for c in caps]
        ws = sznb.workspace(max(sznb.compress_workspace_bytes([f.numel()], [mode]) for f in fields), dev)
        lens = torch.zeros(1, dtype=torch.int64, device=dev)

        def per_field():
            for f, e, c, o in zip(fields, ebs, caps, outs):
                sznb.compress_batch_async([f], e, mode, caps=[c], outs=[o], ws=ws, lens=lens)
        per_field()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        per_field()
        torch.cuda.synchronize()
        p_ms = (time.perf_counter() - t1) * 1e3
    finally:
        sznb.set_workgroups_per_cu(8)
    return {"workload": "512 fields, %.2f GB, sizes log-uniform in [64K, 16M], eb_rel from {1e-3, 1e-4, 1e-5}, "
                        "best-fit" % (raw / 1e9),
            "autotuned": {"block": 1 << ((mode >> 8) & 15), "workgroups_per_cu": wg, "seconds": round(tune_s, 2)},
            "ratio": round(raw / comp, 3), "graph_compress_GBps": _gbps(raw, g_ms),
            "per_field_compress_GBps": _gbps(raw, p_ms), "speedup": round(p_ms / g_ms, 2),
            "graph_ms": round(g_ms, 3), "per_field_ms": round(p_ms, 3)}


def _median_time(fn, reps):
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return sorted(ts)[len(ts) // 2]


def cpu_baseline(host, eb, mode, m, dev, reps=5):
    """The oracle (compress + decompress) on the first m values of each field:
    median of `reps` runs on one host core, the same with one thread per
    field (the oracle's C calls release the interpreter lock), and the
    256 x 2^20 steady-state workload's field size (one 2^20-value random
    walk, LV).  The GPU's bytes for the same sample must be identical."""
    import concurrent.futures as cf

    import oracle
    import torch

    from paper_1711_03888_amd import datagen, sznb
    sample = [h[:m].copy() for h in host]
    streams = {}

    def one(i):
        s = oracle.compress(sample[i], eb, mode)
        oracle.decompress(s)
        streams[i] = s

    def serial():
        for i in range(len(sample)):
            one(i)
    t1 = _median_time(serial, reps)
    threads = min(len(sample), os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(threads) as ex:
        tp = _median_time(lambda: list(ex.map(one, range(len(sample)))), reps)
    got = sznb.compress_batch([torch.from_numpy(x).to(dev) for x in sample], eb, mode)
    exact = all(bytes(g.cpu().numpy()) == streams[i] for i, g in enumerate(got))
    walk = datagen.random_walk()
    c1mode = sznb.PRED_LV | sznb.EB_REL

    def c1():
        oracle.decompress(oracle.compress(walk, 1e-4, c1mode))
    tc1 = _median_time(c1, reps)
    raw = 4.0 * m * len(sample)
    return {"value": round(raw / t1 / 1e9, 5), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": "first %d values of each of the 6 fields, compress + decompress, median of %d runs "
                      "(%.2fs each)" % (m, reps, t1),
            "all_cores": {"value": round(raw / tp / 1e9, 5), "cores": threads,
                          "how": "one thread per field, median of %d" % reps},
            "steady_state_field": {"value": round(4.0 * walk.size / tc1 / 1e9, 5), "cores": 1,
                                   "sample": "one 2^20-value random walk, LV, eb_rel 1e-4, compress + decompress, "
                                             "median of %d" % reps},
            "host_cores": os.cpu_count(), "gpu_bytes_identical_on_sample": exact}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--particles", type=int, default=1 << 26)
    ap.add_argument("--eb", type=float, default=1e-4)
    ap.add_argument("--block-log2", type=int, default=12)
    ap.add_argument("--policy", default="bestfit", choices=["lv", "lcf", "bestfit"])
    ap.add_argument("--cpu-sample", type=int, default=1 << 23, help="values per field timed on the oracle")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-md", action="store_true", help="skip the MD-mode measurement")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-selector measurement")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the steady-state 256 x 1M and the 512-field batched measurements")
    ap.add_argument("--steady-only", action="store_true",
                    help="only the steady-state 256 x 1M measurement (for profiling it on its own)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU; multi-GPU runs are not part of it "
              "(each GPU would compress its own particles independently)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1711_03888_amd import datagen, sznb

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.steady_only:
        walk = datagen.random_walk(1 << 28, seed=7)
        print(json.dumps({"config1_steady": config1_steady(dev, walk, max(3, args.steps), single_call=False)}))
        return
    t_gen = time.time()
    snap = datagen.cosmology(args.particles, seed=2)
    names = list(datagen.FIELD_NAMES)
    print("generated %d particles in %.1fs" % (args.particles, time.time() - t_gen), file=sys.stderr, flush=True)
    host = [snap[k] for k in names]
    fields = [torch.from_numpy(h).to(dev) for h in host]
    n = args.particles
    n_total = n * len(fields)
    pol = {"lv": sznb.PRED_LV, "lcf": sznb.PRED_LCF, "bestfit": sznb.PRED_BESTFIT}[args.policy]
    mode = pol | sznb.EB_REL | sznb.BLOCK_LOG2(args.block_log2)
    caps = [sznb.compress_bound(n, mode)] * len(fields)
    outs = [torch.empty(c, dtype=torch.uint8, device=dev) for c in caps]
    lens = torch.zeros(len(fields), dtype=torch.int64, device=dev)
    ws_c = sznb.workspace(sznb.compress_workspace_bytes([n] * len(fields), [mode] * len(fields)), dev)
    ws_d = sznb.workspace(sznb.decompress_workspace_bytes([n] * len(fields)), dev)
    recon = [torch.empty(n, dtype=torch.float32, device=dev) for _ in fields]

    def compress():
        sznb.compress_batch_async(fields, args.eb, mode, caps=caps, ws=ws_c, outs=outs, lens=lens)

    def decompress():
        sznb.decompress_batch_async(outs, [n] * len(fields), outs=recon, ws=ws_d)

    for _ in range(args.warmup):
        compress()
        decompress()
    torch.cuda.synchronize()
    first, st = sznb.read_status(ws_c, len(fields))
    if first != sznb.OK:
        raise SystemExit("compression failed: %s" % st)
    first, st = sznb.read_status(ws_d, len(fields))
    if first != sznb.OK:
        raise SystemExit("decompression failed: %s" % st)

    # timed region: HIP events bracket only the kernels with algorithmic
    # bytes (a bracket costs the stream a few microseconds between kernels)
    sznb.profile(True, only=["k_range", "k_quant", "k_pack", "d_decode"])
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record()
        compress()
        ev[i][1].record()
        decompress()
        ev[i][2].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sznb.profile(False)
    kern = sznb.profile_summary()
    c_ms = sum(a.elapsed_time(b) for a, b, _ in ev) / args.steps
    d_ms = sum(b.elapsed_time(c) for _, b, c in ev) / args.steps
    ms_step = wall * 1e3 / args.steps
    # every kernel's duration, from the same number of steps run after the
    # timed region with every launch bracketed
    sznb.profile(True)
    for i in range(args.steps):
        compress()
        decompress()
    torch.cuda.synchronize()
    sznb.profile(False)
    kern_all = sznb.profile_summary()

    # results of the last step
    sizes = [int(v) for v in lens.cpu()]
    comp_bytes = sum(sizes)
    ratio = 4.0 * n_total / comp_bytes
    worst = 0.0
    for f, (x, y, s) in enumerate(zip(fields, recon, outs)):
        eb_abs = sznb.stream_info(bytes(s[:128].cpu().numpy()))["eb_abs"]
        err = (x.double() - y.double()).abs().max().item()
        assert err <= eb_abs, (names[f], err, eb_abs)
        worst = max(worst, err / eb_abs)

    # roofline of the dominant kernel
    dom = max((k for k in kern if algorithmic_bytes(k, n_total, comp_bytes)), key=lambda k: kern[k][0])
    avg_ms = kern[dom][0] / kern[dom][1]
    ach = algorithmic_bytes(dom, n_total, comp_bytes) / (avg_ms * 1e-3) / 1e9
    tag = "cosmology_%d_%s_eb%g_S%d" % (n, args.policy, args.eb, 1 << args.block_log2)
    roof = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBPS, 4), "traffic": measured_traffic(dom, tag),
            "algorithmic_bytes": algorithmic_bytes(dom, n_total, comp_bytes), "avg_launch_ms": round(avg_ms, 4)}

    out = {
        "metric": METRIC,
        "value": round(4.0 * n_total / (ms_step * 1e-3) / 1e9, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "cosmology snapshot, %d particles x 6 float32 fields (halos + background, "
                               "8^3 cell order), eb_rel %g, %s predictor per %d-value block"
                               % (n, args.eb, args.policy, 1 << args.block_log2),
                   "particles": n, "fields": 6, "eb_rel": args.eb, "block": 1 << args.block_log2,
                   "policy": args.policy},
        "compress_GBps": round(4.0 * n_total / (c_ms * 1e-3) / 1e9, 2),
        "decompress_GBps": round(4.0 * n_total / (d_ms * 1e-3) / 1e9, 2),
        "ratio": round(ratio, 4),
        "field_ratios": {k: round(4.0 * n / s, 3) for k, s in zip(names, sizes)},
        "max_err_over_eb": round(worst, 6),
        "roofline": roof,
        "kernels_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in sorted(kern_all.items())},
    }

    out["planned"] = planned_section(fields, args.eb, mode, recon, args.steps, sizes)

    if not args.no_batch:
        walk = datagen.random_walk(1 << 28, seed=7)
        out["config1_steady"] = config1_steady(dev, walk, max(3, args.steps))
        out["batched_512"] = batched_512(dev, walk, snap, max(2, args.steps // 2))
        del walk

    if not args.no_learned and args.policy == "bestfit":
        out["learned_selector"] = learned_section(fields, args.eb, args.block_log2, args.steps, c_ms,
                                                  kern["k_quant"][0] / kern["k_quant"][1], ratio)

    if not args.no_md:
        out["md_modes"] = md_modes(dev, args.eb, 5)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(host, args.eb, mode, min(args.cpu_sample, n), dev)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
