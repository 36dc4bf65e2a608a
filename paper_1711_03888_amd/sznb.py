"""Thin ctypes binding of the HIP library ``csrc/libsznb.so``.

Argument marshalling only: device buffers are torch tensors (plumbing for
HBM allocations and the current HIP stream); every step of compression and
decompression runs in the library's kernels.  The library must have been
built (``python -m paper_1711_03888_amd.build``); a missing library raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "csrc", "libsznb.so")

OK, EINVAL, ENONFINITE, EEBTOOSMALL, ENOSPC, ECORRUPT, EDEVICE = 0, -1, -2, -3, -4, -5, -6
PRED_LV, PRED_LCF, PRED_BESTFIT, PRED_LEARNED = 0, 1, 2, 3
EB_REL = 1 << 4
HEADER_BYTES = 128


def BLOCK_LOG2(b: int) -> int:
    return (b & 15) << 8


class SznbError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        super().__init__("sznb error %d (%s)%s" % (code, strerror(code) if _lib else "", (": " + what) if what else ""))
        self.code = code


_lib = None
_u64 = ctypes.c_uint64
_vp = ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("HIP library %s is not built; run python -m paper_1711_03888_amd.build" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        L.sznb_compress_bound.argtypes = [_u64, ctypes.c_uint32]
        L.sznb_compress_bound.restype = _u64
        L.sznb_compress_min_capacity.argtypes = [_u64, ctypes.c_uint32]
        L.sznb_compress_min_capacity.restype = _u64
        L.sznb_compress_workspace_bytes.argtypes = [ctypes.c_int, _vp, _vp]
        L.sznb_compress_workspace_bytes.restype = _u64
        L.sznb_compress.argtypes = [_vp, _u64, ctypes.c_double, ctypes.c_uint32, _vp, _u64, _vp, _vp, _u64, _vp]
        L.sznb_compress_batch.argtypes = [ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _u64, _vp]
        L.sznb_stream_info.argtypes = [_vp, _u64, _vp, _vp, _vp, _vp]
        L.sznb_decompress_workspace_bytes.argtypes = [ctypes.c_int, _vp]
        L.sznb_decompress_workspace_bytes.restype = _u64
        L.sznb_decompress.argtypes = [_vp, _u64, _vp, _u64, _vp, _u64, _vp]
        L.sznb_decompress_batch.argtypes = [ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _u64, _vp]
        L.sznb_decompress_noalloc.argtypes = [_vp, _u64, _vp, _u64, _vp]
        L.sznb_read_status.argtypes = [_vp, ctypes.c_int, _vp, _vp]
        L.sznb_profile.argtypes = [ctypes.c_int]
        L.sznb_profile_summary.argtypes = [ctypes.c_int, _vp, _vp, _vp]
        L.sznb_strerror.argtypes = [ctypes.c_int]
        L.sznb_compress_plan.argtypes = [ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _u64, _vp, _vp]
        L.sznb_decompress_plan.argtypes = [ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _u64, _vp, _vp]
        L.sznb_plan_capture.argtypes = [_vp, _vp]
        L.sznb_plan_launch.argtypes = [_vp, _vp]
        L.sznb_plan_destroy.argtypes = [_vp]
        L.sznb_plan_destroy.restype = None
        L.sznb_set_workgroups_per_cu.argtypes = [ctypes.c_int]
        L.sznb_autotune.argtypes = [ctypes.c_int, _vp, _vp, _vp, ctypes.c_uint32, ctypes.c_char_p, _vp, _vp, _vp]
        L.sznb_set_selector.argtypes = [_vp, ctypes.c_float]
        L.sznb_features_workspace_bytes.argtypes = [ctypes.c_int, _vp, _vp]
        L.sznb_features_workspace_bytes.restype = _u64
        L.sznb_block_features.argtypes = [ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _u64, _vp]
        L.sznb_compress_fallbacks.argtypes = [_vp, ctypes.c_int, _vp, _vp]
        L.sznb_mlp_grad_workspace_bytes.argtypes = [ctypes.c_uint32]
        L.sznb_mlp_grad_workspace_bytes.restype = _u64
        L.sznb_mlp_grad.argtypes = [_vp, _vp, _vp, ctypes.c_uint32, _vp, _vp, _vp, _u64, _vp]
        L.sznb_mlp_adam.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_uint32, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_float, ctypes.c_float, _vp]
        L.sznb_mlp_infer.argtypes = [_vp, _vp, _u64, _vp, _vp, _vp, _vp]
        L.sznb_md_workspace_bytes.argtypes = [ctypes.c_int, _u64]
        L.sznb_md_workspace_bytes.restype = _u64
        L.sznb_md_bound.argtypes = [ctypes.c_int, _u64]
        L.sznb_md_bound.restype = _u64
        L.sznb_md_compress.argtypes = [ctypes.c_int, _vp, _u64, ctypes.c_double, ctypes.c_int, _vp, _u64, _vp, _vp,
                                       _vp, _u64, _vp]
        L.sznb_md_decompress.argtypes = [_vp, _u64, ctypes.c_int, _u64, _vp, _vp, _u64, _vp]
        L.sznb_strerror.restype = ctypes.c_char_p
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().sznb_strerror(code).decode()


def _check(rc: int, what: str = ""):
    if rc != OK:
        raise SznbError(rc, what)


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _arr(ctype, values):
    return (ctype * len(values))(*values)


def compress_bound(n: int, mode: int) -> int:
    return int(lib().sznb_compress_bound(n, mode))


def compress_min_capacity(n: int, mode: int) -> int:
    return int(lib().sznb_compress_min_capacity(n, mode))


def compress_workspace_bytes(ns: Sequence[int], modes: Sequence[int]) -> int:
    return int(lib().sznb_compress_workspace_bytes(len(ns), _arr(_u64, ns), _arr(ctypes.c_uint32, modes)))


def decompress_workspace_bytes(ns: Sequence[int]) -> int:
    return int(lib().sznb_decompress_workspace_bytes(len(ns), _arr(_u64, ns)))


def workspace(nbytes: int, device=None) -> torch.Tensor:
    """Device workspace (the library clears what it needs on every call)."""
    return torch.zeros(max(nbytes, 256), dtype=torch.uint8, device=device or "cuda")


def _field(x: torch.Tensor) -> torch.Tensor:
    if x.dtype != torch.float32 or not x.is_cuda or x.dim() != 1 or not x.is_contiguous():
        raise ValueError("field must be a contiguous 1D float32 CUDA tensor")
    return x


class Compressed:
    """Device-resident compressed streams and their lengths (device words)."""

    def __init__(self, bufs, lens, ws):
        self.bufs = bufs
        self.lens = lens
        self.ws = ws

    def sizes(self):
        return [int(v) for v in self.lens.cpu()]

    def streams(self):
        return [b[:n] for b, n in zip(self.bufs, self.sizes())]


def compress_batch_async(fields: Sequence[torch.Tensor], eb, mode, *, caps=None, ws=None, outs=None,
                         lens=None, stream=None) -> Compressed:
    """Enqueue compression of several fields in one launch sequence."""
    fields = [_field(x) for x in fields]
    nf = len(fields)
    ebs = list(eb) if isinstance(eb, (list, tuple)) else [float(eb)] * nf
    modes = list(mode) if isinstance(mode, (list, tuple)) else [int(mode)] * nf
    ns = [x.numel() for x in fields]
    if caps is None:
        caps = [compress_bound(n, m) for n, m in zip(ns, modes)]
    if outs is None:
        outs = [torch.empty(c, dtype=torch.uint8, device=x.device) for c, x in zip(caps, fields)]
    if lens is None:
        lens = torch.zeros(nf, dtype=torch.int64, device=fields[0].device)
    wsb = compress_workspace_bytes(ns, modes)
    if ws is None or ws.numel() < wsb:
        ws = workspace(wsb, fields[0].device)
    rc = lib().sznb_compress_batch(nf, _arr(_vp, [x.data_ptr() for x in fields]), _arr(_u64, ns),
                                   _arr(ctypes.c_double, ebs), _arr(ctypes.c_uint32, modes),
                                   _arr(_vp, [o.data_ptr() for o in outs]), _arr(_u64, caps),
                                   lens.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream))
    _check(rc, "compress")
    return Compressed(outs, lens, ws)


def read_status(ws: torch.Tensor, nf: int, stream=None):
    st = (ctypes.c_int * nf)()
    first = lib().sznb_read_status(ws.data_ptr(), nf, st, _stream(stream))
    return first, list(st)


def compress_batch(fields, eb, mode, **kw):
    c = compress_batch_async(fields, eb, mode, **kw)
    first, st = read_status(c.ws, len(fields))
    if first != OK:
        raise SznbError(first, "device status %s" % st)
    return c.streams()


def compress(x: torch.Tensor, eb: float, mode: int = PRED_LV | EB_REL, **kw) -> torch.Tensor:
    return compress_batch([x], eb, mode, **kw)[0]


def stream_info(header: bytes):
    n = ctypes.c_uint64(0)
    m = ctypes.c_uint32(0)
    e = ctypes.c_double(0)
    t = ctypes.c_uint64(0)
    buf = ctypes.create_string_buffer(bytes(header[:HEADER_BYTES]), HEADER_BYTES)
    _check(lib().sznb_stream_info(buf, HEADER_BYTES, ctypes.byref(n), ctypes.byref(m), ctypes.byref(e),
                                  ctypes.byref(t)), "stream_info")
    return {"n": n.value, "mode": m.value, "eb_abs": e.value, "total_bytes": t.value}


def decompress_batch_async(streams: Sequence[torch.Tensor], ns: Sequence[int], *, outs=None, ws=None, stream=None):
    nf = len(streams)
    for s in streams:
        if s.dtype != torch.uint8 or not s.is_cuda or not s.is_contiguous():
            raise ValueError("streams must be contiguous uint8 CUDA tensors")
    if outs is None:
        outs = [torch.empty(n, dtype=torch.float32, device=s.device) for n, s in zip(ns, streams)]
    wsb = decompress_workspace_bytes(ns)
    if ws is None or ws.numel() < wsb:
        ws = workspace(wsb, streams[0].device)
    rc = lib().sznb_decompress_batch(nf, _arr(_vp, [s.data_ptr() for s in streams]),
                                     _arr(_u64, [s.numel() for s in streams]),
                                     _arr(_vp, [o.data_ptr() for o in outs]), _arr(_u64, list(ns)),
                                     ws.data_ptr(), ws.numel(), _stream(stream))
    _check(rc, "decompress")
    return outs, ws


def decompress_noalloc(s: torch.Tensor, n: int, *, out=None, stream=None) -> torch.Tensor:
    """sznb_decompress_noalloc: decompression into `out` with the library's
    fixed per-GPU workspace (waits for the stream, raises on a bad status)."""
    if s.dtype != torch.uint8 or not s.is_cuda or not s.is_contiguous():
        raise ValueError("stream must be a contiguous uint8 CUDA tensor")
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=s.device)
    _check(lib().sznb_decompress_noalloc(s.data_ptr(), s.numel(), out.data_ptr(), int(n), _stream(stream)),
           "decompress_noalloc")
    return out


def decompress_batch(streams, ns=None, **kw):
    if ns is None:
        ns = [stream_info(bytes(s[:HEADER_BYTES].cpu().numpy()))["n"] for s in streams]
    outs, ws = decompress_batch_async(streams, ns, **kw)
    first, st = read_status(ws, len(streams))
    if first != OK:
        raise SznbError(first, "device status %s" % st)
    return outs


def decompress(s: torch.Tensor, n: int | None = None, **kw) -> torch.Tensor:
    return decompress_batch([s], None if n is None else [n], **kw)[0]


def profile(enable: bool, only=None) -> None:
    """Bracket every later kernel launch with HIP events (or stop); `only`:
    the kernel names to bracket (each bracket costs the stream a few
    microseconds between kernels), None for every kernel."""
    if enable:
        lib().sznb_profile_kernels(ctypes.c_char_p(",".join(only).encode() if only else None))
    lib().sznb_profile(1 if enable else 0)


def profile_summary(max_kernels: int = 64):
    """{kernel: (total_ms, launches)} of the launches recorded since profile(True)."""
    names = ctypes.create_string_buffer(32 * max_kernels)
    tot = (ctypes.c_double * max_kernels)()
    cnt = (ctypes.c_int * max_kernels)()
    nk = lib().sznb_profile_summary(max_kernels, names, tot, cnt)
    if nk < 0:
        raise SznbError(nk, "profile_summary")
    out = {}
    for i in range(min(nk, max_kernels)):
        nm = names.raw[32 * i:32 * i + 32].split(b"\0", 1)[0].decode()
        out[nm] = (tot[i], cnt[i])
    return out


# ------------------------------------------------ molecular-dynamics modes

MD_SPEED, MD_TRADEOFF, MD_COMPRESSION, MD_CPC2000 = 0, 1, 2, 3
MD_KEY_COORD, MD_KEY_VEL, MD_KEY_ALL = 0, 1, 2
MD_HEADER_BYTES = 96


def md_workspace_bytes(nf: int, n: int) -> int:
    return int(lib().sznb_md_workspace_bytes(nf, n))


def md_bound(nf: int, n: int) -> int:
    return int(lib().sznb_md_bound(nf, n))


def md_mode(kind: int, seg_log2: int | None = None, ignored: int | None = None, key: int = 0) -> int:
    """MD mode word: kind (MD_SPEED .. MD_CPC2000), segment 2^seg_log2
    (10..14, default 14), ignored digits (default 6 for MD_TRADEOFF, else
    0), key fields (MD_KEY_COORD, MD_KEY_VEL, MD_KEY_ALL)."""
    m = kind
    if seg_log2 is not None:
        m |= seg_log2 << 8
    if ignored is not None:
        m |= (ignored + 1) << 12
    return m | (key << 16)


def md_compress_async(fields: Sequence[torch.Tensor], eb_rel: float, mode: int, *, ws=None, out=None, olen=None,
                      perm=None, stream=None):
    """Enqueues an MD compression (x, y, z[, vx, vy, vz]); returns (out,
    device length word, workspace).  The status is read with
    read_status(ws, 1)."""
    fields = [_field(f) for f in fields]
    nf, n = len(fields), fields[0].numel()
    if any(f.numel() != n for f in fields):
        raise ValueError("fields must have equal length")
    dev = fields[0].device
    wsb = md_workspace_bytes(nf, n)
    if ws is None or ws.numel() < wsb:
        ws = workspace(wsb, dev)
    if out is None:
        out = torch.empty(md_bound(nf, n), dtype=torch.uint8, device=dev)
    if olen is None:
        olen = torch.zeros(1, dtype=torch.int64, device=dev)
    rc = lib().sznb_md_compress(nf, _arr(_vp, [f.data_ptr() for f in fields]), n, float(eb_rel), int(mode),
                                out.data_ptr(), out.numel(), olen.data_ptr(),
                                perm.data_ptr() if perm is not None else None, ws.data_ptr(), ws.numel(),
                                _stream(stream))
    _check(rc, "md_compress")
    return out, olen, ws


def md_compress(fields: Sequence[torch.Tensor], eb_rel: float, md_mode: int, *, ws=None, out=None,
                want_perm: bool = False, stream=None):
    """Container of an MD snapshot; returns (bytes tensor, permutation or
    None).  Waits for the stream and raises on a device error."""
    n = fields[0].numel()
    perm = torch.empty(n, dtype=torch.int32, device=fields[0].device) if want_perm else None
    out, olen, ws = md_compress_async(fields, eb_rel, md_mode, ws=ws, out=out, perm=perm, stream=stream)
    first, _ = read_status(ws, 1, stream)
    _check(first, "md_compress")
    return out[:int(olen.item())], perm


def md_decompress_async(blob: torch.Tensor, nf: int, n: int, *, ws=None, outs=None, stream=None):
    """Enqueues an MD decompression; returns (outputs, workspace)."""
    if blob.dtype != torch.uint8 or not blob.is_cuda or not blob.is_contiguous():
        raise ValueError("container must be a contiguous uint8 CUDA tensor")
    dev = blob.device
    wsb = md_workspace_bytes(nf, n)
    if ws is None or ws.numel() < wsb:
        ws = workspace(wsb, dev)
    if outs is None:
        outs = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(nf)]
    rc = lib().sznb_md_decompress(blob.data_ptr(), blob.numel(), nf, n, _arr(_vp, [o.data_ptr() for o in outs]),
                                  ws.data_ptr(), ws.numel(), _stream(stream))
    _check(rc, "md_decompress")
    return outs, ws


def md_decompress(blob: torch.Tensor, nf: int, n: int, *, ws=None, outs=None, stream=None):
    """The particles of an MD container (in its stored order); waits for
    the stream and raises on a device error."""
    outs, ws = md_decompress_async(blob, nf, n, ws=ws, outs=outs, stream=stream)
    first, _ = read_status(ws, 1, stream)
    _check(first, "md_decompress")
    return outs


# ------------------------------------------------------- learned selector

MLP_PARAMS = 1699
N_FEATURES = 16


def set_selector(params, tau: float) -> None:
    """Load the selector of the learned policy on the current device."""
    import numpy as np
    w = np.ascontiguousarray(params, dtype=np.float32)
    if w.size != MLP_PARAMS:
        raise ValueError("selector needs %d parameters" % MLP_PARAMS)
    _check(lib().sznb_set_selector(w.ctypes.data, float(tau)), "set_selector")


def block_features(fields: Sequence[torch.Tensor], eb, mode, *, ws=None, stream=None):
    """(features float32 [blocks, 16], trial costs int64 [blocks, 3], trial
    choice uint8 [blocks]) of every block of the fields, in field order."""
    fields = [_field(f) for f in fields]
    nf = len(fields)
    ebs = [float(eb)] * nf if not isinstance(eb, (list, tuple)) else [float(e) for e in eb]
    modes = [int(mode)] * nf if not isinstance(mode, (list, tuple)) else [int(m) for m in mode]
    ns = [f.numel() for f in fields]
    S = 1 << (((modes[0] >> 8) & 15) or 12)
    nb = sum(-(-n // S) for n in ns)
    dev = fields[0].device
    wsb = int(lib().sznb_features_workspace_bytes(nf, _arr(_u64, ns), _arr(ctypes.c_uint32, modes)))
    if ws is None or ws.numel() < wsb:
        ws = workspace(wsb, dev)
    feat = torch.empty((max(nb, 1), N_FEATURES), dtype=torch.float32, device=dev)
    cost = torch.empty((max(nb, 1), 3), dtype=torch.int64, device=dev)
    label = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev)
    rc = lib().sznb_block_features(nf, _arr(_vp, [f.data_ptr() for f in fields]), _arr(_u64, ns),
                                   _arr(ctypes.c_double, ebs), _arr(ctypes.c_uint32, modes), feat.data_ptr(),
                                   cost.data_ptr(), label.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream))
    _check(rc, "block_features")
    return feat[:nb], cost[:nb], label[:nb]


def compress_fallbacks(ws: torch.Tensor, nf: int, stream=None):
    out = (ctypes.c_uint32 * nf)()
    _check(lib().sznb_compress_fallbacks(ws.data_ptr(), nf, out, _stream(stream)), "compress_fallbacks")
    return list(out)


def mlp_grad(params: torch.Tensor, feat: torch.Tensor, label: torch.Tensor, *, ws=None, grad=None, loss=None,
             stream=None):
    B = feat.shape[0]
    dev = params.device
    wsb = int(lib().sznb_mlp_grad_workspace_bytes(B))
    if ws is None or ws.numel() < wsb:
        ws = workspace(wsb, dev)
    if grad is None:
        grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=dev)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=dev)
    rc = lib().sznb_mlp_grad(params.data_ptr(), feat.data_ptr(), label.data_ptr(), B, grad.data_ptr(),
                             loss.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream))
    _check(rc, "mlp_grad")
    return grad, loss, ws


def mlp_adam(params, m, v, grad, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    rc = lib().sznb_mlp_adam(params.data_ptr(), m.data_ptr(), v.data_ptr(), grad.data_ptr(), int(step), float(lr),
                             float(beta1), float(beta2), float(eps), _stream(stream))
    _check(rc, "mlp_adam")


def mlp_infer(params: torch.Tensor, feat: torch.Tensor, stream=None):
    nb = feat.shape[0]
    dev = feat.device
    logits = torch.empty((max(nb, 1), 3), dtype=torch.float32, device=dev)
    choice = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev)
    margin = torch.empty(max(nb, 1), dtype=torch.float32, device=dev)
    rc = lib().sznb_mlp_infer(params.data_ptr(), feat.data_ptr(), nb, logits.data_ptr(), choice.data_ptr(),
                              margin.data_ptr(), _stream(stream))
    _check(rc, "mlp_infer")
    return logits[:nb], choice[:nb], margin[:nb]


# ----------------------------------------------------------------- plans

class CompressPlan:
    """A field table prepared once; launch() enqueues only kernels, capture()
    records them into a HIP graph that later launches replay.  The input
    tensors may change in place between launches."""

    def __init__(self, fields: Sequence[torch.Tensor], eb, mode, *, stream=None):
        self.fields = [_field(x) for x in fields]
        nf = len(self.fields)
        self.ebs = list(eb) if isinstance(eb, (list, tuple)) else [float(eb)] * nf
        self.modes = list(mode) if isinstance(mode, (list, tuple)) else [int(mode)] * nf
        self.ns = [x.numel() for x in self.fields]
        dev = self.fields[0].device
        self.caps = [compress_bound(n, m) for n, m in zip(self.ns, self.modes)]
        self.outs = [torch.empty(c, dtype=torch.uint8, device=dev) for c in self.caps]
        self.lens = torch.zeros(nf, dtype=torch.int64, device=dev)
        self.ws = workspace(compress_workspace_bytes(self.ns, self.modes), dev)
        self._p = ctypes.c_void_p()
        rc = lib().sznb_compress_plan(nf, _arr(_vp, [x.data_ptr() for x in self.fields]), _arr(_u64, self.ns),
                                      _arr(ctypes.c_double, self.ebs), _arr(ctypes.c_uint32, self.modes),
                                      _arr(_vp, [o.data_ptr() for o in self.outs]), _arr(_u64, self.caps),
                                      self.lens.data_ptr(), self.ws.data_ptr(), self.ws.numel(), _stream(stream),
                                      ctypes.byref(self._p))
        _check(rc, "compress_plan")

    def capture(self, stream):
        _check(lib().sznb_plan_capture(self._p, _stream(stream)), "plan_capture")

    def launch(self, stream=None):
        _check(lib().sznb_plan_launch(self._p, _stream(stream)), "plan_launch")

    def streams(self):
        return [b[:int(v)] for b, v in zip(self.outs, self.lens.cpu())]

    def close(self):
        if self._p:
            lib().sznb_plan_destroy(self._p)
            self._p = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DecompressPlan:
    """Streams (device uint8 tensors) laid out once for decoding; launch()
    enqueues only kernels and capture() records them into a HIP graph."""

    def __init__(self, streams: Sequence[torch.Tensor], ns: Sequence[int], *, outs=None, stream=None):
        self.streams = list(streams)
        self.ns = list(ns)
        dev = self.streams[0].device
        self.outs = outs if outs is not None else [torch.empty(n, dtype=torch.float32, device=dev) for n in self.ns]
        self.ws = workspace(decompress_workspace_bytes(self.ns), dev)
        self._p = ctypes.c_void_p()
        rc = lib().sznb_decompress_plan(len(self.streams), _arr(_vp, [s.data_ptr() for s in self.streams]),
                                        _arr(_u64, [s.numel() for s in self.streams]),
                                        _arr(_vp, [o.data_ptr() for o in self.outs]), _arr(_u64, self.ns),
                                        self.ws.data_ptr(), self.ws.numel(), _stream(stream), ctypes.byref(self._p))
        _check(rc, "decompress_plan")

    def capture(self, stream):
        _check(lib().sznb_plan_capture(self._p, _stream(stream)), "plan_capture")

    def launch(self, stream=None):
        _check(lib().sznb_plan_launch(self._p, _stream(stream)), "plan_launch")

    def close(self):
        if self._p:
            lib().sznb_plan_destroy(self._p)
            self._p = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def set_workgroups_per_cu(wg: int) -> None:
    _check(lib().sznb_set_workgroups_per_cu(int(wg)), "set_workgroups_per_cu")


def autotune(fields: Sequence[torch.Tensor], eb, policy_mode: int, cache_path=None, stream=None):
    """(mode with the chosen block size, workgroups per CU) for these fields."""
    fields = [_field(x) for x in fields]
    nf = len(fields)
    ebs = list(eb) if isinstance(eb, (list, tuple)) else [float(eb)] * nf
    mode = ctypes.c_uint32(0)
    wg = ctypes.c_int(0)
    rc = lib().sznb_autotune(nf, _arr(_vp, [x.data_ptr() for x in fields]), _arr(_u64, [x.numel() for x in fields]),
                             _arr(ctypes.c_double, ebs), int(policy_mode),
                             None if cache_path is None else str(cache_path).encode(), ctypes.byref(mode),
                             ctypes.byref(wg), _stream(stream))
    _check(rc, "autotune")
    return int(mode.value), int(wg.value)
