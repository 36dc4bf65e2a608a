"""ctypes binding of the CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  It builds ``libsznb_oracle.so`` from ``sznb_oracle.c`` with
gcc (``-O2 -ffp-contract=off``) and exposes numpy-level helpers.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sznb_oracle.c")
_LIB = os.path.join(_HERE, "libsznb_oracle.so")
_lib = None

OK, E_INVAL, E_NONFINITE, E_EBSMALL, E_NOSPC, E_CORRUPT = 0, -1, -2, -3, -4, -5
LV, LCF, BESTFIT, LEARNED = 0, 1, 2, 3
EB_REL = 1 << 4


def block_mode(log2_s: int) -> int:
    return (log2_s & 15) << 8


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
                               "-Wall", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        L.sznbref_compress.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_double, ctypes.c_uint32,
                                       ctypes.POINTER(u8p), ctypes.POINTER(ctypes.c_size_t)]
        L.sznbref_compress_blocks.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_double, ctypes.c_uint32,
                                              ctypes.c_void_p, ctypes.POINTER(u8p), ctypes.POINTER(ctypes.c_size_t)]
        L.sznbref_decompress.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(ctypes.POINTER(ctypes.c_float)),
                                         ctypes.POINTER(ctypes.c_uint64)]
        L.sznbref_free.argtypes = [ctypes.c_void_p]
        L.sznbref_params.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_double, ctypes.c_int, ctypes.c_void_p]
        L.sznbref_lattice.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_double, ctypes.c_int, ctypes.c_void_p]
        L.sznbref_residuals.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p]
        L.sznbref_select.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p]
        L.sznbref_block_cost.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p]
        L.sznbref_log_table.argtypes = [ctypes.c_void_p]
        L.sznbref_res_class.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
        L.sznbref_huffman_lengths.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.sznbref_canonical.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.sznbref_reconstruct.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_float]
        L.sznbref_reconstruct.restype = ctypes.c_float
        L.sznbref_features.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64,
                                       ctypes.c_void_p]
        L.sznbref_mlp_logits.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]
        L.sznbref_bf16.argtypes = [ctypes.c_float]
        L.sznbref_bf16.restype = ctypes.c_float
        L.sznbref_select_learned.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64,
                                             ctypes.c_void_p, ctypes.c_float, ctypes.c_void_p, ctypes.c_void_p]
        L.sznbref_compress_learned.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_double, ctypes.c_uint32,
                                               ctypes.c_void_p, ctypes.c_float, ctypes.c_void_p, ctypes.c_void_p]
        L.sznbref_reconstruct_array.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_double, ctypes.c_float,
                                                ctypes.c_void_p]
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__("oracle status %d" % code)
        self.code = code


def _f32(x) -> np.ndarray:
    return np.ascontiguousarray(x, dtype=np.float32)


def compress(x, eb: float, mode: int = LV | EB_REL, pred=None, selector=None) -> bytes:
    """selector = (1699 float32 parameters, tau) for the learned policy."""
    x = _f32(x)
    L = lib()
    out = ctypes.POINTER(ctypes.c_uint8)()
    n = ctypes.c_size_t(0)
    if selector is not None:
        w = np.ascontiguousarray(selector[0], dtype=np.float32)
        assert w.size == MLP_NPARAM
        st = L.sznbref_compress_learned(x.ctypes.data, x.size, eb, mode, w.ctypes.data, float(selector[1]),
                                        ctypes.byref(out), ctypes.byref(n))
    elif pred is None:
        st = L.sznbref_compress(x.ctypes.data, x.size, eb, mode, ctypes.byref(out), ctypes.byref(n))
    else:
        pred = np.ascontiguousarray(pred, dtype=np.uint8)
        st = L.sznbref_compress_blocks(x.ctypes.data, x.size, eb, mode, pred.ctypes.data,
                                       ctypes.byref(out), ctypes.byref(n))
    if st != OK:
        raise OracleError(st)
    data = ctypes.string_at(out, n.value)
    L.sznbref_free(out)
    return data


MLP_NPARAM = 1699
N_FEATURES = 16


def features(q, S: int, P: int) -> np.ndarray:
    """Selector features of every block of a lattice array: float32 [nb, 16]."""
    q = np.ascontiguousarray(q, dtype=np.int32)
    nb = -(-q.size // S)
    out = np.zeros((nb, N_FEATURES), np.float32)
    lib().sznbref_features(q.ctypes.data, q.size, S, int(P), out.ctypes.data)
    return out


def mlp_logits(w, feat) -> np.ndarray:
    """Bit-faithful bfloat16 inference: float32 logits [nb, 3]."""
    w = np.ascontiguousarray(w, dtype=np.float32)
    feat = np.ascontiguousarray(feat, dtype=np.float32).reshape(-1, N_FEATURES)
    out = np.zeros((feat.shape[0], 3), np.float32)
    lib().sznbref_mlp_logits(w.ctypes.data, feat.ctypes.data, feat.shape[0], out.ctypes.data)
    return out


def bf16(x: float) -> float:
    return float(lib().sznbref_bf16(x))


def select_learned(q, S: int, P: int, w, tau: float):
    """(predictor per block, fallback flag per block) of the learned policy."""
    q = np.ascontiguousarray(q, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.float32)
    nb = -(-q.size // S)
    pred = np.zeros(nb, np.uint8)
    fb = np.zeros(nb, np.uint8)
    lib().sznbref_select_learned(q.ctypes.data, q.size, S, int(P), w.ctypes.data, float(tau),
                                 pred.ctypes.data, fb.ctypes.data)
    return pred, fb


def decompress(stream: bytes) -> np.ndarray:
    L = lib()
    buf = np.frombuffer(stream, dtype=np.uint8)
    out = ctypes.POINTER(ctypes.c_float)()
    n = ctypes.c_uint64(0)
    st = L.sznbref_decompress(buf.ctypes.data, buf.size, ctypes.byref(out), ctypes.byref(n))
    if st != OK:
        raise OracleError(st)
    y = np.ctypeslib.as_array(out, shape=(n.value,)).copy() if n.value else np.zeros(0, np.float32)
    L.sznbref_free(out)
    return y


def params(x, eb: float, eb_rel: bool = True) -> dict:
    x = _f32(x)
    out = np.zeros(8, np.float64)
    st = lib().sznbref_params(x.ctypes.data, x.size, eb, int(eb_rel), out.ctypes.data)
    if st != OK:
        raise OracleError(st)
    keys = ("mn", "mx", "R", "eb_abs", "step", "inv", "P", "is_const")
    return dict(zip(keys, out.tolist()))


def lattice(x, eb: float, eb_rel: bool = True) -> np.ndarray:
    x = _f32(x)
    q = np.zeros(x.size, np.int32)
    st = lib().sznbref_lattice(x.ctypes.data, x.size, eb, int(eb_rel), q.ctypes.data)
    if st != OK:
        raise OracleError(st)
    return q


def residuals(q, S: int, k: int) -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=np.int32)
    r = np.zeros(q.size, np.int32)
    lib().sznbref_residuals(q.ctypes.data, q.size, S, k, r.ctypes.data)
    return r


def select(q, S: int):
    q = np.ascontiguousarray(q, dtype=np.int32)
    nb = (q.size + S - 1) // S
    pred = np.zeros(nb, np.uint8)
    costs = np.zeros((nb, 3), np.uint64)
    lib().sznbref_select(q.ctypes.data, q.size, S, pred.ctypes.data, costs.ctypes.data)
    return pred, costs


def block_cost(q, k: int) -> int:
    q = np.ascontiguousarray(q, dtype=np.int32)
    c = np.zeros(1, np.uint64)
    st = lib().sznbref_block_cost(q.ctypes.data, q.size, k, c.ctypes.data)
    if st != OK:
        raise OracleError(st)
    return int(c[0])


def log_table() -> np.ndarray:
    t = np.zeros(16385, np.uint32)
    lib().sznbref_log_table(t.ctypes.data)
    return t


def res_class(r: int):
    c = ctypes.c_int(0)
    e = ctypes.c_int(0)
    lib().sznbref_res_class(int(r), ctypes.byref(c), ctypes.byref(e))
    return c.value, e.value


def huffman_lengths(freq) -> np.ndarray:
    f = np.zeros(65536, np.uint32)
    freq = np.asarray(freq, dtype=np.uint32)
    f[:freq.size] = freq
    ln = np.zeros(65536, np.uint8)
    lib().sznbref_huffman_lengths(f.ctypes.data, ln.ctypes.data)
    return ln


def canonical(lengths):
    ln = np.ascontiguousarray(lengths, dtype=np.uint8)
    code = np.zeros(65536, np.uint32)
    order = np.zeros(65536, np.uint16)
    m = lib().sznbref_canonical(ln.ctypes.data, code.ctypes.data, order.ctypes.data)
    return code, order[:int((ln > 0).sum())], m


def reconstruct(p: int, step: float, mn: float) -> float:
    return float(lib().sznbref_reconstruct(int(p), step, mn))


def reconstruct_array(p, step: float, mn: float) -> np.ndarray:
    p = np.ascontiguousarray(p, dtype=np.int64)
    out = np.zeros(p.size, np.float32)
    lib().sznbref_reconstruct_array(p.ctypes.data, p.size, step, mn, out.ctypes.data)
    return out


# ------------------------------------------------------------ stream parsing

HEADER_FIELDS = (
    ("magic", 0, "4s"), ("version", 4, "<H"), ("policy", 6, "<B"), ("flags", 7, "<B"),
    ("n", 8, "<Q"), ("S", 16, "<I"), ("nblocks", 20, "<I"), ("mn", 24, "<f"), ("mx", 28, "<f"),
    ("eb_abs", 32, "<d"), ("step", 40, "<d"), ("n_sym", 48, "<3I"), ("max_len", 60, "<3B"),
    ("payload_words", 64, "<Q"), ("total_bytes", 72, "<Q"), ("off_pred", 80, "<Q"),
    ("off_pfirst", 88, "<Q"), ("off_cwords", 96, "<Q"), ("off_nesc", 104, "<Q"),
    ("off_books", 112, "<Q"), ("off_payload", 120, "<Q"),
)


def header(stream: bytes) -> dict:
    import struct
    out = {}
    for k, off, fmt in HEADER_FIELDS:
        v = struct.unpack_from(fmt, stream, off)
        out[k] = v if len(v) > 1 else v[0]
    return out
