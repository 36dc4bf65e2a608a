"""Evaluation metrics as the paper defines them.

* compression ratio: original size / compressed size (Problem Statement);
  the "Overall" ratio of a snapshot is total original bytes over total
  compressed bytes (this is how the Overall row of Table 6 is formed);
* pointwise absolute error e_i = |x_i - x~_i| and its maximum; the
  value-range-relative bound eb_rel = eb_abs / R (Problem Statement);
* NRMSE = sqrt(sum e_i^2 / N) / R (Problem Statement);
* PSNR = -20 log10(NRMSE) and bit-rate = 32 / ratio (rate-distortion
  discussion of Sec. 6; the printed formula drops the minus sign, the text
  says higher is better);
* compression / decompression rate in bytes of original data per second.
"""
from __future__ import annotations

import math

import numpy as np


def value_range(x) -> float:
    x = np.asarray(x)
    if x.size == 0:
        return 0.0
    return float(np.float64(x.max()) - np.float64(x.min()))


def ratio(n_values: int, compressed_bytes: int, bytes_per_value: int = 4) -> float:
    return (bytes_per_value * n_values) / float(compressed_bytes)


def overall_ratio(original_bytes, compressed_bytes) -> float:
    return float(np.sum(original_bytes)) / float(np.sum(compressed_bytes))


def overall_from_field_ratios(ratios) -> float:
    """Equal-size fields: total original / total compressed = harmonic mean."""
    r = np.asarray(ratios, dtype=np.float64)
    return float(r.size / np.sum(1.0 / r))


def max_abs_error(x, y) -> float:
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return float(np.max(np.abs(x - y))) if x.size else 0.0


def nrmse(x, y) -> float:
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    R = value_range(x)
    if x.size == 0 or R == 0.0:
        return 0.0
    return float(np.sqrt(np.mean((x - y) ** 2)) / R)


def psnr(x, y) -> float:
    e = nrmse(x, y)
    return math.inf if e == 0.0 else -20.0 * math.log10(e)


def bit_rate(r: float) -> float:
    return 32.0 / r


def rate_gbps(n_values: int, seconds: float, bytes_per_value: int = 4) -> float:
    return bytes_per_value * n_values / seconds / 1e9
