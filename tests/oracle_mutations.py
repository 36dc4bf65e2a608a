"""Mutation check of the oracle's pins (CPU only; not collected by pytest).

Each entry plants one plausible mistake in a copy of the oracle (a dropped
term, a wrong sign or index, a changed tie rule or rounding) and runs the
oracle's CPU pins against the copy.  Every mutation must make at least one
pin fail; the script prints which pin caught it and exits non-zero if any
mutation survives.

    python tests/oracle_mutations.py [name ...]
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = ["tests/test_oracle_pins.py", "tests/test_selector_oracle.py", "tests/test_md_oracle.py"]

# (name, file under oracle/, text, replacement)
MUTATIONS = [
    ("lattice rounds down", "sznb_oracle.c",
     "return (int32_t)floor(t + 0.5);", "return (int32_t)floor(t);"),
    ("guard dropped", "sznb_oracle.c",
     "double g = 2.0 * ulp_f32(am);", "double g = 0.0;"),
    ("reconstruction without fma", "sznb_oracle.c",
     "return (float)fma((double)pi, p->step, (double)p->mn);",
     "return (float)((double)pi * p->step + (double)p->mn);"),
    ("relative bound not scaled by R", "sznb_oracle.c",
     "    p.eb_abs = eb_rel ? eb * p.R : eb;\n    float am", "    p.eb_abs = eb;\n    float am"),
    ("LCF sign", "sznb_oracle.c",
     "else if (k == 1) pred = 2 * d1 - d2;", "else if (k == 1) pred = 2 * d1 + d2;"),
    ("QCF coefficient", "sznb_oracle.c",
     "else pred = 3 * d1 - 3 * d2 + d3;", "else pred = 3 * d1 - 2 * d2 + d3;"),
    ("QCF drops the third term", "sznb_oracle.c",
     "else pred = 3 * d1 - 3 * d2 + d3;", "else pred = 3 * d1 - 3 * d2;"),
    ("warm-up anchors on zero", "sznb_oracle.c",
     "int64_t d1 = j >= 1 ? (int64_t)q[j - 1] - q[0] : 0;", "int64_t d1 = j >= 1 ? (int64_t)q[j - 1] - q[0] : -q[0];"),
    ("LOG table truncated", "sznb_oracle.c",
     "floor(65536.0 * log2((double)m) + 0.5)", "floor(65536.0 * log2((double)m))"),
    ("residual class boundary", "sznb_oracle.c",
     "if (z < 4) { *cls = (int)z; *extra = 0; return; }", "if (z < 8) { *cls = (int)z; *extra = 0; return; }"),
    ("escape without extra bits", "sznb_oracle.c",
     "{ *cls = 32; *extra = 32; return; }", "{ *cls = 32; *extra = 0; return; }"),
    ("selection ties to the highest", "sznb_oracle.c",
     "if (costs[k] < costs[best]) best = k;", "if (costs[k] <= costs[best]) best = k;"),
    ("Huffman ties take the merged node", "sznb_oracle.c",
     "else take_leaf = L[lp].w <= iw[ip];", "else take_leaf = L[lp].w < iw[ip];"),
    ("halving rounds down", "sznb_oracle.c",
     "w[s] = (w[s] + 1) >> 1;", "w[s] = w[s] >> 1;"),
    ("canonical code without shift", "sznb_oracle.c",
     "if (i > 0) c = (c + 1) << (len[order[i]] - len[order[i - 1]]);", "if (i > 0) c = (c + 1);"),
    ("bits packed LSB first", "sznb_oracle.c",
     "if (bit) b->w[pos >> 5] |= 1u << (31 - (pos & 31));", "if (bit) b->w[pos >> 5] |= 1u << (pos & 31);"),
    ("feature 3 sums |Dp|", "sznb_oracle.c", "s1 += a1; s2 += a2;", "s1 += a1; s2 += a1;"),
    ("feature 9 strict", "sznb_oracle.c", "if (a2 <= 1) o2++;", "if (a2 < 1) o2++;"),
    ("feature 11 sums |Dp|", "sznb_oracle.c", "b1 += bitlen32(a1);", "b1 += a1;"),
    ("feature 12 reads Dp", "sznb_oracle.c", "b2 += bitlen32(a2);", "b2 += bitlen32(a1);"),
    ("feature 13 strict", "sznb_oracle.c", "if (a1 >= RADIUS) esc++;", "if (a1 > RADIUS) esc++;"),
    ("sign change counts zeros", "sznb_oracle.c",
     "if ((d1 > 0 && prev < 0) || (d1 < 0 && prev > 0)) sc++;", "if ((d1 >= 0 && prev < 0) || (d1 < 0 && prev >= 0)) sc++;"),
    ("bfloat16 ties away from zero", "sznb_oracle.c",
     "u += 0x7fffu + ((u >> 16) & 1u);", "u += 0x8000u;"),
    ("weights not rounded to bfloat16", "sznb_oracle.c",
     "acc = fmaf(bf16_round(W1[16 * j + k]), x[k], acc);", "acc = fmaf(W1[16 * j + k], x[k], acc);"),
    ("hidden outputs not rounded", "sznb_oracle.c",
     "h2[j] = bf16_round(acc > 0.0f ? acc : 0.0f);", "h2[j] = acc > 0.0f ? acc : 0.0f;"),
    ("fallback on equal margin", "sznb_oracle.c", "if (!(margin >= tau)) {", "if (!(margin > tau)) {"),
    ("decoder adds the residual with the wrong sign", "sznb_oracle.c",
     "int64_t d0 = pred + r[j];", "int64_t d0 = pred - r[j];"),
    ("decoder skips escapes", "sznb_oracle.c",
     "r[j] = (int32_t)get_u32(s, base + 4 * (cwn + esc));", "r[j] = 0;"),
    ("loss summed", "mlp.py",
     "return float(np.mean(lse - z3[np.arange(len(y)), y]))", "return float(np.sum(lse - z3[np.arange(len(y)), y]))"),
    ("loss and gradient summed", "mlp.py", "dz3 /= B\n", "dz3 /= 1\n"),
    ("gradient ignores ReLU", "mlp.py", "dz2 = dh2 * (z2 > 0)", "dz2 = dh2"),
    ("Adam bias correction by beta", "mlp.py",
     "mh = m / (1.0 - beta1 ** step)", "mh = m / (1.0 - beta1)"),
    ("Adam second moment uncorrected", "mlp.py", "vh = v / (1.0 - beta2 ** step)", "vh = v"),
    ("R-index z bit highest", "md.py",
     "key |= bit << np.uint64(3 * j + (2 - c))", "key |= bit << np.uint64(3 * j + c)"),
    ("PRX ignores bits, not digits", "md.py", "sk = key >> np.uint64(3 * k)", "sk = key >> np.uint64(k)"),
    ("six-field key keeps the low bits", "md.py",
     "lattice(f, eb_rel).astype(np.uint64) >> np.uint64(max(0, w - D))",
     "lattice(f, eb_rel).astype(np.uint64) & np.uint64((1 << D) - 1)"),
    ("six-field key with the vz bit highest", "md.py",
     "key |= bit << np.uint64(6 * j + (5 - c))", "key |= bit << np.uint64(6 * j + c)"),
    ("velocity values coded without the minimum", "md.py", "    d = vals - mn\n", "    d = vals\n"),
    ("velocity entry points ignore the segment header", "md.py",
     "starts = vbits + 6 + np.concatenate", "starts = np.concatenate"),
    ("segments of the default size only", "md.py",
     "        perm = segment_order(key, k, seg, digit)", "        perm = segment_order(key, k, SEG, digit)"),
    ("Rice ties to the larger parameter", "md.py",
     "if best_cost is None or cost < best_cost:", "if best_cost is None or cost <= best_cost:"),
    ("Rice cost without the stop bit", "md.py",
     "q.astype(np.int64) + 1 + r).sum())", "q.astype(np.int64) + r).sum())"),
]


def run(mut) -> tuple[bool, str]:
    name, fname, old, new = mut
    tmp = tempfile.mkdtemp(prefix="sznb_mut_")
    try:
        for d in ("oracle", "tests", "paper_1711_03888_amd"):
            shutil.copytree(os.path.join(ROOT, d), os.path.join(tmp, d),
                            ignore=shutil.ignore_patterns("*.so", "_build", "__pycache__", "csrc"))
        shutil.copy(os.path.join(ROOT, "pytest.ini"), tmp)
        path = os.path.join(tmp, "oracle", fname)
        src = open(path).read()
        if src.count(old) < 1:
            return False, "mutation text not found"
        open(path, "w").write(src.replace(old, new, 1))
        r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider"]
                           + PINS, cwd=tmp, capture_output=True, text=True, timeout=900)
        if r.returncode == 0:
            return False, "survived"
        failed = [ln.split(" ")[1] for ln in r.stdout.splitlines() if ln.startswith("FAILED ")]
        return True, failed[0] if failed else "error: " + r.stdout.strip().splitlines()[-1]
    finally:
        shutil.rmtree(tmp, ignore_errors=True)


def main(argv):
    muts = [m for m in MUTATIONS if not argv or m[0] in argv]
    bad = 0
    for m in muts:
        caught, why = run(m)
        bad += not caught
        print("%-38s %s  %s" % (m[0], "caught  " if caught else "SURVIVED", why), flush=True)
    print("%d of %d mutations caught" % (len(muts) - bad, len(muts)))
    return 1 if bad else 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
