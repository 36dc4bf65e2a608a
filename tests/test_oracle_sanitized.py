"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The oracle's decoder is fed corrupt streams by the tests; this builds a copy
of it with -fsanitize=address,undefined (no recovery: any undefined
behaviour aborts), then in a child process round-trips fields through every
policy and decodes a few hundred corrupted and truncated streams, each of
which must give an error status or floats, never a sanitizer report.
"""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = textwrap.dedent('''
    import sys
    import numpy as np
    import oracle
    from paper_1711_03888_amd import datagen
    rng = np.random.default_rng(1)
    xs = [datagen.random_walk(3 * 4096 + 77, seed=2), datagen.cosmology(1 << 14, seed=3)["vx"],
          np.zeros(0, np.float32), np.full(1000, 3.0, np.float32)]
    w = rng.normal(0, 0.5, 1699).astype(np.float32)
    good = []
    for x in xs:
        for mode in (oracle.LV, oracle.LCF, oracle.BESTFIT):
            s = oracle.compress(x, 1e-4, mode | oracle.EB_REL | oracle.block_mode(10))
            y = oracle.decompress(s)
            assert y.size == x.size
            good.append(s)
        s = oracle.compress(x, 1e-4, oracle.LEARNED | oracle.EB_REL, selector=(w, 0.5))
        assert oracle.decompress(s).size == x.size
    bad = 0
    for s in good:
        for t in range(40):
            b = bytearray(s)
            if t % 4 == 3:
                b = b[:int(rng.integers(0, len(b)))]
            else:
                for _ in range(1 + t % 3):
                    i = int(rng.integers(0, len(b))) if len(b) else 0
                    if len(b):
                        b[i] ^= int(rng.integers(1, 256))
            try:
                oracle.decompress(bytes(b))
            except oracle.OracleError:
                bad += 1
    print("sanitized oracle ok, corrupt streams rejected: %d" % bad)
''')


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    for d in ("oracle", "paper_1711_03888_amd"):
        shutil.copytree(os.path.join(ROOT, d), tmp_path / d,
                        ignore=shutil.ignore_patterns("*.so", "_build", "__pycache__", "csrc", "selectors"))
    lib = tmp_path / "oracle" / "libsznb_oracle.so"
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-std=c11", "-fPIC",
                           "-shared", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-o", str(lib), str(tmp_path / "oracle" / "sznb_oracle.c"), "-lm"])
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", PYTHONPATH=str(tmp_path))
    r = subprocess.run([sys.executable, "-c", CHILD], cwd=str(tmp_path), env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "sanitized oracle ok" in r.stdout
