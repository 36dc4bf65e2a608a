"""Pins of the learned-selector oracle: features, bfloat16 inference, the
learned policy's fallback, and the float64 training arithmetic.

Features are pinned by blocks whose statistics are known in closed form and
by a vectorised numpy computation; inference by an exact rational emulation
of each fused multiply-add with torch's own bfloat16 rounding; gradients by
central finite differences; Adam by its first-step closed form.

`tests/oracle_mutations.py` plants one plausible mistake at a time in a copy
of the oracle (a dropped term, a wrong sign, index or tie rule) and checks
that one of these pins fails for each.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_1711_03888_amd import datagen


def test_flog_powers_of_two():
    # F(2^k) = k + 1 exactly: a block whose sampled sum |Dp| is 2^k (samples
    # at positions 0 and 4, m = 2)
    for k in range(0, 20):
        q = np.array([0, 0, 0, 0, 2 ** k], np.int32)
        f = oracle.features(q, 1024, 2 ** 27)[0]
        assert f[2] == float(k + 1) - 2.0  # F(sum|Dp|) - F(m = 2)


def test_features_constant_block():
    q = np.full(4096, 777, np.int32)
    f = oracle.features(q, 4096, 1000)[0]
    assert f[0] == np.float32(777 / 1000)
    assert f[1] == 0
    assert f[4] == 0 and f[5] == 0  # F(0) = 0
    assert f[6] == 1 and f[7] == 1 and f[8] == 1 and f[9] == 1  # of m = 1024 samples
    assert f[10] == 0 and f[13] == 0
    assert f[14] == np.float32(10 + 0xf4 / 256)  # 1000 = 0b1111101000
    assert f[15] == 1


def test_features_ramp_and_zigzag():
    n, c = 4096, 5
    m = n // 4  # sampled positions 0, 4, 8, ...
    ramp = (100 + c * np.arange(n)).astype(np.int32)
    f = oracle.features(ramp, n, 1 << 20)[0]
    # Dp = (0, c, c, ...), D2p = (0, c, 0, 0, ...): on the sample, Dp = 0
    # only at 0 and D2p = 0 everywhere
    assert f[6] == np.float32(1 / m) and f[7] == 1.0
    assert f[4] == 3.25 and f[5] == 0.0  # F(5) = 3 + 0b01/4 = 3.25
    assert f[10] == 0
    zig = (100 + c * (np.arange(n) % 2)).astype(np.int32)
    f = oracle.features(zig, n, 1 << 20)[0]
    # Dp = (0, c, -c, c, ...): at every sampled j >= 4, Dp_j = -c after +c
    assert f[10] == np.float32((m - 1) / m)
    assert f[8] == np.float32(1 / m)


def _features_numpy(q, P):
    q = q.astype(np.int64)
    d = q - q[0]
    dp_all = np.diff(np.concatenate([[0], d]))
    d2 = np.diff(np.concatenate([[0], dp_all]))[::4]
    prev = np.concatenate([[0], dp_all])[:-1][::4]  # Dp at j - 1
    dp = dp_all[::4]
    q = q[::4]
    n = q.size  # m, the sampled positions
    a1, a2 = np.abs(dp), np.abs(d2)

    def F(v):
        v = int(v)
        b = v.bit_length()
        if b == 0:
            return np.float32(0)
        frac = (v >> (b - 9)) & 255 if b >= 9 else (v << (9 - b)) & 255
        return np.float32(b + frac / 256)

    def r(a, b):
        return np.float32(np.float64(a) / np.float64(b))

    Pp = max(int(P), 1)
    sc = int(np.sum((dp > 0) & (prev < 0)) + np.sum((dp < 0) & (prev > 0)))
    bl1 = int(sum(int(v).bit_length() for v in a1))
    bl2 = int(sum(int(v).bit_length() for v in a2))
    fl = F(n)
    return np.array([r(q.sum(), n * Pp), r(q.max() - q.min(), Pp), F(a1.sum()) - fl, F(a2.sum()) - fl,
                     F(a1.max()), F(a2.max()), r((a1 == 0).sum(), n), r((a2 == 0).sum(), n),
                     r((a1 <= 1).sum(), n), r((a2 <= 1).sum(), n), r(sc, n), F(bl1) - fl, F(bl2) - fl,
                     r((a1 >= 32768).sum(), n), F(Pp), 1.0], np.float32)


@pytest.mark.parametrize("S", [1024, 4096])
def test_features_match_vectorised_numpy(S):
    x = datagen.random_walk(3 * S + 333, seed=21)
    q = oracle.lattice(x, 1e-4)
    P = oracle.params(x, 1e-4)["P"]
    got = oracle.features(q, S, P)
    for b in range(got.shape[0]):
        want = _features_numpy(q[b * S:(b + 1) * S], P)
        assert np.array_equal(got[b], want), (b, got[b], want)


def test_bf16_matches_torch_rounding():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    vals = rng.normal(0, 10, 2000).astype(np.float32)
    # exact ties between two bfloat16 values, both parities
    ties = (np.arange(1, 200, dtype=np.uint32) << 16 | 0x8000).view(np.float32)
    vals = np.concatenate([vals, ties, -ties, np.float32([0.0, -0.0, 1e-40, 3e38])])
    ref = torch.from_numpy(vals).to(torch.bfloat16).to(torch.float32).numpy()
    got = np.array([oracle.bf16(float(v)) for v in vals], np.float32)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def _round_f32(x: Fraction) -> np.float32:
    """float32 nearest to the rational x, ties to even."""
    c = np.float32(float(x))
    best = None
    for cand in (np.nextafter(c, np.float32(-np.inf)), c, np.nextafter(c, np.float32(np.inf))):
        err = abs(Fraction(float(cand)) - x)
        key = (err, int(np.float32(cand).view(np.uint32)) & 1)
        if best is None or key < best[0]:
            best = (key, cand)
    return np.float32(best[1])


def _infer_exact(w, feat):
    torch = pytest.importorskip("torch")

    def bf(v):
        return np.float32(torch.tensor([float(v)], dtype=torch.float32).to(torch.bfloat16).float().item())

    p = mlp.unpack(w)
    x = [bf(v) for v in feat]

    def layer(W, b, inp, relu):
        out = []
        for j in range(W.shape[0]):
            acc = np.float32(b[j])
            for k in range(W.shape[1]):
                acc = _round_f32(Fraction(float(bf(np.float32(W[j, k])))) * Fraction(float(inp[k]))
                                 + Fraction(float(acc)))
            out.append(bf(max(acc, np.float32(0))) if relu else acc)
        return out

    h1 = layer(p["W1"], p["b1"], x, True)
    h2 = layer(p["W2"], p["b2"], h1, True)
    return np.array(layer(p["W3"], p["b3"], h2, False), np.float32)


def test_mlp_inference_exact_emulation():
    rng = np.random.default_rng(5)
    w = rng.normal(0, 0.4, mlp.NPARAM).astype(np.float32)
    x = datagen.random_walk(4 * 1024, seed=8)
    q = oracle.lattice(x, 1e-3)
    feat = oracle.features(q, 1024, oracle.params(x, 1e-3)["P"])
    feat = np.concatenate([feat, rng.normal(0, 3, (3, 16)).astype(np.float32)])
    got = oracle.mlp_logits(w, feat)
    for b in range(feat.shape[0]):
        assert np.array_equal(got[b].view(np.uint32), _infer_exact(w, feat[b]).view(np.uint32)), b


def test_learned_policy_extremes():
    rng = np.random.default_rng(6)
    w = rng.normal(0, 0.5, mlp.NPARAM).astype(np.float32)
    x = datagen.random_walk(8 * 1024 + 50, seed=9)
    eb = 1e-3
    q = oracle.lattice(x, eb)
    P = oracle.params(x, eb)["P"]
    S = 1024
    exh = oracle.select(q, S)[0]
    pred_inf, fb_inf = oracle.select_learned(q, S, P, w, float("inf"))
    assert fb_inf.all() and np.array_equal(pred_inf, exh)
    pred_ninf, fb_ninf = oracle.select_learned(q, S, P, w, float("-inf"))
    logits = oracle.mlp_logits(w, oracle.features(q, S, P))
    assert not fb_ninf.any() and np.array_equal(pred_ninf, np.argmax(logits, axis=1))
    # tau = +inf gives the best-fit stream, up to the policy byte
    mode = oracle.EB_REL | oracle.block_mode(10)
    s_l = bytearray(oracle.compress(x, eb, oracle.LEARNED | mode, selector=(w, float("inf"))))
    s_b = oracle.compress(x, eb, oracle.BESTFIT | mode)
    assert s_l[6] == 3 and s_b[6] == 2
    s_l[6] = 2
    assert bytes(s_l) == s_b
    y = oracle.decompress(bytes(oracle.compress(x, eb, oracle.LEARNED | mode, selector=(w, 0.0))))
    assert np.abs(y.astype(np.float64) - x).max() <= oracle.params(x, eb)["eb_abs"]


def test_gradient_finite_differences():
    rng = np.random.default_rng(11)
    w = rng.normal(0, 0.5, mlp.NPARAM)
    x = rng.normal(0, 1, (40, 16))
    y = rng.integers(0, 3, 40)
    g = mlp.grad(w, x, y)
    h = 1e-6
    idx = np.concatenate([rng.choice(mlp.NPARAM, 60, replace=False), [511, 543, 1567, 1599, 1695, 1698]])
    for i in idx:
        e = np.zeros(mlp.NPARAM)
        e[i] = h
        fd = (mlp.loss(w + e, x, y) - mlp.loss(w - e, x, y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(g[i]), (i, fd, g[i])


def test_adam_first_step():
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    w0 = np.array([1.0, 1.0, 1.0, 1.0])
    w1, m, v = mlp.adam(w0, np.zeros(4), np.zeros(4), g, 1, 0.01)
    # bias-corrected first moments are g and g^2: a step of lr * g / (|g| + eps)
    assert np.allclose(w1, w0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


# ---- closed-form blocks for the features the ramp, zigzag and constant
# blocks leave untouched (3, 9, 11, 12, 13).  S = 1024, sampled positions
# j = 0, 4, ..., 1020 (m = 256, F(m) = 9).  Values of F are worked by hand:
# F(v) = bit length + (the 8 bits after the leading one) / 256.

def _feat(q):
    return oracle.features(np.asarray(q, np.int32), 1024, 1 << 21)[0]


def test_features_triangular_block():
    # p_j = j(j-1)/2: Dp_j = j - 1 (j >= 1), D2p_j = 1 (j >= 2), D2p_1 = 0.
    # Samples: D2p = 0 at j = 0, 1 at the 255 others.
    j = np.arange(1024, dtype=np.int64)
    f = _feat(j * (j - 1) // 2)
    # feature 3: F(sum |D2p|) - F(m) = F(255) - 9; 255 = 0b11111111 -> 8 + 254/256
    assert f[3] == np.float32(-2 / 256)
    # feature 9: every sample has |D2p| <= 1 (a "< 1" would give 1/256)
    assert f[9] == 1.0
    assert f[7] == np.float32(1 / 256)
    # feature 12: sum of bit lengths of |D2p| = 255 -> the same value as feature 3
    assert f[12] == np.float32(-2 / 256)
    # feature 11: sum over k = 1..255 of bitlen(4k - 1)
    #   = 2*1 + 3*1 + 4*2 + 5*4 + 6*8 + 7*16 + 8*32 + 9*64 + 10*127 = 2295
    #   2295 = 0b100011110111 -> 12 + 0b00011110/256 = 12 + 30/256
    assert f[11] == np.float32(3 + 30 / 256)
    assert f[5] == 1.0  # F(max |D2p|) = F(1) = 1


def test_features_square_block():
    # p_j = j^2: D2p_j = 2 for j >= 2; samples: 0 at j = 0, 2 at the others
    j = np.arange(1024, dtype=np.int64)
    f = _feat(j * j)
    # feature 3: F(510) - 9; 510 = 0b111111110 -> 9 + 0b11111110/256 = 9 + 254/256
    assert f[3] == np.float32(254 / 256)
    # feature 9: only the first sample has |D2p| <= 1
    assert f[9] == np.float32(1 / 256)
    # feature 12: sum of bitlen(2) = 2 * 255 = 510, the same F
    assert f[12] == np.float32(254 / 256)
    assert f[5] == 2.0  # F(2)


@pytest.mark.parametrize("amp,count", [(32768, 255), (32767, 0), (40000, 255)])
def test_features_escape_count(amp, count):
    # p alternates 0, amp: |Dp| = amp at every sample after the first
    f = _feat(amp * (np.arange(1024) % 2))
    assert f[13] == np.float32(count / 256)
    assert f[8] == np.float32(1 / 256)


# ---- training arithmetic: known values

def test_loss_known_values():
    w = np.zeros(mlp.NPARAM)
    x = np.random.default_rng(1).normal(0, 1, (7, 16))
    # zero weights: equal logits, the loss of each row is ln 3 (mean, not sum)
    assert abs(mlp.loss(w, x, np.array([0, 1, 2, 0, 1, 2, 2])) - np.log(3.0)) < 1e-15
    # a logit margin of 50 through the last bias: the labelled class costs
    # ln(1 + 2 e^-50) ~ 3.9e-22, another class 50 + ln(1 + ... ) ~ 50
    p = mlp.unpack(w)
    p["b3"][:] = [50.0, 0.0, 0.0]
    w = mlp.pack(p)
    assert mlp.loss(w, x[:1], np.array([0])) < 1e-20
    assert abs(mlp.loss(w, x[:1], np.array([1])) - 50.0) < 1e-12
    # mixed labels average the two: (ln(e^50 + 2) - 50 + ln(e^50 + 2)) / 2
    lse = 50.0 + np.log1p(2 * np.exp(-50.0))
    assert abs(mlp.loss(w, x[:2], np.array([0, 2])) - (lse - 50.0 + lse) / 2) < 1e-12


def test_adam_constant_gradient_many_steps():
    # with a constant gradient the bias-corrected moments are exactly g and
    # g^2 at every step t (m_t = (1 - b1^t) g, v_t = (1 - b2^t) g^2), so each
    # step moves by lr g / (|g| + eps); a correction by b instead of b^t
    # fails from t = 2 on
    g = np.array([0.5, -2.0, 1e-3, 3.0])
    w = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    for t in range(1, 11):
        w_prev = w
        w, m, v = mlp.adam(w, m, v, g, t, 0.01)
        assert np.allclose(m, (1 - 0.9 ** t) * g, rtol=1e-14, atol=0)
        assert np.allclose(v, (1 - 0.999 ** t) * g * g, rtol=1e-12, atol=0)
        assert np.allclose(w - w_prev, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=0), t


def test_fallback_only_below_tau():
    # all weights 0 and output biases (1, 0, 0): every block's logits are
    # exactly (1, 0, 0), margin 1.  A margin equal to tau is trusted; one
    # just below tau falls back to the exhaustive trial.
    p = mlp.unpack(np.zeros(mlp.NPARAM))
    p["b3"][:] = [1.0, 0.0, 0.0]
    w = mlp.pack(p).astype(np.float32)
    j = np.arange(3 * 1024, dtype=np.int64)
    q = (5 * j * j % 7919).astype(np.int32)
    pred, fb = oracle.select_learned(q, 1024, 1 << 20, w, 1.0)
    assert not fb.any() and (pred == 0).all()
    pred, fb = oracle.select_learned(q, 1024, 1 << 20, w, float(np.nextafter(np.float32(1), np.float32(2))))
    assert fb.all() and np.array_equal(pred, oracle.select(q, 1024)[0])
