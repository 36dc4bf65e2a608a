"""Training of the learned predictor selector on the GPU.

The selector (16 block features -> 32 -> 32 -> 3 logits) replaces the
exhaustive trial of the best-fit policy; its labels are the trial's own
choices.  Training data are synthetic fields from the random-walk and
cosmology generators; features, trial costs and labels come from the
library's feature kernel, the gradient and the Adam step from its training
kernels.  Host code only shuffles, standardises and slices the data set.

  python -m paper_1711_03888_amd.selector OUT.json [--data nbody|md] [--steps K]

writes the parameters (feature standardisation folded into the first
layer), the fallback threshold tau and the training record.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

from . import datagen

FORMAT_VERSION = 1
# the feature definition the parameters are trained for (see sznb.h)
FEATURE_SPEC = ("sample j=0 mod 4, m positions: sum p/(m P'); (max p-min p)/P'; F(sum|Dp|)-F(m); "
                "F(sum|D2p|)-F(m); F(max|Dp|); F(max|D2p|); #(Dp=0)/m; #(D2p=0)/m; #(|Dp|<=1)/m; #(|D2p|<=1)/m; "
                "#(Dp_j Dp_j-1<0)/m; F(sum bitlen|Dp|)-F(m); F(sum bitlen|D2p|)-F(m); #(|Dp|>=32768)/m; F(P'); 1")
FEATURE_HASH = hashlib.sha256(FEATURE_SPEC.encode()).hexdigest()[:16]
EBS = (1e-3, 1e-4, 1e-5)


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights, zero biases, flat in the library's order."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_out, fan_in in ((32, 16), (32, 32), (3, 32)):
        lim = np.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-lim, lim, size=fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def generate_fields(n_walk: int, n_cosmo: int, seed: int, walk_n=1 << 20, cosmo_n=1 << 22):
    """(field, eb_rel) pairs: random-walk fields and cosmology snapshots (all
    six fields of each), bounds drawn from {1e-3, 1e-4, 1e-5}."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_walk):
        out.append((datagen.random_walk(walk_n, seed=seed * 1000 + i), float(rng.choice(EBS))))
    for i in range(n_cosmo):
        halos = max(1, int(round(20000 * cosmo_n / float(1 << 26))))
        snap = datagen.cosmology(cosmo_n, seed=seed * 1000 + 500 + i, n_halos=halos)
        for name in datagen.FIELD_NAMES:
            out.append((snap[name], float(rng.choice(EBS))))
    return out


def generate_md_fields(n_snap: int, seed: int, cells=(32, 32, 64)):
    """(field, eb_rel) pairs of FCC snapshots (the three coordinates)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_snap):
        snap = datagen.md_lattice(cells=cells, seed=seed * 1000 + i)
        for name in datagen.FIELD_NAMES[:3]:
            out.append((snap[name], float(rng.choice(EBS[:2]))))
    return out


def block_data(fields, mode, dev):
    """Features, trial costs and labels of every block of the fields."""
    import torch

    from . import sznb
    feats, costs, labels = [], [], []
    for x, eb in fields:
        t = torch.from_numpy(np.ascontiguousarray(x, np.float32)).to(dev)
        f, c, l = sznb.block_features([t], eb, mode)
        feats.append(f.cpu().numpy())
        costs.append(c.cpu().numpy())
        labels.append(l.cpu().numpy())
    return np.concatenate(feats), np.concatenate(costs), np.concatenate(labels)


def fold_standardisation(params: np.ndarray, mean: np.ndarray, std: np.ndarray) -> np.ndarray:
    """Parameters trained on (x - mean) / std rewritten for raw features x."""
    p = params.astype(np.float64).copy()
    W1 = p[0:512].reshape(32, 16)
    b1 = p[512:544]
    b1 -= W1 @ (mean / std)
    W1 /= std[None, :]
    p[0:512] = W1.reshape(-1)
    p[512:544] = b1
    return p.astype(np.float32)


def choose_tau(margin, choice, cost, label, budget=0.002):
    """Smallest tau whose remaining regret (blocks trusted to the network
    that it gets wrong) stays within `budget` of the exhaustive total."""
    best = cost[np.arange(len(label)), label].astype(np.float64)
    regret = cost[np.arange(len(label)), choice].astype(np.float64) - best
    total = best.sum()
    order = np.argsort(-margin)  # most confident first
    cum = np.cumsum(regret[order])
    ok = cum <= budget * total
    # trust the k most confident blocks, k the longest prefix within budget
    k = int(np.argmin(ok)) if not ok.all() else len(ok)
    if k == len(ok):
        return 0.0  # every block may be trusted: fall back on exact ties only
    return float(margin[order[k]]) + 1e-6


def train(feat, label, *, steps=2000, batch=4096, lr=3e-3, seed=0, dev="cuda", log=None):
    """Adam on the mean cross-entropy with the library's kernels; returns the
    parameters for raw features and the loss curve."""
    import torch

    from . import sznb
    mean = feat.mean(axis=0).astype(np.float64)
    std = feat.std(axis=0).astype(np.float64)
    std[std < 1e-6] = 1.0
    mean[15] = 0.0  # the constant feature keeps its role as a bias input
    std[15] = 1.0
    xs = ((feat - mean) / std).astype(np.float32)
    rng = np.random.default_rng(seed)
    perm = rng.permutation(len(label))
    xs_d = torch.from_numpy(np.ascontiguousarray(xs[perm])).to(dev)
    y_d = torch.from_numpy(np.ascontiguousarray(label[perm].astype(np.uint8))).to(dev)
    params = torch.from_numpy(init_params(seed)).to(dev)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    nb = len(label)
    batch = min(batch, nb)
    ws = grad = loss = None
    curve = []
    for step in range(1, steps + 1):
        i = ((step - 1) * batch) % max(1, nb - batch + 1)
        grad, loss, ws = sznb.mlp_grad(params, xs_d[i:i + batch], y_d[i:i + batch], ws=ws, grad=grad, loss=loss)
        sznb.mlp_adam(params, m, v, grad, step, lr)
        if step % max(1, steps // 20) == 0 or step == 1:
            curve.append((step, float(loss.item())))
            if log:
                log("step %d loss %.5f" % curve[-1])
    return fold_standardisation(params.cpu().numpy(), mean, std), curve


def evaluate(params, feat, cost, label, dev="cuda"):
    """Choices, margins and accuracy of the bfloat16 inference on a set."""
    import torch

    from . import sznb
    p = torch.from_numpy(params).to(dev)
    f = torch.from_numpy(np.ascontiguousarray(feat)).to(dev)
    _, choice, margin = sznb.mlp_infer(p, f)
    choice = choice.cpu().numpy().astype(np.int64)
    margin = margin.cpu().numpy()
    return choice, margin, float((choice == label).mean())


def save(path, params, tau, record):
    with open(path, "w") as fh:
        json.dump({"version": FORMAT_VERSION, "feature_hash": FEATURE_HASH, "tau": tau,
                   "params": [float(v) for v in params], "record": record}, fh, indent=1)


SELECTORS = {name: os.path.join(os.path.dirname(os.path.abspath(__file__)), "selectors", name + ".json")
             for name in ("nbody", "md")}


def load(path):
    with open(path) as fh:
        d = json.load(fh)
    if d.get("version") != FORMAT_VERSION or d.get("feature_hash") != FEATURE_HASH:
        raise ValueError("selector file %s was trained for another feature definition" % path)
    return np.asarray(d["params"], np.float32), float(d["tau"]), d.get("record", {})


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("out")
    ap.add_argument("--walk-fields", type=int, default=64)
    ap.add_argument("--cosmo-snapshots", type=int, default=4)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--seed", type=int, default=100)
    ap.add_argument("--data", choices=["nbody", "md"], default="nbody",
                    help="random-walk and cosmology fields, or FCC coordinate fields")
    ap.add_argument("--md-snapshots", type=int, default=48)
    args = ap.parse_args(argv)
    import torch

    from . import sznb
    dev = torch.device("cuda:0")
    t0 = time.time()
    if args.data == "md":
        fields = generate_md_fields(args.md_snapshots, args.seed)
    else:
        fields = generate_fields(args.walk_fields, args.cosmo_snapshots, args.seed)
    mode = sznb.PRED_BESTFIT | sznb.EB_REL
    feat, cost, label = block_data(fields, mode, dev)
    print("blocks %d, labels LV/LCF/QCF %s, %.1fs" % (len(label), np.bincount(label, minlength=3).tolist(),
                                                      time.time() - t0), flush=True)
    rng = np.random.default_rng(args.seed + 1)
    idx = rng.permutation(len(label))
    n_val = max(1, len(label) // 20)
    val, tr = idx[:n_val], idx[n_val:]
    params, curve = train(feat[tr], label[tr], steps=args.steps, batch=args.batch, seed=args.seed, dev=dev,
                          log=lambda s: print(s, flush=True))
    choice, margin, acc = evaluate(params, feat[val], cost[val], label[val], dev)
    tau = choose_tau(margin, choice, cost[val], label[val])
    fb = float((margin < tau).mean())
    record = {"blocks": int(len(label)), "label_histogram": np.bincount(label, minlength=3).tolist(),
              "train_blocks": int(len(tr)), "heldout_blocks": int(n_val), "heldout_accuracy": acc,
              "heldout_fallback_rate": fb, "loss_curve": curve, "steps": args.steps, "batch": args.batch,
              "seed": args.seed, "data": args.data, "walk_fields": args.walk_fields,
              "cosmo_snapshots": args.cosmo_snapshots, "md_snapshots": args.md_snapshots,
              "train_seconds": round(time.time() - t0, 1)}
    save(args.out, params, tau, record)
    print(json.dumps({k: v for k, v in record.items() if k != "loss_curve"}), "tau", tau, flush=True)


if __name__ == "__main__":
    sys.exit(main())
