"""Seeded synthetic particle fields.

These generators stand in for the paper's HACC (cosmology) and AMDF
(molecular dynamics) snapshots (Table 1), which are not available; they
reproduce the shapes, value distributions and orderings described for the
workloads and contain none of the compressor's arithmetic.  Every tensor is
float32 numpy, generated with ``numpy.random.default_rng(seed)``; the GPU
path receives the same bytes.

* ``random_walk``   -- one field: a random walk with N(0, 0.01) steps plus
  U(-0.005, 0.005) noise, wrapped into [0, 256) (1 Mi values by default).
* ``cosmology``     -- six fields xx yy zz vx vy vz: 20k Poisson halo centres
  in a [0,256)^3 box with Gaussian offsets (sigma 0.5) for 70% of the
  particles and a uniform background for 30%, stored in 8^3 spatial-cell
  order; velocities are a halo bulk N(0,300) plus thermal N(0,100).
* ``md_lattice``    -- three coordinate fields of an FCC lattice (a = 3.6)
  with N(0, 0.05) thermal displacements in lattice-index order, 5% of the
  256-atom blocks internally permuted.
* ``batch_spec`` / ``batch_field`` -- uneven fields drawn from the two
  generators above; ``batch_from_sources`` cuts the same batch out of one
  long random walk and one cosmology snapshot (much faster to generate).
* ``steady_fields`` -- many equal random-walk fields cut from one long walk.
"""
from __future__ import annotations

import numpy as np

FIELD_NAMES = ("xx", "yy", "zz", "vx", "vy", "vz")


def random_walk(n: int = 1 << 20, seed: int = 1) -> np.ndarray:
    rng = np.random.default_rng(seed)
    steps = rng.normal(0.0, 0.01, size=n)
    noise = rng.uniform(-0.005, 0.005, size=n)
    x = np.mod(np.cumsum(steps) + noise, 256.0)
    f = x.astype(np.float32)
    f[f >= np.float32(256.0)] = np.float32(0.0)
    return f


def cosmology(n: int = 1 << 26, seed: int = 2, n_halos: int | None = None,
              box: float = 256.0) -> dict[str, np.ndarray]:
    """Halo + background particles in 8^3 cell order (HACC stand-in)."""
    rng = np.random.default_rng(seed)
    if n_halos is None:
        n_halos = max(1, int(round(20000 * n / float(1 << 26))))
    n_halo_p = int(round(0.7 * n))
    n_bg = n - n_halo_p
    centres = rng.uniform(0.0, box, size=(n_halos, 3))
    bulk = rng.normal(0.0, 300.0, size=(n_halos, 3))
    hid = np.sort(rng.integers(0, n_halos, size=n_halo_p))  # grouped by halo id
    pos = np.empty((n, 3), dtype=np.float64)
    vel = np.empty((n, 3), dtype=np.float64)
    pos[:n_halo_p] = centres[hid] + rng.normal(0.0, 0.5, size=(n_halo_p, 3))
    vel[:n_halo_p] = bulk[hid] + rng.normal(0.0, 100.0, size=(n_halo_p, 3))
    pos[n_halo_p:] = rng.uniform(0.0, box, size=(n_bg, 3))
    vel[n_halo_p:] = rng.normal(0.0, 300.0, size=(n_bg, 3)) + rng.normal(0.0, 100.0, size=(n_bg, 3))
    np.mod(pos, box, out=pos)
    cell = np.minimum((pos // (box / 8.0)).astype(np.int64), 7)
    key = (cell[:, 0] * 8 + cell[:, 1]) * 8 + cell[:, 2]
    order = np.argsort(key, kind="stable")
    out = {}
    for k, name in enumerate(FIELD_NAMES[:3]):
        f = pos[order, k].astype(np.float32)
        f[f >= np.float32(box)] = np.float32(0.0)
        out[name] = f
    for k, name in enumerate(FIELD_NAMES[3:]):
        out[name] = vel[order, k].astype(np.float32)
    return out


def md_lattice(cells=(64, 64, 128), a: float = 3.6, sigma: float = 0.05,
               seed: int = 3, shuffle_frac: float = 0.05, blk: int = 256,
               velocities: bool = False) -> dict[str, np.ndarray]:
    """FCC lattice in lattice-index order with thermal noise (AMDF stand-in).
    With velocities, also Maxwell-Boltzmann velocity components N(0, 1) per
    atom, drawn from their own generator (the coordinates do not change)."""
    rng = np.random.default_rng(seed)
    ci, cj, ck = cells
    basis = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]])
    i, j, k, b = np.meshgrid(np.arange(ci), np.arange(cj), np.arange(ck), np.arange(4), indexing="ij")
    i, j, k, b = (v.reshape(-1) for v in (i, j, k, b))
    n = i.size
    pos = np.stack([i, j, k], axis=1).astype(np.float64) + basis[b]
    pos = pos * a + rng.normal(0.0, sigma, size=(n, 3))
    nblk = n // blk
    chosen = rng.choice(nblk, size=int(round(shuffle_frac * nblk)), replace=False)
    perm = np.arange(n)
    for c in np.sort(chosen):
        perm[c * blk:(c + 1) * blk] = c * blk + rng.permutation(blk)
    pos = pos[perm]
    out = {name: pos[:, d].astype(np.float32) for d, name in enumerate(FIELD_NAMES[:3])}
    if velocities:
        vel = np.random.default_rng(seed + 1000).normal(0.0, 1.0, size=(n, 3))[perm]
        out.update({name: vel[:, d].astype(np.float32) for d, name in enumerate(FIELD_NAMES[3:])})
    return out


def batch_spec(n_fields: int = 512, seed: int = 4, lo: float = 16.0, hi: float = 24.0):
    """Sizes, relative bounds and generator kinds of a batch of uneven fields."""
    ss = np.random.SeedSequence(seed)
    children = ss.spawn(n_fields)
    specs = []
    for f, child in enumerate(children):
        rng = np.random.default_rng(child)
        nf = int(round(2.0 ** rng.uniform(lo, hi)))
        eb = float(rng.choice([1e-3, 1e-4, 1e-5]))
        sub_seed = int(rng.integers(0, 2**31 - 1))
        specs.append({"index": f, "n": nf, "eb_rel": eb, "seed": sub_seed,
                      "kind": "walk" if f % 2 == 0 else "cosmo", "field": (f // 2) % 6})
    return specs


def batch_field(spec) -> np.ndarray:
    if spec["kind"] == "walk":
        return random_walk(spec["n"], seed=spec["seed"])
    n = spec["n"]
    halos = max(1, int(round(20000 * n / float(1 << 26))))
    snap = cosmology(n, seed=spec["seed"], n_halos=halos)
    return snap[FIELD_NAMES[spec["field"]]]


def rebased(w: np.ndarray) -> np.ndarray:
    """A slice of a long random walk restarted at zero and wrapped into
    [0, 256), as a fresh walk of that length would be."""
    f = np.mod(w.astype(np.float64) - float(w[0]), 256.0).astype(np.float32)
    f[f >= np.float32(256.0)] = np.float32(0.0)
    return f


def steady_fields(walk: np.ndarray, n: int = 1 << 20, nf: int = 256) -> list[np.ndarray]:
    """nf distinct random-walk fields of n values: consecutive slices of one
    long walk, each restarted at zero."""
    return [rebased(walk[i * n:(i + 1) * n]) for i in range(nf)]


def batch_from_sources(walk: np.ndarray, cosmo: dict, specs=None, seed: int = 4):
    """The uneven batch of ``batch_spec`` cut from existing data: even fields
    are slices of a long random walk (restarted at zero), odd fields slices
    of the named field of a cosmology snapshot, at offsets drawn from
    ``default_rng(seed)``.  Returns (specs, list of float32 arrays)."""
    specs = batch_spec() if specs is None else specs
    rng = np.random.default_rng(seed)
    out = []
    for sp in specs:
        n = sp["n"]
        src = walk if sp["kind"] == "walk" else cosmo[FIELD_NAMES[sp["field"]]]
        off = int(rng.integers(0, (src.size - n) // 4 + 1)) * 4
        out.append(rebased(src[off:off + n]) if sp["kind"] == "walk" else src[off:off + n])
    return specs, out
