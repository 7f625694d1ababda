"""Seeded synthetic workloads standing in for the paper's molecules and boxes.

The paper times TensorNet on real molecules and random particle clouds
(Sec. 3.3, Table 2 and the inference-time figure; Sec. 2.5.1 for the
neighbour benchmarks).  None of those structures ship with the paper, so
every workload here is drawn from a seeded NumPy PCG64 generator with the
same shape: atoms of species {H, C, N, O} at a liquid-like number density of
0.1 atoms per cubic angstrom, placed by random sequential addition with a
hard minimum separation of 0.9 angstrom.

Nothing in this module evaluates the model: it only draws numbers and lays
out arrays (positions float32 [N,3], species int32 [N], system index int32
[N] sorted ascending, and an optional rectangular box float64 [3,3]).
"""

from __future__ import annotations

import functools
import math

import numpy as np

DENSITY = 0.1          # atoms per cubic angstrom
DMIN = 0.9             # minimum pair separation, angstrom
SPECIES = np.array([1, 6, 7, 8], dtype=np.int32)
MASS_BY_Z = {1: 1.008, 6: 12.011, 7: 14.007, 8: 15.999}   # amu
KB_EV = 8.617333262e-5          # Boltzmann constant, eV/K
EV_PER_AMU_A2_FS2 = 9.648533212e-3   # (eV/angstrom)/amu expressed in angstrom/fs^2

# Five workloads (positions seed 1000+i, weights seed 2000+i).
CONFIGS = {
    0: dict(kind="molecule", n_atoms=48, F=64, K=32, L=2, r_c=4.5, max_z=100,
            precision="f64", desc="one isolated 48-atom molecule, hidden 64, 2 layers, cutoff 4.5 A"),
    1: dict(kind="box", n_atoms=6000, F=128, K=32, L=2, r_c=5.0, max_z=100,
            precision="f32", desc="periodic cubic box of 6000 atoms, hidden 128, 2 layers, cutoff 5 A"),
    2: dict(kind="batch", n_mol=512, size_lo=8, size_hi=64, noise=0.0, F=128, K=32, L=2, r_c=5.0,
            max_z=100, precision="f32",
            desc="512 isolated molecules of 8-64 atoms, hidden 128, 2 layers, cutoff 5 A"),
    3: dict(kind="box", n_atoms=100_000, box_len=100.0, F=128, K=32, L=2, r_c=5.0, max_z=100,
            precision="f32", desc="periodic cubic box of 100000 atoms (100 A), hidden 128, 2 layers, cutoff 5 A"),
    4: dict(kind="batch", n_mol=64, size_lo=16, size_hi=128, noise=0.05, F=128, K=32, L=3, r_c=5.0,
            max_z=100, precision="f32",
            desc="64 molecules of 16-128 atoms with 0.05 A noise, hidden 128, 3 layers, cutoff 5 A"),
}


def _rsa_ball(rng: np.random.Generator, n: int, radius: float, dmin: float) -> np.ndarray:
    """Random sequential addition of n points in a ball, min separation dmin."""
    pts = np.empty((n, 3), dtype=np.float64)
    k = 0
    d2min = dmin * dmin
    while k < n:
        c = rng.uniform(-radius, radius, size=3)
        if c @ c > radius * radius:
            continue
        if k:
            diff = pts[:k] - c
            if np.min(np.einsum("ij,ij->i", diff, diff)) < d2min:
                continue
        pts[k] = c
        k += 1
    return pts


def _rsa_box(rng: np.random.Generator, n: int, box_len: float, dmin: float) -> np.ndarray:
    """Random sequential addition of n points in a periodic cube, min image separation dmin."""
    nc = max(1, int(math.floor(box_len / dmin)))
    side = box_len / nc
    slots = 8   # a cube of side >= dmin holds at most 8 points that are dmin apart
    grid = np.full((nc, nc, nc, slots), -1, dtype=np.int64)
    fill = np.zeros((nc, nc, nc), dtype=np.int64)
    pts = np.empty((n, 3), dtype=np.float64)
    offs = np.array([(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)], dtype=np.int64)
    d2min = dmin * dmin
    k = 0
    while k < n:
        c = rng.uniform(0.0, box_len, size=3)
        cell = np.minimum((c / side).astype(np.int64), nc - 1)
        if k:
            nb = (cell[None, :] + offs) % nc
            cand = grid[nb[:, 0], nb[:, 1], nb[:, 2]].ravel()
            cand = cand[cand >= 0]
            if cand.size:
                diff = pts[cand] - c
                diff -= box_len * np.round(diff / box_len)
                if np.min(np.einsum("ij,ij->i", diff, diff)) < d2min:
                    continue
        pts[k] = c
        grid[cell[0], cell[1], cell[2], fill[cell[0], cell[1], cell[2]]] = k
        fill[cell[0], cell[1], cell[2]] += 1
        k += 1
    return pts


def single_molecule(n: int, seed: int, density: float = DENSITY, dmin: float = DMIN):
    """One isolated molecule: n atoms uniform in a ball of radius (3n/(4 pi rho))^(1/3)."""
    rng = np.random.default_rng(seed)
    radius = (3.0 * n / (4.0 * math.pi * density)) ** (1.0 / 3.0)
    pos = _rsa_ball(rng, n, radius, dmin)
    z = SPECIES[rng.integers(0, len(SPECIES), size=n)]
    return dict(pos=pos.astype(np.float32), z=z.astype(np.int32),
                batch=np.zeros(n, dtype=np.int32), box=None, n_systems=1)


def molecule_batch(n_mol: int, size_lo: int, size_hi: int, seed: int, noise: float = 0.0,
                   density: float = DENSITY, dmin: float = DMIN):
    """n_mol isolated molecules with sizes iid uniform on {size_lo..size_hi}.

    Every molecule is centred on the origin, so they overlap in space and only
    the system index keeps them apart.  The system index is sorted.
    """
    rng = np.random.default_rng(seed)
    sizes = rng.integers(size_lo, size_hi + 1, size=n_mol)
    pos, z, batch = [], [], []
    for s, n in enumerate(sizes):
        radius = (3.0 * n / (4.0 * math.pi * density)) ** (1.0 / 3.0)
        p = _rsa_ball(rng, int(n), radius, dmin)
        if noise > 0.0:
            p = p + rng.normal(0.0, noise, size=p.shape)
        pos.append(p)
        z.append(SPECIES[rng.integers(0, len(SPECIES), size=int(n))])
        batch.append(np.full(int(n), s, dtype=np.int32))
    return dict(pos=np.concatenate(pos).astype(np.float32), z=np.concatenate(z).astype(np.int32),
                batch=np.concatenate(batch).astype(np.int32), box=None, n_systems=int(n_mol))


def periodic_box(n: int, seed: int, box_len: float | None = None, density: float = DENSITY,
                 dmin: float = DMIN):
    """n atoms in a periodic cube of side (n/rho)^(1/3) (or box_len), positions in [0, L)."""
    rng = np.random.default_rng(seed)
    if box_len is None:
        box_len = (n / density) ** (1.0 / 3.0)
    pos = _rsa_box(rng, n, box_len, dmin)
    z = SPECIES[rng.integers(0, len(SPECIES), size=n)]
    box = np.diag([box_len, box_len, box_len]).astype(np.float64)
    return dict(pos=pos.astype(np.float32), z=z.astype(np.int32),
                batch=np.zeros(n, dtype=np.int32), box=box, n_systems=1)


def random_cloud(n: int, n_batches: int, seed: int, neighbors: float = 64.0, cutoff: float = 5.0):
    """Neighbour-search benchmark shape: n points iid uniform in a periodic cube whose density puts
    `neighbors` points within `cutoff` of a point on average, split into n_batches systems of
    (nearly) equal size by contiguous index ranges (sorted batch vector), so every system is spread
    over the whole box."""
    rng = np.random.default_rng(seed)
    density = neighbors / (4.0 / 3.0 * math.pi * cutoff ** 3)
    box_len = (n / density) ** (1.0 / 3.0)
    pos = rng.uniform(0.0, box_len, size=(n, 3))
    batch = (np.arange(n, dtype=np.int64) * n_batches // max(n, 1)).astype(np.int32)
    box = np.diag([box_len, box_len, box_len]).astype(np.float64)
    return dict(pos=pos.astype(np.float32), batch=batch, box=box, n_systems=int(n_batches))


@functools.lru_cache(maxsize=8)
def _config_cached(cfg: int):
    c = CONFIGS[cfg]
    seed = 1000 + cfg
    if c["kind"] == "molecule":
        d = single_molecule(c["n_atoms"], seed)
    elif c["kind"] == "box":
        d = periodic_box(c["n_atoms"], seed, box_len=c.get("box_len"))
    else:
        d = molecule_batch(c["n_mol"], c["size_lo"], c["size_hi"], seed, noise=c["noise"])
    return d


def make_config(cfg: int) -> dict:
    """Inputs and model sizes of workload `cfg` (0..4); arrays are fresh copies."""
    d = _config_cached(cfg)
    c = CONFIGS[cfg]
    out = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in d.items()}
    out.update({k: c[k] for k in ("F", "K", "L", "r_c", "max_z", "precision", "desc")})
    out["weight_seed"] = 2000 + cfg
    return out


def make_weights(F: int, K: int, L: int, max_z: int = 100, seed: int = 0) -> dict:
    """Random TensorNet parameters, FP64, drawn in the fixed blob order.

    Every Linear weight and bias is iid N(0, 1/fan_in); the species embedding
    is N(0, 1); LayerNorm scales are 1 and shifts 0.
    """
    from .blob import tensor_layout
    rng = np.random.default_rng(seed)
    out = {}
    for name, shape, init, fan_in in tensor_layout(F, K, L, max_z):
        if init == "normal_fanin":
            out[name] = rng.normal(0.0, 1.0 / math.sqrt(fan_in), size=shape)
        elif init == "normal":
            out[name] = rng.normal(0.0, 1.0, size=shape)
        elif init == "ones":
            out[name] = np.ones(shape)
        elif init == "zeros":
            out[name] = np.zeros(shape)
        else:
            raise ValueError(init)
    return out


def maxwell_boltzmann(z: np.ndarray, temperature: float = 300.0, seed: int = 4003) -> np.ndarray:
    """Velocities (angstrom/fs, float32 [N,3]) at `temperature`, zero net momentum."""
    rng = np.random.default_rng(seed)
    m = np.array([MASS_BY_Z[int(a)] for a in z], dtype=np.float64)
    sigma = np.sqrt(KB_EV * temperature * EV_PER_AMU_A2_FS2 / m)
    v = rng.normal(0.0, 1.0, size=(len(z), 3)) * sigma[:, None]
    v -= (m[:, None] * v).sum(0) / m.sum()
    return v.astype(np.float32)


def masses(z: np.ndarray) -> np.ndarray:
    return np.array([MASS_BY_Z[int(a)] for a in z], dtype=np.float64)
