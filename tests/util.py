"""Small shared helpers for the tests (inputs and error metrics; no model arithmetic)."""

from __future__ import annotations

import math

import numpy as np

from synth import make_weights, write_blob
from synth.generators import _rsa_ball, _rsa_box, SPECIES


def small_blob(F=16, K=8, L=2, max_z=100, r_c=4.5, seed=7, r_lo=0.0):
    w = make_weights(F, K, L, max_z, seed=seed)
    return write_blob(w, F, K, L, max_z, r_c, r_lo=r_lo)


def random_molecule(n, seed, density=0.1, dmin=0.9):
    rng = np.random.default_rng(seed)
    radius = (3.0 * n / (4.0 * math.pi * density)) ** (1.0 / 3.0)
    pos = _rsa_ball(rng, n, radius, dmin)
    z = SPECIES[rng.integers(0, 4, size=n)].astype(np.int32)
    return pos, z


def random_box(n, seed, box_len, dmin=0.9):
    rng = np.random.default_rng(seed)
    pos = _rsa_box(rng, n, box_len, dmin)
    z = SPECIES[rng.integers(0, 4, size=n)].astype(np.int32)
    return pos, z, np.diag([box_len] * 3).astype(np.float64)


def random_rotation(seed, reflect=False):
    rng = np.random.default_rng(seed)
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    if reflect:
        q = q @ np.diag([1.0, 1.0, -1.0])
    return q


def rel_energy_err(E, E_ref):
    E = np.asarray(E, dtype=np.float64)
    E_ref = np.asarray(E_ref, dtype=np.float64)
    return float(np.max(np.abs(E - E_ref) / np.abs(E_ref)))


def rel_rms(Fv, F_ref):
    Fv = np.asarray(Fv, dtype=np.float64)
    F_ref = np.asarray(F_ref, dtype=np.float64)
    return float(np.linalg.norm(Fv - F_ref) / np.linalg.norm(F_ref))


def random_triclinic_cell(seed, cutoff, scale=(2.1, 3.2)):
    """A reduced triclinic cell (rows a, b, c; lower triangular) with random tilts and every
    height between scale[0] and scale[1] times the cutoff (scaled up if a draw is too flat)."""
    from oracle.neighbors import cell_heights
    rng = np.random.default_rng(seed)
    ax, by, cz = cutoff * rng.uniform(scale[0], scale[1], size=3)
    H = np.array([[ax, 0.0, 0.0],
                  [rng.uniform(-0.5, 0.5) * ax, by, 0.0],
                  [rng.uniform(-0.5, 0.5) * ax, rng.uniform(-0.5, 0.5) * by, cz]])
    h = cell_heights(H)
    if h.min() < 2.0 * cutoff:
        H = H * (2.0 * cutoff / h.min()) * 1.01
    return H


def random_in_cell(n, seed, H, dmin=0.9):
    """n points in the cell H (rows), no two closer than dmin under the nearest image."""
    from oracle.neighbors import nearest_image_d2
    rng = np.random.default_rng(seed)
    pts = np.zeros((0, 3))
    while len(pts) < n:
        p = rng.uniform(0.0, 1.0, size=(1, 3)) @ H
        if len(pts) and nearest_image_d2(np.repeat(p, len(pts), 0), pts, H, reach=1).min() < dmin * dmin:
            continue
        pts = np.concatenate([pts, p])
    z = SPECIES[rng.integers(0, 4, size=n)].astype(np.int32)
    return pts, z
