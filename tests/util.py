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


def energy_errors_r21(E, E_ref, abs_sum, floor=0.1):
    """Per-system energy errors |E - E_ref| / max(|E_ref|, floor * sum_i |eps_i|), with sum_i |eps_i| the
    per-atom energy magnitudes of the system.  A sum whose condition number sum_i |eps_i| / |E_ref| exceeds
    1 / floor is judged against floor * sum_i |eps_i|: the rounding of the per-atom terms scales with that,
    not with the cancelled result.  The denominator is continuous in E_ref.  Returns (errors, mask of the
    ill-conditioned systems)."""
    E = np.asarray(E, dtype=np.float64)
    E_ref = np.asarray(E_ref, dtype=np.float64)
    abs_sum = np.asarray(abs_sum, dtype=np.float64)
    near = np.abs(E_ref) < floor * abs_sum
    den = np.maximum(np.abs(E_ref), floor * abs_sum)
    return np.abs(E - E_ref) / den, near


def oracle_energy_forces_r21(oracle, pos, z, batch, box, S):
    """The oracle's (E [S], F, sum_i |eps_i| per system)."""
    cap = {}
    E, F = oracle.energy_forces(pos, z, batch, box, S, capture=cap)
    abs_sum = np.zeros(S)
    np.add.at(abs_sum, np.asarray(batch), np.abs(cap["atom_energy"].numpy()))
    return E, F, abs_sum


def max_atom_dev(Fv, F_ref):
    """Largest per-atom force deviation relative to the largest reference force."""
    d = np.asarray(Fv, np.float64) - np.asarray(F_ref, np.float64)
    return float(np.sqrt((d * d).sum(1)).max() / np.sqrt((np.asarray(F_ref, np.float64) ** 2).sum(1)).max())


def poison_workspace(model, n, S, max_pairs, box=None, precision="fp32", path="fused"):
    """Fill the model's workspace with 0xFF bytes (NaN in FP32 and FP64) before a parity call, so a
    kernel reading scratch it did not write shows up as a wrong result."""
    buf = model.ws.get(model.workspace_bytes(n, S, max_pairs, box=box, precision=precision, path=path))
    buf.fill_(0xFF)


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
