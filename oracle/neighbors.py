"""O1: the neighbour pair set, written from its definition.

Sec. 2.5.1 of the paper defines the neighbour list as every pair of atoms of
the same system (batch member) closer than the cutoff, without self pairs,
with rectangular and triclinic periodic boundaries by the minimum image, as an
upper-bounded list padded with -1.  The reading used here:

  P = {(i, j) : i < j, batch_i == batch_j, d_ij^2 < r_c^2}

  isolated systems   v = r_j - r_i
  periodic cell      rows a = (a_x, 0, 0), b = (b_x, b_y, 0), c = (c_x, c_y, c_z)
                     in reduced form (|b_x|, |c_x| <= a_x / 2, |c_y| <= b_y / 2),
                     every cell height >= 2 r_c; the minimum image of D = r_j - r_i
                     is taken along c, then b, then a:
                       v = D - c rint(D_z / c_z);  v -= b rint(v_y / b_y);
                       v -= a rint(v_x / a_x)
                     (for a rectangular box this is v_a = D_a - L_a rint(D_a / L_a))

For a reduced cell and distances below half the smallest cell height, this
sequential reduction returns the nearest lattice image; `nearest_image_d2`
enumerates the images directly and the tests compare the two.

The arithmetic is pinned so that a GPU implementation can match the set bit
for bit: inputs promoted to float64, rint rounds half to even, every product
(lattice component * rint(.)) is rounded before the subtraction, and
d^2 = (v_x*v_x + v_y*v_y) + v_z*v_z with every product rounded (no fused
multiply-add).  Every numpy ufunc call below rounds its result, so this code
follows that order literally.

`brute_force_pairs` is the O(N^2) definition.  `cell_list_pairs` only prunes
candidate pairs by binning fractional coordinates (cells at least as high as
the cutoff) and then applies the same predicate; it is checked against the
brute force in the tests.
"""

from __future__ import annotations

import math

import numpy as np


def lattice(box):
    """The periodic cell as a [3, 3] float64 array of rows a, b, c (None for isolated systems).
    Rows must be lower triangular and in reduced form."""
    if box is None:
        return None
    H = np.asarray(box, dtype=np.float64).reshape(3, 3).copy()
    if H[0, 1] != 0.0 or H[0, 2] != 0.0 or H[1, 2] != 0.0:
        raise ValueError("cell rows must be lower triangular: a along x, b in the xy plane")
    if not (H[0, 0] > 0.0 and H[1, 1] > 0.0 and H[2, 2] > 0.0):
        raise ValueError("cell diagonal must be positive")
    if abs(H[1, 0]) > 0.5 * H[0, 0] or abs(H[2, 0]) > 0.5 * H[0, 0] or abs(H[2, 1]) > 0.5 * H[1, 1]:
        raise ValueError("cell is not in reduced form")
    return H


def cell_heights(H):
    """Distances between opposite faces of the cell (1 / |reciprocal vector|)."""
    inv = np.linalg.inv(H)
    return 1.0 / np.linalg.norm(inv, axis=0)


def min_image(delta: np.ndarray, H) -> np.ndarray:
    """Minimum image of displacements [n, 3] (float64), in the pinned operation order."""
    if H is None:
        return delta
    dx, dy, dz = delta[:, 0].copy(), delta[:, 1].copy(), delta[:, 2].copy()
    kz = np.rint(dz / H[2, 2])
    dx = dx - H[2, 0] * kz
    dy = dy - H[2, 1] * kz
    dz = dz - H[2, 2] * kz
    ky = np.rint(dy / H[1, 1])
    dx = dx - H[1, 0] * ky
    dy = dy - H[1, 1] * ky
    kx = np.rint(dx / H[0, 0])
    dx = dx - H[0, 0] * kx
    return np.stack([dx, dy, dz], axis=1)


def _d2(pi: np.ndarray, pj: np.ndarray, H) -> np.ndarray:
    """Squared minimum-image distance in float64, in the pinned operation order."""
    delta = min_image(pj.astype(np.float64) - pi.astype(np.float64), H)
    vx, vy, vz = delta[:, 0], delta[:, 1], delta[:, 2]
    return (vx * vx + vy * vy) + vz * vz


def nearest_image_d2(pi: np.ndarray, pj: np.ndarray, H, reach: int = 2) -> np.ndarray:
    """Squared distance to the nearest periodic image, by enumerating lattice translations
    n_a a + n_b b + n_c c with |n| <= reach around the displacement whose fractional
    coordinates are rounded into [-1/2, 1/2] (the definition, for the tests)."""
    delta = pj.astype(np.float64) - pi.astype(np.float64)
    frac = delta @ np.linalg.inv(H)
    delta = delta - np.rint(frac) @ H
    best = np.full(len(delta), np.inf)
    rng = range(-reach, reach + 1)
    for na in rng:
        for nb in rng:
            for nc in rng:
                t = na * H[0] + nb * H[1] + nc * H[2]
                v = delta + t
                best = np.minimum(best, (v * v).sum(1))
    return best


def _canonical(i: np.ndarray, j: np.ndarray) -> np.ndarray:
    out = np.stack([i, j], axis=1).astype(np.int64)
    if out.size == 0:
        return out.reshape(0, 2)
    order = np.lexsort((out[:, 1], out[:, 0]))
    return out[order]


def brute_force_pairs(pos, batch, box, cutoff: float) -> np.ndarray:
    """Every pair i<j checked: same system first, then distance.  Returns [P,2] int64, sorted."""
    pos = np.asarray(pos)
    batch = np.asarray(batch)
    n = len(pos)
    H = lattice(box)
    rc2 = np.float64(cutoff) * np.float64(cutoff)
    ii, jj = [], []
    chunk = max(1, 4_000_000 // max(n, 1))
    for start in range(0, n, chunk):
        rows = np.arange(start, min(n, start + chunk))
        i = np.repeat(rows, n)
        j = np.tile(np.arange(n), len(rows))
        keep = (j > i) & (batch[i] == batch[j])
        i, j = i[keep], j[keep]
        m = _d2(pos[i], pos[j], H) < rc2
        ii.append(i[m])
        jj.append(j[m])
    if not ii:
        return np.zeros((0, 2), dtype=np.int64)
    return _canonical(np.concatenate(ii), np.concatenate(jj))


def cell_list_pairs(pos, batch, box, cutoff: float) -> np.ndarray:
    """Same set as `brute_force_pairs`, candidates pruned by a cell grid (side >= cutoff)."""
    pos = np.asarray(pos)
    batch = np.asarray(batch)
    n = len(pos)
    if n == 0:
        return np.zeros((0, 2), dtype=np.int64)
    H = lattice(box)
    p64 = pos.astype(np.float64)
    if H is not None:
        # cells at least as high as the cutoff (with a relative margin, so rounding in the
        # binning can never put two atoms closer than the cutoff two cells apart): two atoms
        # within the cutoff then differ by at most one cell along every fractional axis
        nc = np.maximum(1, np.floor(cell_heights(H) / (cutoff * (1.0 + 1e-6))).astype(np.int64))
        frac = p64 @ np.linalg.inv(H)
        frac = frac - np.floor(frac)
        cell3 = np.minimum(np.floor(frac * nc).astype(np.int64), nc - 1)
        offs = []
        for a in range(3):
            if nc[a] == 1:
                offs.append([0])
            elif nc[a] == 2:
                offs.append([0, 1])
            else:
                offs.append([-1, 0, 1])
    else:
        lo = p64.min(0)
        span = p64.max(0) - lo
        side = cutoff * (1.0 + 1e-6)
        nc = np.maximum(1, np.floor(span / side).astype(np.int64) + 1)
        cell3 = np.minimum(np.floor((p64 - lo) / side).astype(np.int64), nc - 1)
        offs = [[-1, 0, 1]] * 3
    lin = (cell3[:, 0] * nc[1] + cell3[:, 1]) * nc[2] + cell3[:, 2]
    order = np.argsort(lin, kind="stable")
    ncell = int(np.prod(nc))
    count = np.bincount(lin, minlength=ncell)
    start = np.concatenate([[0], np.cumsum(count)[:-1]])
    rc2 = np.float64(cutoff) * np.float64(cutoff)
    ii, jj = [], []
    for ox in offs[0]:
        for oy in offs[1]:
            for oz in offs[2]:
                c = cell3 + np.array([ox, oy, oz])
                if H is not None:
                    c = c % nc
                    valid = np.ones(n, dtype=bool)
                else:
                    valid = np.all((c >= 0) & (c < nc), axis=1)
                    c = np.clip(c, 0, nc - 1)
                cl = (c[:, 0] * nc[1] + c[:, 1]) * nc[2] + c[:, 2]
                cnt = np.where(valid, count[cl], 0)
                tot = int(cnt.sum())
                if tot == 0:
                    continue
                i = np.repeat(np.arange(n), cnt)
                first = np.repeat(start[cl], cnt)
                k = np.arange(tot) - np.repeat(np.cumsum(cnt) - cnt, cnt)
                j = order[first + k]
                keep = (j > i) & (batch[i] == batch[j])
                i, j = i[keep], j[keep]
                m = _d2(pos[i], pos[j], H) < rc2
                ii.append(i[m])
                jj.append(j[m])
    if not ii:
        return np.zeros((0, 2), dtype=np.int64)
    return _canonical(np.concatenate(ii), np.concatenate(jj))


def neighbor_pairs(pos, batch, box, cutoff: float) -> np.ndarray:
    """The pair set of O1 as a sorted [P,2] int64 array (brute force when small)."""
    n = len(pos)
    if n <= 2000:
        return brute_force_pairs(pos, batch, box, cutoff)
    if box is None:
        # Isolated systems: the brute force inside each system is exact and cheap.
        batch = np.asarray(batch)
        bounds = np.flatnonzero(np.diff(batch)) + 1
        starts = np.concatenate([[0], bounds])
        ends = np.concatenate([bounds, [n]])
        if len(starts) > 1 and np.all(np.diff(batch) >= 0):
            out = []
            for s, e in zip(starts, ends):
                if e - s > 2000:
                    p = cell_list_pairs(pos[s:e], batch[s:e], None, cutoff)
                else:
                    p = brute_force_pairs(pos[s:e], batch[s:e], None, cutoff)
                out.append(p + s)
            return _canonical(*np.concatenate(out).T) if out else np.zeros((0, 2), np.int64)
    return cell_list_pairs(pos, batch, box, cutoff)


def min_cell_count(box, cutoff):
    """Cells per axis of the oracle's grid (used by tests that need ncell < 3)."""
    return np.maximum(1, np.floor(cell_heights(lattice(box)) / (cutoff * (1.0 + 1e-6))).astype(np.int64))


__all__ = ["brute_force_pairs", "cell_list_pairs", "neighbor_pairs", "min_cell_count", "lattice", "cell_heights",
           "min_image", "nearest_image_d2", "math"]
