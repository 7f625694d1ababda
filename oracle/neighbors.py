"""O1: the neighbour pair set, written from its definition.

Sec. 2.5.1 of the paper defines the neighbour list as every pair of atoms of
the same system (batch member) closer than the cutoff, without self pairs,
with rectangular (and triclinic) periodic boundaries by the minimum image,
as an upper-bounded list padded with -1.  The reading used here:

  P = {(i, j) : i < j, batch_i == batch_j, d_ij^2 < r_c^2}

  isolated systems   v = r_j - r_i
  rectangular box    v_a = D_a - L_a * rint(D_a / L_a),  D_a = x_ja - x_ia

The arithmetic is pinned so that a GPU implementation can match the set bit
for bit: inputs promoted to float64, rint rounds half to even, the product
L_a * rint(.) is rounded before the subtraction, and
d^2 = (v_x*v_x + v_y*v_y) + v_z*v_z with every product rounded (no fused
multiply-add).  Every numpy ufunc call below rounds its result, so this code
follows that order literally.

`brute_force_pairs` is the O(N^2) definition.  `cell_list_pairs` only prunes
candidate pairs by spatial binning and then applies the same predicate; it is
checked against the brute force in the tests.
"""

from __future__ import annotations

import math

import numpy as np


def _box_lengths(box):
    if box is None:
        return None
    b = np.asarray(box, dtype=np.float64).reshape(3, 3)
    off = b - np.diag(np.diag(b))
    if np.any(off != 0.0):
        raise NotImplementedError("only rectangular boxes")
    return np.diag(b).copy()


def _d2(pi: np.ndarray, pj: np.ndarray, lengths) -> np.ndarray:
    """Squared minimum-image distance in float64, in the pinned operation order."""
    delta = pj.astype(np.float64) - pi.astype(np.float64)
    if lengths is not None:
        q = delta / lengths
        shift = lengths * np.rint(q)
        delta = delta - shift
    vx, vy, vz = delta[:, 0], delta[:, 1], delta[:, 2]
    return (vx * vx + vy * vy) + vz * vz


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
    lengths = _box_lengths(box)
    rc2 = np.float64(cutoff) * np.float64(cutoff)
    ii, jj = [], []
    chunk = max(1, 4_000_000 // max(n, 1))
    for start in range(0, n, chunk):
        rows = np.arange(start, min(n, start + chunk))
        i = np.repeat(rows, n)
        j = np.tile(np.arange(n), len(rows))
        keep = (j > i) & (batch[i] == batch[j])
        i, j = i[keep], j[keep]
        m = _d2(pos[i], pos[j], lengths) < rc2
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
    lengths = _box_lengths(box)
    p64 = pos.astype(np.float64)
    if lengths is not None:
        # side >= cutoff with a relative margin, so rounding in the binning
        # can never put two atoms closer than the cutoff two cells apart
        nc = np.maximum(1, np.floor(lengths / (cutoff * (1.0 + 1e-6))).astype(np.int64))
        side = lengths / nc
        wrapped = p64 - lengths * np.floor(p64 / lengths)
        cell3 = np.minimum(np.floor(wrapped / side).astype(np.int64), nc - 1)
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
                if lengths is not None:
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
                m = _d2(pos[i], pos[j], lengths) < rc2
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
    """Cells per side of the oracle's grid (used by tests that need ncell < 3)."""
    lengths = _box_lengths(box)
    return np.maximum(1, np.floor(lengths / (cutoff * (1.0 + 1e-6))).astype(np.int64))


__all__ = ["brute_force_pairs", "cell_list_pairs", "neighbor_pairs", "min_cell_count", "math"]
