"""Pins of the oracle's neighbour set (O1): brute force by explicit periodic images,
the cell-list accelerator against the brute force, relabelling and batch isolation.
"""

import itertools

import numpy as np
import pytest

from oracle.neighbors import brute_force_pairs, cell_list_pairs, neighbor_pairs, min_cell_count
from tests.util import random_box, random_molecule


def image_enumeration_pairs(pos, batch, box_len, cutoff):
    """Independent definition: minimum over the 27 lattice images of |r_j - r_i + n L|."""
    pos = np.asarray(pos, dtype=np.float64)
    n = len(pos)
    out = []
    shifts = np.array(list(itertools.product((-1, 0, 1), repeat=3)), dtype=np.float64) * box_len
    for i in range(n):
        for j in range(i + 1, n):
            if batch[i] != batch[j]:
                continue
            # wrap the raw difference into [-L/2, L/2) first, so 27 images suffice
            d = pos[j] - pos[i]
            d = d - box_len * np.floor(d / box_len + 0.5)
            best = np.min(np.sum((d[None, :] + shifts) ** 2, axis=1))
            if best < cutoff * cutoff:
                out.append((i, j))
    return np.array(out, dtype=np.int64).reshape(-1, 2)


@pytest.mark.parametrize("box_len,n,seed", [(9.0, 60, 1), (10.5, 90, 2), (13.6, 200, 3), (18.0, 300, 4)])
def test_p1_brute_force_matches_image_enumeration(box_len, n, seed):
    cutoff = 4.5
    pos, _, box = random_box(n, seed, box_len)
    # put some atoms outside [0, L) to exercise the minimum image on unwrapped input
    rng = np.random.default_rng(seed)
    pos = pos + box_len * rng.integers(-2, 3, size=pos.shape)
    pos = pos.astype(np.float32)
    batch = np.zeros(n, dtype=np.int32)
    ref = image_enumeration_pairs(pos, batch, box_len, cutoff)
    got = brute_force_pairs(pos, batch, box, cutoff)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("box_len,n,seed", [(9.0, 60, 11), (10.0, 80, 12), (13.0, 180, 13), (14.0, 250, 14),
                                           (22.0, 1000, 15)])
def test_p1_cell_list_matches_brute_force_periodic(box_len, n, seed):
    cutoff = 4.5
    pos, _, box = random_box(n, seed, box_len)
    pos = pos.astype(np.float32)
    batch = np.zeros(n, dtype=np.int32)
    nc = min_cell_count(box, cutoff)
    assert nc.min() >= 1
    a = brute_force_pairs(pos, batch, box, cutoff)
    b = cell_list_pairs(pos, batch, box, cutoff)
    assert np.array_equal(a, b)


def test_p1_cell_counts_cover_small_grids():
    # the parametrised boxes above include 1 and 2 cells per side
    assert list(min_cell_count(np.diag([9.0] * 3), 4.5)) == [1, 1, 1]
    assert list(min_cell_count(np.diag([10.0] * 3), 4.5)) == [2, 2, 2]
    assert list(min_cell_count(np.diag([14.0] * 3), 4.5)) == [3, 3, 3]


def test_p1_isolated_cluster_cell_list():
    pos, _ = random_molecule(300, 21)
    pos = pos.astype(np.float32)
    batch = np.zeros(300, dtype=np.int32)
    a = brute_force_pairs(pos, batch, None, 5.0)
    b = cell_list_pairs(pos, batch, None, 5.0)
    assert np.array_equal(a, b)
    # explicit O(N^2) check on the isolated set
    p = pos.astype(np.float64)
    ref = [(i, j) for i in range(300) for j in range(i + 1, 300)
           if ((p[j] - p[i]) ** 2).sum() < 25.0]
    assert np.array_equal(a, np.array(ref))


def test_p2_lattice_shift_and_relabel():
    box_len, cutoff = 13.0, 4.5
    pos, _, box = random_box(150, 31, box_len)
    pos = pos.astype(np.float32)
    batch = np.zeros(150, dtype=np.int32)
    base = {tuple(p) for p in brute_force_pairs(pos, batch, box, cutoff)}
    # lattice shift of a few atoms (exact in float32 for these magnitudes)
    shifted = pos.copy()
    shifted[:10] += np.float32(box_len) * np.array([1, -1, 2], dtype=np.float32)
    got = {tuple(p) for p in brute_force_pairs(shifted, batch, box, cutoff)}
    assert got == base
    # relabelling
    perm = np.random.default_rng(0).permutation(150)
    inv = np.argsort(perm)
    got = brute_force_pairs(pos[perm], batch, box, cutoff)
    mapped = {tuple(sorted((perm[i], perm[j]))) for i, j in got}
    assert mapped == base
    assert np.all(inv[perm] == np.arange(150))


def test_p2_batch_isolation_and_additivity():
    # two overlapping molecules: pairs never cross systems, and each system's set
    # equals the set of that molecule alone
    p1, _ = random_molecule(40, 41)
    p2, _ = random_molecule(55, 42)
    pos = np.concatenate([p1, p2]).astype(np.float32)
    batch = np.array([0] * 40 + [1] * 55, dtype=np.int32)
    got = brute_force_pairs(pos, batch, None, 5.0)
    assert np.all(batch[got[:, 0]] == batch[got[:, 1]])
    a = brute_force_pairs(p1.astype(np.float32), np.zeros(40, np.int32), None, 5.0)
    b = brute_force_pairs(p2.astype(np.float32), np.zeros(55, np.int32), None, 5.0) + 40
    assert np.array_equal(got, np.concatenate([a, b]))
    # the batched dispatcher returns the same set
    assert np.array_equal(neighbor_pairs(pos, batch, None, 5.0), got)


def test_strict_cutoff_and_no_self_pairs():
    pos = np.array([[0, 0, 0], [4.5, 0, 0], [0, 4.4999995, 0], [0, 0, 0]], dtype=np.float32)
    batch = np.zeros(4, dtype=np.int32)
    got = {tuple(p) for p in brute_force_pairs(pos, batch, None, 4.5)}
    # exactly at the cutoff is excluded, just inside is included; coincident atoms pair
    assert (0, 1) not in got
    assert (0, 2) in got and (2, 3) in got and (0, 3) in got
    assert all(i < j for i, j in got)


def test_rint_half_to_even():
    # Delta / L exactly 0.5 and -0.5: rint gives 0 and -0 (half to even), so the
    # minimum image keeps |v| = L/2 and the pair at exactly half a box is found
    box_len = 10.0
    pos = np.array([[0, 0, 0], [5.0, 0, 0], [0, 0, 4.0], [-5.0, 0, 0]], dtype=np.float32)
    got = brute_force_pairs(pos, np.zeros(4, np.int32), np.diag([box_len] * 3), 5.01)
    # (1,3) are 10 apart = one full box: distance 0 after the image shift
    assert {tuple(p) for p in got} == {(0, 1), (0, 2), (0, 3), (1, 3)}


# ---------------------------------------------------------------- triclinic cells
from oracle.neighbors import lattice, nearest_image_d2  # noqa: E402
from tests.util import random_in_cell, random_triclinic_cell  # noqa: E402


def enumeration_pairs_cell(pos, batch, H, cutoff):
    """Independent definition for any cell: nearest image by enumerating lattice translations."""
    pos = np.asarray(pos, dtype=np.float64)
    n = len(pos)
    i, j = np.triu_indices(n, 1)
    keep = batch[i] == batch[j]
    i, j = i[keep], j[keep]
    d2 = nearest_image_d2(pos[i], pos[j], H, reach=3)
    m = d2 < cutoff * cutoff
    return np.stack([i[m], j[m]], 1).astype(np.int64), d2


@pytest.mark.parametrize("seed,n", [(31, 60), (32, 120), (33, 200), (34, 300)])
def test_p1_triclinic_sequential_image_is_nearest(seed, n):
    cutoff = 4.5
    H = random_triclinic_cell(seed, cutoff)
    pos, _ = random_in_cell(n, seed, H)
    rng = np.random.default_rng(seed)
    # unwrapped input: shift atoms by random lattice vectors
    pos = (pos + rng.integers(-2, 3, size=(n, 3)) @ H).astype(np.float32)
    batch = np.zeros(n, dtype=np.int32)
    ref, _ = enumeration_pairs_cell(pos, batch, H, cutoff)
    got = brute_force_pairs(pos, batch, H, cutoff)
    assert len(ref) > 0
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("seed,n,scale", [(41, 60, (2.0, 2.3)), (42, 150, (2.5, 3.5)), (43, 400, (3.0, 4.5)),
                                          (44, 1200, (5.0, 6.0))])
def test_p1_triclinic_cell_list_matches_brute_force(seed, n, scale):
    cutoff = 4.5
    H = random_triclinic_cell(seed, cutoff, scale)
    pos, _ = random_in_cell(n, seed, H, dmin=0.5)
    pos = pos.astype(np.float32)
    batch = np.zeros(n, dtype=np.int32)
    a = brute_force_pairs(pos, batch, H, cutoff)
    b = cell_list_pairs(pos, batch, H, cutoff)
    assert len(a) > 0
    assert np.array_equal(a, b)


def test_p2_triclinic_lattice_shift():
    cutoff = 4.5
    H = random_triclinic_cell(45, cutoff)
    pos, _ = random_in_cell(150, 45, H)
    batch = np.zeros(150, dtype=np.int32)
    a = brute_force_pairs(pos, batch, H, cutoff)
    k = np.random.default_rng(46).integers(-1, 2, size=(150, 3))
    b = brute_force_pairs(pos + k @ H, batch, H, cutoff)
    assert np.array_equal(a, b)


def test_triclinic_cell_validation():
    with pytest.raises(ValueError):
        lattice(np.array([[10.0, 1.0, 0.0], [0.0, 10.0, 0.0], [0.0, 0.0, 10.0]]))   # not lower triangular
    with pytest.raises(ValueError):
        lattice(np.array([[10.0, 0.0, 0.0], [6.0, 10.0, 0.0], [0.0, 0.0, 10.0]]))   # not reduced
    H = lattice(np.array([[10.0, 0.0, 0.0], [5.0, 10.0, 0.0], [-5.0, 5.0, 10.0]]))
    assert H.shape == (3, 3)


def test_zero_tilt_cell_is_the_rectangular_box():
    pos, _, box = random_box(200, 47, 13.0)
    batch = np.zeros(200, dtype=np.int32)
    a = brute_force_pairs(pos.astype(np.float32), batch, box, 4.5)
    ref = image_enumeration_pairs(pos.astype(np.float32), batch, 13.0, 4.5)
    assert np.array_equal(a, ref)
