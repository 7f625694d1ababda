"""GPU neighbour search (tn_build_neighbors) against the oracle's pair set: bit-exact
as sorted sets, including tiny boxes with 1-3 cells per side, padding, overflow,
empty inputs, float64 positions and the 100k-atom box."""

import numpy as np
import pytest
import torch

from oracle.neighbors import brute_force_pairs, neighbor_pairs
from paper_2402_17660_amd import _lib as L
from paper_2402_17660_amd import build_neighbors
from synth import make_config, random_cloud
from tests.util import random_box, random_molecule

pytestmark = pytest.mark.gpu


def gpu_pairs(dev, pos, batch, box, cutoff, max_pairs, f64=False, method="auto"):
    p = torch.tensor(np.asarray(pos), dtype=torch.float64 if f64 else torch.float32, device=dev)
    b = torch.tensor(np.asarray(batch), dtype=torch.int32, device=dev)
    pairs, n_pairs, status = build_neighbors(p, b, cutoff, max_pairs, box=box, check=False, method=method)
    torch.cuda.synchronize()
    return pairs.cpu().numpy(), int(n_pairs.item()), int(status.item())


def check_against_oracle(dev, pos, batch, box, cutoff, slack=1000, f64=False, method="auto"):
    ref = neighbor_pairs(np.asarray(pos, dtype=np.float64 if f64 else np.float32), batch, box, cutoff)
    max_pairs = len(ref) + slack
    pr, n, st = gpu_pairs(dev, pos, batch, box, cutoff, max_pairs, f64=f64, method=method)
    assert st == 0, st
    assert n == len(ref)
    got = pr[:, :n].T.astype(np.int64)
    assert np.all(got[:, 0] < got[:, 1])
    got = got[np.lexsort((got[:, 1], got[:, 0]))]
    assert np.array_equal(got, ref)          # the same set, compared as sorted canonical pairs
    assert np.all(pr[:, n:] == -1)
    return ref


@pytest.mark.parametrize("cfg", [0, 1, 2])
def test_workload_pair_sets(dev, cfg):
    c = make_config(cfg)
    print(f"neighbours cfg={cfg} N={len(c['pos'])}", flush=True)
    check_against_oracle(dev, c["pos"], c["batch"], c["box"], c["r_c"])


def test_100k_box_pair_set(dev):
    c = make_config(3)
    ref = check_against_oracle(dev, c["pos"], c["batch"], c["box"], c["r_c"], slack=50_000)
    assert len(ref) > 2_500_000


@pytest.mark.parametrize("box_len,n,seed", [(9.0, 60, 1), (10.0, 90, 2), (13.6, 200, 3), (17.0, 300, 4)])
def test_tiny_boxes_unwrapped_input(dev, box_len, n, seed):
    pos, _, box = random_box(n, seed, box_len)
    rng = np.random.default_rng(seed)
    pos = (pos + box_len * rng.integers(-2, 3, size=pos.shape)).astype(np.float32)
    check_against_oracle(dev, pos, np.zeros(n, np.int32), box, 4.5)


def test_float64_positions(dev):
    pos, _, box = random_box(300, 5, 15.0)
    check_against_oracle(dev, pos.astype(np.float64), np.zeros(300, np.int32), box, 4.5, f64=True)
    mol, _ = random_molecule(64, 6)
    check_against_oracle(dev, mol.astype(np.float64), np.zeros(64, np.int32), None, 5.0, f64=True)


def test_periodic_batch_isolation(dev):
    # two systems sharing one box: one cell list, no cross-system pairs
    p1, _, box = random_box(150, 7, 16.0)
    p2, _, _ = random_box(120, 8, 16.0)
    pos = np.concatenate([p1, p2]).astype(np.float32)
    batch = np.array([0] * 150 + [1] * 120, np.int32)
    ref = check_against_oracle(dev, pos, batch, box, 4.5)
    assert np.all(batch[ref[:, 0]] == batch[ref[:, 1]])


def test_max_pairs_independence_and_padding(dev):
    c = make_config(0)
    ref = brute_force_pairs(c["pos"], c["batch"], None, c["r_c"])
    outs = []
    for mp in (len(ref), len(ref) + 1, 4 * len(ref)):
        pr, n, st = gpu_pairs(dev, c["pos"], c["batch"], None, c["r_c"], mp)
        assert st == 0 and n == len(ref)
        assert np.all(pr[:, n:] == -1)
        outs.append(pr[:, :n])
    assert all(np.array_equal(outs[0], o) for o in outs[1:])   # same pairs in the same order


def test_deterministic_order_in_a_box(dev):
    c = make_config(1)
    a, n1, _ = gpu_pairs(dev, c["pos"], c["batch"], c["box"], c["r_c"], 200_000)
    b, n2, _ = gpu_pairs(dev, c["pos"], c["batch"], c["box"], c["r_c"], 200_000)
    assert n1 == n2 and np.array_equal(a, b)


def test_overflow_reports_true_count(dev):
    c = make_config(1)
    ref = neighbor_pairs(c["pos"], c["batch"], c["box"], c["r_c"])
    pr, n, st = gpu_pairs(dev, c["pos"], c["batch"], c["box"], c["r_c"], len(ref) - 1)
    assert st & L.TN_STATUS_OVERFLOW
    assert n == len(ref)
    assert np.all(pr == -1)
    pr, n, st = gpu_pairs(dev, c["pos"], c["batch"], c["box"], c["r_c"], 0)
    assert st & L.TN_STATUS_OVERFLOW and n == len(ref)


def test_empty_and_single_atom(dev):
    pr, n, st = gpu_pairs(dev, np.zeros((0, 3)), np.zeros(0, np.int32), None, 5.0, 16)
    assert n == 0 and st == 0 and np.all(pr == -1)
    pr, n, st = gpu_pairs(dev, np.zeros((1, 3)), np.zeros(1, np.int32), np.diag([12.0] * 3), 5.0, 16)
    assert n == 0 and st == 0 and np.all(pr == -1)


def test_unsorted_batch_flagged(dev):
    pos, _ = random_molecule(40, 9)
    batch = np.array([1] * 20 + [0] * 20, np.int32)
    pr, n, st = gpu_pairs(dev, pos, batch, None, 5.0, 4000)
    assert st & L.TN_STATUS_BATCH
    ref = brute_force_pairs(pos.astype(np.float32), batch, None, 5.0)
    assert n == len(ref)
    got = pr[:, :n].T
    assert np.array_equal(got[np.lexsort((got[:, 1], got[:, 0]))], ref)


def test_nonfinite_position_flagged(dev):
    pos, _, box = random_box(50, 10, 12.0)
    pos = pos.astype(np.float32)
    pos[3, 1] = np.nan
    pr, n, st = gpu_pairs(dev, pos, np.zeros(50, np.int32), box, 4.5, 4000)
    assert st & L.TN_STATUS_NONFINITE
    assert not np.any(pr[:, :n] == 3)


# ---------------------------------------------------------------- search strategies
# The benchmark shape of the neighbour-search study: a uniform random cloud with 64
# neighbours per point on average in a periodic cube, split into systems by index range.
@pytest.mark.parametrize("method", ["cell", "brute"])
@pytest.mark.parametrize("n,n_batches,seed", [(2000, 1, 11), (2000, 2, 12), (3000, 64, 13), (777, 5, 14),
                                              (130, 1, 15)])
def test_random_cloud_strategies(dev, method, n, n_batches, seed):
    c = random_cloud(n, n_batches, seed)
    print(f"random cloud n={n} batches={n_batches} method={method}", flush=True)
    ref = check_against_oracle(dev, c["pos"], c["batch"], c["box"], 5.0, method=method)
    assert np.all(c["batch"][ref[:, 0]] == c["batch"][ref[:, 1]])


def test_strategy_order_is_deterministic(dev):
    c = random_cloud(1500, 3, 16)
    mp = 60_000
    for method in ("cell", "brute"):
        a = gpu_pairs(dev, c["pos"], c["batch"], c["box"], 5.0, mp, method=method)
        b = gpu_pairs(dev, c["pos"], c["batch"], c["box"], 5.0, mp, method=method)
        assert a[2] == 0 and a[1] == b[1]
        assert np.array_equal(a[0], b[0])
    # the brute force keeps the caller's order: pairs come sorted by (i, j)
    pr, n, _ = gpu_pairs(dev, c["pos"], c["batch"], c["box"], 5.0, mp, method="brute")
    got = pr[:, :n].T.astype(np.int64)
    assert np.array_equal(got, got[np.lexsort((got[:, 1], got[:, 0]))])


def test_strategy_overflow_reports_true_count(dev):
    c = random_cloud(1000, 1, 17)
    ref = neighbor_pairs(c["pos"], c["batch"], c["box"], 5.0)
    for method in ("cell", "brute"):
        pr, n, st = gpu_pairs(dev, c["pos"], c["batch"], c["box"], 5.0, len(ref) - 10, method=method)
        assert n == len(ref)
        assert st & L.TN_STATUS_OVERFLOW
        assert np.all(pr == -1)


def test_cell_strategy_needs_a_box(dev):
    mol, _ = random_molecule(20, 18)
    with pytest.raises(Exception):
        gpu_pairs(dev, mol, np.zeros(20, np.int32), None, 5.0, 1000, method="cell")


# ---------------------------------------------------------------- triclinic cells
from tests.util import random_in_cell, random_triclinic_cell  # noqa: E402


@pytest.mark.parametrize("method", ["auto", "brute"])
@pytest.mark.parametrize("seed,n,scale", [(71, 60, (2.0, 2.3)), (72, 150, (2.4, 3.4)), (73, 400, (3.0, 4.5)),
                                          (74, 1500, (5.0, 7.0))])
def test_triclinic_pair_sets(dev, method, seed, n, scale):
    H = random_triclinic_cell(seed, 4.5, scale)
    pos, _ = random_in_cell(n, seed, H, dmin=0.5)
    pos = (pos + np.random.default_rng(seed).integers(-2, 3, size=pos.shape) @ H).astype(np.float32)
    print(f"triclinic pairs n={n} seed={seed} method={method}", flush=True)
    check_against_oracle(dev, pos, np.zeros(n, np.int32), H, 4.5, method=method)


def test_triclinic_two_systems_one_cell(dev):
    H = random_triclinic_cell(75, 4.5, (3.0, 3.5))
    p1, _ = random_in_cell(200, 75, H)
    p2, _ = random_in_cell(150, 76, H)
    pos = np.concatenate([p1, p2]).astype(np.float32)
    batch = np.array([0] * 200 + [1] * 150, np.int32)
    ref = check_against_oracle(dev, pos, batch, H, 4.5)
    assert np.all(batch[ref[:, 0]] == batch[ref[:, 1]])


@pytest.mark.parametrize("method", ["auto", "brute"])
def test_exact_cutoff_distance_is_excluded(dev, method):
    # d^2 == r_c^2 exactly in FP64 (3-4-5 and axis-aligned pairs) is not a pair; one float32 ulp
    # inside is; coincident atoms are (d = 0 < r_c); the same decisions as the oracle's pins
    pos = np.array([[0, 0, 0], [3, 4, 0], [0, 0, 5], [0, 4.9999995, 0], [0, 0, 0], [-3, 0, -4]], np.float32)
    got = check_against_oracle(dev, pos, np.zeros(len(pos), np.int32), None, 5.0, method=method)
    s = {tuple(p) for p in got}
    assert (0, 1) not in s and (0, 2) not in s and (0, 5) not in s
    assert (0, 3) in s and (0, 4) in s
    # across a periodic face: x = 0.5 and x = 7.5 in a 12 A box are 5 A apart through the face
    box = np.diag([12.0, 12.0, 12.0])
    pos = np.array([[0.5, 6, 6], [7.5, 6, 6], [7.5000005, 6, 6], [6, 0.25, 6], [6, 7.25, 6]], np.float32)
    for m in (("auto", "brute") if method == "auto" else ("brute",)):
        got = check_against_oracle(dev, pos, np.zeros(len(pos), np.int32), box, 5.0, method=m)
        s = {tuple(p) for p in got}
        assert (0, 1) not in s and (3, 4) not in s
        assert (0, 2) in s


def test_half_box_displacements_round_half_to_even(dev):
    # Delta / L exactly +1/2 and -1/2 (rint rounds both to zero): the minimum-image vector keeps
    # |v| = L/2, which at r_c = L/2 is exactly the cutoff and is excluded; atoms a whole box
    # apart coincide; the remaining pairs are ordinary.  Cell list and brute force agree with
    # the oracle on every pair
    box_len = 10.0
    box = np.diag([box_len] * 3)
    pos = np.array([[0, 0, 0], [5, 0, 0], [0, 0, 4], [-5, 0, 0], [0, 5, 0], [0, -5, 0], [2.5, 2.5, 2.5],
                    [0, 0, -5], [10, 0, 3], [1, 1, 1]], np.float32)
    for method in ("auto", "brute"):
        got = check_against_oracle(dev, pos, np.zeros(len(pos), np.int32), box, 5.0, method=method)
        s = {tuple(p) for p in got}
        assert (0, 1) not in s and (0, 3) not in s and (0, 4) not in s and (0, 5) not in s and (0, 7) not in s
        assert (1, 3) in s and (4, 5) in s     # a whole box apart: distance 0
        assert (0, 2) in s and (0, 9) in s
