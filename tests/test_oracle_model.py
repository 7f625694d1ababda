"""Pins of the oracle's network (O3-O6).

* P-6/P-18: an independent evaluator for atoms on one line.  Along the z axis
  every feature matrix stays in the commutative algebra spanned by
  {1, J = A0(z), S = S0(z)} with J^2 = S - 2/3, JS = SJ = -J/3, S^2 = S/3 + 2/9,
  and norms ||a 1 + b J + c S|| = 3a^2 + 2b^2 + 2c^2/3.  The evaluator below
  runs the whole network on those three coefficient vectors per atom (numpy,
  no 3x3 matrices) and must agree with the oracle, energies and forces.
* P-8 O(3) invariance/equivariance incl. reflections, P-9 permutation,
  P-10 zero net force and torque, P-11 central finite differences,
  P-12 continuity through the cutoff, P-13 batch additivity, P-14 supercell,
  P-15 lattice-shift invariance, P-19 the YM-only negative control.
"""

import math

import numpy as np
import pytest
import torch

from oracle import TensorNetOracle, decompose
from synth import make_config, make_weights, write_blob
from tests.util import random_box, random_molecule, random_rotation, small_blob


# ----------------------------------------------------------------------------- P-6 / P-18
def _silu(x):
    return x / (1.0 + np.exp(-x))


def _ln(x, g, b):
    m = x.mean()
    v = ((x - m) ** 2).mean()
    return (x - m) / np.sqrt(v + 1e-5) * g + b


def _prod(x, y):
    """Product in the {1, J, S} algebra (commutative)."""
    xa, xb, xc = x
    ya, yb, yc = y
    return (xa * ya - 2.0 / 3.0 * xb * yb + 2.0 / 9.0 * xc * yc,
            xa * yb + xb * ya - (xb * yc + xc * yb) / 3.0,
            xa * yc + xc * ya + xb * yb + xc * yc / 3.0)


def _nrm(x):
    return 3 * x[0] ** 2 + 2 * x[1] ** 2 + 2.0 / 3.0 * x[2] ** 2


def collinear_energy(zpos, species, w, F, K, L, r_c, r_lo=0.0):
    """Energy of atoms at (0, 0, zpos[k]) computed in the {1, J, S} coefficient algebra."""
    n = len(zpos)
    alpha = 5.0 / (r_c - r_lo)
    start = math.exp(-(r_c - r_lo))
    mu = np.array([start + (1 - start) * k / (K - 1) for k in range(K)])
    beta = (2.0 / K * (1 - start)) ** -2
    edges = []
    for i in range(n):
        for j in range(n):
            if i != j and abs(zpos[j] - zpos[i]) < r_c:
                d = abs(zpos[j] - zpos[i])
                sgn = 1.0 if zpos[j] > zpos[i] else -1.0
                phi = 0.5 * (math.cos(math.pi * d / r_c) + 1.0)
                e = phi * np.exp(-beta * (np.exp(-alpha * (d - r_lo)) - mu) ** 2)
                edges.append((i, j, sgn, phi, e))
    Emb = w["emb.E"]
    X = [[np.zeros(F), np.zeros(F), np.zeros(F)] for _ in range(n)]
    for i, j, sgn, phi, e in edges:
        Zij = w["emb.Wz"] @ np.concatenate([Emb[species[i]], Emb[species[j]]]) + w["emb.bz"]
        f0 = w["emb.W0"] @ e + w["emb.b0"]
        a, b, c = f0[:F], f0[F:2 * F], f0[2 * F:]
        X[i][0] += phi * Zij * a
        X[i][1] += phi * Zij * b * sgn
        X[i][2] += phi * Zij * c
    for i in range(n):
        nn = _ln(_nrm(X[i]), w["emb.ln_g"], w["emb.ln_b"])
        g = _silu(w["emb.W2"] @ _silu(w["emb.W1"] @ nn + w["emb.b1"]) + w["emb.b2"])
        X[i] = [g[:F] * (w["emb.WI"] @ X[i][0]), g[F:2 * F] * (w["emb.WA"] @ X[i][1]),
                g[2 * F:] * (w["emb.WS"] @ X[i][2])]
    for l in range(L):
        p = f"layer{l}."
        Xb = [[c / (_nrm(x) + 1.0) for c in x] for x in X]
        Y = [[w[p + "W1I"] @ x[0], w[p + "W1A"] @ x[1], w[p + "W1S"] @ x[2]] for x in Xb]
        M = [[np.zeros(F), np.zeros(F), np.zeros(F)] for _ in range(n)]
        for i, j, sgn, phi, e in edges:
            t = _silu(w[p + "Wa"] @ e + w[p + "ba"])
            t = _silu(w[p + "Wb"] @ t + w[p + "bb"])
            t = phi * _silu(w[p + "Wc"] @ t + w[p + "bc"])
            for k in range(3):
                M[i][k] += t[k * F:(k + 1) * F] * Y[j][k]
        newX = []
        for i in range(n):
            P = [2.0 * c for c in _prod(Y[i], M[i])]      # Y M + M Y = 2 Y M here
            Pb = [c / (_nrm(P) + 1.0) for c in P]
            dX = [w[p + "W2I"] @ Pb[0], w[p + "W2A"] @ Pb[1], w[p + "W2S"] @ Pb[2]]
            sq = _prod(dX, dX)
            newX.append([Xb[i][k] + dX[k] + sq[k] for k in range(3)])
        X = newX
    E = 0.0
    for i in range(n):
        q = np.concatenate([3 * X[i][0] ** 2, 2 * X[i][1] ** 2, 2.0 / 3.0 * X[i][2] ** 2])
        q = _ln(q, w["out.ln_g"], w["out.ln_b"])
        x = _silu(w["out.Wo"] @ q + w["out.bo"])
        E += float((w["out.W2"] @ _silu(w["out.Wh"] @ x + w["out.bh"]) + w["out.b2"])[0])
    return E


def _oracle_line(zpos, species, blob):
    o = TensorNetOracle(blob)
    pos = np.zeros((len(zpos), 3))
    pos[:, 2] = zpos
    E, F = o.energy_forces(pos, np.array(species, dtype=np.int32), np.zeros(len(zpos), np.int32), None, 1)
    return E[0], F


@pytest.mark.parametrize("L", [0, 1, 2])
def test_p6_dimer_closed_form(L):
    F, K, r_c = 8, 6, 4.5
    w = make_weights(F, K, L, 100, seed=11 + L)
    blob = write_blob(w, F, K, L, 100, r_c)
    d = 1.7
    E, Fo = _oracle_line([0.0, d], [6, 8], blob)
    ref = collinear_energy([0.0, d], [6, 8], w, F, K, L, r_c)
    assert abs(E - ref) <= 1e-12 * max(1.0, abs(ref))
    h = 1e-5
    dE = (collinear_energy([0.0, d + h], [6, 8], w, F, K, L, r_c)
          - collinear_energy([0.0, d - h], [6, 8], w, F, K, L, r_c)) / (2 * h)
    # F_1 = -F_2 = E'(d) vhat with vhat = +z
    assert np.allclose(Fo[:, :2], 0.0, atol=1e-13)
    assert abs(Fo[0, 2] - dE) < 1e-8 * max(1.0, abs(dE))
    assert abs(Fo[1, 2] + dE) < 1e-8 * max(1.0, abs(dE))


def test_p6_collinear_chain_all_layers():
    F, K, L, r_c = 12, 8, 2, 5.0
    w = make_weights(F, K, L, 100, seed=5)
    blob = write_blob(w, F, K, L, 100, r_c)
    zpos = [0.0, 1.1, 2.9, 4.2, 7.5, 8.6]
    species = [1, 6, 7, 8, 6, 1]
    E, Fo = _oracle_line(zpos, species, blob)
    ref = collinear_energy(zpos, species, w, F, K, L, r_c)
    assert abs(E - ref) <= 1e-12 * max(1.0, abs(ref))
    h = 1e-5
    for k in (0, 2, 5):
        zp = list(zpos); zp[k] += h
        zm = list(zpos); zm[k] -= h
        dE = (collinear_energy(zp, species, w, F, K, L, r_c) - collinear_energy(zm, species, w, F, K, L, r_c)) / (2 * h)
        assert abs(Fo[k, 2] + dE) < 1e-7 * max(1.0, np.abs(Fo).max())


# ----------------------------------------------------------------------------- O(3), permutation, sums
@pytest.fixture(scope="module")
def mol():
    pos, z = random_molecule(30, 101)
    return pos, z


@pytest.mark.parametrize("reflect", [False, True])
def test_p8_o3_invariance_and_equivariance(mol, reflect):
    pos, z = mol
    blob = small_blob(F=16, K=8, L=2, seed=3)
    o = TensorNetOracle(blob)
    batch = np.zeros(len(pos), np.int32)
    cap0, cap1 = {}, {}
    E0, F0 = o.energy_forces(pos, z, batch, None, 1, capture=cap0)
    Q = random_rotation(7, reflect=reflect)
    t = np.array([0.3, -1.2, 2.5])
    pos2 = pos @ Q.T + t
    E1, F1 = o.energy_forces(pos2, z, batch, None, 1, capture=cap1)
    assert abs(E1[0] - E0[0]) <= 1e-11 * abs(E0[0])
    assert np.allclose(F1, F0 @ Q.T, atol=1e-10 * np.abs(F0).max())
    Qt = torch.tensor(Q)
    det = float(np.linalg.det(Q))
    for key in ("X_emb", "X_layer0", "X_layer1"):
        I0, A0, S0 = decompose(cap0[key])
        I1, A1, S1 = decompose(cap1[key])
        scale = cap0[key].abs().max()
        assert torch.allclose(I1, I0, atol=1e-11 * scale)
        assert torch.allclose(S1, Qt @ S0 @ Qt.T, atol=1e-11 * scale)
        assert torch.allclose(A1, det * (Qt @ A0 @ Qt.T), atol=1e-11 * scale)


def test_p19_negative_control_left_product(mol):
    pos, z = mol
    blob = small_blob(F=16, K=8, L=2, seed=3)
    bad = TensorNetOracle(blob, product="left")
    batch = np.zeros(len(pos), np.int32)
    E0 = bad.energy(pos, z, batch, None, 1)[0]
    Er = bad.energy(pos @ random_rotation(7).T, z, batch, None, 1)[0]
    Ef = bad.energy(pos @ random_rotation(7, reflect=True).T, z, batch, None, 1)[0]
    assert abs(Er - E0) <= 1e-11 * abs(E0)          # still rotation invariant
    assert abs(Ef - E0) > 1e-6 * abs(E0)            # but not reflection invariant


def test_p9_permutation(mol):
    pos, z = mol
    o = TensorNetOracle(small_blob(F=16, K=8, L=2, seed=4))
    batch = np.zeros(len(pos), np.int32)
    E0, F0 = o.energy_forces(pos, z, batch, None, 1)
    perm = np.random.default_rng(5).permutation(len(pos))
    E1, F1 = o.energy_forces(pos[perm], z[perm], batch, None, 1)
    assert abs(E1[0] - E0[0]) <= 1e-12 * abs(E0[0])
    assert np.allclose(F1, F0[perm], atol=1e-12 * np.abs(F0).max())


def test_p10_net_force_and_torque(mol):
    pos, z = mol
    o = TensorNetOracle(small_blob(F=16, K=8, L=2, seed=6))
    batch = np.zeros(len(pos), np.int32)
    _, Fv = o.energy_forces(pos, z, batch, None, 1)
    scale = np.abs(Fv).max()
    assert np.allclose(Fv.sum(0), 0.0, atol=1e-12 * scale * len(pos))
    torque = np.cross(pos.astype(np.float64), Fv).sum(0)
    assert np.allclose(torque, 0.0, atol=1e-11 * scale * len(pos))
    # periodic: net force zero
    pb, zb, box = random_box(100, 8, 10.0)
    _, Fp = o.energy_forces(pb, zb, np.zeros(100, np.int32), box, 1)
    assert np.allclose(Fp.sum(0), 0.0, atol=1e-12 * np.abs(Fp).max() * 100)


def _fd_check(o, pos, z, box, coords, h=1e-5):
    batch = np.zeros(len(pos), np.int32)
    _, Fv = o.energy_forces(pos, z, batch, box, 1)
    pos = pos.astype(np.float64)
    pairs = o.pairs(pos, batch, box)
    worst = 0.0
    for (a, c) in coords:
        p1 = pos.copy(); p1[a, c] += h
        p2 = pos.copy(); p2[a, c] -= h
        # fixed pair set: the displaced atom does not cross the cutoff at this h
        fd = -(o.energy(p1, z, batch, box, 1, pairs=pairs)[0] - o.energy(p2, z, batch, box, 1, pairs=pairs)[0]) / (2 * h)
        worst = max(worst, abs(fd - Fv[a, c]))
    return worst / np.abs(Fv).max()


def test_p11_finite_differences_workload0():
    c = make_config(0)
    w = make_weights(c["F"], c["K"], c["L"], c["max_z"], seed=c["weight_seed"])
    o = TensorNetOracle(write_blob(w, c["F"], c["K"], c["L"], c["max_z"], c["r_c"]))
    rng = np.random.default_rng(9)
    coords = [(int(rng.integers(0, 48)), int(rng.integers(0, 3))) for _ in range(10)]
    assert _fd_check(o, c["pos"].astype(np.float64), c["z"], None, coords) <= 1e-7


def test_p11_finite_differences_periodic():
    pos, z, box = random_box(100, 12, 10.0)
    o = TensorNetOracle(small_blob(F=16, K=8, L=2, seed=13))
    rng = np.random.default_rng(10)
    coords = [(int(rng.integers(0, 100)), int(rng.integers(0, 3))) for _ in range(8)]
    assert _fd_check(o, pos, z, box, coords) <= 1e-7


def test_p12_continuity_through_cutoff():
    # The jump of E and F when a pair crosses r_c is that pair's whole contribution
    # evaluated at d -> r_c.  Place atom 0 just inside r_c of atom 1 and evaluate
    # with and without that pair in the list: the difference must vanish.
    o = TensorNetOracle(small_blob(F=16, K=8, L=2, seed=14, r_c=4.5))
    pos, z = random_molecule(12, 15)
    pos = pos.astype(np.float64)
    u = pos[0] - pos[1]
    u /= np.linalg.norm(u)
    pos[0] = pos[1] + 4.5 * (1 - 1e-7) * u
    batch = np.zeros(12, np.int32)
    pairs = o.pairs(pos, batch, None)
    key = (0, 1)
    assert any(tuple(p) == key for p in pairs)
    without = np.array([p for p in pairs if tuple(p) != key])
    E1, F1 = o.energy_forces(pos, z, batch, None, 1, pairs=pairs)
    E0, F0 = o.energy_forces(pos, z, batch, None, 1, pairs=without)
    assert abs(E1[0] - E0[0]) <= 1e-12
    assert np.abs(F1 - F0).max() <= 1e-6


def test_p13_batch_additivity():
    o = TensorNetOracle(small_blob(F=16, K=8, L=2, seed=16))
    p1, z1 = random_molecule(20, 17)
    p2, z2 = random_molecule(27, 18)
    pos = np.concatenate([p1, p2])
    z = np.concatenate([z1, z2])
    batch = np.array([0] * 20 + [1] * 27, np.int32)
    E, Fv = o.energy_forces(pos, z, batch, None, 2)
    Ea, Fa = o.energy_forces(p1, z1, np.zeros(20, np.int32), None, 1)
    Eb, Fb = o.energy_forces(p2, z2, np.zeros(27, np.int32), None, 1)
    assert np.allclose(E, [Ea[0], Eb[0]], rtol=1e-13, atol=0)
    assert np.allclose(Fv, np.concatenate([Fa, Fb]), atol=1e-13)


def test_p14_supercell():
    r_c = 3.0
    o = TensorNetOracle(small_blob(F=16, K=8, L=2, seed=19, r_c=r_c))
    L_box = (30 / 0.1) ** (1 / 3)
    pos, z, box = random_box(30, 20, L_box)
    E, Fv = o.energy_forces(pos, z, np.zeros(30, np.int32), box, 1)
    shifts = np.array([(a, b, c) for a in (0, 1) for b in (0, 1) for c in (0, 1)], dtype=np.float64) * L_box
    pos8 = np.concatenate([pos + s for s in shifts])
    z8 = np.tile(z, 8)
    E8, F8 = o.energy_forces(pos8, z8, np.zeros(240, np.int32), box * 2, 1)
    assert abs(E8[0] - 8 * E[0]) <= 1e-11 * abs(8 * E[0])
    assert np.allclose(F8, np.tile(Fv, (8, 1)), atol=1e-11 * np.abs(Fv).max())


def test_p15_lattice_shift_invariance():
    o = TensorNetOracle(small_blob(F=16, K=8, L=2, seed=21))
    pos, z, box = random_box(100, 22, 10.0)
    E, Fv = o.energy_forces(pos, z, np.zeros(100, np.int32), box, 1)
    k = np.random.default_rng(23).integers(-2, 3, size=pos.shape)
    E2, F2 = o.energy_forces(pos + 10.0 * k, z, np.zeros(100, np.int32), box, 1)
    assert abs(E2[0] - E[0]) <= 1e-12 * abs(E[0])
    assert np.allclose(F2, Fv, atol=1e-12 * np.abs(Fv).max())


# ---------------------------------------------------------------- triclinic cells
from tests.util import random_in_cell, random_triclinic_cell  # noqa: E402


def test_p14_supercell_triclinic():
    r_c = 3.0
    o = TensorNetOracle(small_blob(F=16, K=8, L=2, seed=51, r_c=r_c))
    H = random_triclinic_cell(52, r_c, (2.1, 2.6))
    pos, z = random_in_cell(30, 52, H)
    E, Fv = o.energy_forces(pos, z, np.zeros(30, np.int32), H, 1)
    shifts = np.array([(a, b, c) for a in (0, 1) for b in (0, 1) for c in (0, 1)], dtype=np.float64) @ H
    pos8 = np.concatenate([pos + s for s in shifts])
    z8 = np.tile(z, 8)
    E8, F8 = o.energy_forces(pos8, z8, np.zeros(240, np.int32), 2 * H, 1)
    assert abs(E8[0] - 8 * E[0]) <= 1e-11 * abs(8 * E[0])
    assert np.allclose(F8, np.tile(Fv, (8, 1)), atol=1e-11 * np.abs(Fv).max())


def test_p15_lattice_shift_invariance_triclinic():
    o = TensorNetOracle(small_blob(F=16, K=8, L=2, seed=53))
    H = random_triclinic_cell(54, 4.5)
    pos, z = random_in_cell(80, 54, H)
    E, Fv = o.energy_forces(pos, z, np.zeros(80, np.int32), H, 1)
    k = np.random.default_rng(55).integers(-2, 3, size=pos.shape)
    E2, F2 = o.energy_forces(pos + k @ H, z, np.zeros(80, np.int32), H, 1)
    assert abs(E2[0] - E[0]) <= 1e-12 * abs(E[0])
    assert np.allclose(F2, Fv, atol=1e-12 * np.abs(Fv).max())


def test_p11_finite_differences_triclinic():
    o = TensorNetOracle(small_blob(F=16, K=8, L=2, seed=56))
    H = random_triclinic_cell(57, 4.5)
    pos, z = random_in_cell(40, 57, H)
    batch = np.zeros(40, np.int32)
    _, Fv = o.energy_forces(pos, z, batch, H, 1)
    pairs = o.pairs(pos, batch, H)
    h = 1e-5
    rng = np.random.default_rng(58)
    for a in rng.choice(40, size=4, replace=False):
        for ax in range(3):
            p1, p2 = pos.copy(), pos.copy()
            p1[a, ax] += h
            p2[a, ax] -= h
            fd = -(o.energy(p1, z, batch, H, 1, pairs=pairs)[0] - o.energy(p2, z, batch, H, 1, pairs=pairs)[0]) / (2 * h)
            assert abs(fd - Fv[a, ax]) <= 1e-7 * max(1.0, np.abs(Fv).max())
