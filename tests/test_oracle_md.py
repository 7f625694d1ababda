"""Pins of the oracle's velocity-Verlet integrator (oracle/md.py) against what fixes it
independently: the SI constants behind the unit factor, exact motion under a constant force,
the analytic harmonic oscillator and the method's second order, free flight through periodic
(rectangular and triclinic) boundaries, time reversibility and energy conservation with the
oracle's TensorNet forces."""

import math

import numpy as np
import pytest
import scipy.constants as sc

from oracle import TensorNetOracle
from oracle.md import ACCEL, kinetic_energy, tensornet_forces, velocity_verlet, wrap
from synth import maxwell_boltzmann
from synth.generators import masses
from tests.util import random_box, random_in_cell, random_molecule, random_triclinic_cell, small_blob


def test_unit_factor_from_codata():
    # (eV / angstrom) / amu in angstrom / fs^2 from scipy's CODATA values (the atomic mass
    # constant moved by 1.4e-9 relative between the 2018 and 2022 adjustments)
    ref = sc.electron_volt / sc.angstrom / sc.atomic_mass * (sc.femto ** 2 / sc.angstrom)
    assert abs(ACCEL / ref - 1.0) < 1e-8


def test_constant_force_is_integrated_exactly():
    rng = np.random.default_rng(1)
    n = 7
    x0, v0 = rng.normal(size=(n, 3)), 0.01 * rng.normal(size=(n, 3))
    m = rng.uniform(1.0, 16.0, size=n)
    Fc = rng.normal(size=(n, 3))
    dt, steps = 0.7, 25
    x, v, pot, kin = velocity_verlet(lambda x: (0.0, Fc), x0, v0, m, None, dt, steps)
    a = ACCEL * Fc / m[:, None]
    t = dt * steps
    assert np.allclose(x, x0 + v0 * t + 0.5 * a * t * t, rtol=0, atol=1e-12)
    assert np.allclose(v, v0 + a * t, rtol=0, atol=1e-14)
    assert len(pot) == len(kin) == steps + 1


def test_harmonic_oscillator_second_order():
    m = np.array([2.0])
    k = 3.0   # eV / A^2
    w = math.sqrt(k * ACCEL / m[0])
    x0, v0 = np.array([[0.3, -0.1, 0.2]]), np.array([[0.01, 0.02, -0.015]])
    T = 40.0

    def err(dt):
        n = int(round(T / dt))
        x, v, _, _ = velocity_verlet(lambda x: (0.5 * k * float((x * x).sum()), -k * x), x0, v0, m, None, dt, n)
        ref = x0 * math.cos(w * T) + v0 / w * math.sin(w * T)
        return float(np.abs(x - ref).max())

    e1, e2 = err(0.4), err(0.2)
    assert e1 < 1e-2
    assert 3.6 < e1 / e2 < 4.4   # global error O(dt^2)


@pytest.mark.parametrize("triclinic", [False, True])
def test_free_flight_wraps_into_the_cell(triclinic):
    rng = np.random.default_rng(5)
    H = random_triclinic_cell(5, 4.5) if triclinic else np.diag([11.0, 12.0, 13.0])
    n = 20
    x0 = rng.uniform(0, 1, size=(n, 3)) @ H
    v0 = rng.normal(size=(n, 3)) * 0.8   # several boxes over the run
    dt, steps = 1.0, 30
    x, v, _, _ = velocity_verlet(lambda x: (0.0, np.zeros_like(x)), x0, v0, np.ones(n), H, dt, steps)
    s = x @ np.linalg.inv(H)
    assert (s >= 0).all() and (s < 1).all()
    # the unwrapped straight line and the wrapped result differ by a lattice vector
    k = (x0 + v0 * dt * steps - x) @ np.linalg.inv(H)
    assert np.abs(k - np.round(k)).max() < 1e-9
    assert np.array_equal(v, v0)


def test_wrap_is_a_lattice_shift():
    H = random_triclinic_cell(9, 4.5)
    rng = np.random.default_rng(9)
    x = rng.normal(size=(50, 3)) * 30
    k = (x - wrap(x, H)) @ np.linalg.inv(H)
    assert np.abs(k - np.round(k)).max() < 1e-9


def test_time_reversibility_with_tensornet_forces():
    pos, z = random_molecule(16, 71)
    o = TensorNetOracle(small_blob(F=16, K=8, L=1))
    batch = np.zeros(len(z), np.int32)
    fn = tensornet_forces(o, z, batch, None)
    m = masses(z)
    v0 = maxwell_boltzmann(z, 300.0, seed=72).astype(np.float64)
    x1, v1, _, _ = velocity_verlet(fn, pos.astype(np.float64), v0, m, None, 0.5, 6)
    x2, v2, _, _ = velocity_verlet(fn, x1, -v1, m, None, 0.5, 6)
    assert np.abs(x2 - pos).max() < 1e-10
    assert np.abs(v2 + v0).max() < 1e-10
    assert np.abs(x1 - pos).max() > 1e-3   # the atoms did move


def test_energy_conservation_with_tensornet_forces():
    pos, z, box = random_box(40, 73, 9.5)
    o = TensorNetOracle(small_blob(F=16, K=8, L=1))
    batch = np.zeros(len(z), np.int32)
    fn = tensornet_forces(o, z, batch, box)
    m = masses(z)
    v0 = maxwell_boltzmann(z, 300.0, seed=74).astype(np.float64)

    def drift(dt, T=4.0):
        _, _, pot, kin = velocity_verlet(fn, pos.astype(np.float64), v0, m, box, dt, int(round(T / dt)))
        tot = np.array(pot) + np.array(kin)
        return float(np.abs(tot - tot[0]).max()), float(np.ptp(kin))

    d1, swing = drift(0.5)
    d2, _ = drift(0.25)
    assert d1 < 0.05 * swing          # total energy far steadier than its kinetic part
    assert 2.5 < d1 / d2 < 5.5        # and its error shrinks as dt^2


def test_kinetic_energy_units():
    # equipartition at the generator's temperature: <KE> = 3/2 N k_B T
    z = np.array([1, 6, 7, 8] * 2500, dtype=np.int32)
    v = maxwell_boltzmann(z, 300.0, seed=4003).astype(np.float64)
    ke = kinetic_energy(v, masses(z))
    expect = 1.5 * len(z) * sc.k / sc.electron_volt * 300.0
    assert abs(ke / expect - 1.0) < 0.03
