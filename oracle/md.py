"""Velocity-Verlet molecular dynamics on the oracle's forces, in float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper runs TensorNet as the force field of molecular dynamics (Sec. 3.2) and
captures whole steps into CUDA graphs to remove launch overhead (Sec. 2.5); it does
not print its integrator.  The reading used here is the textbook velocity-Verlet
step in angstrom, femtosecond, amu and eV units:

    v <- v + (dt/2) * c * F(x) / m
    x <- x + dt * v,  then wrapped into the periodic cell
    F <- F(x)        (neighbour list rebuilt from the wrapped positions)
    v <- v + (dt/2) * c * F(x) / m

where c converts (eV/angstrom)/amu into angstrom/fs^2.  Wrapping maps every atom into
the cell: fractional coordinates s = x H^-1 (H the rows a, b, c) are reduced to [0, 1).
It leaves energies and forces unchanged, since the model sees positions only through the
minimum image.
"""

from __future__ import annotations

import numpy as np

# c = (1 eV / 1 angstrom) / 1 amu in angstrom / fs^2, from the SI values of the
# elementary charge (J per eV) and the atomic mass constant (kg per amu):
#   1 eV/(A amu) = 1.602176634e-19 J / (1e-10 m * 1.66053906660e-27 kg) in m/s^2,
#   and 1 m/s^2 = 1e10 A / 1e30 fs^2.
EV_J = 1.602176634e-19
AMU_KG = 1.66053906660e-27
ACCEL = EV_J / (1e-10 * AMU_KG) * 1e10 / 1e30


def wrap(pos: np.ndarray, box) -> np.ndarray:
    """Positions mapped into the cell: fractional coordinates reduced to [0, 1)."""
    if box is None:
        return pos
    H = np.asarray(box, dtype=np.float64)
    s = pos @ np.linalg.inv(H)
    s -= np.floor(s)
    return s @ H


def kinetic_energy(vel: np.ndarray, masses: np.ndarray) -> float:
    """Sum of m v^2 / 2 in eV (v in angstrom/fs, m in amu)."""
    return float(0.5 * (masses[:, None] * np.asarray(vel, np.float64) ** 2).sum() / ACCEL)


def velocity_verlet(force_fn, pos, vel, masses, box, dt: float, n_steps: int):
    """n_steps velocity-Verlet steps.  force_fn(x) -> (potential energy, forces [N,3]) in eV, eV/A.

    Returns (positions, velocities, potential energies, kinetic energies), the energy lists
    holding the start and every step's end (n_steps + 1 entries each)."""
    x = np.array(pos, dtype=np.float64)
    v = np.array(vel, dtype=np.float64)
    m = np.asarray(masses, dtype=np.float64)[:, None]
    e_pot, f = force_fn(x)
    pot, kin = [float(e_pot)], [kinetic_energy(v, m[:, 0])]
    for _ in range(n_steps):
        v = v + 0.5 * dt * ACCEL * f / m
        x = wrap(x + dt * v, box)
        e_pot, f = force_fn(x)
        v = v + 0.5 * dt * ACCEL * f / m
        pot.append(float(e_pot))
        kin.append(kinetic_energy(v, m[:, 0]))
    return x, v, pot, kin


def tensornet_forces(oracle, z, batch, box, n_systems: int = 1):
    """force_fn for velocity_verlet: the oracle's total energy and forces (neighbours rebuilt on every call)."""
    def fn(x):
        E, F = oracle.energy_forces(x, z, batch, box, n_systems)
        return float(np.sum(E)), F
    return fn


__all__ = ["ACCEL", "wrap", "kinetic_energy", "velocity_verlet", "tensornet_forces"]
