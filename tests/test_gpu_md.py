"""Captured velocity-Verlet MD on the GPU against the oracle's FP64 velocity-Verlet
trajectory (oracle/md.py: same kick, drift, wrap and rebuilt neighbours, oracle forces),
element by element after several steps, in a rectangular box and a triclinic cell."""

import numpy as np
import pytest
import torch

from oracle import TensorNetOracle
from oracle.md import tensornet_forces, velocity_verlet
from paper_2402_17660_amd import TensorNet, capture
from synth import maxwell_boltzmann
from synth.generators import masses
from tests.util import random_box, random_in_cell, random_triclinic_cell, small_blob

pytestmark = pytest.mark.gpu

# FP32 positions carry about 1e-6 A of rounding per step; forces agree to ~1e-6 relative:
# after 10 steps of 1 fs the trajectories stay within 1e-4 A and 1e-4 relative in velocity
POS_TOL = 1e-4
VEL_TOL = 1e-4


def _min_image_dev(a, b, H):
    d = (np.asarray(a, np.float64) - np.asarray(b, np.float64)) @ np.linalg.inv(H)
    d -= np.round(d)
    return float(np.abs(d @ H).max())


@pytest.mark.parametrize("kind", ["rectangular", "triclinic"])
def test_md_trajectory_matches_oracle(dev, kind):
    n, steps, dt = 150, 10, 1.0
    if kind == "rectangular":
        pos0, z, H = random_box(n, 91, 12.0)
    else:
        H = random_triclinic_cell(92, 4.5, (2.5, 2.8))
        pos0, z = random_in_cell(n, 92, H)
    pos0 = pos0.astype(np.float32)
    blob = small_blob(F=64, K=32, L=2, seed=93, r_c=4.5)
    m_amu = masses(z)
    vel0 = maxwell_boltzmann(z, 300.0, seed=94)
    batch = np.zeros(n, np.int32)
    print(f"md parity {kind}: n={n} steps={steps}", flush=True)

    model = TensorNet(blob, dev)
    pos = torch.tensor(pos0, device=dev)
    zt = torch.tensor(z, dtype=torch.int32, device=dev)
    bt = torch.tensor(batch, device=dev)
    vel = torch.tensor(vel0, device=dev)
    im = torch.tensor((1.0 / m_amu).astype(np.float32), device=dev)
    mp = 40 * n
    E, Fo = model.energy_forces(pos, zt, bt, 1, box=H, max_pairs=mp, precision="fp32")
    g, E_out, F_out, n_pairs, status = capture(model, pos, zt, bt, 1, box=H, max_pairs=mp, precision="fp32",
                                               n_steps=steps, vel=vel, inv_mass=im, dt_fs=dt, forces_out=Fo)
    g.replay()
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    p_gpu, v_gpu, e_gpu = pos.cpu().numpy(), vel.cpu().numpy(), float(E_out[0])
    g.close()
    model.close()

    o = TensorNetOracle(blob)
    x, v, pot, kin = velocity_verlet(tensornet_forces(o, z, batch, H), pos0.astype(np.float64),
                                     vel0.astype(np.float64), m_amu, H, dt, steps)
    moved = _min_image_dev(x, pos0, H)
    dpos = _min_image_dev(p_gpu, x, H)
    dvel = float(np.linalg.norm(v_gpu - v) / np.linalg.norm(v))
    de = abs(e_gpu - pot[-1]) / abs(pot[-1])
    print(f"  moved {moved:.3e} A; position dev {dpos:.2e} A, velocity rel {dvel:.2e}, final E_pot rel {de:.2e}",
          flush=True)
    assert moved > 1e-2
    assert dpos <= POS_TOL
    assert dvel <= VEL_TOL
    assert de <= 1e-5
    frac = p_gpu.astype(np.float64) @ np.linalg.inv(H)
    assert frac.min() >= -1e-6 and frac.max() < 1.0 + 1e-6


def test_capture_without_forces_starts_from_the_current_forces(dev):
    """capture(n_steps>0) without forces_out computes F(pos) first instead of kicking with zeros."""
    n = 100
    pos0, z, H = random_box(n, 95, 10.0)
    pos0 = pos0.astype(np.float32)
    blob = small_blob(F=64, K=32, L=2, seed=96, r_c=4.5)
    m_amu = masses(z)
    vel0 = maxwell_boltzmann(z, 300.0, seed=97)
    zt = torch.tensor(z, dtype=torch.int32, device=dev)
    bt = torch.zeros(n, dtype=torch.int32, device=dev)
    im = torch.tensor((1.0 / m_amu).astype(np.float32), device=dev)
    model = TensorNet(blob, dev)
    out = []
    for explicit in (True, False):
        pos = torch.tensor(pos0, device=dev)
        vel = torch.tensor(vel0, device=dev)
        Fo = None
        if explicit:
            _, Fo = model.energy_forces(pos, zt, bt, 1, box=H, max_pairs=40 * n, precision="fp32")
        g, _, _, _, status = capture(model, pos, zt, bt, 1, box=H, max_pairs=40 * n, precision="fp32", n_steps=3,
                                     vel=vel, inv_mass=im, dt_fs=1.0, forces_out=Fo)
        g.replay()
        torch.cuda.synchronize()
        assert int(status.item()) == 0
        out.append((pos.cpu().numpy(), vel.cpu().numpy()))
        g.close()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    model.close()
