"""HIP-graph capture: a captured energy+forces evaluation replays to the eager result
(several replays with eager work in between), and captured velocity-Verlet MD is
consistent between one n-step graph and n one-step replays, conserves momentum and
keeps the total energy to within the integrator's error."""

import numpy as np
import pytest
import torch

from paper_2402_17660_amd import TensorNet, capture
from synth import make_config, make_weights, write_blob
from synth.generators import MASS_BY_Z
from tests.util import random_box, small_blob

pytestmark = pytest.mark.gpu


def _inputs(dev, pos, z, batch):
    return (torch.tensor(pos, dtype=torch.float32, device=dev), torch.tensor(z, dtype=torch.int32, device=dev),
            torch.tensor(batch, dtype=torch.int32, device=dev))


@pytest.mark.parametrize("cfg,precision", [(0, "fp32"), (2, "fp32"), (2, "bf16"), (1, "fp32")])
def test_captured_energy_forces_replays(dev, cfg, precision):
    c = make_config(cfg)
    m = TensorNet(write_blob(make_weights(c["F"], c["K"], c["L"], c["max_z"], seed=c["weight_seed"]),
                             c["F"], c["K"], c["L"], c["max_z"], c["r_c"]), dev)
    pos, z, batch = _inputs(dev, c["pos"], c["z"], c["batch"])
    mp = 64 * len(c["pos"]) if cfg != 1 else 170_000
    E0, F0 = m.energy_forces(pos, z, batch, c["n_systems"], box=c["box"], max_pairs=mp, precision=precision)
    E0, F0 = E0.cpu().numpy(), F0.cpu().numpy()
    g, E, Fo, n_pairs, status = capture(m, pos, z, batch, c["n_systems"], box=c["box"], max_pairs=mp,
                                        precision=precision)
    for rep in range(3):
        E.zero_()
        Fo.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert int(status.item()) == 0
        assert np.array_equal(E.cpu().numpy(), E0), rep
        assert np.array_equal(Fo.cpu().numpy(), F0), rep
        # unrelated eager work between replays
        m.energy_forces(pos, z, batch, c["n_systems"], box=c["box"], max_pairs=mp, precision=precision)
    g.close()


def _md_setup(dev, seed=3):
    pos, z, box = random_box(200, seed, 13.0)
    rng = np.random.default_rng(seed)
    m_amu = np.array([MASS_BY_Z[int(a)] for a in z])
    vel = rng.normal(0.0, 0.01, size=(200, 3)).astype(np.float32)
    vel -= (m_amu[:, None] * vel).sum(0) / m_amu.sum()
    return pos.astype(np.float32), z, box, vel.astype(np.float32), (1.0 / m_amu).astype(np.float32), m_amu


def test_md_graph_consistency_and_conservation(dev):
    model = TensorNet(small_blob(F=64, K=32, L=2, seed=5, r_c=4.5), dev)
    pos0, z, box, vel0, inv_m, m_amu = _md_setup(dev)
    batch = np.zeros(200, np.int32)
    runs = []
    for n_steps, replays in ((10, 1), (1, 10)):
        pos, zt, bt = _inputs(dev, pos0, z, batch)
        vel = torch.tensor(vel0, device=dev)
        im = torch.tensor(inv_m, device=dev)
        E, Fo = model.energy_forces(pos, zt, bt, 1, box=box, max_pairs=20000, precision="fp32")
        E_start = float(E[0])
        ke_start = 0.5 * float((torch.tensor(m_amu, device=dev)[:, None] * vel.double() ** 2).sum()) / 9.648533212e-3
        g, E_out, F_out, n_pairs, status = capture(model, pos, zt, bt, 1, box=box, max_pairs=20000, precision="fp32",
                                                   n_steps=n_steps, vel=vel, inv_mass=im, dt_fs=0.1,
                                                   forces_out=Fo)
        for _ in range(replays):
            g.replay()
        torch.cuda.synchronize()
        assert int(status.item()) == 0
        runs.append((pos.cpu().numpy(), vel.cpu().numpy(), float(E_out[0]), E_start, ke_start))
        g.close()
    (p1, v1, e1, es, ks), (p2, v2, e2, _, _) = runs
    assert np.array_equal(p1, p2) and np.array_equal(v1, v2) and e1 == e2
    mom = (m_amu[:, None] * v1.astype(np.float64)).sum(0)
    assert np.abs(mom).max() < 1e-4
    ke_end = 0.5 * float((m_amu[:, None] * v1.astype(np.float64) ** 2).sum()) / 9.648533212e-3
    drift = abs((e1 + ke_end) - (es + ks))
    print(f"MD: E_pot {es:.6f} -> {e1:.6f}, E_kin {ks:.6f} -> {ke_end:.6f}, total drift {drift:.3e}", flush=True)
    assert drift < 1e-3 * max(1.0, abs(es))


def test_md_triclinic_cell_wraps_and_conserves(dev):
    from tests.util import random_in_cell, random_triclinic_cell
    H = random_triclinic_cell(81, 4.5, (2.6, 3.0))
    pos0, z = random_in_cell(200, 81, H)
    rng = np.random.default_rng(82)
    m_amu = np.array([MASS_BY_Z[int(a)] for a in z])
    vel0 = rng.normal(0.0, 0.01, size=(200, 3))
    vel0 -= (m_amu[:, None] * vel0).sum(0) / m_amu.sum()
    model = TensorNet(small_blob(F=64, K=32, L=2, seed=83, r_c=4.5), dev)
    batch = np.zeros(200, np.int32)
    pos, zt, bt = _inputs(dev, pos0, z, batch)
    vel = torch.tensor(vel0.astype(np.float32), device=dev)
    im = torch.tensor((1.0 / m_amu).astype(np.float32), device=dev)
    E, Fo = model.energy_forces(pos, zt, bt, 1, box=H, max_pairs=20000, precision="fp32")
    es = float(E[0])
    ks = 0.5 * float((m_amu[:, None] * vel0 ** 2).sum()) / 9.648533212e-3
    g, E_out, F_out, n_pairs, status = capture(model, pos, zt, bt, 1, box=H, max_pairs=20000, precision="fp32",
                                               n_steps=20, vel=vel, inv_mass=im, dt_fs=0.1, forces_out=Fo)
    g.replay()
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    p = pos.cpu().numpy().astype(np.float64)
    frac = p @ np.linalg.inv(H)
    assert frac.min() >= -1e-5 and frac.max() <= 1.0 + 1e-5      # wrapped into the cell
    v1 = vel.cpu().numpy().astype(np.float64)
    ke = 0.5 * float((m_amu[:, None] * v1 ** 2).sum()) / 9.648533212e-3
    drift = abs((float(E_out[0]) + ke) - (es + ks))
    print(f"triclinic MD: E_pot {es:.6f} -> {float(E_out[0]):.6f}, total drift {drift:.3e}", flush=True)
    assert drift < 1e-3 * max(1.0, abs(es))
    g.close()
