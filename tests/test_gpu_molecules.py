"""The molecule path (one launch in which a workgroup owns whole isolated systems) against the
FP64 oracle and against the fused path, whose arithmetic it shares stage for stage: FP32 results
must be the same bits as the fused path's on the same inputs; BF16 results (whose FP32 islands
are compiled into two different kernels, where the compiler may fuse multiply-adds
differently) within 1e-6 of the energy and 1e-5 of the largest force.  Also: uneven
batches with empty and one-atom systems, the proportional pair budget and its overflow
flag, rejection of periodic boxes, and graph capture.  Workspaces are NaN-filled before
each call."""

import os

import numpy as np
import pytest
import torch

from oracle import TensorNetOracle
from paper_2402_17660_amd import TensorNet, TensorNetError, capture
from paper_2402_17660_amd import _lib as L
from synth import make_config, make_weights, write_blob
from tests.util import (energy_errors_r21, max_atom_dev, oracle_energy_forces_r21, poison_workspace, random_molecule,
                        rel_rms, small_blob)

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL = {"fp32": (1e-6, 1e-5), "bf16": (None, 2e-2)}


def cfg_blob(c):
    return write_blob(make_weights(c["F"], c["K"], c["L"], c["max_z"], seed=c["weight_seed"]), c["F"], c["K"],
                      c["L"], c["max_z"], c["r_c"])


def same_as_fused(precision, E, F, Ef, Ff):
    if precision == "fp32":
        return np.array_equal(E, Ef) and np.array_equal(F, Ff)
    return (np.abs(E - Ef).max() <= 1e-6 * np.abs(Ef).max()
            and np.abs(F - Ff).max() <= 1e-5 * np.abs(Ff).max())


def run(dev, m, pos, z, batch, S, precision, path, max_pairs):
    p = torch.tensor(np.asarray(pos), dtype=torch.float32, device=dev)
    zt = torch.tensor(np.asarray(z), dtype=torch.int32, device=dev)
    bt = torch.tensor(np.asarray(batch), dtype=torch.int32, device=dev)
    poison_workspace(m, len(p), S, max_pairs, precision=precision, path=path)
    E, F = m.energy_forces(p, zt, bt, S, max_pairs=max_pairs, precision=precision, path=path)
    return E.cpu().numpy(), F.cpu().numpy(), int(m.n_pairs.item())


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_molecule48_oracle_and_fused_bits(dev, precision):
    c = make_config(0)
    m = TensorNet(cfg_blob(c), dev)
    g = np.load(os.path.join(GOLDEN, "oracle_cfg0.npz"))
    mp = 32 * len(c["pos"])
    E, F, npairs = run(dev, m, c["pos"], c["z"], c["batch"], 1, precision, "molecule", mp)
    Ef, Ff, npf = run(dev, m, c["pos"], c["z"], c["batch"], 1, precision, "fused", mp)
    assert npairs == npf == int(g["n_pairs"])
    ee = abs(E[0] - g["E"][0]) / abs(g["E"][0])
    fe = rel_rms(F, g["F"])
    print(f"molecule path cfg0 {precision}: energy rel err {ee:.3e}, force rel RMS {fe:.3e}", flush=True)
    te, tf = TOL[precision]
    if te is not None:
        assert ee <= te
    assert fe <= tf
    assert same_as_fused(precision, E, F, Ef, Ff)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_512_molecules_oracle_and_fused_bits(dev, precision):
    c = make_config(2)
    g = np.load(os.path.join(GOLDEN, "oracle_cfg2.npz"))
    m = TensorNet(cfg_blob(c), dev)
    mp = 32 * len(c["pos"])
    E, F, npairs = run(dev, m, c["pos"], c["z"], c["batch"], c["n_systems"], precision, "molecule", mp)
    assert int(m.status.item()) == 0
    assert npairs == int(g["n_pairs"])
    Ef, Ff, _ = run(dev, m, c["pos"], c["z"], c["batch"], c["n_systems"], precision, "fused", mp)
    ee = float(np.max(np.abs(E - g["E"]) / np.abs(g["E"])))
    fe = rel_rms(F, g["F"])
    print(f"molecule path cfg2 {precision}: energy rel err {ee:.3e}, force rel RMS {fe:.3e}, max atom dev "
          f"{max_atom_dev(F, g['F']):.3e}", flush=True)
    te, tf = TOL[precision]
    if te is not None:
        assert ee <= te
    assert fe <= tf
    if precision == "bf16":
        assert max_atom_dev(F, g["F"]) <= 0.1
    assert same_as_fused(precision, E, F, Ef, Ff)


def test_uneven_batch_with_empty_and_single_atom_systems(dev):
    parts = [random_molecule(n, 300 + n) for n in (17, 1, 64, 5, 33)]
    blob = small_blob(F=64, K=32, L=2, seed=77)
    m = TensorNet(blob, dev)
    # systems 0..6 with system 2 and system 5 empty
    sys_of = [0, 1, 3, 4, 6]
    pos = np.concatenate([p for p, _ in parts]).astype(np.float32)
    z = np.concatenate([q for _, q in parts])
    batch = np.concatenate([np.full(len(p), s, np.int32) for s, (p, _) in zip(sys_of, parts)])
    S = 7
    E_ref, F_ref, abs_sum = oracle_energy_forces_r21(TensorNetOracle(blob), pos, z, batch, None, S)
    E, F, _ = run(dev, m, pos, z, batch, S, "fp32", "molecule", 32 * len(pos))
    assert int(m.status.item()) == 0
    assert E[2] == 0.0 and E[5] == 0.0
    nz = [s for s in range(S) if s not in (2, 5)]
    errs, _ = energy_errors_r21(E[nz], E_ref[nz], abs_sum[nz])
    fe = rel_rms(F, F_ref)
    print(f"uneven batch: energy errors {errs}, force rel RMS {fe:.3e}", flush=True)
    assert errs.max() <= 1e-6 and fe <= 1e-5
    assert np.all(F[17] == 0.0)   # the lone atom has no neighbours
    Ef, Ff, _ = run(dev, m, pos, z, batch, S, "fp32", "fused", 32 * len(pos))
    assert np.array_equal(E, Ef) and np.array_equal(F, Ff)


def test_pair_budget_split_and_overflow(dev):
    c = make_config(0)
    m = TensorNet(cfg_blob(c), dev)
    g = np.load(os.path.join(GOLDEN, "oracle_cfg0.npz"))
    true_pairs = int(g["n_pairs"])
    p = torch.tensor(c["pos"], dtype=torch.float32, device=dev)
    zt = torch.tensor(c["z"], dtype=torch.int32, device=dev)
    bt = torch.tensor(c["batch"], dtype=torch.int32, device=dev)
    m.energy_forces(p, zt, bt, 1, max_pairs=true_pairs - 20, precision="fp32", path="molecule", check=False)
    assert int(m.status.item()) & L.TN_STATUS_OVERFLOW
    assert int(m.n_pairs.item()) == true_pairs
    # exactly enough slots (the budget rounds up to whole 16-pair blocks) is not an overflow
    m.energy_forces(p, zt, bt, 1, max_pairs=true_pairs, precision="fp32", path="molecule")
    assert int(m.status.item()) == 0


def test_periodic_box_is_unsupported(dev):
    c = make_config(0)
    m = TensorNet(cfg_blob(c), dev)
    p = torch.tensor(c["pos"], dtype=torch.float32, device=dev)
    zt = torch.tensor(c["z"], dtype=torch.int32, device=dev)
    bt = torch.tensor(c["batch"], dtype=torch.int32, device=dev)
    with pytest.raises(TensorNetError):
        m.energy_forces(p, zt, bt, 1, box=np.diag([30.0] * 3), max_pairs=4096, precision="fp32", path="molecule")
    with pytest.raises(TensorNetError):
        m.energy_forces(p.double(), zt, bt, 1, max_pairs=4096, precision="fp64", path="molecule")


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_molecule_path_in_a_graph(dev, precision):
    c = make_config(2)
    m = TensorNet(cfg_blob(c), dev)
    p = torch.tensor(c["pos"], dtype=torch.float32, device=dev)
    zt = torch.tensor(c["z"], dtype=torch.int32, device=dev)
    bt = torch.tensor(c["batch"], dtype=torch.int32, device=dev)
    mp = 32 * len(c["pos"])
    E0, F0 = m.energy_forces(p, zt, bt, c["n_systems"], max_pairs=mp, precision=precision, path="molecule")
    E0, F0 = E0.cpu().numpy(), F0.cpu().numpy()
    gr, E, Fo, n_pairs, status = capture(m, p, zt, bt, c["n_systems"], max_pairs=mp, precision=precision,
                                         path="molecule")
    for rep in range(3):
        E.zero_()
        Fo.zero_()
        gr.replay()
        torch.cuda.synchronize()
        assert int(status.item()) == 0
        assert np.array_equal(E.cpu().numpy(), E0), rep
        assert np.array_equal(Fo.cpu().numpy(), F0), rep
        m.energy_forces(p, zt, bt, c["n_systems"], max_pairs=mp, precision=precision, path="fused")
    gr.close()
