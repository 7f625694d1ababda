"""GPU training step (loss and weight gradient, tn_train_grad) against the FP64 oracle's
double-autograd gradient (oracle.train).

Bars: in FP64 the dual-number pass differs from the oracle only by rounding order, so the
loss is held to 1e-11 relative and every gradient tensor to 1e-10 of its largest entry
(measured: below 1e-14).  In FP32 every step runs in single precision (unit roundoff 6e-8)
through sums of up to a few thousand terms and about twenty layers of products, so errors of
order 1e-6 are expected; the bars are 2e-5 of each tensor's largest entry and 2e-6 on the
loss (measured: 3e-6 and 2e-7).
"""

import numpy as np
import pytest
import torch

from oracle import TensorNetOracle
from oracle.train import training_loss_and_grad
from paper_2402_17660_amd import TensorNet
from tests.util import random_box, random_molecule, small_blob

pytestmark = pytest.mark.gpu

BARS = {"fp64": (1e-11, 1e-10), "fp32": (2e-6, 2e-5)}


def _molecules(sizes, seed):
    parts = [random_molecule(n, seed + n) for n in sizes]
    pos = np.concatenate([p for p, _ in parts])
    z = np.concatenate([q for _, q in parts])
    batch = np.concatenate([np.full(len(p), s, np.int32) for s, (p, _) in enumerate(parts)])
    return pos, z, batch


def _gpu(dev, blob, pos, z, batch, box, S, E_ref, F_ref, precision, w_energy=1.0, w_force=1.0):
    m = TensorNet(blob, dev)
    pdt = torch.float64 if precision == "fp64" else torch.float32
    t = lambda a, dt: torch.tensor(np.asarray(a), dtype=dt, device=dev)
    loss, E, F, g = m.train_grad(t(pos, pdt), t(z, torch.int32), t(batch, torch.int32), S, t(E_ref, torch.float64),
                                 t(F_ref, torch.float64), box=box, precision=precision, w_energy=w_energy,
                                 w_force=w_force)
    grads = {k: v.cpu().numpy() for k, v in m.split_params(g).items()}
    return float(loss.item()), E.cpu().numpy(), F.cpu().numpy().astype(np.float64), grads, g


def _check(label, precision, loss, grads, loss_ref, grads_ref):
    tl, tg = BARS[precision]
    assert set(grads) == set(grads_ref)
    worst, where = 0.0, None
    for k, ref in grads_ref.items():
        scale = np.abs(ref).max()
        err = np.abs(grads[k] - ref).max() / scale if scale > 0 else np.abs(grads[k]).max()
        if err > worst:
            worst, where = err, k
    lerr = abs(loss - loss_ref) / abs(loss_ref)
    print(f"{label}: loss {loss:.6e} rel err {lerr:.2e}; worst gradient tensor {where} rel err {worst:.2e}",
          flush=True)
    assert lerr <= tl, (label, lerr)
    assert worst <= tg, (label, where, worst)


def _case(sizes, F, K, L, seed):
    pos, z, batch = _molecules(sizes, seed)
    S = len(sizes)
    E_ref, F_ref = TensorNetOracle(small_blob(F=F, K=K, L=L, seed=seed + 1000)).energy_forces(pos, z, batch, None, S)
    blob = small_blob(F=F, K=K, L=L, seed=seed + 2000)
    return pos, z, batch, S, E_ref, F_ref, blob


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("sizes,F,K,L", [((9, 14), 16, 8, 2), ((12, 17, 23, 31, 40, 8, 19), 32, 16, 2)])
def test_gradient_matches_oracle_molecules(dev, precision, sizes, F, K, L):
    pos, z, batch, S, E_ref, F_ref, blob = _case(sizes, F, K, L, 3)
    loss_ref, g_ref = training_loss_and_grad(TensorNetOracle(blob), pos, z, batch, None, S, E_ref, F_ref)
    loss, E, Fo, grads, _ = _gpu(dev, blob, pos, z, batch, None, S, E_ref, F_ref, precision)
    _check(f"molecules {sizes} F={F} {precision}", precision, loss, grads, loss_ref, g_ref)


@pytest.mark.parametrize("w_energy,w_force", [(0.3, 0.0), (0.0, 2.0)])
def test_loss_weights(dev, w_energy, w_force):
    pos, z, batch, S, E_ref, F_ref, blob = _case((11, 20, 7), 16, 8, 2, 5)
    loss_ref, g_ref = training_loss_and_grad(TensorNetOracle(blob), pos, z, batch, None, S, E_ref, F_ref,
                                             w_energy=w_energy, w_force=w_force)
    loss, _, _, grads, _ = _gpu(dev, blob, pos, z, batch, None, S, E_ref, F_ref, "fp64", w_energy, w_force)
    _check(f"weights {w_energy}:{w_force}", "fp64", loss, grads, loss_ref, g_ref)


def test_gradient_matches_oracle_periodic_box(dev):
    """600 atoms in a periodic box: the cell list reorders atoms, so seeds and position
    tangents go through the permutation."""
    pos, z, box = random_box(600, 77, (600 / 0.1) ** (1 / 3))
    batch = np.zeros(len(pos), np.int32)
    E_ref, F_ref = TensorNetOracle(small_blob(F=16, K=8, L=1, seed=78)).energy_forces(pos, z, batch, box, 1)
    blob = small_blob(F=16, K=8, L=1, seed=79)
    loss_ref, g_ref = training_loss_and_grad(TensorNetOracle(blob), pos, z, batch, box, 1, E_ref, F_ref)
    loss, _, _, grads, _ = _gpu(dev, blob, pos, z, batch, box, 1, E_ref, F_ref, "fp64")
    _check("periodic box 600", "fp64", loss, grads, loss_ref, g_ref)


def test_zero_loss_and_gradient_at_own_predictions(dev):
    """Targets equal to the step's own predictions: loss and every gradient entry exactly zero."""
    pos, z, batch, S, E_ref, F_ref, blob = _case((13, 9, 21), 16, 8, 2, 9)
    for precision in ("fp64", "fp32"):
        _, E, Fo, _, _ = _gpu(dev, blob, pos, z, batch, None, S, E_ref, F_ref, precision)
        loss, _, _, _, g = _gpu(dev, blob, pos, z, batch, None, S, E, Fo, precision)
        assert loss == 0.0, precision
        assert bool((g == 0).all()), precision


def test_deterministic(dev):
    pos, z, batch, S, E_ref, F_ref, blob = _case((15, 22), 16, 8, 2, 11)
    a = _gpu(dev, blob, pos, z, batch, None, S, E_ref, F_ref, "fp32")[4]
    b = _gpu(dev, blob, pos, z, batch, None, S, E_ref, F_ref, "fp32")[4]
    assert torch.equal(a, b)


def test_empty_input(dev):
    m = TensorNet(small_blob(F=16, K=8, L=2, seed=4), dev)
    e = torch.empty(0, dtype=torch.float64, device=dev)
    loss, E, Fo, g = m.train_grad(torch.empty((0, 3), dtype=torch.float64, device=dev),
                                  torch.empty(0, dtype=torch.int32, device=dev),
                                  torch.empty(0, dtype=torch.int32, device=dev), 0, e,
                                  torch.empty((0, 3), dtype=torch.float64, device=dev), precision="fp64")
    assert float(loss.item()) == 0.0
    assert g.numel() == m.param_count() and bool((g == 0).all())


def _cfg4_blob(seed):
    from synth import make_config, make_weights, write_blob
    c = make_config(4)
    return write_blob(make_weights(c["F"], c["K"], c["L"], c["max_z"], seed=seed), c["F"], c["K"], c["L"],
                      c["max_z"], c["r_c"])


def test_full_model_size_sample_matches_oracle(dev):
    """The training workload's model (hidden 128, 3 layers, 32 RBF, student weights) on three of its
    molecules, targets from the teacher network in the oracle."""
    from synth import make_config
    c = make_config(4)
    sel = np.isin(c["batch"], [0, 1, 2])
    pos, z, batch = c["pos"][sel].astype(np.float64), c["z"][sel], c["batch"][sel]
    E_ref, F_ref = TensorNetOracle(_cfg4_blob(3000)).energy_forces(pos, z, batch, None, 3)
    blob = _cfg4_blob(c["weight_seed"])
    loss_ref, g_ref = training_loss_and_grad(TensorNetOracle(blob), pos, z, batch, None, 3, E_ref, F_ref)
    for precision in ("fp64", "fp32"):
        loss, _, _, grads, _ = _gpu(dev, blob, pos, z, batch, None, 3, E_ref, F_ref, precision)
        _check(f"hidden 128 x 3 layers, 3 molecules {precision}", precision, loss, grads, loss_ref, g_ref)


def test_full_batch_fp32_against_fp64(dev):
    """All 64 molecules (4759 atoms) with seeded random targets: the FP32 step against the FP64 step,
    to the FP32 bars (a property of the arithmetic that holds at any size)."""
    from synth import make_config
    c = make_config(4)
    rng = np.random.default_rng(4004)
    S = c["n_systems"]
    E_ref = rng.normal(0.0, 10.0, size=S)
    F_ref = rng.normal(0.0, 1.0, size=(len(c["pos"]), 3))
    blob = _cfg4_blob(c["weight_seed"])
    mp = 20 * len(c["pos"])   # about 13 unordered pairs per atom in these molecules
    ref = _gpu_mp(dev, blob, c, E_ref, F_ref, "fp64", mp)
    got = _gpu_mp(dev, blob, c, E_ref, F_ref, "fp32", mp)
    _check("full batch fp32 vs fp64", "fp32", got[0], got[3], ref[0], ref[3])


def _gpu_mp(dev, blob, c, E_ref, F_ref, precision, max_pairs):
    m = TensorNet(blob, dev)
    pdt = torch.float64 if precision == "fp64" else torch.float32
    t = lambda a, dt: torch.tensor(np.asarray(a), dtype=dt, device=dev)
    loss, E, F, g = m.train_grad(t(c["pos"], pdt), t(c["z"], torch.int32), t(c["batch"], torch.int32),
                                 c["n_systems"], t(E_ref, torch.float64), t(F_ref, torch.float64),
                                 max_pairs=max_pairs, precision=precision)
    return float(loss.item()), E, F, {k: v.cpu().numpy() for k, v in m.split_params(g).items()}


def test_gradient_matches_oracle_triclinic_cell(dev):
    """A reduced triclinic cell: the minimum image shifts the dual displacement's value by a
    lattice vector and leaves its tangent alone."""
    from tests.util import random_in_cell, random_triclinic_cell
    H = random_triclinic_cell(131, 4.5)
    pos, z = random_in_cell(300, 132, H)
    batch = np.zeros(len(pos), np.int32)
    E_ref, F_ref = TensorNetOracle(small_blob(F=16, K=8, L=1, seed=133)).energy_forces(pos, z, batch, H, 1)
    blob = small_blob(F=16, K=8, L=1, seed=134)
    loss_ref, g_ref = training_loss_and_grad(TensorNetOracle(blob), pos, z, batch, H, 1, E_ref, F_ref)
    loss, _, _, grads, _ = _gpu(dev, blob, pos, z, batch, H, 1, E_ref, F_ref, "fp64")
    _check("triclinic cell 300", "fp64", loss, grads, loss_ref, g_ref)


def test_pair_budget_overflow_is_flagged(dev):
    """Too small a pair budget: the step returns, the status word carries the overflow bit."""
    from paper_2402_17660_amd import TensorNetError
    pos, z, batch, S, E_ref, F_ref, blob = _case((9, 14), 16, 8, 2, 3)
    m = TensorNet(blob, dev)
    t = lambda a, dt: torch.tensor(np.asarray(a), dtype=dt, device=dev)
    m.train_grad(t(pos, torch.float64), t(z, torch.int32), t(batch, torch.int32), S, t(E_ref, torch.float64),
                 t(F_ref, torch.float64), precision="fp64")
    m.ws.buf.fill_(0x7F)   # stale workspace: no pair index may be read from it after an overflow
    with pytest.raises(TensorNetError, match="pair overflow"):
        m.train_grad(t(pos, torch.float64), t(z, torch.int32), t(batch, torch.int32), S, t(E_ref, torch.float64),
                     t(F_ref, torch.float64), max_pairs=16, precision="fp64")
    assert int(m.n_pairs.item()) > 16


def test_systems_without_pairs(dev):
    """A one-atom system and a two-atom system farther apart than the cutoff sit between two
    molecules: their energies depend on the species only, their forces are zero."""
    parts = [random_molecule(12, 41), (np.zeros((1, 3)), np.array([6], np.int32)),
             (np.array([[0.0, 0.0, 0.0], [6.0, 0.0, 0.0]]), np.array([1, 8], np.int32)), random_molecule(9, 42)]
    pos = np.concatenate([p for p, _ in parts])
    z = np.concatenate([q for _, q in parts]).astype(np.int32)
    batch = np.concatenate([np.full(len(p), s, np.int32) for s, (p, _) in enumerate(parts)])
    S = len(parts)
    E_ref, F_ref = TensorNetOracle(small_blob(F=16, K=8, L=2, seed=43)).energy_forces(pos, z, batch, None, S)
    blob = small_blob(F=16, K=8, L=2, seed=44)
    loss_ref, g_ref = training_loss_and_grad(TensorNetOracle(blob), pos, z, batch, None, S, E_ref, F_ref)
    for precision in ("fp64", "fp32"):
        loss, _, _, grads, _ = _gpu(dev, blob, pos, z, batch, None, S, E_ref, F_ref, precision)
        _check(f"systems without pairs {precision}", precision, loss, grads, loss_ref, g_ref)


def test_training_step_in_a_hip_graph(dev):
    """The step allocates nothing and never synchronises, so it can be captured: replays (with
    eager work and synchronisation between them) reproduce the eager gradient bit for bit."""
    pos, z, batch, S, E_ref, F_ref, blob = _case((12, 17, 23), 64, 16, 2, 13)
    m = TensorNet(blob, dev)
    t = lambda a, dt: torch.tensor(np.asarray(a), dtype=dt, device=dev)
    args = (t(pos, torch.float32), t(z, torch.int32), t(batch, torch.int32), S, t(E_ref, torch.float64),
            t(F_ref, torch.float64))
    grad = torch.empty(m.param_count(), dtype=torch.float64, device=dev)
    _, _, _, eager = m.train_grad(*args, precision="fp32")
    eager = eager.clone()
    m.train_grad(*args, precision="fp32", check=False, grad_out=grad)   # workspace sized before capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        m.train_grad(*args, precision="fp32", check=False, grad_out=grad)
    for _ in range(3):
        grad.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        m.check()
        assert torch.equal(grad, eager)
        m.train_grad(args[0].double(), *args[1:], precision="fp64")   # eager work between replays


def test_more_than_a_million_pairs(dev):
    """A batch past 1,048,576 pairs (which the earlier 16-row block limit refused): 600 copies of
    a set of molecules have the same mean losses as one copy, so the loss and every gradient
    tensor must agree with the single copy's up to FP32 summation order; energies and forces
    match tn_energy_forces on the same inputs."""
    sizes = (40, 55, 64, 31, 48)
    pos, z, batch, S, E_ref, F_ref, blob = _case(sizes, 128, 32, 2, 11)
    reps = 600
    posr = np.tile(pos, (reps, 1))
    zr = np.tile(z, reps)
    batchr = np.concatenate([batch + r * S for r in range(reps)]).astype(np.int32)
    Er, Fr = np.tile(E_ref, reps), np.tile(F_ref, (reps, 1))
    m = TensorNet(blob, dev)
    t = lambda a, dt: torch.tensor(np.asarray(a), dtype=dt, device=dev)
    loss1, _, _, g1 = m.train_grad(t(pos, torch.float32), t(z, torch.int32), t(batch, torch.int32), S,
                                   t(E_ref, torch.float64), t(F_ref, torch.float64), max_pairs=40 * len(pos),
                                   precision="fp32")
    # a budget just above the true count (the dual workspace is about 60 KB per pair slot)
    mp = int(int(m.n_pairs.item()) * reps * 1.02) + 1024
    lossr, Eo, Fo, gr = m.train_grad(t(posr, torch.float32), t(zr, torch.int32), t(batchr, torch.int32), S * reps,
                                     t(Er, torch.float64), t(Fr, torch.float64), max_pairs=mp, precision="fp32")
    n_pairs = int(m.n_pairs.item())
    assert n_pairs > (1 << 20), n_pairs
    E2, F2 = m.energy_forces(t(posr, torch.float32), t(zr, torch.int32), t(batchr, torch.int32), S * reps,
                             max_pairs=mp, precision="fp32")
    assert torch.equal(Eo, E2) and torch.equal(Fo, F2)
    g1n, grn = g1.cpu().numpy(), gr.cpu().numpy()
    lerr = abs(float(lossr.item()) - float(loss1.item())) / abs(float(loss1.item()))
    gerr = float(np.abs(grn - g1n).max() / np.abs(g1n).max())
    print(f"{n_pairs} pairs: loss rel diff {lerr:.2e}, gradient max diff / max {gerr:.2e}", flush=True)
    assert lerr <= 1e-5 and gerr <= 1e-4
