"""Pins of the training-step oracle (energy + force loss, parameter gradient by double
autograd): central finite differences of the loss in single parameters, zero loss and zero
gradient at the targets' own weights, and invariance of loss and gradient under a rotation
of the inputs with the force targets rotated alike."""

import numpy as np
import pytest

from oracle import TensorNetOracle
from oracle.train import training_loss, training_loss_and_grad
from oracle.blob import read_blob
from synth import make_weights, write_blob
from tests.util import random_molecule, random_rotation, small_blob


def _batch(seed):
    parts = [random_molecule(n, seed + n) for n in (9, 14)]
    pos = np.concatenate([p for p, _ in parts])
    z = np.concatenate([q for _, q in parts])
    batch = np.concatenate([np.full(len(p), s, np.int32) for s, (p, _) in enumerate(parts)])
    return pos, z, batch


def _targets(seed, pos, z, batch):
    teacher = TensorNetOracle(small_blob(F=16, K=8, L=2, seed=seed))
    return teacher.energy_forces(pos, z, batch, None, 2)


def _perturbed_blob(blob, name, index, delta):
    """The same blob with one entry of one tensor shifted by delta (rewritten through synth)."""
    hyper, w = read_blob(blob)
    tensors = {k: v.numpy().copy() for k, v in w.items()}
    tensors[name].reshape(-1)[index] += delta
    return write_blob(tensors, hyper["F"], hyper["K"], hyper["L"], hyper["max_z"], hyper["r_c"])


@pytest.mark.parametrize("name", ["emb.E", "emb.Wz", "emb.W0", "emb.ln_g", "emb.W2", "emb.WA",
                                  "layer0.Wa", "layer0.bc", "layer1.W1S", "layer1.W2I", "out.Wo", "out.b2"])
def test_gradient_matches_central_differences(name):
    pos, z, batch = _batch(3)
    E_ref, F_ref = _targets(101, pos, z, batch)
    blob = small_blob(F=16, K=8, L=2, seed=102)
    model = TensorNetOracle(blob)
    pairs = model.pairs(pos, batch, None)
    loss, grads = training_loss_and_grad(model, pos, z, batch, None, 2, E_ref, F_ref, pairs=pairs)
    g = grads[name].reshape(-1)
    rng = np.random.default_rng(hash(name) % 2**32)
    idx = int(rng.integers(0, g.size)) if name != "emb.E" else int(np.flatnonzero(np.abs(g) > 0)[0])
    h = 1e-5
    lp = training_loss(TensorNetOracle(_perturbed_blob(blob, name, idx, h)), pos, z, batch, None, 2, E_ref, F_ref,
                       pairs=pairs)
    lm = training_loss(TensorNetOracle(_perturbed_blob(blob, name, idx, -h)), pos, z, batch, None, 2, E_ref, F_ref,
                       pairs=pairs)
    fd = (lp - lm) / (2 * h)
    assert abs(fd - g[idx]) <= 1e-6 * max(abs(fd), 1e-3 * loss), (name, idx, fd, g[idx])


def test_zero_loss_and_gradient_at_the_targets_weights():
    pos, z, batch = _batch(5)
    blob = small_blob(F=16, K=8, L=2, seed=103)
    model = TensorNetOracle(blob)
    E_ref, F_ref = model.energy_forces(pos, z, batch, None, 2)
    loss, grads = training_loss_and_grad(model, pos, z, batch, None, 2, E_ref, F_ref)
    assert loss == 0.0
    assert all(np.all(g == 0.0) for g in grads.values())


def test_loss_and_gradient_rotation_invariant():
    pos, z, batch = _batch(7)
    E_ref, F_ref = _targets(104, pos, z, batch)
    model = TensorNetOracle(small_blob(F=16, K=8, L=2, seed=105))
    Q = random_rotation(106, reflect=True)
    l0, g0 = training_loss_and_grad(model, pos, z, batch, None, 2, E_ref, F_ref)
    l1, g1 = training_loss_and_grad(model, pos @ Q.T + 2.5, z, batch, None, 2, E_ref, F_ref @ Q.T)
    assert abs(l1 - l0) <= 1e-12 * abs(l0)
    for k in g0:
        assert np.allclose(g1[k], g0[k], rtol=1e-9, atol=1e-12 * max(1.0, np.abs(g0[k]).max())), k


def test_every_blob_tensor_gets_a_gradient():
    pos, z, batch = _batch(9)
    E_ref, F_ref = _targets(107, pos, z, batch)
    model = TensorNetOracle(small_blob(F=16, K=8, L=2, seed=108))
    _, grads = training_loss_and_grad(model, pos, z, batch, None, 2, E_ref, F_ref)
    hyper, w = read_blob(small_blob(F=16, K=8, L=2, seed=108))
    assert set(grads) == set(w)
    for k, v in w.items():
        assert grads[k].shape == tuple(v.shape)
        if k != "emb.E":     # rows of species that do not occur stay zero
            assert np.any(grads[k] != 0.0), k
