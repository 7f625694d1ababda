"""Training-step oracle: the energy + force loss and its parameter gradient.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper trains TensorNet on energies and forces together, the forces being
the negative position gradient of the energy, which makes the parameter
gradient of the force term a second derivative (Sec. 2.5: training needs a
double backward through the force computation; Sec. 3 losses combine energy
and force errors).  The reading used here (weights 1:1, mean squared errors):

  loss = w_E mean_s (E_s - E_s^ref)^2 + w_F mean_{i,a} (F_ia - F_ia^ref)^2,
  F = -d(sum_s E_s)/dr,

with the gradient with respect to every tensor of the weight blob taken by
torch autograd in float64: the forces are formed with create_graph=True and
the loss is differentiated through them.
"""

from __future__ import annotations

import numpy as np
import torch

from .model import DT, TensorNetOracle


def training_loss_and_grad(model: TensorNetOracle, pos, z, batch, box, n_systems, E_ref, F_ref,
                           w_energy: float = 1.0, w_force: float = 1.0, pairs=None):
    """(loss, {tensor name: gradient as a float64 numpy array of the tensor's shape})."""
    names = list(model.w.keys())
    params = {k: v.detach().clone().requires_grad_(True) for k, v in model.w.items()}
    saved = model.w
    model.w = params
    try:
        p = torch.as_tensor(np.asarray(pos, dtype=np.float64)).clone().requires_grad_(True)
        if pairs is None:
            pairs = model.pairs(np.asarray(pos), batch, box)
        E = model.energy_t(p, z, batch, box, n_systems, pairs=pairs)
        (g,) = torch.autograd.grad(E.sum(), p, create_graph=True)
        Fo = -g
        E_ref_t = torch.as_tensor(np.asarray(E_ref, dtype=np.float64), dtype=DT)
        F_ref_t = torch.as_tensor(np.asarray(F_ref, dtype=np.float64), dtype=DT)
        loss = w_energy * ((E - E_ref_t) ** 2).mean() + w_force * ((Fo - F_ref_t) ** 2).mean()
        grads = torch.autograd.grad(loss, [params[k] for k in names], allow_unused=True)
    finally:
        model.w = saved
    out = {}
    for k, gk in zip(names, grads):
        out[k] = (gk.detach().numpy() if gk is not None else np.zeros(tuple(params[k].shape)))
    return float(loss.detach()), out


def training_loss(model: TensorNetOracle, pos, z, batch, box, n_systems, E_ref, F_ref,
                  w_energy: float = 1.0, w_force: float = 1.0, pairs=None) -> float:
    """The loss alone (forces by first-order autograd), for finite-difference pins."""
    E, Fo = model.energy_forces(pos, z, batch, box, n_systems, pairs=pairs)
    return float(w_energy * np.mean((E - np.asarray(E_ref)) ** 2) + w_force * np.mean((Fo - np.asarray(F_ref)) ** 2))


__all__ = ["training_loss_and_grad", "training_loss"]
