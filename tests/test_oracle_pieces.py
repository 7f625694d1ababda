"""Pins of the oracle's building blocks: closed forms (P-3, P-4, P-5, P-7), library
special cases (LayerNorm, SiLU, cross product), the parameter count the paper prints
(P-17) and the blob parser's error handling.
"""

import math
import struct

import numpy as np
import pytest
import torch

from oracle import (cosine_cutoff, decompose, expnorm_constants, expnorm_rbf, layer_norm, read_blob,
                    silu, skew, sym_traceless_outer, symmetric_product, tensor_norm)
from oracle.model import parameter_count
from synth import make_weights, write_blob
from tests.util import small_blob

DT = torch.float64


def test_p3_cutoff_closed_forms():
    r_c = 4.5
    d = torch.tensor([0.0, r_c / 2, r_c - 1e-12, r_c, r_c + 1.0], dtype=DT, requires_grad=True)
    phi = cosine_cutoff(d, r_c)
    assert phi[0].item() == 1.0
    assert abs(phi[1].item() - 0.5) < 1e-15
    assert abs(phi[2].item()) < 1e-20
    assert phi[3].item() == 0.0 and phi[4].item() == 0.0
    (g,) = torch.autograd.grad(phi.sum(), d)
    assert abs(g[2].item()) < 1e-11          # phi'(r_c) = 0
    assert abs(g[1].item() + math.pi / (2 * r_c)) < 1e-14   # phi'(r_c/2) = -pi/(2 r_c)


@pytest.mark.parametrize("K,r_lo,r_c", [(32, 0.0, 5.0), (32, 0.0, 4.5), (8, 0.5, 3.0)])
def test_p3_expnorm_constants_and_peaks(K, r_lo, r_c):
    alpha, mu, beta = expnorm_constants(K, r_lo, r_c)
    assert alpha == 5.0 / (r_c - r_lo)
    assert abs(mu[0].item() - math.exp(-(r_c - r_lo))) < 1e-16 and abs(mu[-1].item() - 1.0) < 1e-15
    assert torch.allclose(mu[1:] - mu[:-1], torch.full((K - 1,), (1 - math.exp(-(r_c - r_lo))) / (K - 1), dtype=DT),
                          rtol=0, atol=1e-15)
    assert torch.allclose(beta, torch.full((K,), ((2 / K) * (1 - math.exp(-(r_c - r_lo)))) ** -2, dtype=DT))
    # e_k / phi equals 1 exactly where exp(-alpha (d - r_lo)) = mu_k, i.e. d_k = r_lo - ln(mu_k)/alpha
    dk = r_lo - torch.log(mu) / alpha
    inside = dk < r_c
    e = expnorm_rbf(dk[inside], K, r_lo, r_c)
    ratio = e / cosine_cutoff(dk[inside], r_c)[:, None]
    idx = torch.arange(K)[inside]
    assert torch.allclose(ratio[torch.arange(len(idx)), idx], torch.ones(len(idx), dtype=DT), atol=1e-12)
    assert torch.all(ratio <= 1.0 + 1e-12)


def test_p4_skew_and_symmetric_outer():
    rng = np.random.default_rng(0)
    u = torch.tensor(rng.normal(size=(20, 3)), dtype=DT)
    u = u / u.norm(dim=-1, keepdim=True)
    w = torch.tensor(rng.normal(size=(20, 3)), dtype=DT)
    A0 = skew(u)
    assert torch.allclose((A0 @ w[..., None])[..., 0], torch.linalg.cross(u, w), atol=1e-14)
    S0 = sym_traceless_outer(u)
    assert torch.allclose(S0, S0.transpose(-1, -2))
    assert torch.allclose(S0.diagonal(dim1=-2, dim2=-1).sum(-1), torch.zeros(20, dtype=DT), atol=1e-15)
    assert torch.allclose((S0 @ u[..., None])[..., 0], 2.0 / 3.0 * u, atol=1e-15)
    perp = torch.linalg.cross(u, w)
    assert torch.allclose((S0 @ perp[..., None])[..., 0], -perp / 3.0, atol=1e-14)
    eye = torch.eye(3, dtype=DT)
    assert tensor_norm(eye).item() == 3.0
    assert torch.allclose(tensor_norm(A0), torch.full((20,), 2.0, dtype=DT))
    assert torch.allclose(tensor_norm(S0), torch.full((20,), 2.0 / 3.0, dtype=DT))


def test_p5_decomposition_exact_and_orthogonal():
    rng = np.random.default_rng(1)
    X = torch.tensor(rng.normal(size=(50, 3, 3)), dtype=DT)
    I, A, S = decompose(X)
    assert torch.allclose(I + A + S, X, atol=1e-15)
    for P, Q in ((I, A), (I, S), (A, S)):
        assert torch.allclose((P * Q).sum((-2, -1)), torch.zeros(50, dtype=DT), atol=1e-14)
    assert torch.allclose(tensor_norm(X), tensor_norm(I) + tensor_norm(A) + tensor_norm(S))
    # projections are idempotent and land in the right subspaces
    for k, part in enumerate((I, A, S)):
        assert torch.allclose(decompose(part)[k], part, atol=1e-15)
    assert torch.allclose(A, -A.transpose(-1, -2))
    assert torch.allclose(S, S.transpose(-1, -2))
    assert torch.allclose(S.diagonal(dim1=-2, dim2=-1).sum(-1), torch.zeros(50, dtype=DT), atol=1e-14)
    # I is a multiple of the identity with the same trace
    assert torch.allclose(I.diagonal(dim1=-2, dim2=-1).sum(-1), X.diagonal(dim1=-2, dim2=-1).sum(-1))


def test_p7_normalisation_and_product():
    rng = np.random.default_rng(2)
    X = torch.tensor(rng.normal(size=(100, 3, 3)) * rng.uniform(0, 100, size=(100, 1, 1)), dtype=DT)
    Xb = X / (tensor_norm(X) + 1.0)[..., None, None]
    assert torch.all(tensor_norm(Xb) < 1.0)
    M = torch.tensor(rng.normal(size=(10, 3, 3)), dtype=DT)
    eye = torch.eye(3, dtype=DT).expand(10, 3, 3)
    assert torch.allclose(symmetric_product(eye, M), 2.0 * M)
    # brute-force entries of Y M + M Y
    Y = torch.tensor(rng.normal(size=(3, 3)), dtype=DT)
    Mm = torch.tensor(rng.normal(size=(3, 3)), dtype=DT)
    ref = torch.zeros(3, 3, dtype=DT)
    for a in range(3):
        for b in range(3):
            ref[a, b] = sum(Y[a, c] * Mm[c, b] + Mm[a, c] * Y[c, b] for c in range(3))
    assert torch.allclose(symmetric_product(Y, Mm), ref)


def test_layer_norm_and_silu_match_library():
    rng = np.random.default_rng(3)
    x = torch.tensor(rng.normal(size=(7, 24)) * 5 + 2, dtype=DT)
    g = torch.tensor(rng.normal(size=24), dtype=DT)
    b = torch.tensor(rng.normal(size=24), dtype=DT)
    ref = torch.nn.functional.layer_norm(x, (24,), g, b, eps=1e-5)
    assert torch.allclose(layer_norm(x, g, b), ref, atol=1e-13)
    assert torch.allclose(silu(x), torch.nn.functional.silu(x), atol=1e-14)


def test_p17_parameter_count_matches_paper():
    path = __file__.replace("test_oracle_pieces.py", "golden/param_count.txt")
    row = [ln for ln in open(path) if ln.strip() and not ln.startswith("#")][0].split()
    F, K, L, max_z, lo, hi = map(int, row)
    blob = write_blob(make_weights(F, K, L, max_z, seed=0), F, K, L, max_z, 5.0)
    n = parameter_count(blob)
    assert lo <= n <= hi
    assert n == 3_967_233


@pytest.mark.parametrize("F,K,L,count", [(128, 32, 0, 297_857), (128, 32, 1, 532_097), (128, 32, 2, 766_337),
                                         (128, 32, 3, 1_000_577), (64, 32, 2, 200_897)])
def test_p17_parameter_counts_of_workloads(F, K, L, count):
    blob = write_blob(make_weights(F, K, L, 100, seed=0), F, K, L, 100, 5.0)
    assert parameter_count(blob) == count


def test_blob_parser_rejects_bad_input():
    blob = small_blob()
    hyper, w = read_blob(blob)
    assert hyper["F"] == 16 and hyper["K"] == 8 and hyper["L"] == 2 and hyper["r_c"] == 4.5
    with pytest.raises(ValueError):
        read_blob(b"XXXXXXXX" + blob[8:])
    with pytest.raises(ValueError):
        read_blob(blob[:-8])
    with pytest.raises(ValueError):
        read_blob(blob + b"\0" * 8)
    bad_version = blob[:8] + struct.pack("<I", 2) + blob[12:]
    with pytest.raises(ValueError):
        read_blob(bad_version)
