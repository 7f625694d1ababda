"""O2-O6: TensorNet energy and forces, plain FP64 on full 3x3 matrices.

What the paper fixes (TorchMD-Net 2.0, Sec. 2.1.1 "TensorNet"; Sec. 2.4 hyper
parameter listing; Sec. 2 model composition; Tables S3 and S4):
  * an O(3)-equivariant message-passing network whose per-atom features are
    rank-2 Cartesian tensors (F channels of 3x3 matrices), decomposed into a
    scalar (trace) part I, an antisymmetric (vector) part A and a symmetric
    traceless part S;
  * node-level 3x3 matrix products in place of Clebsch-Gordan products, in
    the symmetric order required by the O(3) group of Tables S3/S4;
  * exp-normal radial basis ("expnorm", not trainable), cosine cutoff with
    lower cutoff 0, SiLU activations, max_z = 100 species rows;
  * a scalar output network whose per-atom values are summed per system, and
    forces as the negative position gradient of that sum (Sec. 2).

The paper prints no equations for TensorNet, so the concrete formulas below
are a reading of that description (the points where a choice was needed are
listed in the design notes of the repository):

  norm        ||X|| = sum_ab X_ab^2  (squared Frobenius norm, per channel)
  mixing      (W . T)_f = sum_g W_fg T_g, applied to every matrix entry
  geometry    v_ij = r_j - r_i (minimum image), d, vhat = v/d
  cutoff      phi(d) = (cos(pi d / r_c) + 1) / 2
  basis       e_k = phi(d) exp(-beta_k (exp(-alpha (d - r_lo)) - mu_k)^2),
              alpha = 5/(r_c - r_lo), mu = linspace(exp(-(r_c - r_lo)), 1, K),
              beta_k = (2 (1 - exp(-(r_c - r_lo))) / K)^-2
  embedding   Z_ij = W_z [E_zi ; E_zj] + b_z;  (a,b,c) = split(W0 e + b0)
              X_i = sum_j phi Z_ij (a 1 + b A0(vhat) + c S0(vhat))
              n_i = LN(||X_i||);  (gI,gA,gS) = split(silu(W2 silu(W1 n + b1) + b2))
              X_i <- gI (W_I I(X_i)) + gA (W_A A(X_i)) + gS (W_S S(X_i))
  layer       Xb = X / (||X|| + 1);  Y = W1_I I(Xb) + W1_A A(Xb) + W1_S S(Xb)
              h = phi silu(Wc silu(Wb silu(Wa e + ba) + bb) + bc) = (hI,hA,hS)
              M_i = sum_j hI I(Y_j) + hA A(Y_j) + hS S(Y_j)
              P = Y M + M Y;  Pb = P / (||P|| + 1)
              dX = W2_I I(Pb) + W2_A A(Pb) + W2_S S(Pb);  X <- Xb + dX + dX dX
  output      q = LN([||I(X)||; ||A(X)||; ||S(X)||]);  x = silu(Wo q + bo)
              eps_i = w2 . silu(Wh x + bh) + b2;   E_s = sum_{i in s} eps_i
  forces      F_i = -d(sum_s E_s)/d r_i   (torch.autograd, float64)

This file is test infrastructure: it must not be imported by the product path.
"""

from __future__ import annotations

import math

import numpy as np
import torch
from torch.utils.checkpoint import checkpoint

from .blob import read_blob
from .neighbors import lattice, neighbor_pairs

DT = torch.float64
_EYE = torch.eye(3, dtype=DT)


# ---------------------------------------------------------------- tensor algebra
def decompose(X):
    """I/A/S parts of 3x3 matrices (Sec. 2.1.1): trace, antisymmetric, symmetric traceless."""
    tr = X.diagonal(dim1=-2, dim2=-1).sum(-1)
    I = (tr / 3.0)[..., None, None] * _EYE
    Xt = X.transpose(-1, -2)
    A = 0.5 * (X - Xt)
    S = 0.5 * (X + Xt) - I
    return I, A, S


def tensor_norm(X):
    """Squared Frobenius norm over the last two axes."""
    return (X * X).sum((-2, -1))


def skew(u):
    """A0(u): the antisymmetric matrix with A0(u) w = u x w."""
    ux, uy, uz = u.unbind(-1)
    zero = torch.zeros_like(ux)
    return torch.stack([
        torch.stack([zero, -uz, uy], -1),
        torch.stack([uz, zero, -ux], -1),
        torch.stack([-uy, ux, zero], -1),
    ], -2)


def sym_traceless_outer(u):
    """S0(u) = u u^T - 1/3 (symmetric traceless part of the outer product of a unit vector)."""
    return u[..., :, None] * u[..., None, :] - _EYE / 3.0


def symmetric_product(Y, M):
    """Y M + M Y per channel: the node-level 3x3 product in its O(3) (reflection-safe) order."""
    return Y @ M + M @ Y


def mix(W, T):
    """Channel mixing (W . T)_f = sum_g W_fg T_g on [N, F, 3, 3]."""
    return torch.einsum("fg,ngab->nfab", W, T)


# ---------------------------------------------------------------- scalar pieces
def cosine_cutoff(d, r_c):
    """phi(d) = (cos(pi d / r_c) + 1)/2 for d < r_c, else 0 (cutoff_lower = 0, Sec. 2.4)."""
    return 0.5 * (torch.cos(math.pi * d / r_c) + 1.0) * (d < r_c).to(d.dtype)


def expnorm_constants(K, r_lo, r_c):
    """alpha, mu[K], beta[K] of the exp-normal basis (rbf_type 'expnorm', Sec. 2.4)."""
    alpha = 5.0 / (r_c - r_lo)
    start = math.exp(-(r_c - r_lo))
    mu = torch.tensor([start + (1.0 - start) * k / (K - 1) for k in range(K)], dtype=DT) if K > 1 \
        else torch.tensor([start], dtype=DT)
    beta = torch.full((K,), (2.0 / K * (1.0 - start)) ** -2, dtype=DT)
    return alpha, mu, beta


def expnorm_rbf(d, K, r_lo, r_c):
    """e_k(d) = phi(d) exp(-beta_k (exp(-alpha (d - r_lo)) - mu_k)^2), shape [E, K]."""
    alpha, mu, beta = expnorm_constants(K, r_lo, r_c)
    u = torch.exp(-alpha * (d - r_lo))[:, None]
    return cosine_cutoff(d, r_c)[:, None] * torch.exp(-beta * (u - mu) ** 2)


def silu(x):
    """SiLU activation x * sigmoid(x) (activation 'silu', Sec. 2.4)."""
    return x / (1.0 + torch.exp(-x))


def layer_norm(x, g, b, eps=1e-5):
    """LayerNorm over the last axis, population variance, eps 1e-5, affine g/b."""
    mean = x.mean(-1, keepdim=True)
    var = ((x - mean) ** 2).mean(-1, keepdim=True)
    return (x - mean) / torch.sqrt(var + eps) * g + b


def linear(x, W, b=None):
    y = x @ W.T
    return y if b is None else y + b


# ---------------------------------------------------------------- per-edge blocks
def _embed_edges(rbf, phi, vhat, zrow_recv, zrow_send, w, F):
    """phi Z_ij (a 1 + b A0(vhat) + c S0(vhat)) for a chunk of directed edges, [E, F, 3, 3]."""
    Zij = linear(torch.cat([zrow_recv, zrow_send], -1), w["emb.Wz"], w["emb.bz"])
    f0 = linear(rbf, w["emb.W0"], w["emb.b0"])
    a, b, c = f0[:, :F], f0[:, F:2 * F], f0[:, 2 * F:]
    base = (a[..., None, None] * _EYE
            + b[..., None, None] * skew(vhat)[:, None]
            + c[..., None, None] * sym_traceless_outer(vhat)[:, None])
    return (phi[:, None] * Zij)[..., None, None] * base


def _edge_filter(rbf, phi, w, prefix, F):
    """h = phi * silu(Wc silu(Wb silu(Wa e + ba) + bb) + bc), split into (hI, hA, hS)."""
    t = silu(linear(rbf, w[prefix + "Wa"], w[prefix + "ba"]))
    t = silu(linear(t, w[prefix + "Wb"], w[prefix + "bb"]))
    t = silu(linear(t, w[prefix + "Wc"], w[prefix + "bc"]))
    h = phi[:, None] * t
    return h[:, :F], h[:, F:2 * F], h[:, 2 * F:]


def _message_edges(rbf, phi, send, Yi, Ya, Ys, w, prefix, F):
    hI, hA, hS = _edge_filter(rbf, phi, w, prefix, F)
    return (hI[..., None, None] * Yi[send] + hA[..., None, None] * Ya[send]
            + hS[..., None, None] * Ys[send])


# ---------------------------------------------------------------- the model
class TensorNetOracle:
    """FP64 TensorNet (readings O2-O6) over a weight blob.

    product="sym" is the O(3) product Y M + M Y.  product="left" (Y M only) is
    a deliberately wrong variant kept for the negative-control test.
    """

    def __init__(self, blob: bytes, product: str = "sym", edge_chunk: int = 16384):
        self.hyper, self.w = read_blob(blob)
        if product not in ("sym", "left"):
            raise ValueError(product)
        self.product = product
        self.edge_chunk = edge_chunk

    @property
    def F(self):
        return self.hyper["F"]

    def pairs(self, pos, batch, box):
        return neighbor_pairs(np.asarray(pos), np.asarray(batch), box, self.hyper["r_c"])

    # -- forward ------------------------------------------------------------
    def energy_t(self, pos, z, batch, box, n_systems, pairs=None, capture=None):
        """Per-system energies [S] (float64 torch) from positions `pos` (float64 torch, may require grad)."""
        h = self.hyper
        w = self.w
        F, K, L = h["F"], h["K"], h["L"]
        r_lo, r_c = h["r_lo"], h["r_c"]
        N = pos.shape[0]
        z = torch.as_tensor(np.asarray(z), dtype=torch.long)
        batch_t = torch.as_tensor(np.asarray(batch), dtype=torch.long)
        if pairs is None:
            pairs = self.pairs(pos.detach().numpy(), batch, box)
        pairs = torch.as_tensor(np.asarray(pairs), dtype=torch.long).reshape(-1, 2)
        # directed edges: receiver i collects from sender j, both directions of each pair
        recv = torch.cat([pairs[:, 0], pairs[:, 1]])
        send = torch.cat([pairs[:, 1], pairs[:, 0]])

        v = pos[send] - pos[recv]
        if box is not None:
            # minimum image in the reduced cell: along c, then b, then a (round = half to even)
            H = torch.as_tensor(lattice(box), dtype=DT)
            v = v - torch.round(v[:, 2:3] / H[2, 2]) * H[2]
            v = v - torch.round(v[:, 1:2] / H[1, 1]) * H[1]
            v = v - torch.round(v[:, 0:1] / H[0, 0]) * H[0]
        d = torch.sqrt((v * v).sum(-1))
        vhat = v / d[:, None]
        phi = cosine_cutoff(d, r_c)
        rbf = expnorm_rbf(d, K, r_lo, r_c)

        zrow = w["emb.E"][z]
        E_edges = recv.shape[0]
        chunk = self.edge_chunk if (self.edge_chunk and E_edges > self.edge_chunk) else max(E_edges, 1)
        use_ckpt = E_edges > chunk

        # O3: embedding
        X = torch.zeros(N, F, 3, 3, dtype=DT)
        for s in range(0, E_edges, chunk):
            sl = slice(s, s + chunk)
            args = (rbf[sl], phi[sl], vhat[sl], zrow[recv[sl]], zrow[send[sl]])
            contrib = (checkpoint(_embed_edges, *args, w, F, use_reentrant=False) if use_ckpt
                       else _embed_edges(*args, w, F))
            X = X.index_add(0, recv[sl], contrib)
        n0 = layer_norm(tensor_norm(X), w["emb.ln_g"], w["emb.ln_b"])
        g = silu(linear(silu(linear(n0, w["emb.W1"], w["emb.b1"])), w["emb.W2"], w["emb.b2"]))
        gI, gA, gS = g[:, :F], g[:, F:2 * F], g[:, 2 * F:]
        I, A, S = decompose(X)
        X = (gI[..., None, None] * mix(w["emb.WI"], I) + gA[..., None, None] * mix(w["emb.WA"], A)
             + gS[..., None, None] * mix(w["emb.WS"], S))
        if capture is not None:
            capture["X_emb"] = X.detach().clone()

        # O4: interaction layers
        for l in range(L):
            p = f"layer{l}."
            Xb = X / (tensor_norm(X) + 1.0)[..., None, None]
            I, A, S = decompose(Xb)
            Y = mix(w[p + "W1I"], I) + mix(w[p + "W1A"], A) + mix(w[p + "W1S"], S)
            Yi, Ya, Ys = decompose(Y)
            M = torch.zeros(N, F, 3, 3, dtype=DT)
            for s in range(0, E_edges, chunk):
                sl = slice(s, s + chunk)
                args = (rbf[sl], phi[sl], send[sl], Yi, Ya, Ys)
                msg = (checkpoint(_message_edges, *args, w, p, F, use_reentrant=False) if use_ckpt
                       else _message_edges(*args, w, p, F))
                M = M.index_add(0, recv[sl], msg)
            P = symmetric_product(Y, M) if self.product == "sym" else Y @ M
            Pb = P / (tensor_norm(P) + 1.0)[..., None, None]
            I, A, S = decompose(Pb)
            dX = mix(w[p + "W2I"], I) + mix(w[p + "W2A"], A) + mix(w[p + "W2S"], S)
            X = Xb + dX + dX @ dX
            if capture is not None:
                capture[f"X_layer{l}"] = X.detach().clone()

        # O5: output network and per-system sum
        I, A, S = decompose(X)
        q = layer_norm(torch.cat([tensor_norm(I), tensor_norm(A), tensor_norm(S)], -1),
                       w["out.ln_g"], w["out.ln_b"])
        x = silu(linear(q, w["out.Wo"], w["out.bo"]))
        eps = linear(silu(linear(x, w["out.Wh"], w["out.bh"])), w["out.W2"], w["out.b2"])[:, 0]
        if capture is not None:
            capture["atom_energy"] = eps.detach().clone()
        E = torch.zeros(n_systems, dtype=DT).index_add(0, batch_t, eps)
        return E

    # -- convenience ----------------------------------------------------------
    def energy(self, pos, z, batch, box, n_systems, pairs=None, capture=None):
        """Per-system energies as a float64 numpy array."""
        p = torch.as_tensor(np.asarray(pos, dtype=np.float64))
        with torch.no_grad():
            return self.energy_t(p, z, batch, box, n_systems, pairs=pairs, capture=capture).numpy()

    def energy_forces(self, pos, z, batch, box, n_systems, pairs=None, capture=None):
        """(E [S], F [N,3]) as float64 numpy arrays; F = -dE/dpos by autograd (O6)."""
        p = torch.as_tensor(np.asarray(pos, dtype=np.float64)).clone().requires_grad_(True)
        if pairs is None:
            pairs = self.pairs(np.asarray(pos), batch, box)
        E = self.energy_t(p, z, batch, box, n_systems, pairs=pairs, capture=capture)
        (grad,) = torch.autograd.grad(E.sum(), p)
        return E.detach().numpy(), (-grad).numpy()


def parameter_count(blob: bytes) -> int:
    _, w = read_blob(blob)
    return int(sum(t.numel() for t in w.values()))
