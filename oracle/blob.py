"""Oracle-side parser of the weight blob (independent of the C library's parser).

Byte layout: 8-byte magic "TNETBLOB", eight little-endian u32 (version, F, K,
L, max_z, activation, 0, 0), two f64 (r_lo, r_c), then float64 tensors.  The
tensor order is spelled out here again, by hand, rather than imported, so a
mistake in the writer's order is caught when the two disagree on a size.
"""

from __future__ import annotations

import struct

import numpy as np
import torch


def _order(F, K, L, max_z):
    o = [("emb.E", (max_z, F)), ("emb.Wz", (F, 2 * F)), ("emb.bz", (F,)),
         ("emb.W0", (3 * F, K)), ("emb.b0", (3 * F,)), ("emb.ln_g", (F,)), ("emb.ln_b", (F,)),
         ("emb.W1", (2 * F, F)), ("emb.b1", (2 * F,)), ("emb.W2", (3 * F, 2 * F)), ("emb.b2", (3 * F,)),
         ("emb.WI", (F, F)), ("emb.WA", (F, F)), ("emb.WS", (F, F))]
    for l in range(L):
        p = f"layer{l}."
        o += [(p + "Wa", (F, K)), (p + "ba", (F,)), (p + "Wb", (2 * F, F)), (p + "bb", (2 * F,)),
              (p + "Wc", (3 * F, 2 * F)), (p + "bc", (3 * F,)),
              (p + "W1I", (F, F)), (p + "W1A", (F, F)), (p + "W1S", (F, F)),
              (p + "W2I", (F, F)), (p + "W2A", (F, F)), (p + "W2S", (F, F))]
    o += [("out.ln_g", (3 * F,)), ("out.ln_b", (3 * F,)), ("out.Wo", (F, 3 * F)), ("out.bo", (F,)),
          ("out.Wh", (F // 2, F)), ("out.bh", (F // 2,)), ("out.W2", (1, F // 2)), ("out.b2", (1,))]
    return o


def read_blob(blob: bytes):
    """Return (hyper dict, {name: float64 torch tensor})."""
    if len(blob) < 56 or blob[:8] != b"TNETBLOB":
        raise ValueError("not a TensorNet weight blob")
    version, F, K, L, max_z, act, _, _ = struct.unpack_from("<8I", blob, 8)
    r_lo, r_c = struct.unpack_from("<2d", blob, 40)
    if version != 1 or act != 1:
        raise ValueError("unsupported blob version/activation")
    hyper = dict(F=F, K=K, L=L, max_z=max_z, r_lo=r_lo, r_c=r_c)
    off = 56
    w = {}
    for name, shape in _order(F, K, L, max_z):
        n = int(np.prod(shape))
        if off + 8 * n > len(blob):
            raise ValueError("blob truncated")
        arr = np.frombuffer(blob, dtype="<f8", count=n, offset=off).reshape(shape)
        w[name] = torch.from_numpy(arr.copy())
        off += 8 * n
    if off != len(blob):
        raise ValueError("blob has trailing bytes")
    return hyper, w
