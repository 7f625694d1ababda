"""Weight blob: the byte format that carries one TensorNet's parameters.

Layout (little endian):

    offset  size  field
    0       8     magic b"TNETBLOB"
    8       4     u32 version (= 1)
    12      4     u32 F      hidden channels (even)
    16      4     u32 K      radial basis functions
    20      4     u32 L      interaction layers (0 allowed)
    24      4     u32 max_z  rows of the species embedding
    28      4     u32 activation id (1 = SiLU, the only one defined)
    32      8     two reserved u32, zero
    40      8     f64 r_lo   lower cutoff (angstrom)
    48      8     f64 r_c    upper cutoff (angstrom)
    56      ...   the tensors of `tensor_layout`, in that order, f64, row major

A Linear map y = W x + b stores W as [out, in].  The blob is the contract
between the generator, the FP64 oracle and the C library; each of the last
two parses it on its own.  Only hyper-parameters and learnable tensors are
stored: the radial-basis constants follow from (K, r_lo, r_c) and are derived
independently by each consumer.
"""

from __future__ import annotations

import struct

import numpy as np

BLOB_MAGIC = b"TNETBLOB"
BLOB_VERSION = 1
HEADER_BYTES = 56


def tensor_layout(F: int, K: int, L: int, max_z: int):
    """[(name, shape, init, fan_in)] in blob order."""
    if F % 2:
        raise ValueError("F must be even")
    t = []

    def lin(prefix, n_out, n_in, bias=True):
        t.append((prefix.replace("#", "W"), (n_out, n_in), "normal_fanin", n_in))
        if bias:
            t.append((prefix.replace("#", "b"), (n_out,), "normal_fanin", n_in))

    t.append(("emb.E", (max_z, F), "normal", 1))
    lin("emb.#z", F, 2 * F)
    lin("emb.#0", 3 * F, K)
    t.append(("emb.ln_g", (F,), "ones", 1))
    t.append(("emb.ln_b", (F,), "zeros", 1))
    lin("emb.#1", 2 * F, F)
    lin("emb.#2", 3 * F, 2 * F)
    for part in "IAS":
        t.append((f"emb.W{part}", (F, F), "normal_fanin", F))
    for l in range(L):
        lin(f"layer{l}.#a", F, K)
        lin(f"layer{l}.#b", 2 * F, F)
        lin(f"layer{l}.#c", 3 * F, 2 * F)
        for part in "IAS":
            t.append((f"layer{l}.W1{part}", (F, F), "normal_fanin", F))
        for part in "IAS":
            t.append((f"layer{l}.W2{part}", (F, F), "normal_fanin", F))
    t.append(("out.ln_g", (3 * F,), "ones", 1))
    t.append(("out.ln_b", (3 * F,), "zeros", 1))
    lin("out.#o", F, 3 * F)
    lin("out.#h", F // 2, F)
    lin("out.#2", 1, F // 2)
    return t


def write_blob(weights: dict, F: int, K: int, L: int, max_z: int, r_c: float, r_lo: float = 0.0) -> bytes:
    """Serialise `weights` (name -> float64 array) into blob bytes."""
    head = BLOB_MAGIC + struct.pack("<8I", BLOB_VERSION, F, K, L, max_z, 1, 0, 0) + struct.pack("<2d", r_lo, r_c)
    assert len(head) == HEADER_BYTES
    parts = [head]
    for name, shape, _, _ in tensor_layout(F, K, L, max_z):
        a = np.ascontiguousarray(np.asarray(weights[name], dtype="<f8"))
        if a.shape != tuple(shape):
            raise ValueError(f"{name}: shape {a.shape} != {shape}")
        parts.append(a.tobytes())
    return b"".join(parts)
