"""Python binding over the C ABI: argument marshalling only.

Torch tensors provide device memory and the current HIP stream; every step of
the computation runs in libtensornet.so.  There is no CPU fallback: without
the built library or a GPU these functions raise.
"""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L

_PREC = {"fp32": L.TN_FP32, "bf16": L.TN_BF16, "fp64": L.TN_FP64}
_PATH = {"fused": L.TN_FUSED, "plain": L.TN_PLAIN, "molecule": L.TN_MOLECULE}


class TensorNetError(RuntimeError):
    pass


def _check(rc: int, what: str):
    if rc != L.TN_OK:
        raise TensorNetError(f"{what}: {L.status_string(rc)} ({rc})")


def _status_bits(word: int) -> str:
    names = [(L.TN_STATUS_OVERFLOW, "pair overflow"), (L.TN_STATUS_BATCH, "bad batch vector"),
             (L.TN_STATUS_Z, "atomic number out of range"), (L.TN_STATUS_NONFINITE, "non-finite value")]
    return ", ".join(n for b, n in names if word & b) or "ok"


def _box_arg(box):
    if box is None:
        return None, None
    arr = (ctypes.c_double * 9)(*np.asarray(box, dtype=np.float64).reshape(9).tolist())
    return arr, ctypes.cast(arr, ctypes.c_void_p)


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _require_device(t: torch.Tensor, name: str, dtype, device):
    if not t.is_cuda or t.device != device:
        raise TensorNetError(f"{name} must live on {device}")
    if t.dtype != dtype:
        raise TensorNetError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise TensorNetError(f"{name} must be contiguous")


class Workspace:
    """Grow-only device scratch buffer (a uint8 tensor)."""

    def __init__(self, device):
        self.device = device
        self.buf = None

    def get(self, nbytes: int) -> torch.Tensor:
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=self.device)
        return self.buf


_NBR = {"auto": L.TN_NBR_AUTO, "cell": L.TN_NBR_CELL, "brute": L.TN_NBR_BRUTE}


def build_neighbors(pos: torch.Tensor, batch: torch.Tensor, cutoff: float, max_pairs: int, box=None,
                    check: bool = True, ws: Workspace | None = None, method: str = "auto", out=None):
    """Unordered neighbour pairs (tn_build_neighbors_method): returns (pairs [2, max_pairs] int32, n_pairs,
    status).  method: "auto", "cell" or "brute"; out: optional (pairs, n_pairs, status) tensors to fill."""
    device = pos.device
    pos_f64 = pos.dtype == torch.float64
    _require_device(pos, "pos", torch.float64 if pos_f64 else torch.float32, device)
    _require_device(batch, "batch", torch.int32, device)
    n = pos.shape[0]
    boxarr, boxp = _box_arg(box)
    nbytes = L.lib().tn_neighbor_workspace_bytes(n, max_pairs, boxp, float(cutoff))
    if nbytes == 0:
        raise TensorNetError("invalid neighbour-search request (box or sizes)")
    ws = ws or Workspace(device)
    buf = ws.get(nbytes)
    if out is None:
        pairs = torch.empty((2, max_pairs), dtype=torch.int32, device=device)
        n_pairs = torch.zeros(1, dtype=torch.int64, device=device)
        status = torch.zeros(1, dtype=torch.int32, device=device)
    else:
        pairs, n_pairs, status = out
    rc = L.lib().tn_build_neighbors_method(_stream(device), n, _ptr(pos), int(pos_f64), _ptr(batch), boxp,
                                           float(cutoff), max_pairs, _ptr(pairs), _ptr(n_pairs), _ptr(status),
                                           _ptr(buf), buf.numel(), _NBR[method])
    _check(rc, "tn_build_neighbors_method")
    if check:
        word = int(status.item())
        if word & ~L.TN_STATUS_OVERFLOW:
            raise TensorNetError(f"neighbour search: {_status_bits(word)}")
    return pairs, n_pairs, status


class TensorNet:
    """A TensorNet model on one GPU (tn_model_create over a weight blob)."""

    def __init__(self, blob: bytes, device: int | str | torch.device = 0):
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self._blob = bytes(blob)
        h = ctypes.c_void_p()
        buf = ctypes.create_string_buffer(self._blob, len(self._blob))
        _check(L.lib().tn_model_create(ctypes.cast(buf, ctypes.c_void_p), len(self._blob), self.device.index,
                                       ctypes.byref(h)), "tn_model_create")
        self._h = h
        F, K, Ly, Z = (ctypes.c_int32() for _ in range(4))
        rlo, rc = ctypes.c_double(), ctypes.c_double()
        _check(L.lib().tn_model_info(self._h, ctypes.byref(F), ctypes.byref(K), ctypes.byref(Ly), ctypes.byref(Z),
                                     ctypes.byref(rlo), ctypes.byref(rc)), "tn_model_info")
        self.F, self.K, self.L, self.max_z = F.value, K.value, Ly.value, Z.value
        self.r_lo, self.r_c = rlo.value, rc.value
        self.ws = Workspace(self.device)
        self.n_pairs = torch.zeros(1, dtype=torch.int64, device=self.device)
        self.status = torch.zeros(1, dtype=torch.int32, device=self.device)

    def close(self):
        if getattr(self, "_h", None):
            L.lib().tn_model_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self, n_atoms, n_systems, max_pairs, box=None, precision="fp32", path="fused",
                        forces=True) -> int:
        _, boxp = _box_arg(box)
        return int(L.lib().tn_workspace_bytes(self._h, n_atoms, n_systems, max_pairs, boxp, _PREC[precision],
                                              _PATH[path], int(forces)))

    def _run(self, pos, z, batch, n_systems, box, max_pairs, precision, path, forces, check, energy_out=None,
             forces_out=None):
        dev = self.device
        pdt = torch.float64 if precision == "fp64" else torch.float32
        _require_device(pos, "pos", pdt, dev)
        _require_device(z, "z", torch.int32, dev)
        _require_device(batch, "batch", torch.int32, dev)
        n = pos.shape[0]
        if max_pairs is None:
            max_pairs = max(64 * n, 1)
        boxarr, boxp = _box_arg(box)
        nbytes = L.lib().tn_workspace_bytes(self._h, n, n_systems, max_pairs, boxp, _PREC[precision], _PATH[path],
                                            int(forces))
        if nbytes == 0:
            raise TensorNetError(f"invalid request (precision={precision}, path={path}, box, sizes)")
        buf = self.ws.get(nbytes)
        E = energy_out if energy_out is not None else torch.empty(n_systems, dtype=torch.float64, device=dev)
        args_head = (self._h, _stream(dev), n, n_systems, _ptr(pos), _ptr(z), _ptr(batch), boxp, max_pairs,
                     _PREC[precision], _PATH[path], _ptr(E))
        if forces:
            Fo = forces_out if forces_out is not None else torch.empty((n, 3), dtype=pdt, device=dev)
            rc = L.lib().tn_energy_forces(*args_head, _ptr(Fo), _ptr(self.n_pairs), _ptr(self.status), _ptr(buf),
                                          buf.numel())
            _check(rc, "tn_energy_forces")
        else:
            Fo = None
            rc = L.lib().tn_energy(*args_head, _ptr(self.n_pairs), _ptr(self.status), _ptr(buf), buf.numel())
            _check(rc, "tn_energy")
        if check:
            self.check()
        return E, Fo

    def check(self):
        """Synchronise and raise if the device status word is non-zero."""
        word = int(self.status.item())
        if word:
            raise TensorNetError(f"device status {word}: {_status_bits(word)} (n_pairs={int(self.n_pairs.item())})")

    def energy(self, pos, z, batch, n_systems, box=None, max_pairs=None, precision="fp32", path="fused",
               check=True, out=None):
        return self._run(pos, z, batch, n_systems, box, max_pairs, precision, path, False, check, energy_out=out)[0]

    def energy_forces(self, pos, z, batch, n_systems, box=None, max_pairs=None, precision="fp32", path="fused",
                      check=True, energy_out=None, forces_out=None):
        return self._run(pos, z, batch, n_systems, box, max_pairs, precision, path, True, check,
                         energy_out=energy_out, forces_out=forces_out)

    def param_shapes(self):
        """(name, shape) of every tensor of the weight blob, in blob order: the layout of the flat gradient
        tn_train_grad writes."""
        F, K, Z = self.F, self.K, self.max_z
        out = [("emb.E", (Z, F)), ("emb.Wz", (F, 2 * F)), ("emb.bz", (F,)), ("emb.W0", (3 * F, K)),
               ("emb.b0", (3 * F,)), ("emb.ln_g", (F,)), ("emb.ln_b", (F,)), ("emb.W1", (2 * F, F)),
               ("emb.b1", (2 * F,)), ("emb.W2", (3 * F, 2 * F)), ("emb.b2", (3 * F,)), ("emb.WI", (F, F)),
               ("emb.WA", (F, F)), ("emb.WS", (F, F))]
        for layer in range(self.L):
            p = f"layer{layer}."
            out += [(p + "Wa", (F, K)), (p + "ba", (F,)), (p + "Wb", (2 * F, F)), (p + "bb", (2 * F,)),
                    (p + "Wc", (3 * F, 2 * F)), (p + "bc", (3 * F,)), (p + "W1I", (F, F)), (p + "W1A", (F, F)),
                    (p + "W1S", (F, F)), (p + "W2I", (F, F)), (p + "W2A", (F, F)), (p + "W2S", (F, F))]
        out += [("out.ln_g", (3 * F,)), ("out.ln_b", (3 * F,)), ("out.Wo", (F, 3 * F)), ("out.bo", (F,)),
                ("out.Wh", (F // 2, F)), ("out.bh", (F // 2,)), ("out.W2", (1, F // 2)), ("out.b2", (1,))]
        return out

    def split_params(self, flat: torch.Tensor) -> dict:
        """Views of a flat blob-ordered tensor (a gradient from train_grad) by tensor name."""
        out, off = {}, 0
        for name, shape in self.param_shapes():
            n = int(np.prod(shape))
            out[name] = flat[off:off + n].view(shape)
            off += n
        if off != flat.numel():
            raise TensorNetError(f"expected {off} values, got {flat.numel()}")
        return out

    def param_count(self) -> int:
        return int(L.lib().tn_param_count(self._h))

    def train_grad(self, pos, z, batch, n_systems, energy_ref, forces_ref, box=None, max_pairs=None,
                   precision="fp64", w_energy=1.0, w_force=1.0, check=True, grad_out=None):
        """One training step's loss and weight gradient (tn_train_grad).  Returns (loss [1] float64, energies,
        forces, grad [param_count] float64), all on the device."""
        dev = self.device
        pdt = torch.float64 if precision == "fp64" else torch.float32
        _require_device(pos, "pos", pdt, dev)
        _require_device(z, "z", torch.int32, dev)
        _require_device(batch, "batch", torch.int32, dev)
        _require_device(energy_ref, "energy_ref", torch.float64, dev)
        _require_device(forces_ref, "forces_ref", torch.float64, dev)
        n = pos.shape[0]
        if max_pairs is None:
            max_pairs = max(64 * n, 1)
        boxarr, boxp = _box_arg(box)
        nbytes = L.lib().tn_train_workspace_bytes(self._h, n, n_systems, max_pairs, boxp, _PREC[precision])
        if nbytes == 0:
            raise TensorNetError(f"invalid training request (precision={precision}, box, sizes)")
        buf = self.ws.get(nbytes)
        loss = torch.empty(1, dtype=torch.float64, device=dev)
        E = torch.empty(n_systems, dtype=torch.float64, device=dev)
        Fo = torch.empty((n, 3), dtype=pdt, device=dev)
        grad = grad_out if grad_out is not None else torch.empty(self.param_count(), dtype=torch.float64,
                                                                 device=dev)
        rc = L.lib().tn_train_grad(self._h, _stream(dev), n, n_systems, _ptr(pos), _ptr(z), _ptr(batch), boxp,
                                   max_pairs, _PREC[precision], _ptr(energy_ref), _ptr(forces_ref), float(w_energy),
                                   float(w_force), _ptr(loss), _ptr(E), _ptr(Fo), _ptr(grad), _ptr(self.n_pairs),
                                   _ptr(self.status), _ptr(buf), buf.numel())
        _check(rc, "tn_train_grad")
        if check:
            self.check()
        return loss, E, Fo, grad

    @staticmethod
    def pair_variant_count(precision="fp32") -> int:
        return int(L.lib().tn_pair_variant_count(_PREC[precision]))

    def set_pair_variant(self, precision="fp32", forward=-1, reverse=-1):
        """Force the fused pair kernels' tile shapes (tn_model_set_pair_variant); -1 = tuned/default."""
        _check(L.lib().tn_model_set_pair_variant(self._h, _PREC[precision], int(forward), int(reverse)),
               "tn_model_set_pair_variant")

    def autotune(self, pos, z, batch, n_systems, box=None, max_pairs=None, precision="fp32", reps=10):
        """Time every pair-tile shape on these inputs (tn_autotune) and keep the fastest for this pair-budget
        class; returns (forward shape, reverse shape).  Synchronises; never call it under capture."""
        dev = self.device
        _require_device(pos, "pos", torch.float32, dev)
        _require_device(z, "z", torch.int32, dev)
        _require_device(batch, "batch", torch.int32, dev)
        n = pos.shape[0]
        if max_pairs is None:
            max_pairs = max(64 * n, 1)
        boxarr, boxp = _box_arg(box)
        nbytes = L.lib().tn_workspace_bytes(self._h, n, n_systems, max_pairs, boxp, _PREC[precision],
                                            _PATH["fused"], 1)
        if nbytes == 0:
            raise TensorNetError(f"invalid request (precision={precision}, box, sizes)")
        buf = self.ws.get(nbytes)
        E = torch.empty(n_systems, dtype=torch.float64, device=dev)
        Fo = torch.empty((n, 3), dtype=torch.float32, device=dev)
        chosen = (ctypes.c_int32 * 2)()
        rc = L.lib().tn_autotune(self._h, _stream(dev), n, n_systems, _ptr(pos), _ptr(z), _ptr(batch), boxp,
                                 max_pairs, _PREC[precision], _ptr(E), _ptr(Fo), _ptr(self.n_pairs),
                                 _ptr(self.status), _ptr(buf), buf.numel(), int(reps),
                                 ctypes.cast(chosen, ctypes.c_void_p))
        _check(rc, "tn_autotune")
        self.check()
        return int(chosen[0]), int(chosen[1])


class Graph:
    """An instantiated HIP graph (tn_md_capture); keeps every buffer it uses alive."""

    def __init__(self, handle, device, keep):
        self._h = handle
        self.device = device
        self._keep = keep

    def replay(self):
        _check(L.lib().tn_graph_replay(self._h, _stream(self.device)), "tn_graph_replay")

    def close(self):
        if getattr(self, "_h", None):
            L.lib().tn_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def capture(model: "TensorNet", pos, z, batch, n_systems, box=None, max_pairs=None, precision="fp32",
            path="fused", n_steps=0, vel=None, inv_mass=None, dt_fs=1.0, energy_out=None, forces_out=None):
    """Record one energy+forces evaluation (n_steps=0) or n_steps velocity-Verlet steps into a graph.

    For MD, forces_out must hold F(pos) when the graph is first replayed; without it the forces of the
    current positions are computed here, before the capture.  Returns (graph, energy, forces, n_pairs, status); the tensors are the graph's outputs.
    """
    dev = model.device
    pdt = torch.float64 if precision == "fp64" else torch.float32
    _require_device(pos, "pos", pdt, dev)
    _require_device(z, "z", torch.int32, dev)
    _require_device(batch, "batch", torch.int32, dev)
    n = pos.shape[0]
    if max_pairs is None:
        max_pairs = max(64 * n, 1)
    boxarr, boxp = _box_arg(box)
    need = L.lib().tn_workspace_bytes(model._h, n, n_systems, max_pairs, boxp, _PREC[precision], _PATH[path], 1)
    if need == 0:
        raise TensorNetError("invalid capture request")
    ws = torch.empty(int(need) + 4096, dtype=torch.uint8, device=dev)
    E = energy_out if energy_out is not None else torch.empty(n_systems, dtype=torch.float64, device=dev)
    if forces_out is not None:
        Fo = forces_out
    elif n_steps > 0:
        # the first half kick of a replay needs F(pos) on entry
        _, Fo = model.energy_forces(pos, z, batch, n_systems, box=box, max_pairs=max_pairs, precision=precision,
                                    path=path)
    else:
        Fo = torch.zeros((n, 3), dtype=pdt, device=dev)
    n_pairs = torch.zeros(1, dtype=torch.int64, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    if n_steps > 0:
        _require_device(vel, "vel", torch.float32, dev)
        _require_device(inv_mass, "inv_mass", torch.float32, dev)
    h = ctypes.c_void_p()
    torch.cuda.synchronize(dev)
    # capture on a side stream (the legacy default stream cannot be captured)
    side = torch.cuda.Stream(dev)
    with torch.cuda.stream(side):
        rc = L.lib().tn_md_capture(model._h, _stream(dev), n, n_systems, _ptr(pos), _ptr(vel), _ptr(inv_mass),
                                   _ptr(z), _ptr(batch), boxp, float(dt_fs), int(n_steps), max_pairs,
                                   _PREC[precision], _PATH[path], _ptr(E), _ptr(Fo), _ptr(n_pairs), _ptr(status),
                                   _ptr(ws), ws.numel(), ctypes.byref(h))
    _check(rc, "tn_md_capture")
    keep = (pos, z, batch, vel, inv_mass, ws, E, Fo, n_pairs, status, side)
    return Graph(h, dev, keep), E, Fo, n_pairs, status


class TensorNetEF(torch.autograd.Function):
    """E = TensorNetEF.apply(model, pos, z, batch, n_systems, box, max_pairs, precision, path).

    Backward returns dL/dpos = -F * dL/dE[batch] from the library's forces.
    """

    @staticmethod
    def forward(ctx, model, pos, z, batch, n_systems, box, max_pairs, precision, path):
        E, Fo = model.energy_forces(pos.detach(), z, batch, n_systems, box=box, max_pairs=max_pairs,
                                    precision=precision, path=path)
        ctx.save_for_backward(Fo, batch)
        return E

    @staticmethod
    def backward(ctx, gE):
        Fo, batch = ctx.saved_tensors
        g = -(Fo.to(torch.float64) * gE[batch.long()][:, None]).to(Fo.dtype)
        return None, g, None, None, None, None, None, None, None
