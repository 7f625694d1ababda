"""tn_energy_forces_static (the entry point that allocates nothing; its scratch is the library's
static device array) against tn_energy_forces with a caller workspace: two calls in a row, the
second with a smaller input, must give the same bits; requests larger than the static scratch are
rejected on the host."""

import ctypes

import numpy as np
import pytest
import torch

from paper_2402_17660_amd import TensorNet
from paper_2402_17660_amd import _lib as L
from tests.util import random_box, random_molecule, small_blob

pytestmark = pytest.mark.gpu

_PREC = {"fp32": L.TN_FP32, "bf16": L.TN_BF16, "fp64": L.TN_FP64}
_PATH = {"fused": L.TN_FUSED, "plain": L.TN_PLAIN}


def _vp(t):
    return ctypes.c_void_p(t.data_ptr())


def static_call(model, pos, z, batch, S, box, max_pairs, precision, path):
    """One tn_energy_forces_static call through the C ABI; returns (rc, E, F, n_pairs, status)."""
    dev = model.device
    n = pos.shape[0]
    E = torch.full((S,), float("nan"), dtype=torch.float64, device=dev)
    Fo = torch.full((n, 3), float("nan"), dtype=pos.dtype, device=dev)
    n_pairs = torch.zeros(1, dtype=torch.int64, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    boxarr = None if box is None else (ctypes.c_double * 9)(*np.asarray(box, np.float64).reshape(9).tolist())
    rc = L.lib().tn_energy_forces_static(model._h, torch.cuda.current_stream(dev).cuda_stream, n, S, _vp(pos),
                                         _vp(z), _vp(batch), None if boxarr is None else ctypes.cast(boxarr,
                                                                                                      ctypes.c_void_p),
                                         max_pairs, _PREC[precision], _PATH[path], _vp(E), _vp(Fo), _vp(n_pairs),
                                         _vp(status))
    torch.cuda.synchronize(dev)
    return rc, E, Fo, n_pairs, status


def _inputs(dev, pos, z, precision, S=1, batch=None):
    pdt = torch.float64 if precision == "fp64" else torch.float32
    p = torch.tensor(pos, dtype=pdt, device=dev)
    zt = torch.tensor(z, dtype=torch.int32, device=dev)
    b = np.zeros(len(pos), np.int32) if batch is None else batch
    return p, zt, torch.tensor(b, dtype=torch.int32, device=dev)


@pytest.mark.parametrize("precision,path", [("fp32", "fused"), ("bf16", "fused"), ("fp64", "plain")])
def test_static_matches_workspace_entry_point(dev, precision, path):
    blob = small_blob(F=64, K=32, L=2, seed=91)
    m = TensorNet(blob, dev)
    # a larger input first (a periodic box), then a smaller one (an isolated molecule): the second call
    # runs on scratch that still holds the first call's contents
    pb, zb, box = random_box(150, 92, 12.0)
    pm, zm = random_molecule(30, 93)
    cases = [(pb, zb, box, 150 * 20), (pm, zm, None, 30 * 32)]
    for pos, z, bx, mp in cases:
        need = m.workspace_bytes(len(pos), 1, mp, box=bx, precision=precision, path=path)
        assert 0 < need <= L.TN_STATIC_WS_BYTES, need
        p, zt, bt = _inputs(dev, pos, z, precision)
        rc, E, Fo, n_pairs, status = static_call(m, p, zt, bt, 1, bx, mp, precision, path)
        assert rc == L.TN_OK, L.status_string(rc)
        assert int(status.item()) == 0
        E_ref, F_ref = m.energy_forces(p, zt, bt, 1, box=bx, max_pairs=mp, precision=precision, path=path)
        torch.cuda.synchronize(dev)
        print(f"static {precision}/{path} n={len(pos)}: E={float(E[0]):.10f} (workspace call "
              f"{float(E_ref[0]):.10f}), {int(n_pairs.item())} pairs, workspace {need} bytes", flush=True)
        assert int(n_pairs.item()) == int(m.n_pairs.item())
        assert torch.equal(E, E_ref)
        assert torch.equal(Fo, F_ref)


def test_static_rejects_requests_beyond_its_scratch(dev):
    blob = small_blob(F=64, K=32, L=2, seed=91)
    m = TensorNet(blob, dev)
    pm, zm = random_molecule(30, 93)
    p, zt, bt = _inputs(dev, pm, zm, "fp32")
    big = 1 << 22   # a pair budget whose workspace is far beyond the static scratch
    assert m.workspace_bytes(30, 1, big, precision="fp32", path="fused") > L.TN_STATIC_WS_BYTES
    rc, E, Fo, n_pairs, status = static_call(m, p, zt, bt, 1, None, big, "fp32", "fused")
    assert rc == L.TN_E_WORKSPACE
    assert torch.isnan(E).all() and torch.isnan(Fo).all()   # nothing was enqueued
    # a valid call afterwards still works
    rc, E, Fo, _, status = static_call(m, p, zt, bt, 1, None, 30 * 32, "fp32", "fused")
    assert rc == L.TN_OK and int(status.item()) == 0 and torch.isfinite(Fo).all()
