"""Write the oracle's energies and forces for the larger workloads.

Calls only the FP64 oracle and the seeded generators; run from the repository
root:  python tests/golden/make_golden.py [cfg ...]
Each file holds E [S], F [N,3] (float64) and the pair count of the oracle's
neighbour set, for the workload of the same number (synth.CONFIGS).  For the
100k-atom box (workload 3), oracle_cfg3_sampled.npz holds exact forces of atoms
near two centres (see sampled_forces_periodic) and oracle_cfg3_energy.npz the
whole box's energy from the forward pass alone (argument 33 writes only that).
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import TensorNetOracle  # noqa: E402
from synth import make_config, make_weights, write_blob  # noqa: E402


def sampled_forces_periodic(cfg, centres=(0, 50_000), radius=35.0, core=5.0):
    """Exact oracle forces for atoms near a few centres of a large periodic box.

    The force on atom i depends only on atoms within 2(L+1) r_c of i (the energy of atom k
    sees atoms within (L+1) r_c of k, and F_i sums over those k).  An isolated cluster of
    radius `radius` around a centre, with coordinates unwrapped by the minimum image,
    therefore gives the periodic box's exact forces for every atom within
    radius - 2(L+1) r_c of the centre.
    """
    c = make_config(cfg)
    w = make_weights(c["F"], c["K"], c["L"], c["max_z"], seed=c["weight_seed"])
    o = TensorNetOracle(write_blob(w, c["F"], c["K"], c["L"], c["max_z"], c["r_c"]))
    reach = 2 * (c["L"] + 1) * c["r_c"]
    assert radius - reach >= core
    box_len = np.diag(c["box"])
    pos = c["pos"].astype(np.float64)
    idx_all, F_all = [], []
    for ci in centres:
        t = time.time()
        d = pos - pos[ci]
        d -= box_len * np.round(d / box_len)
        r = np.sqrt((d * d).sum(1))
        sel = np.flatnonzero(r < radius)
        # cluster coordinates: the minimum-image vectors from the centre, as float32 like the input
        cpos = (d[sel]).astype(np.float32)
        E, F = o.energy_forces(cpos, c["z"][sel], np.zeros(len(sel), np.int32), None, 1)
        keep = r[sel] < core
        idx_all.append(sel[keep])
        F_all.append(F[keep])
        print(f"cfg {cfg}: cluster around {ci}: {len(sel)} atoms, {keep.sum()} exact rows, "
              f"{time.time() - t:.1f}s", flush=True)
    path = os.path.join(HERE, f"oracle_cfg{cfg}_sampled.npz")
    np.savez_compressed(path, idx=np.concatenate(idx_all), F=np.concatenate(F_all),
                        n_pairs=np.int64(len(o.pairs(c["pos"], c["batch"], c["box"]))))
    print(f"-> {path}", flush=True)


def box_energy(cfg):
    """The oracle's energy of a whole periodic box (forward only, no autograd), with the sum of
    the per-atom energy magnitudes: the denominator for a near-cancelling sum."""
    c = make_config(cfg)
    w = make_weights(c["F"], c["K"], c["L"], c["max_z"], seed=c["weight_seed"])
    o = TensorNetOracle(write_blob(w, c["F"], c["K"], c["L"], c["max_z"], c["r_c"]))
    t = time.time()
    pairs = o.pairs(c["pos"], c["batch"], c["box"])
    cap = {}
    E = o.energy(c["pos"], c["z"], c["batch"], c["box"], c["n_systems"], pairs=pairs, capture=cap)
    eps = cap["atom_energy"].numpy()
    path = os.path.join(HERE, f"oracle_cfg{cfg}_energy.npz")
    np.savez_compressed(path, E=E, abs_atom_energy_sum=np.array([np.abs(eps).sum()]),
                        n_pairs=np.int64(len(pairs)))
    print(f"cfg {cfg}: N={len(c['pos'])} pairs={len(pairs)} E={E} sum|eps|={np.abs(eps).sum():.6f} "
          f"{time.time() - t:.1f}s -> {path}", flush=True)


def main(cfgs):
    for cfg in cfgs:
        if cfg == 3:
            sampled_forces_periodic(cfg)
            box_energy(cfg)
            continue
        if cfg == 33:   # the 100k-atom box's energy alone
            box_energy(3)
            continue
        c = make_config(cfg)
        w = make_weights(c["F"], c["K"], c["L"], c["max_z"], seed=c["weight_seed"])
        o = TensorNetOracle(write_blob(w, c["F"], c["K"], c["L"], c["max_z"], c["r_c"]))
        t = time.time()
        pairs = o.pairs(c["pos"], c["batch"], c["box"])
        E, F = o.energy_forces(c["pos"], c["z"], c["batch"], c["box"], c["n_systems"], pairs=pairs)
        path = os.path.join(HERE, f"oracle_cfg{cfg}.npz")
        np.savez_compressed(path, E=E, F=F, n_pairs=np.int64(len(pairs)))
        print(f"cfg {cfg}: N={len(c['pos'])} pairs={len(pairs)} {time.time() - t:.1f}s -> {path}", flush=True)


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or [1, 2])
