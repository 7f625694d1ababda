"""Write the oracle's energies and forces for the larger workloads.

Calls only the FP64 oracle and the seeded generators; run from the repository
root:  python tests/golden/make_golden.py [cfg ...]
Each file holds E [S], F [N,3] (float64) and the pair count of the oracle's
neighbour set, for the workload of the same number (synth.CONFIGS).
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import TensorNetOracle  # noqa: E402
from synth import make_config, make_weights, write_blob  # noqa: E402


def main(cfgs):
    for cfg in cfgs:
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
