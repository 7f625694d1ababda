"""Benchmark: TensorNet energy+forces atom-steps/s on one MI355X.

One step = one full energy-and-forces evaluation (cell-list neighbour search,
embedding, interaction layers, output network, reverse sweep for forces) of
the periodic 6000-atom box (hidden 128, 2 layers, 32 RBF, cutoff 5 A) with all
inputs resident in HBM.  Prints one JSON line on stdout.

The timed variants are the fused path (FP32, BF16) and the plain unfused path
(FP32).  `value` is the fused FP32 path when it is available.  Each variant's
result is compared with the FP64 oracle's stored energies and forces.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "TensorNet energy+forces atom-steps/s, fused vs plain, at stated force error"
PEAK = {"fp32": 157.3e12, "bf16": 2.5e15, "fp64": 78.6e12}   # dense MFMA peaks, FLOP/s
HBM_PEAK = 8.0e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_flops_per_atom_step(F, K, L, p):
    """Forward FLOPs per atom (edge filter once per unordered pair, p = pairs/atom); E+F = 2x."""
    fwd = (p * (6 * K * F + L * 2 * (K * F + 2 * F * F + 6 * F * F)) + 2 * p * 20 * F + L * 2 * p * 18 * F
           + 34 * F * F + L * (36 * F * F + 162 * F) + 2 * (3 * F * F + F * F / 2 + F / 2))
    return 2.0 * fwd


def edge_filter_flops_per_pair(F, K):
    return 2.0 * (K * F + 2 * F * F + 6 * F * F)


# timed kernels of each path: {timer name: algorithmic FLOP per unordered pair per launch}
def timed_kernels(path, F, K, L):
    if path == "plain":
        return {"plain_edge_gemm_c": 2.0 * (2 * F) * (3 * F)}
    per_pair = 2.0 * K * 3 * F + L * edge_filter_flops_per_pair(F, K)
    return {"edge_fwd": per_pair, "edge_bwd": per_pair}


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "edge_kernels_fp32_box6000_hbm_counters.md")


def measured_traffic(kernel, precision):
    """HBM bytes per launch of the dominant kernel from the committed counter summary, or None when
    there is none for it or the kernel sources changed since the counters were taken."""
    import hashlib
    if kernel != "edge_bwd" or precision != "fp32" or not os.path.exists(TRAFFIC_SUMMARY):
        return None
    fields = {}
    for line in open(TRAFFIC_SUMMARY):
        k, _, v = line.strip().partition(": ")
        if k in ("edge_bwd_traffic_bytes", "kernel_sources_sha256"):
            fields[k] = v
    csrc = os.path.join(ROOT, "paper_2402_17660_amd", "csrc")
    h = hashlib.sha256(b"".join(open(os.path.join(csrc, n), "rb").read()
                                for n in ("tn_pair.hip", "tn_mfma.h", "tn_device.h", "tn_internal.h"))).hexdigest()
    if fields.get("kernel_sources_sha256") != h or "edge_bwd_traffic_bytes" not in fields:
        return None
    return float(fields["edge_bwd_traffic_bytes"])


def cpu_baseline(n_atoms, F, K, L, r_c, seed):
    import numpy as np
    import torch
    from oracle import TensorNetOracle
    from synth import make_weights, periodic_box, write_blob
    box_in = periodic_box(n_atoms, seed=5001)
    o = TensorNetOracle(write_blob(make_weights(F, K, L, 100, seed=seed), F, K, L, 100, r_c))
    pairs = o.pairs(box_in["pos"], box_in["batch"], box_in["box"])
    t = time.perf_counter()
    o.energy_forces(box_in["pos"], box_in["z"], box_in["batch"], box_in["box"], 1, pairs=pairs)
    dt = time.perf_counter() - t
    return dict(value=n_atoms / dt, unit="atom-steps/s", cores=torch.get_num_threads(), kind="oracle",
                sample=f"one FP64 energy+forces evaluation of a {n_atoms}-atom periodic box at 0.1 atoms/A^3 "
                       f"(same model sizes, {len(pairs)} pairs), {dt:.1f} s incl. autograd; neighbour list excluded")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--variants", default="fused:fp32,fused:bf16,plain:fp32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-atoms", type=int, default=3000)
    ap.add_argument("--budget", type=float, default=1.05, help="max_pairs = budget * true pair count")
    ap.add_argument("--extra", default="batch,md,table2,nbr,train",
                    help="extra workloads: batch (512 molecules, captured), md (100 captured velocity-Verlet steps, "
                         "100k atoms), table2 (the paper's Table 2 sizes and 0/1/2 layers, captured), nbr "
                         "(neighbour-search study on random clouds), train (one training step on 64 molecules, "
                         "loss on energies and forces, exact weight gradient); 'none' = none")
    ap.add_argument("--md-steps", type=int, default=100)
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="after the timed variants, copy this many MiB device-to-device once (a reference "
                         "dispatch of known size for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); run it with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2402_17660_amd import TensorNet, TensorNetError, lib
    from synth import make_config, make_weights, write_blob

    cfg = 1
    c = make_config(cfg)
    F, K, L, r_c = c["F"], c["K"], c["L"], c["r_c"]
    N = len(c["pos"])
    dev = torch.device("cuda", 0)
    blob = write_blob(make_weights(F, K, L, c["max_z"], seed=c["weight_seed"]), F, K, L, c["max_z"], r_c)
    model = TensorNet(blob, dev)
    pos = torch.tensor(c["pos"], device=dev)
    z = torch.tensor(c["z"], device=dev)
    batch = torch.tensor(c["batch"], device=dev)
    box = c["box"]
    golden = np.load(os.path.join(ROOT, "tests", "golden", f"oracle_cfg{cfg}.npz"))

    # static pair budget from one untimed call
    model.energy_forces(pos, z, batch, 1, box=box, max_pairs=64 * N, precision="fp32", path="plain")
    n_pairs = int(model.n_pairs.item())
    max_pairs = int(math.ceil(args.budget * n_pairs / 1024.0) * 1024)
    log(f"workload: N={N} pairs={n_pairs} max_pairs={max_pairs}")

    L_ = lib()
    results = []
    for spec in args.variants.split(","):
        path, prec = spec.split(":")
        try:
            E_out = torch.empty(1, dtype=torch.float64, device=dev)
            F_out = torch.empty((N, 3), dtype=torch.float32, device=dev)
            run = lambda: model.energy_forces(pos, z, batch, 1, box=box, max_pairs=max_pairs, precision=prec,
                                              path=path, check=False, energy_out=E_out, forces_out=F_out)
            run()
            model.check()
            # pick the pair-tile shapes for this workload (setup, outside the timed region)
            shapes = (model.autotune(pos, z, batch, 1, box=box, max_pairs=max_pairs, precision=prec, reps=10)
                      if path == "fused" else None)
        except TensorNetError as e:
            log(f"{path}/{prec}: unavailable ({e})")
            results.append(dict(path=path, precision=prec, available=False))
            continue
        for _ in range(args.warmup):
            run()
        torch.cuda.synchronize()
        timers = timed_kernels(path, F, K, L)
        L_.tn_timing_reset()
        L_.tn_timing_enable(1)
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record()
        for _ in range(args.steps):
            run()
        stop.record()
        torch.cuda.synchronize()
        L_.tn_timing_enable(0)
        ms = start.elapsed_time(stop) / args.steps
        import ctypes
        kernels = []
        for timer, flop_per_pair in timers.items():
            tot, cnt = ctypes.c_double(), ctypes.c_int64()
            L_.tn_timing_read(timer.encode(), ctypes.byref(tot), ctypes.byref(cnt))
            kernel_ms = tot.value / max(cnt.value, 1)
            flop_per_launch = flop_per_pair * n_pairs
            achieved = flop_per_launch / (kernel_ms * 1e-3) if cnt.value else None
            kernels.append(dict(name=timer, launches_per_step=cnt.value / args.steps, avg_ms=kernel_ms,
                                ms_per_step=tot.value / args.steps, flop_per_launch=flop_per_launch,
                                achieved_tflops=(achieved / 1e12) if achieved else None,
                                peak_tflops=PEAK[prec] / 1e12))
        model.check()
        E = E_out.cpu().numpy()
        Fo = F_out.double().cpu().numpy()
        e_err = float(np.max(np.abs(E - golden["E"]) / np.abs(golden["E"])))
        f_err = float(np.linalg.norm(Fo - golden["F"]) / np.linalg.norm(golden["F"]))
        dom = max(kernels, key=lambda k: k["ms_per_step"])
        res = dict(path=path, precision=prec, available=True, ms_per_step=ms, value=N / (ms * 1e-3),
                   energy_rel_err=e_err, force_rel_rms=f_err, kernel=dom, kernels=kernels,
                   pair_tile_shapes=dict(forward=shapes[0], reverse=shapes[1]) if shapes else None)
        log(f"{path}/{prec}: {ms:.3f} ms/step, {res['value']:.3e} atom-steps/s, E err {e_err:.2e}, "
            + (f"tile shapes {shapes}, " if shapes else "") +
            f"F err {f_err:.2e}, " + ", ".join(f"{k['name']} {k['avg_ms']:.3f} ms/launch "
                                               f"({k['achieved_tflops'] or 0:.1f} TFLOP/s)" for k in kernels))
        results.append(res)

    if args.copy_probe > 0:
        n = args.copy_probe * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe} MiB read + {args.copy_probe} MiB written in one dispatch")
        del src, dst

    avail = [r for r in results if r.get("available")]
    head = next((r for r in avail if r["path"] == "fused" and r["precision"] == "fp32"), None) or avail[0]
    k = head["kernel"]
    roofline = dict(bound="mfma", achieved=k["achieved_tflops"], peak=k["peak_tflops"], unit="TFLOP/s",
                    frac=(k["achieved_tflops"] / k["peak_tflops"]) if k["achieved_tflops"] else None,
                    traffic=measured_traffic(k["name"], head["precision"]),
                    kernel=k["name"], avg_launch_ms=k["avg_ms"], flop_per_launch=k["flop_per_launch"])
    p_atom = n_pairs / N
    step_flop = algorithmic_flops_per_atom_step(F, K, L, p_atom) * N
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host ...")
        cpu = cpu_baseline(args.cpu_atoms, F, K, L, r_c, c["weight_seed"])
    extra = {}
    for name in [e for e in args.extra.split(",") if e and e != "none"]:
        try:
            extra[name] = EXTRA[name](args, dev)
        except Exception as e:   # an extra workload never hides the headline line
            log(f"extra workload {name} failed: {e!r}")
            extra[name] = dict(error=repr(e))
    out = dict(metric=METRIC, value=head["value"], unit="atom-steps/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=head["ms_per_step"], higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="f32" if head["precision"] == "fp32" else head["precision"],
               data="synthetic",
               config=dict(workload="periodic cubic box, 6000 atoms at 0.1/A^3, Z in {H,C,N,O}; TensorNet hidden 128, "
                                    "2 layers, 32 RBF, cutoff 5 A; energy+forces incl. cell-list neighbour search",
                           n_atoms=N, n_pairs=n_pairs, max_pairs=max_pairs, path=head["path"],
                           precision=head["precision"]),
               roofline=roofline, cpu_baseline=cpu,
               step_algorithmic_tflop=step_flop / 1e12,
               step_tflops=step_flop / (head["ms_per_step"] * 1e-3) / 1e12,
               errors=dict(energy_rel=head["energy_rel_err"], force_rel_rms=head["force_rel_rms"]),
               variants=results, extra=extra)
    print(json.dumps(out), flush=True)


def _blob_for(c):
    from synth import make_weights, write_blob
    return write_blob(make_weights(c["F"], c["K"], c["L"], c["max_z"], seed=c["weight_seed"]),
                      c["F"], c["K"], c["L"], c["max_z"], c["r_c"])


def extra_batch(args, dev):
    """512 isolated molecules of 8-64 atoms: one captured graph per evaluation, FP32 vs BF16."""
    import numpy as np
    import torch
    from paper_2402_17660_amd import TensorNet, capture
    from synth import make_config
    c = make_config(2)
    N = len(c["pos"])
    golden = np.load(os.path.join(ROOT, "tests", "golden", "oracle_cfg2.npz"))
    model = TensorNet(_blob_for(c), dev)
    pos = torch.tensor(c["pos"], device=dev)
    z = torch.tensor(c["z"], device=dev)
    batch = torch.tensor(c["batch"], device=dev)
    mp = int(math.ceil(1.05 * int(golden["n_pairs"]) / 1024.0) * 1024)
    out = dict(workload="512 isolated molecules, sizes uniform 8-64 atoms (centred at the origin), hidden 128, "
                        "2 layers, cutoff 5 A; one captured HIP graph per energy+forces call",
               n_atoms=N, n_pairs=int(golden["n_pairs"]), max_pairs=mp)
    for prec in ("fp32", "bf16"):
        shapes = model.autotune(pos, z, batch, c["n_systems"], max_pairs=mp, precision=prec, reps=3)
        g, E, Fo, n_pairs, status = capture(model, pos, z, batch, c["n_systems"], max_pairs=mp, precision=prec)
        for _ in range(3):
            g.replay()
        torch.cuda.synchronize()
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 20
        start.record()
        for _ in range(reps):
            g.replay()
        stop.record()
        torch.cuda.synchronize()
        ms = start.elapsed_time(stop) / reps
        Ev = E.cpu().numpy()
        Fv = Fo.double().cpu().numpy()
        out[prec] = dict(ms_per_step=ms, value=N / (ms * 1e-3), status=int(status.item()), pair_tile_shapes=shapes,
                         energy_rel_err=float(np.max(np.abs(Ev - golden["E"]) / np.abs(golden["E"]))),
                         force_rel_rms=float(np.linalg.norm(Fv - golden["F"]) / np.linalg.norm(golden["F"])))
        log(f"batch/{prec}: {ms:.3f} ms/step, {out[prec]['value']:.3e} atom-steps/s, "
            f"E err {out[prec]['energy_rel_err']:.2e}, F err {out[prec]['force_rel_rms']:.2e}")
        g.close()
    return out


def extra_md(args, dev):
    """100k-atom periodic box: n captured velocity-Verlet steps (dt 1 fs), neighbours rebuilt every step."""
    import numpy as np
    import torch
    from paper_2402_17660_amd import TensorNet, capture
    from synth import make_config, maxwell_boltzmann
    from synth.generators import masses
    c = make_config(3)
    N = len(c["pos"])
    model = TensorNet(_blob_for(c), dev)
    z = torch.tensor(c["z"], device=dev)
    batch = torch.tensor(c["batch"], device=dev)
    m_amu = masses(c["z"])
    inv_m = torch.tensor((1.0 / m_amu).astype(np.float32), device=dev)
    out = dict(workload=f"periodic cubic box of 100000 atoms (100 A), hidden 128, 2 layers, cutoff 5 A; "
                        f"{args.md_steps} velocity-Verlet steps (dt 1 fs) in one HIP graph, neighbour search every "
                        f"step; Maxwell-Boltzmann velocities at 300 K", n_atoms=N, steps=args.md_steps)
    for prec in ("fp32", "bf16"):
        pos = torch.tensor(c["pos"], device=dev)
        vel = torch.tensor(maxwell_boltzmann(c["z"]), device=dev)
        E0, F0 = model.energy_forces(pos, z, batch, 1, box=c["box"], max_pairs=32 * N, precision=prec)
        n0 = int(model.n_pairs.item())
        mp = int(math.ceil(1.10 * n0 / 1024.0) * 1024)
        rms_f0 = float(torch.sqrt((F0.double() ** 2).mean()))
        shapes = model.autotune(pos, z, batch, 1, box=c["box"], max_pairs=mp, precision=prec, reps=2)
        g, E, Fo, n_pairs, status = capture(model, pos, z, batch, 1, box=c["box"], max_pairs=mp, precision=prec,
                                            n_steps=args.md_steps, vel=vel, inv_mass=inv_m, dt_fs=1.0,
                                            forces_out=F0)
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        g.replay()
        stop.record()
        torch.cuda.synchronize()
        ms = start.elapsed_time(stop)
        st = int(status.item())
        out[prec] = dict(ms_per_replay=ms, ms_per_step=ms / args.md_steps, pair_tile_shapes=shapes,
                         value=N * args.md_steps / (ms * 1e-3), status=st, initial_pairs=n0, max_pairs=mp,
                         final_pairs=int(n_pairs.item()), initial_rms_force=rms_f0,
                         energy_start=float(E0[0]), energy_end=float(E[0]))
        log(f"md/{prec}: {args.md_steps} steps in {ms:.1f} ms ({ms / args.md_steps:.3f} ms/step, "
            f"{out[prec]['value']:.3e} atom-steps/s), status {st}, pairs {n0} -> {int(n_pairs.item())}")
        g.close()
    return out


# Table 2 of the paper: TensorNet E+F, one molecule per call, cutoff 4.5 A, hidden 128, 32 RBF,
# pair budget 32 N; the paper's "Graph" column (RTX 4090, Msteps/day) for 0/1/2 layers.
TABLE2 = [("alanine dipeptide", 22, (172.80, 84.71, 56.47)), ("testosterone", 49, (154.29, 63.53, 39.82)),
          ("chignolin", 166, (77.14, 26.02, 15.57)), ("DHFR", 2489, (5.65, 1.69, 1.00)),
          ("factor IX", 5807, (2.33, 0.70, 0.42))]


def _time_replays(g, reps):
    import torch
    for _ in range(10):
        g.replay()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        g.replay()
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / reps


def extra_table2(args, dev):
    """Synthetic molecules of the Table 2 sizes (random H/C/N/O, 0.1 atoms/A^3), 0/1/2 interaction layers,
    captured graphs, FP32 fused; plus the cost of the static pair budget (32 N, as in the paper) against an
    exact one, in workspace bytes and in time."""
    import torch
    from paper_2402_17660_amd import TensorNet, capture
    from synth import make_weights, single_molecule, write_blob
    rows = []
    for name, n, paper_g in TABLE2:
        mol = single_molecule(n, seed=7000 + n)
        pos = torch.tensor(mol["pos"], device=dev)
        z = torch.tensor(mol["z"], device=dev)
        batch = torch.tensor(mol["batch"], device=dev)
        for L in (0, 1, 2):
            model = TensorNet(write_blob(make_weights(128, 32, L, 100, seed=8000 + L), 128, 32, L, 100, 4.5), dev)
            reps = 50 if n < 1000 else 20
            g, E, Fo, n_pairs, status = capture(model, pos, z, batch, 1, max_pairs=32 * n, precision="fp32")
            ms = _time_replays(g, reps)
            st = int(status.item())
            np_true = int(n_pairs.item())
            g.close()
            g, E, Fo, n_pairs, status = capture(model, pos, z, batch, 1, max_pairs=max(np_true, 1),
                                                precision="fp32")
            ms_exact = _time_replays(g, reps)
            st |= int(status.item())
            g.close()
            ws_static = model.workspace_bytes(n, 1, 32 * n)
            ws_exact = model.workspace_bytes(n, 1, max(np_true, 1))
            msteps_day = 86400.0 / (ms * 1e-3) / 1e6
            rows.append(dict(molecule=name, atoms=n, layers=L, pairs=np_true, ms_per_step=ms,
                             msteps_per_day=msteps_day, atom_steps_per_s=n / (ms * 1e-3), status=st,
                             ms_per_step_exact_budget=ms_exact, workspace_mb_static=ws_static / 2**20,
                             workspace_mb_exact=ws_exact / 2**20,
                             paper_graph_msteps_per_day_rtx4090=paper_g[L]))
            log(f"table2 {name} ({n} atoms, {np_true} pairs) {L}L: {ms * 1e3:.1f} us/step "
                f"({ms_exact * 1e3:.1f} with an exact pair budget), {msteps_day:.2f} Msteps/day "
                f"(paper RTX 4090 Graph: {paper_g[L]}); workspace {ws_static / 2**20:.1f} MB static vs "
                f"{ws_exact / 2**20:.1f} MB exact")
            model.close()
    return dict(workload="synthetic stand-ins for the Table 2 molecules (sizes 22-5807 atoms), cutoff 4.5 A, "
                         "hidden 128, 32 RBF, 0/1/2 layers, max_pairs 32 N (and the exact pair count), fused FP32, "
                         "one captured HIP graph per step",
                rows=rows)


def extra_nbr(args, dev):
    """Neighbour-search study, cell list vs brute force, on uniform random clouds with 64 neighbours per
    point (cutoff 5 A, periodic cube): an N sweep at 1, 2 and 64 systems, and 32768 points split into
    1..1024 systems.  Times eager calls (all launches of one search) with preallocated outputs."""
    import torch
    from paper_2402_17660_amd import Workspace, build_neighbors
    from synth import random_cloud

    def time_search(c, method, reps):
        n = len(c["pos"])
        pos = torch.tensor(c["pos"], device=dev)
        batch = torch.tensor(c["batch"], device=dev)
        mp = 40 * n
        ws = Workspace(dev)
        out = (torch.empty((2, mp), dtype=torch.int32, device=dev), torch.zeros(1, dtype=torch.int64, device=dev),
               torch.zeros(1, dtype=torch.int32, device=dev))
        call = lambda: build_neighbors(pos, batch, 5.0, mp, box=c["box"], check=False, ws=ws, method=method,
                                       out=out)
        for _ in range(3):
            call()
        torch.cuda.synchronize()
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(reps):
            call()
        stop.record()
        torch.cuda.synchronize()
        return start.elapsed_time(stop) / reps, int(out[1].item()), int(out[2].item())

    def row(n, nb, seed):
        c = random_cloud(n, nb, seed)
        r = dict(points=n, systems=nb)
        for method in ("cell", "brute"):
            if method == "brute" and n // nb > 65536:
                continue
            ms, pairs, st = time_search(c, method, 20)
            r[f"{method}_ms"] = ms
            r[f"{method}_pairs"] = pairs
            r[f"{method}_status"] = st
        log(f"nbr {n} points / {nb} systems: cell {r['cell_ms']:.3f} ms"
            + (f", brute {r['brute_ms']:.3f} ms" if "brute_ms" in r else "") + f", {r['cell_pairs']} pairs")
        return r

    sweep = [row(1 << k, nb, 9000 + 100 * nb + k) for nb in (1, 2, 64) for k in range(8, 21) if (1 << k) >= 4 * nb]
    split = [row(32768, 1 << b, 9500 + b) for b in range(0, 11)]
    return dict(workload="uniform random clouds, 64 neighbours per point on average within 5 A, periodic cube; "
                         "points split into systems by index range; cell list vs brute force (brute force up to "
                         "65536 points per system)", sweep=sweep, batch_split=split)


def timing(L_, name):
    """(total ms, launches) of a named scope in the library's timing registry."""
    import ctypes
    tot, cnt = ctypes.c_double(), ctypes.c_int64()
    L_.tn_timing_read(name.encode(), ctypes.byref(tot), ctypes.byref(cnt))
    return tot.value, cnt.value


def train_wgrad_flops(F, K, L, n_atoms, n_pairs, max_z):
    """Algorithmic FLOPs of the training step's parameter adjoints (outer products of layer adjoints with layer
    inputs) on dual numbers: per weight entry and row, one value product and two tangent products (6 FLOP)."""
    pair = n_pairs * (L * (F * K + 2 * F * F + 6 * F * F) + 3 * F * K)
    node = n_atoms * ((1 + 2 * L) * 9 * F * F + 2 * F * F + 6 * F * F + 3 * F * F + (F // 2) * F)
    species = 2 * max_z * F * F
    return 6.0 * (pair + node + species)


def train_cpu_baseline(c, n_mol):
    """The oracle's training step (double autograd, FP64) on the first n_mol molecules of the workload."""
    import numpy as np
    import torch
    from oracle import TensorNetOracle
    from oracle.train import training_loss_and_grad
    from synth import make_weights, write_blob
    sel = c["batch"] < n_mol
    pos, z, batch = c["pos"][sel].astype(np.float64), c["z"][sel], c["batch"][sel]
    blob = lambda seed: write_blob(make_weights(c["F"], c["K"], c["L"], c["max_z"], seed=seed), c["F"], c["K"],
                                   c["L"], c["max_z"], c["r_c"])
    E_ref, F_ref = TensorNetOracle(blob(3000)).energy_forces(pos, z, batch, None, n_mol)
    student = TensorNetOracle(blob(c["weight_seed"]))
    t = time.perf_counter()
    training_loss_and_grad(student, pos, z, batch, None, n_mol, E_ref, F_ref)
    dt = time.perf_counter() - t
    n = int(sel.sum())
    return dict(value=n / dt, unit="atoms/s", cores=torch.get_num_threads(), kind="oracle",
                sample=f"one FP64 training step (loss, forces, weight gradient by double autograd) on the first {n_mol} "
                       f"molecules of the workload ({n} atoms), {dt:.1f} s; teacher targets excluded")


def extra_train(args, dev):
    """One training step: 64 molecules of 16-128 atoms (0.05 A noise), hidden 128, 3 layers, cutoff 5 A; loss =
    mean squared energy error + mean squared force error against a teacher network of the same shape (seed 3000),
    and the exact gradient of that loss with respect to every weight of the student (tn_train_grad: energies and
    forces, then the dual-number reverse sweep to the weights).  FP32 (the workload's precision) and FP64."""
    import torch
    from paper_2402_17660_amd import TensorNet, build_neighbors, lib
    from synth import make_config, make_weights, write_blob
    c = make_config(4)
    N, S = len(c["pos"]), c["n_systems"]
    pos32 = torch.tensor(c["pos"], device=dev)
    z = torch.tensor(c["z"], device=dev)
    batch = torch.tensor(c["batch"], device=dev)
    _, n_pairs, _ = build_neighbors(pos32, batch, c["r_c"], 64 * N)
    true_pairs = int(n_pairs.item())
    mp = int(math.ceil(1.05 * true_pairs / 1024.0) * 1024)
    teacher = TensorNet(write_blob(make_weights(c["F"], c["K"], c["L"], c["max_z"], seed=3000), c["F"], c["K"],
                                   c["L"], c["max_z"], c["r_c"]), dev)
    E_t, F_t = teacher.energy_forces(pos32, z, batch, S, max_pairs=mp, precision="fp32", path="fused")
    E_ref, F_ref = E_t.clone(), F_t.double()
    teacher.close()
    student = TensorNet(_blob_for(c), dev)
    out = dict(workload="64 molecules, sizes uniform 16-128 atoms, 0.05 A noise; hidden 128, 3 layers, 32 RBF, "
                        "cutoff 5 A; one training step = loss on energies and forces + exact weight gradient",
               n_atoms=N, n_systems=S, n_pairs=true_pairs, max_pairs=mp, n_params=student.param_count())
    grads = {}
    L_ = lib()
    wflop = train_wgrad_flops(c["F"], c["K"], c["L"], N, true_pairs, c["max_z"])
    for prec in ("fp32", "fp64"):
        pos = pos32 if prec == "fp32" else pos32.double()
        for _ in range(2):
            loss, E, Fo, g = student.train_grad(pos, z, batch, S, E_ref, F_ref, max_pairs=mp, precision=prec)
        torch.cuda.synchronize()
        reps = 10
        L_.tn_timing_reset()
        L_.tn_timing_enable(1)
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(reps):
            student.train_grad(pos, z, batch, S, E_ref, F_ref, max_pairs=mp, precision=prec, check=False,
                               grad_out=g)
        stop.record()
        torch.cuda.synchronize()
        L_.tn_timing_enable(0)
        student.check()
        ms = start.elapsed_time(stop) / reps
        wg_ms, wg_launches = timing(L_, "train_wgrad")
        wg_ms /= reps
        grads[prec] = g.clone()
        achieved = wflop / (wg_ms * 1e-3) / 1e12 if wg_ms > 0 else None
        peak = PEAK[prec] / 1e12
        out[prec] = dict(ms_per_step=ms, atom_steps_per_s=N / (ms * 1e-3), loss=float(loss.item()),
                         grad_norm=float(g.norm().item()),
                         roofline=dict(bound="mfma", kernel="k_wgrad_mfma (parameter adjoints, dual)",
                                       achieved=achieved, peak=peak, unit="TFLOP/s",
                                       frac=achieved / peak if achieved else None, traffic=None,
                                       ms_per_step=wg_ms, launches_per_step=wg_launches / reps,
                                       flop_per_step=wflop))
        log(f"train/{prec}: {ms:.2f} ms per training step ({N / (ms * 1e-3):.3e} atoms/s), loss "
            f"{out[prec]['loss']:.6e}, |grad| {out[prec]['grad_norm']:.6e}; parameter adjoints {wg_ms:.2f} ms "
            f"({achieved:.1f} TFLOP/s of {peak:.1f})")
    d = (grads["fp32"] - grads["fp64"]).abs().max() / grads["fp64"].abs().max()
    out["fp32_vs_fp64_grad_max_rel"] = float(d.item())
    # the inference step on the same inputs, for the training overhead
    for _ in range(2):
        student.energy_forces(pos32, z, batch, S, max_pairs=mp, precision="fp32", path="fused")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        student.energy_forces(pos32, z, batch, S, max_pairs=mp, precision="fp32", path="fused", check=False)
    torch.cuda.synchronize()
    out["energy_forces_fused_fp32_ms"] = (time.perf_counter() - t0) / 10 * 1e3
    student.close()
    if not args.no_cpu_baseline:
        log("timing the oracle's training step on the host ...")
        out["cpu_baseline"] = train_cpu_baseline(c, 20)
    return out


EXTRA = {"batch": extra_batch, "md": extra_md, "table2": extra_table2, "nbr": extra_nbr, "train": extra_train}


if __name__ == "__main__":
    main()
