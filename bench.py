"""Benchmark: TensorNet energy+forces atom-steps/s on one MI355X.

One step = one full energy-and-forces evaluation (cell-list neighbour search, embedding,
interaction layers, output network, reverse sweep for forces) of the periodic box of
100,000 atoms (100 A cube at 0.1 atoms/A^3; hidden 128, 2 layers, 32 RBF, cutoff 5 A), with
all inputs resident in HBM.  The timed variants are the fused path (FP32, BF16) and the plain
unfused path (FP32); `value` is the fused FP32 path.  Each variant is checked against the FP64
oracle's stored values for this box: the whole box's energy and the exact forces of the atoms
near two centres.

The LAST line on stdout is one compact JSON object (the headline).  The extra workloads (the
48-atom anchor, the 6000-atom box, the 512-molecule batch, 100 velocity-Verlet steps, the
Table 2 sizes, the neighbour-search study, the training step) print one JSON line each on
stderr, and all of them are written to --extra-out when given.
"""

from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "TensorNet energy+forces atom-steps/s, fused vs plain, at stated force error"
PEAK = {"fp32": 157.3e12, "bf16": 2.5e15, "fp64": 78.6e12}   # dense MFMA peaks, FLOP/s
HBM_PEAK = 8.0e12
HEADLINE_CFG = 3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_flops_per_atom_step(F, K, L, p):
    """E+F FLOPs per atom (edge filter once per unordered pair, p = pairs/atom): 2x the forward."""
    fwd = (p * (6 * K * F + L * 2 * (K * F + 2 * F * F + 6 * F * F)) + 2 * p * 20 * F + L * 2 * p * 18 * F
           + 34 * F * F + L * (36 * F * F + 162 * F) + 2 * (3 * F * F + F * F / 2 + F / 2))
    return 2.0 * fwd


def algorithmic_bytes_per_atom_step(F, L, p):
    """HBM bytes per atom-step under ideal reuse (FP32 state): per layer write Y, read Y once, save X,
    read it back, write and read the adjoint; the embedding; the pair list in every pass; I/O."""
    return (6 * L + 2) * 9 * F * 4 + 2 * (L + 1) * 8 * p + 56


def edge_filter_flops_per_pair(F, K):
    return 2.0 * (K * F + 2 * F * F + 6 * F * F)


# timed kernels of each path: {timer name: algorithmic FLOP per unordered pair per launch}
def timed_kernels(path, F, K, L):
    if path == "plain":
        return {"plain_edge_gemm_c": 2.0 * (2 * F) * (3 * F)}
    per_pair = 2.0 * K * 3 * F + L * edge_filter_flops_per_pair(F, K)
    return {"edge_fwd": per_pair, "edge_bwd": per_pair}


KERNEL_NAMES = {"edge_fwd": "k_pair_fwd", "edge_bwd": "k_pair_bwd", "plain_edge_gemm_c": "k_gemm_mfma"}
PAIR_SOURCES = ("tn_pair.hip", "tn_pairtile.h", "tn_mfma.h", "tn_device.h", "tn_internal.h")


def kernel_code_hash():
    """sha256 of the pair kernels' sources with comments and blank space removed, so that a
    comment-only edit keeps a counter summary valid while any code change invalidates it."""
    csrc = os.path.join(ROOT, "paper_2402_17660_amd", "csrc")
    h = hashlib.sha256()
    for name in PAIR_SOURCES:
        text = open(os.path.join(csrc, name)).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def traffic_summary_path(precision):
    return os.path.join(ROOT, "profiles", f"pair_kernels_{precision}_box100k_hbm_counters.md")


def measured_traffic(timer, precision):
    """HBM bytes per launch of a pair kernel from the committed counter summary of this workload,
    or None when there is none or the kernel code changed since the counters were taken."""
    path = traffic_summary_path(precision)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        k, _, v = line.strip().strip("`").partition(": ")
        fields[k.strip()] = v.strip()
    if fields.get("kernel_code_sha256") != kernel_code_hash():
        return None
    v = fields.get(f"{timer}_traffic_bytes")
    return float(v) if v else None


def cpu_baseline(c, weight_seed, n_atoms=3000, reps=2):
    """The FP64 oracle on a bounded sample of the headline workload: periodic boxes of n_atoms drawn
    by the same generator (0.1 atoms/A^3, H/C/N/O, 0.9 A minimum separation) with the headline's
    weights, timed over `reps` energy+forces evaluations."""
    import torch
    from oracle import TensorNetOracle
    from synth import make_weights, periodic_box, write_blob
    box_in = periodic_box(n_atoms, seed=5000 + HEADLINE_CFG)
    o = TensorNetOracle(write_blob(make_weights(c["F"], c["K"], c["L"], c["max_z"], seed=weight_seed),
                                   c["F"], c["K"], c["L"], c["max_z"], c["r_c"]))
    pairs = o.pairs(box_in["pos"], box_in["batch"], box_in["box"])
    t = time.perf_counter()
    for _ in range(reps):
        o.energy_forces(box_in["pos"], box_in["z"], box_in["batch"], box_in["box"], 1, pairs=pairs)
    dt = time.perf_counter() - t
    return dict(value=n_atoms * reps / dt, unit="atom-steps/s", cores=torch.get_num_threads(), kind="oracle",
                sample=f"{reps} FP64 energy+forces evaluations (autograd forces) of a {n_atoms}-atom periodic box "
                       f"drawn like the 100k-atom box (same density, species, model and weights; {len(pairs)} "
                       f"pairs), {dt:.1f} s; the oracle's cost per atom does not depend on the box size; "
                       f"neighbour list excluded")


def timed_run(run, steps, warmup, timers, L_):
    """Warm-up, then `steps` calls between two events on the current stream with the library's kernel
    events enabled (the dominant kernels' launch durations, on their launch stream), then the same
    number of calls without kernel events (their overhead).  Returns (ms/step, ms/step without kernel
    events, {timer: (avg ms per launch, launches per step)})."""
    import torch
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    L_.tn_timing_reset()
    L_.tn_timing_enable(1)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        run()
    stop.record()
    torch.cuda.synchronize()
    L_.tn_timing_enable(0)
    ms = start.elapsed_time(stop) / steps
    kern = {}
    for timer in timers:
        tot, cnt = ctypes.c_double(), ctypes.c_int64()
        L_.tn_timing_read(timer.encode(), ctypes.byref(tot), ctypes.byref(cnt))
        kern[timer] = (tot.value / max(cnt.value, 1), cnt.value / steps)
    L_.tn_timing_reset()
    start.record()
    for _ in range(steps):
        run()
    stop.record()
    torch.cuda.synchronize()
    return ms, start.elapsed_time(stop) / steps, kern


def box_errors(E, Fo, golden_E, golden_F):
    """Errors of the 100k-atom box against the oracle: energy relative to |E| and to sum |eps_i| (the
    per-atom energy magnitudes; the denominator for a near-cancelling sum), relative RMS of the exact
    sampled forces, the largest sampled per-atom force deviation relative to the largest sampled
    force, and the net force per atom relative to the RMS force."""
    import numpy as np
    out = dict(energy_rel=None, energy_rel_sum_abs=None)
    if golden_E is not None:
        e = abs(float(E[0]) - float(golden_E["E"][0]))
        out["energy_rel"] = e / abs(float(golden_E["E"][0]))
        out["energy_rel_sum_abs"] = e / float(golden_E["abs_atom_energy_sum"][0])
    idx, Fs = golden_F["idx"], golden_F["F"]
    d = Fo[idx] - Fs
    out["force_rel_rms"] = float(np.linalg.norm(d) / np.linalg.norm(Fs))
    out["force_max_atom_dev_rel"] = float(np.sqrt((d * d).sum(1)).max() / np.sqrt((Fs * Fs).sum(1)).max())
    out["force_sampled_atoms"] = int(len(idx))
    out["net_force_rel"] = float(np.linalg.norm(Fo.sum(0)) / len(Fo) / np.sqrt((Fo * Fo).sum(1).mean()))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--variants", default="fused:fp32,fused:bf16,plain:fp32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-atoms", type=int, default=3000)
    ap.add_argument("--cpu-reps", type=int, default=2)
    ap.add_argument("--budget", type=float, default=1.05, help="max_pairs = budget * true pair count")
    ap.add_argument("--extra", default="anchor,box6000,batch,md,table2,nbr,train",
                    help="extra workloads: anchor (the 48-atom molecule, FP64 plain and FP32 fused), box6000 "
                         "(the 6000-atom box, all variants), batch (512 molecules, captured), md (100 captured "
                         "velocity-Verlet steps on the 100k-atom box), table2 (the paper's Table 2 sizes and 0/1/2 "
                         "layers, captured), nbr (neighbour-search study on random clouds), train (one training "
                         "step on 64 molecules); 'none' = none")
    ap.add_argument("--extra-out", default=None, help="write the extra workloads' results to this JSON file")
    ap.add_argument("--md-steps", type=int, default=100)
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="after the timed variants, copy this many MiB device-to-device once (a reference "
                         "dispatch of known size for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); this build runs on one GPU, "
              f"run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2402_17660_amd import TensorNet, TensorNetError, lib
    from synth import make_config, make_weights, write_blob

    cfg = HEADLINE_CFG
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
    gdir = os.path.join(ROOT, "tests", "golden")
    golden_F = np.load(os.path.join(gdir, f"oracle_cfg{cfg}_sampled.npz"))
    epath = os.path.join(gdir, f"oracle_cfg{cfg}_energy.npz")
    golden_E = np.load(epath) if os.path.exists(epath) else None
    n_pairs = int(golden_F["n_pairs"])
    max_pairs = int(math.ceil(args.budget * n_pairs / 1024.0) * 1024)
    log(f"workload: N={N} pairs={n_pairs} max_pairs={max_pairs}")
    p_atom = n_pairs / N
    step_flop = algorithmic_flops_per_atom_step(F, K, L, p_atom) * N
    step_bytes = algorithmic_bytes_per_atom_step(F, L, p_atom) * N

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
            if int(model.n_pairs.item()) != n_pairs:
                raise TensorNetError(f"pair count {int(model.n_pairs.item())} != oracle's {n_pairs}")
            # pick the pair-tile shapes for this workload (setup, outside the timed region)
            shapes = (model.autotune(pos, z, batch, 1, box=box, max_pairs=max_pairs, precision=prec, reps=3)
                      if path == "fused" else None)
        except TensorNetError as e:
            log(f"{path}/{prec}: unavailable ({e})")
            results.append(dict(path=path, precision=prec, available=False, error=str(e)))
            continue
        timers = timed_kernels(path, F, K, L)
        ms, ms_plain, kern = timed_run(run, args.steps, args.warmup, timers, L_)
        kernels = []
        for timer, flop_per_pair in timers.items():
            avg_ms, per_step = kern[timer]
            flop_per_launch = flop_per_pair * n_pairs
            achieved = flop_per_launch / (avg_ms * 1e-3) if per_step else None
            kernels.append(dict(name=timer, kernel=KERNEL_NAMES[timer], launches_per_step=per_step, avg_ms=avg_ms,
                                ms_per_step=avg_ms * per_step, flop_per_launch=flop_per_launch,
                                achieved_tflops=(achieved / 1e12) if achieved else None,
                                peak_tflops=PEAK[prec] / 1e12,
                                frac=(achieved / PEAK[prec]) if achieved else None))
        model.check()
        err = box_errors(E_out.cpu().numpy(), F_out.double().cpu().numpy(), golden_E, golden_F)
        dom = max(kernels, key=lambda k: k["ms_per_step"])
        step_tflops = step_flop / (ms * 1e-3) / 1e12
        res = dict(path=path, precision=prec, available=True, ms_per_step=ms, ms_per_step_no_kernel_events=ms_plain,
                   value=N / (ms * 1e-3), errors=err, kernel=dom, kernels=kernels,
                   step=dict(algorithmic_tflop=step_flop / 1e12, tflops=step_tflops,
                             mfma_frac=step_tflops * 1e12 / PEAK[prec],
                             algorithmic_gb=step_bytes / 1e9,
                             hbm_frac=step_bytes / (ms * 1e-3) / HBM_PEAK),
                   pair_tile_shapes=dict(forward=shapes[0], reverse=shapes[1]) if shapes else None)
        log(f"{path}/{prec}: {ms:.3f} ms/step ({ms_plain:.3f} without kernel events), {res['value']:.3e} "
            f"atom-steps/s, step {step_tflops:.1f} TFLOP/s, errors {err}, "
            + (f"tile shapes {shapes}, " if shapes else "")
            + ", ".join(f"{k['name']} {k['avg_ms']:.3f} ms/launch ({k['achieved_tflops'] or 0:.1f} TFLOP/s)"
                        for k in kernels))
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
    model.close()
    del model
    torch.cuda.empty_cache()

    avail = [r for r in results if r.get("available")]
    if not avail:
        raise SystemExit("no variant ran")
    head = next((r for r in avail if r["path"] == "fused" and r["precision"] == "fp32"), None) or avail[0]
    k = head["kernel"]
    roofline = dict(bound="mfma", achieved=k["achieved_tflops"], peak=k["peak_tflops"], unit="TFLOP/s",
                    frac=k["frac"], traffic=measured_traffic(k["name"], head["precision"]),
                    kernel=k["kernel"], avg_launch_ms=k["avg_ms"], flop_per_launch=k["flop_per_launch"],
                    step_mfma_frac=head["step"]["mfma_frac"], step_hbm_frac=head["step"]["hbm_frac"])
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host ...")
        cpu = cpu_baseline(c, c["weight_seed"], args.cpu_atoms, args.cpu_reps)
    extra = {}
    for name in [e for e in args.extra.split(",") if e and e != "none"]:
        try:
            extra[name] = EXTRA[name](args, dev)
        except Exception as e:   # an extra workload never hides the headline line
            log(f"extra workload {name} failed: {e!r}")
            extra[name] = dict(error=repr(e))
        torch.cuda.empty_cache()
    if args.extra_out:
        with open(args.extra_out, "w") as f:
            json.dump(dict(headline_variants=results, extra=extra), f, indent=1)

    def brief(r):
        if not r.get("available"):
            return dict(path=r["path"], precision=r["precision"], available=False)
        e = r["errors"]
        return dict(path=r["path"], precision=r["precision"], ms_per_step=round(r["ms_per_step"], 4),
                    value=r["value"], energy_rel=e["energy_rel"], force_rel_rms=e["force_rel_rms"],
                    force_max_atom_dev_rel=e["force_max_atom_dev_rel"],
                    step_mfma_frac=round(r["step"]["mfma_frac"], 4),
                    kernel=r["kernel"]["kernel"], kernel_frac=r["kernel"]["frac"] and round(r["kernel"]["frac"], 4))

    out = dict(metric=METRIC, value=head["value"], unit="atom-steps/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=head["ms_per_step"], higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="f32" if head["precision"] == "fp32" else head["precision"],
               data="synthetic",
               config=dict(workload="periodic cubic box of 100000 atoms (100 A, 0.1 atoms/A^3, Z in {H,C,N,O}); "
                                    "TensorNet hidden 128, 2 layers, 32 RBF, cutoff 5 A; energy+forces incl. "
                                    "cell-list neighbour search",
                           n_atoms=N, n_pairs=n_pairs, max_pairs=max_pairs, path=head["path"],
                           precision=head["precision"]),
               roofline=roofline, cpu_baseline=cpu, errors=head["errors"],
               variants=[brief(r) for r in results],
               extra_summary={k: summarize(k, v) for k, v in extra.items()})
    print(json.dumps(out), flush=True)


def summarize(name, r):
    """A few key numbers of an extra workload for the headline line."""
    if "error" in r:
        return dict(error=r["error"][:200])
    f = lambda x, n=4: (float(f"{x:.{n}g}") if isinstance(x, (int, float)) and x is not None else x)
    if name == "anchor":
        return [dict(variant=f"{q['path']}/{q['precision']}", us_graph=f(q["us_per_call_graph"]),
                     us_eager=f(q["us_per_call_eager"]), energy_rel=f(q["energy_rel_err"], 2),
                     force_rel_rms=f(q["force_rel_rms"], 2)) for q in r["rows"]]
    if name == "box6000":
        return [dict(variant=f"{q['path']}/{q['precision']}", ms=f(q["ms_per_step"]), value=f(q["value"]),
                     energy_rel=f(q["energy_rel_err"], 2), force_rel_rms=f(q["force_rel_rms"], 2)) for q in r["rows"]]
    if name == "batch":
        return {p: dict(ms=f(r[p]["ms_per_step"]), value=f(r[p]["value"]), energy_rel=f(r[p]["energy_rel_err"], 2),
                        force_rel_rms=f(r[p]["force_rel_rms"], 2))
                for p in ("fp32", "bf16", "molecule_fp32", "molecule_bf16") if p in r}
    if name == "md":
        return {p: dict(ms_per_step=f(r[p]["ms_per_step"]), value=f(r[p]["value"]), status=r[p]["status"],
                        total_energy_max_dev_eV=f(r[p]["total_max_dev"]), min_pair_distance=f(r[p]["min_pair_distance"]),
                        temperature_K=[f(r[p]["temperature_start_K"]), f(r[p]["temperature_end_K"])])
                for p in ("fp32", "bf16") if p in r}
    if name == "table2":
        return {f"{q['atoms']}/{q['layers']}L": f(q["ms_per_step"] * 1e3) for q in r["rows"]}
    if name == "nbr":
        return {f"{q['points']}pts/{q['systems']}sys": [f(q.get("cell_ms")), f(q.get("brute_ms"))]
                for q in r["sweep"] if q["points"] in (1024, 1 << 20)}
    if name == "train":
        return {p: dict(ms=f(r[p]["ms_per_step"]), wgrad_frac=f(r[p]["roofline"]["frac"], 3)) for p in ("fp32", "fp64")
                if p in r}
    return None


def _blob_for(c):
    from synth import make_weights, write_blob
    return write_blob(make_weights(c["F"], c["K"], c["L"], c["max_z"], seed=c["weight_seed"]),
                      c["F"], c["K"], c["L"], c["max_z"], c["r_c"])


def extra_batch(args, dev):
    """512 isolated molecules of 8-64 atoms: one captured graph per evaluation, FP32 vs BF16, with the fused
    path (one launch per operation over the whole batch) and the molecule path (one launch in which a
    workgroup owns each molecule; pair budget 32 per atom)."""
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
    for prec, path in (("fp32", "fused"), ("bf16", "fused"), ("fp32", "molecule"), ("bf16", "molecule")):
        key = prec if path == "fused" else f"molecule_{prec}"
        shapes = None
        if path == "fused":
            shapes = model.autotune(pos, z, batch, c["n_systems"], max_pairs=mp, precision=prec, reps=3)
        g, E, Fo, n_pairs, status = capture(model, pos, z, batch, c["n_systems"],
                                            max_pairs=mp if path == "fused" else 32 * N, precision=prec, path=path)
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
        out[key] = dict(ms_per_step=ms, value=N / (ms * 1e-3), status=int(status.item()), pair_tile_shapes=shapes,
                        energy_rel_err=float(np.max(np.abs(Ev - golden["E"]) / np.abs(golden["E"]))),
                        force_rel_rms=float(np.linalg.norm(Fv - golden["F"]) / np.linalg.norm(golden["F"])))
        log(f"batch/{path}/{prec}: {ms:.3f} ms/step, {out[key]['value']:.3e} atom-steps/s, "
            f"E err {out[key]['energy_rel_err']:.2e}, F err {out[key]['force_rel_rms']:.2e}")
        g.close()
    return out


def extra_md(args, dev):
    """100k-atom periodic box: n captured velocity-Verlet steps (dt 1 fs), neighbours rebuilt every step.
    The timed replay runs all steps in one graph.  A second pass from the same start replays a one-step
    graph n times and records after every step the potential, kinetic and total energy and the minimum
    pair distance; its end state is compared with the timed replay's."""
    import numpy as np
    import torch
    from paper_2402_17660_amd import TensorNet, build_neighbors, capture
    from synth import make_config, maxwell_boltzmann
    from synth.generators import EV_PER_AMU_A2_FS2, masses
    c = make_config(3)
    N = len(c["pos"])
    model = TensorNet(_blob_for(c), dev)
    z = torch.tensor(c["z"], device=dev)
    batch = torch.tensor(c["batch"], device=dev)
    m_amu = masses(c["z"])
    inv_m = torch.tensor((1.0 / m_amu).astype(np.float32), device=dev)
    m_t = torch.tensor(m_amu, device=dev)
    box_len = float(c["box"][0, 0])
    out = dict(workload=f"periodic cubic box of 100000 atoms (100 A), hidden 128, 2 layers, cutoff 5 A; "
                        f"{args.md_steps} velocity-Verlet steps (dt 1 fs) in one HIP graph, neighbour search every "
                        f"step; Maxwell-Boltzmann velocities at 300 K", n_atoms=N, steps=args.md_steps)

    def kinetic(vel):
        return float(0.5 * (m_t[:, None] * vel.double() ** 2).sum() / EV_PER_AMU_A2_FS2)

    def min_distance(p, mp):
        pairs, npair, _ = build_neighbors(p, batch, c["r_c"], mp, box=c["box"])
        k = int(npair.item())
        i, j = pairs[0, :k].long(), pairs[1, :k].long()
        v = p[j].double() - p[i].double()
        v -= box_len * torch.round(v / box_len)
        return float(torch.sqrt((v * v).sum(1)).min())

    for prec in ("fp32", "bf16"):
        pos0 = torch.tensor(c["pos"], device=dev)
        vel0 = torch.tensor(maxwell_boltzmann(c["z"]), device=dev)
        pos, vel = pos0.clone(), vel0.clone()
        E0, F0 = model.energy_forces(pos, z, batch, 1, box=c["box"], max_pairs=32 * N, precision=prec)
        n0 = int(model.n_pairs.item())
        mp = int(math.ceil(1.10 * n0 / 1024.0) * 1024)
        rms_f0 = float(torch.sqrt((F0.double() ** 2).mean()))
        shapes = model.autotune(pos, z, batch, 1, box=c["box"], max_pairs=mp, precision=prec, reps=2)
        F_start = F0.clone()
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
        pos_end, vel_end = pos.clone(), vel.clone()
        g.close()
        del g
        # diagnostics: the same trajectory one step per replay
        pos.copy_(pos0)
        vel.copy_(vel0)
        Fo.copy_(F_start)
        g1, E1, F1, np1, st1 = capture(model, pos, z, batch, 1, box=c["box"], max_pairs=mp, precision=prec,
                                       n_steps=1, vel=vel, inv_mass=inv_m, dt_fs=1.0, forces_out=Fo)
        ke0 = kinetic(vel)
        pe, ke, dmin = [float(E0[0])], [ke0], [min_distance(pos, mp)]
        st_diag = 0
        for _ in range(args.md_steps):
            g1.replay()
            st_diag |= int(st1.item())
            pe.append(float(E1[0]))
            ke.append(kinetic(vel))
            dmin.append(min_distance(pos, mp))
        g1.close()
        tot = [a + b for a, b in zip(pe, ke)]
        same = float((pos - pos_end).abs().max())
        out[prec] = dict(ms_per_replay=ms, ms_per_step=ms / args.md_steps, pair_tile_shapes=shapes,
                         value=N * args.md_steps / (ms * 1e-3), status=st, status_diagnostic_pass=st_diag,
                         initial_pairs=n0, max_pairs=mp, final_pairs=int(n_pairs.item()), initial_rms_force=rms_f0,
                         potential_start=pe[0], potential_end=pe[-1], kinetic_start=ke[0], kinetic_end=ke[-1],
                         total_start=tot[0], total_end=tot[-1],
                         total_max_dev=max(abs(t - tot[0]) for t in tot),
                         temperature_start_K=2.0 * ke[0] / (3.0 * N * 8.617333262e-5),
                         temperature_end_K=2.0 * ke[-1] / (3.0 * N * 8.617333262e-5),
                         min_pair_distance=min(dmin), min_pair_distance_start=dmin[0],
                         pairs_below_0p5A=bool(min(dmin) < 0.5),
                         diagnostic_pass_end_pos_max_diff=same)
        log(f"md/{prec}: {args.md_steps} steps in {ms:.1f} ms ({ms / args.md_steps:.3f} ms/step, "
            f"{out[prec]['value']:.3e} atom-steps/s), status {st}, pairs {n0} -> {int(n_pairs.item())}; "
            f"E_pot {pe[0]:.2f} -> {pe[-1]:.2f}, E_kin {ke[0]:.2f} -> {ke[-1]:.2f}, E_tot {tot[0]:.2f} -> "
            f"{tot[-1]:.2f} eV (max dev {out[prec]['total_max_dev']:.3f}), min pair distance {min(dmin):.4f} A, "
            f"one-step replays end {same:.2e} A from the timed replay")
        del pos, vel, E, Fo, n_pairs, status, E1, F1, np1, st1
    model.close()
    return out


def extra_anchor(args, dev):
    """The correctness anchor: one isolated 48-atom molecule (hidden 64, 2 layers, cutoff 4.5 A).  The plain
    path in FP64, the fused path in FP32 (and BF16) and the molecule path (one launch, a workgroup per
    molecule) in FP32 and BF16, eager calls and one captured graph per call; microseconds per energy+forces
    call, errors against the oracle's stored values."""
    import numpy as np
    import torch
    from paper_2402_17660_amd import TensorNet, capture
    from synth import make_config
    c = make_config(0)
    N = len(c["pos"])
    golden = np.load(os.path.join(ROOT, "tests", "golden", "oracle_cfg0.npz"))
    model = TensorNet(_blob_for(c), dev)
    z = torch.tensor(c["z"], device=dev)
    batch = torch.tensor(c["batch"], device=dev)
    mp = 32 * N
    out = dict(workload="one isolated 48-atom molecule, hidden 64, 2 layers, 32 RBF, cutoff 4.5 A; max_pairs 32 N",
               n_atoms=N, n_pairs=int(golden["n_pairs"]), rows=[])
    for path, prec in (("plain", "fp64"), ("fused", "fp32"), ("fused", "bf16"), ("plain", "fp32"), ("molecule", "fp32"),
                       ("molecule", "bf16")):
        pdt = torch.float64 if prec == "fp64" else torch.float32
        pos = torch.tensor(c["pos"], dtype=pdt, device=dev)
        E_out = torch.empty(1, dtype=torch.float64, device=dev)
        F_out = torch.empty((N, 3), dtype=pdt, device=dev)
        run = lambda: model.energy_forces(pos, z, batch, 1, max_pairs=mp, precision=prec, path=path, check=False,
                                          energy_out=E_out, forces_out=F_out)
        run()
        model.check()
        for _ in range(20):
            run()
        torch.cuda.synchronize()
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 200
        start.record()
        for _ in range(reps):
            run()
        stop.record()
        torch.cuda.synchronize()
        us_eager = start.elapsed_time(stop) / reps * 1e3
        e_err = abs(float(E_out[0]) - float(golden["E"][0])) / abs(float(golden["E"][0]))
        f_err = float(np.linalg.norm(F_out.double().cpu().numpy() - golden["F"]) / np.linalg.norm(golden["F"]))
        g, E, Fo, n_pairs, status = capture(model, pos, z, batch, 1, max_pairs=mp, precision=prec, path=path)
        us_graph = _time_replays(g, reps) * 1e3
        st = int(status.item())
        g_err = abs(float(E[0]) - float(golden["E"][0])) / abs(float(golden["E"][0]))
        g.close()
        row = dict(path=path, precision=prec, us_per_call_eager=us_eager, us_per_call_graph=us_graph,
                   atom_steps_per_s_graph=N / (us_graph * 1e-6), energy_rel_err=e_err, force_rel_rms=f_err,
                   graph_energy_rel_err=g_err, status=st)
        out["rows"].append(row)
        log(f"anchor {path}/{prec}: {us_eager:.1f} us eager, {us_graph:.1f} us per graph replay, E err {e_err:.2e}, "
            f"F err {f_err:.2e}")
    model.close()
    return out


def extra_box6000(args, dev):
    """The 6000-atom periodic box (39.15 A, hidden 128, 2 layers, cutoff 5 A): eager energy+forces calls incl.
    the neighbour search, fused FP32/BF16 and plain FP32, errors against the oracle's stored values."""
    import numpy as np
    import torch
    from paper_2402_17660_amd import TensorNet, lib
    from synth import make_config
    c = make_config(1)
    N = len(c["pos"])
    golden = np.load(os.path.join(ROOT, "tests", "golden", "oracle_cfg1.npz"))
    n_pairs = int(golden["n_pairs"])
    mp = int(math.ceil(1.05 * n_pairs / 1024.0) * 1024)
    model = TensorNet(_blob_for(c), dev)
    pos = torch.tensor(c["pos"], device=dev)
    z = torch.tensor(c["z"], device=dev)
    batch = torch.tensor(c["batch"], device=dev)
    L_ = lib()
    step_flop = algorithmic_flops_per_atom_step(c["F"], c["K"], c["L"], n_pairs / N) * N
    out = dict(workload="periodic cubic box of 6000 atoms (39.15 A), hidden 128, 2 layers, 32 RBF, cutoff 5 A; "
                        "energy+forces incl. cell-list neighbour search", n_atoms=N, n_pairs=n_pairs, max_pairs=mp,
               rows=[])
    for path, prec in (("fused", "fp32"), ("fused", "bf16"), ("plain", "fp32")):
        E_out = torch.empty(1, dtype=torch.float64, device=dev)
        F_out = torch.empty((N, 3), dtype=torch.float32, device=dev)
        run = lambda: model.energy_forces(pos, z, batch, 1, box=c["box"], max_pairs=mp, precision=prec, path=path,
                                          check=False, energy_out=E_out, forces_out=F_out)
        run()
        model.check()
        shapes = model.autotune(pos, z, batch, 1, box=c["box"], max_pairs=mp, precision=prec, reps=5) \
            if path == "fused" else None
        timers = timed_kernels(path, c["F"], c["K"], c["L"])
        ms, ms_plain, kern = timed_run(run, 50, 10, timers, L_)
        model.check()
        Fo = F_out.double().cpu().numpy()
        d = Fo - golden["F"]
        row = dict(path=path, precision=prec, ms_per_step=ms, ms_per_step_no_kernel_events=ms_plain,
                   value=N / (ms * 1e-3), pair_tile_shapes=shapes,
                   energy_rel_err=abs(float(E_out[0]) - float(golden["E"][0])) / abs(float(golden["E"][0])),
                   force_rel_rms=float(np.linalg.norm(d) / np.linalg.norm(golden["F"])),
                   force_max_atom_dev_rel=float(np.sqrt((d * d).sum(1)).max()
                                                / np.sqrt((golden["F"] ** 2).sum(1)).max()),
                   step_mfma_frac=step_flop / (ms * 1e-3) / PEAK[prec],
                   kernels={t: dict(avg_ms=a, launches_per_step=n,
                                    frac=(timers[t] * n_pairs / (a * 1e-3) / PEAK[prec]) if n else None)
                            for t, (a, n) in kern.items()})
        out["rows"].append(row)
        log(f"box6000 {path}/{prec}: {ms:.3f} ms/step, {row['value']:.3e} atom-steps/s, E err "
            f"{row['energy_rel_err']:.2e}, F err {row['force_rel_rms']:.2e}")
    model.close()
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
            model.close()
    log("table2 us/step (0L/1L/2L): " + "; ".join(
        f"{n}: " + "/".join(f"{r['ms_per_step'] * 1e3:.0f}" for r in rows if r["atoms"] == n) for _, n, _ in TABLE2))
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
        return r

    sweep = [row(1 << k, nb, 9000 + 100 * nb + k) for nb in (1, 2, 64) for k in range(8, 21) if (1 << k) >= 4 * nb]
    split = [row(32768, 1 << b, 9500 + b) for b in range(0, 11)]
    log("nbr 1M points cell list: " + ", ".join(f"{r['systems']} systems {r['cell_ms']:.2f} ms" for r in sweep
                                                 if r["points"] == 1 << 20))
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
    inputs) on dual numbers: per weight entry and row, the two tangent products the loss gradient needs
    (4 FLOP); the value part is not formed."""
    pair = n_pairs * (L * (F * K + 2 * F * F + 6 * F * F) + 3 * F * K)
    node = n_atoms * ((1 + 2 * L) * 9 * F * F + 2 * F * F + 6 * F * F + 3 * F * F + (F // 2) * F)
    species = 2 * max_z * F * F
    return 4.0 * (pair + node + species)


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


EXTRA = {"anchor": extra_anchor, "box6000": extra_box6000, "batch": extra_batch, "md": extra_md, "table2": extra_table2, "nbr": extra_nbr, "train": extra_train}


if __name__ == "__main__":
    main()
