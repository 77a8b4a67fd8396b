#!/usr/bin/env python3
"""Throughput of the fused lattice-Boltzmann + raspberry-coupling step on one MI355X.

Default workload: a 128x128x256 box holding a cylindrical pore of radius 40 along z
(1,286,144 fluid nodes), thermal fluid (kT = 4e-5) with counter-based noise, 32 raspberry
spheres of radius 2-6 (about 15k beads), FP32 populations stored shifted by w_i rho0.
One step = body half kick/drift, bead coupling + force spreading, body force/torque sums
and second half kick, fused collide-and-stream of every fluid node.  Inputs are synthetic
and resident in HBM before timing; the steps run as HIP-graph replays.

Prints one JSON line.  `value` = fluid-node updates per second / 1e6 (MLUPS) over the timed
steps.  `roofline` is for the dominant kernel, node_step (the update of every fluid node; its
few leading workgroups finish the bodies): algorithmic bytes 152 B (FP32) per fluid node (19
populations read + written) divided by its mean duration from HIP events recorded around each
launch on the library's stream, in a separate eager window of the same run.  `cpu_baseline` times the FP64 CPU oracle on a few steps of the same box.
"""
import argparse
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0
ROOT = os.path.dirname(os.path.abspath(__file__))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"])
    ap.add_argument("--timing-steps", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--graph-steps", type=int, default=100,
                    help="steps per HIP-graph replay (0 = eager launches, for profilers)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="before the run, copy a buffer of this many MiB three times with a "
                         "plain device copy (reference for hardware byte counters)")
    return ap.parse_args()


def algorithmic_bytes_per_node(precision):
    return 19 * 2 * (4 if precision == "f32" else 8)


def traffic_from_profiles(kernel_tag):
    """HBM bytes per launch measured with rocprofv3 PMC counters (profiles/*.json), if the
    record matches the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(kernel_tag)
        if not rec:
            return None
        import hashlib
        src = open(os.path.join(ROOT, "paper_1604_01829_amd", "csrc", "lbrb_kernels.hip"),
                   "rb").read() + open(os.path.join(ROOT, "paper_1604_01829_amd", "csrc",
                                                    "lbrb_core.h"), "rb").read()
        if hashlib.sha256(src).hexdigest()[:16] != rec.get("source_hash"):
            return None
        return rec.get("bytes_per_launch")
    except Exception:
        return None


def cpu_baseline(wl, seconds):
    """The FP64 oracle on the same box: one step to size the sample, then as many steps as
    fit in about `seconds`."""
    sys.path.insert(0, ROOT)
    from oracle import pyoracle as po
    from tests.helpers import oracle_from_workload
    orc = oracle_from_workload(wl)
    rep = wl["replicas"][0]
    n_fluid = int((rep["mask"] == 0).sum()) if rep["mask"] is not None else \
        rep["shape"][0] * rep["shape"][1] * rep["shape"][2]
    t0 = time.perf_counter()
    orc.step(1)
    t1 = time.perf_counter() - t0
    k = max(1, int(seconds / max(t1, 1e-3)) - 1)
    t0 = time.perf_counter()
    orc.step(k)
    dt = time.perf_counter() - t0
    return {"value": round(n_fluid * k / dt / 1e6, 3), "unit": "MLUPS", "cores": po.num_threads(),
            "kind": "oracle",
            "sample": f"{k} steps (after 1 sizing step) of the same box, FP64, {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    sys.path.insert(0, ROOT)
    import torch
    from paper_1604_01829_amd import lbrb
    from paper_1604_01829_amd import workloads as W

    dev = torch.device("cuda:0")
    if args.copy_calibration_mb > 0:
        n = args.copy_calibration_mb * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize(dev)
        del a, b
    wl = W.workload(2)
    sim = lbrb.simulation_from_workload(wl, precision=args.precision)
    n_nodes, n_fluid = sim.node_counts(0)
    n_beads = sum(b["offsets"].shape[0] for b in wl["replicas"][0]["bodies"])
    sim.set_graph_steps(args.graph_steps)

    sim.step(args.warmup)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize(dev)
    dt = time.perf_counter() - t0
    t, _, _, rc = sim.observables(0, check=False)
    mlups = n_fluid * args.steps / dt / 1e6

    # kernel timing window: eager launches bracketed by HIP events on the library's stream
    sim.set_timing(True)
    sim.step(args.timing_steps)
    kt = sim.kernel_times()
    sim.set_timing(False)
    # node_step: every fluid node's update (its leading workgroups finish the bodies)
    node_s = kt["node_ms"] / max(1, kt["node_launches"]) / 1e3
    # couple: bead coupling and force spreading
    couple_s = kt["couple_ms"] / max(1, kt["couple_launches"]) / 1e3
    bpn = algorithmic_bytes_per_node(args.precision)
    achieved = bpn * n_fluid / node_s / 1e9
    tag = f"node_step_{args.precision}_pore128x128x256"
    traffic = traffic_from_profiles(tag)

    out = {
        "metric": "MLUPS (D3Q19 LB + raspberry coupling) and % HBM roofline",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": "pore 128x128x256 (radius 40, 1,286,144 fluid nodes), 32 raspberry "
                               "spheres R~U[2,6], thermal kT=4e-5, FP32 shifted populations"
                   if args.precision == "f32" else "same pore workload, FP64 populations",
                   "fluid_nodes": n_fluid, "all_nodes": n_nodes, "beads": n_beads,
                   "bodies": len(wl["replicas"][0]["bodies"]), "graph_steps": args.graph_steps,
                   "finite_after_run": bool(t["finite"]) and rc == 0},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": "node_step",
                     "algorithmic_bytes_per_launch": bpn * n_fluid,
                     "mean_launch_us": round(node_s * 1e6, 3),
                     "couple_mean_launch_us": round(couple_s * 1e6, 3)},
    }
    sim.close()
    del sim
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
