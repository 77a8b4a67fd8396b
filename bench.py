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
few leading workgroups finish the bodies): algorithmic bytes 152 B (FP32) or 304 B (FP64) per
fluid node (19 populations read + written) divided by its mean duration from HIP events
recorded by the dispatch of each launch on the library's stream, in a separate eager window of the same
run.  `cpu_baseline` times the FP64 CPU oracle on a few steps of the same box.

`compare` (default workload only) measures, on the same GPU in the same process:
  fp64            the same workload with FP64 populations;
  batched_fp32    512 uneven pore replicas (sides 32-64, one ellipsoid each, thermal) in one
                  batch, 100-step graph replays, with its node_step roofline;
  plain_fp64      a sample of those replicas run one context at a time in FP64;
  box256_fp32/64  the 256^3 periodic box with 16 ellipsoids (larger than the on-package
                  cache, so its node_step bandwidth is HBM bandwidth);
  adjoint         64^3 box, fixed sphere of 401 beads, 200-step window with checkpoints every
                  20 steps: the reverse pass (forward + recompute + reverse) against 200
                  forward steps; and the same window with every state kept (no recompute).
"""
import argparse
import hashlib
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0
ROOT = os.path.dirname(os.path.abspath(__file__))
WORKLOAD_TAGS = {2: "pore128x128x256", 3: "box256", 4: "batch512"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"])
    ap.add_argument("--workload", type=int, default=2, choices=[2, 3, 4],
                    help="2 = pore with 32 spheres (default), 3 = 256^3 box with 16 "
                         "ellipsoids, 4 = 512 pore replicas")
    ap.add_argument("--timing-steps", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--graph-steps", type=int, default=100,
                    help="steps per HIP-graph replay (0 = eager launches, for profilers)")
    ap.add_argument("--step-policy", default="auto", choices=["auto", "serial", "overlap"],
                    help="how the main workload's fluid step is launched (lb_set_step_policy)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="before the run, copy a buffer of this many MiB three times with a "
                         "plain device copy (reference for hardware byte counters)")
    return ap.parse_args()


def algorithmic_bytes_per_node(precision):
    return 19 * 2 * (4 if precision == "f32" else 8)


def kernel_source_hash():
    """sha256 (first 16 hex) of the sources the step kernels are built from."""
    h = hashlib.sha256()
    for name in ("lbrb_kernels.hip", "lbrb_core.h", "lbrb_device.h", "lbrb_layout.h"):
        h.update(open(os.path.join(ROOT, "paper_1604_01829_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel_tag):
    """HBM bytes per launch measured with rocprofv3 PMC counters (profiles/traffic.json), if
    the record matches the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(kernel_tag)
        if not rec or kernel_source_hash() != rec.get("source_hash"):
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


def measure(sim, steps, warmup, timing_steps, graph_steps, precision, policy=None):
    """Timed graph-replayed steps, then an eager window with per-launch HIP events.  In the
    overlapped step both launches update nodes (the coupling runs inside the first, the body
    finishing inside the second); node_us is then their sum per step and couple_us is 0."""
    import torch
    if policy is not None:
        sim.set_step_policy(policy)
    overlapped = sim.step_overlapped()
    n_nodes = n_fluid = 0
    for r in range(len(sim.shapes)):
        a, b = sim.node_counts(r)
        n_nodes += a
        n_fluid += b
    sim.set_graph_steps(graph_steps)
    sim.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    finite = True
    for r in range(len(sim.shapes)):
        t, _, _, rc = sim.observables(r, check=False)
        finite = finite and bool(t["finite"]) and rc == 0
    sim.set_timing(True)
    sim.step(timing_steps)
    kt = sim.kernel_times()
    sim.set_timing(False)
    if overlapped:
        node_s = kt["node_ms"] / timing_steps / 1e3
        couple_s = 0.0
    else:
        node_s = kt["node_ms"] / max(1, kt["node_launches"]) / 1e3
        couple_s = kt["couple_ms"] / max(1, kt["couple_launches"]) / 1e3
    bpn = algorithmic_bytes_per_node(precision)
    achieved = bpn * n_fluid / node_s / 1e9
    return {"mlups": n_fluid * steps / dt / 1e6, "all_node_mlups": n_nodes * steps / dt / 1e6,
            "ms_per_step": dt / steps * 1e3, "n_fluid": n_fluid, "n_nodes": n_nodes,
            "finite": finite, "node_us": node_s * 1e6, "couple_us": couple_s * 1e6,
            "node_gbs": achieved, "bytes_per_launch": bpn * n_fluid, "overlapped": overlapped}


def compare_runs(args):
    import numpy as np
    import torch
    from paper_1604_01829_amd import lbrb
    from paper_1604_01829_amd import workloads as W

    out = {}
    # same pore workload, FP32, with the overlapped step (coupling alongside the node update
    # of the tiles without spread force; body finishing alongside the remaining tiles)
    wl2 = W.workload(2)
    sim = lbrb.simulation_from_workload(wl2, precision="f32")
    m = measure(sim, 2000, 200, 100, 100, "f32", policy=lbrb.LB_STEP_OVERLAP)
    sim.close()
    out["overlapped_step_fp32"] = {"mlups": round(m["mlups"], 1),
                                   "ms_per_step": round(m["ms_per_step"], 5),
                                   "node_update_us_per_step": round(m["node_us"], 2),
                                   "overlapped": m["overlapped"]}
    # same pore workload, FP64 populations
    wl2 = W.workload(2)
    sim = lbrb.simulation_from_workload(wl2, precision="f64")
    m = measure(sim, 1000, 100, 100, 100, "f64")
    sim.close()
    out["fp64"] = {"mlups": round(m["mlups"], 1), "ms_per_step": round(m["ms_per_step"], 5),
                   "node_step_us": round(m["node_us"], 2),
                   "node_step_frac": round(m["node_gbs"] / HBM_PEAK_GBS, 4),
                   "overlapped": m["overlapped"]}
    # 512 uneven pore replicas in one batch, FP32
    wl4 = W.workload(4)
    sim = lbrb.simulation_from_workload(wl4, precision="f32")
    m = measure(sim, 400, 100, 100, 100, "f32")
    sim.close()
    out["batched_fp32"] = {
        "replicas": len(wl4["replicas"]), "fluid_nodes": m["n_fluid"], "all_nodes": m["n_nodes"],
        "mlups": round(m["mlups"], 1), "all_node_mlups": round(m["all_node_mlups"], 1),
        "ms_per_step": round(m["ms_per_step"], 5), "node_step_us": round(m["node_us"], 2),
        "node_step_frac": round(m["node_gbs"] / HBM_PEAK_GBS, 4),
        "couple_us": round(m["couple_us"], 2), "finite": m["finite"],
        "overlapped": m["overlapped"]}
    del sim
    torch.cuda.empty_cache()
    # the plain path: a sample of the same replicas, one FP64 context at a time
    rng = np.random.default_rng(1)
    sample = sorted(rng.choice(len(wl4["replicas"]), 16, replace=False).tolist())
    upd, tsum = 0, 0.0
    for r in sample:
        sim = lbrb.simulation_from_workload(wl4, precision="f64", replicas=[r])
        sim.set_graph_steps(100)
        sim.step(100)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(200)
        torch.cuda.synchronize()
        tsum += time.perf_counter() - t0
        upd += sim.node_counts(0)[1] * 200
        sim.close()
    out["plain_fp64"] = {"replicas_sampled": len(sample), "mlups": round(upd / tsum / 1e6, 1)}
    out["batched_fp32_over_plain_fp64"] = round(out["batched_fp32"]["mlups"] /
                                                out["plain_fp64"]["mlups"], 2)
    # 256^3 box, 16 ellipsoids: HBM-resident
    wl3 = W.workload(3)
    for prec in ("f32", "f64"):
        sim = lbrb.simulation_from_workload(wl3, precision=prec)
        m = measure(sim, 400, 100, 100, 100, prec)
        sim.close()
        del sim
        torch.cuda.empty_cache()
        out["box256_" + prec] = {"mlups": round(m["mlups"], 1),
                                 "ms_per_step": round(m["ms_per_step"], 5),
                                 "node_step_us": round(m["node_us"], 2),
                                 "node_step_gbs": round(m["node_gbs"], 1),
                                 "node_step_frac": round(m["node_gbs"] / HBM_PEAK_GBS, 4),
                                 "overlapped": m["overlapped"],
                                 "traffic": traffic_from_profiles(f"node_step_{prec}_box256")}
    # the paper's integration scheme on the same pore: 2 MD steps per fluid step, inner
    # excluded-volume layers on the spheres and WCA pore beads (eps = kT)
    wlm = W.confined_md_workload(substeps=2)
    sim = lbrb.simulation_from_workload(wlm, precision="f32")
    m = measure(sim, 1000, 100, 100, 100, "f32")
    sim.close()
    out["confined_md_fp32"] = {
        "md_steps_per_fluid_step": 2,
        "pore_sites": int(wlm["replicas"][0]["wall_sites"][0].shape[0]),
        "ev_sites": int(sum(b["ev"][0].shape[0] for b in wlm["replicas"][0]["bodies"])),
        "mlups": round(m["mlups"], 1), "ms_per_step": round(m["ms_per_step"], 5),
        "node_step_us": round(m["node_us"], 2), "couple_us": round(m["couple_us"], 2),
        "finite": m["finite"]}
    # raspberry construction: the paper's 15 ellipsoids of revolution (volume of a radius-4.25
    # sphere, aspect ratios 1/10 .. 10), outer and inner shells relaxed together, 20,000 steps
    from paper_1604_01829_amd import construction as CN
    phis = [1 / 10, 1 / 5, 1 / 4, 1 / 3, 1 / 2, 2 / 3, 4 / 5, 9 / 10, 10 / 9, 5 / 4, 3 / 2, 2, 4, 5, 10]
    axes, init = [], []
    for k, phi in enumerate(phis):
        bb = (4.25 ** 3 / phi) ** (1 / 3)
        for d in (0.0, 0.5):
            ax = (phi * bb - d, bb - d, bb - d)
            axes.append(ax)
            init.append(CN.separated_shell(*ax, CN.shell_count(*ax), seed=k))
    CN.relax_shells(axes, init, n_steps=10)              # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    CN.relax_shells(axes, init, n_steps=20000)
    torch.cuda.synchronize()
    t_c = time.perf_counter() - t0
    out["construction"] = {"shells": len(axes), "beads": int(sum(len(p) for p in init)),
                           "steps": 20000, "seconds": round(t_c, 3),
                           "us_per_step": round(t_c / 20000 * 1e6, 2)}
    # trajectory analysis: 32 bodies, 20,000 frames (seeded synthetic poses around the pore
    # axis), 1000 lags of every MSD
    from paper_1604_01829_amd import analysis as AN
    F, NB, LAGS = 20000, 32, 1000
    traj = torch.as_tensor(W.synthetic_trajectory(F, NB, seed=5, centre=(64.0, 64.0),
                                                  radius=(2.0, 30.0)), device="cuda:0").contiguous()
    ref = np.tile([1.0, 0.0, 0.0], (NB, 1))
    edges = np.linspace(0.0, 32.0, 9)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, (time.perf_counter() - t0) * 1e3

    lab, t_lab = timed(lambda: AN.lab_frame(traj))
    _, t_msd3 = timed(lambda: AN.msd(lab, LAGS))
    bod, t_body = timed(lambda: AN.body_frame(traj))
    _, t_msd6 = timed(lambda: AN.msd(bod, LAGS))
    _, t_rot = timed(lambda: AN.rotation_msd(traj, ref, LAGS))
    (pf, rad), t_pore = timed(lambda: AN.pore_frame(traj, (64.0, 64.0)))
    _, t_bin = timed(lambda: AN.binned_msd(pf, rad, edges, LAGS))
    terms = NB * sum(F - k for k in range(1, LAGS + 1))      # (origin, lag) pairs per body set
    out["analysis"] = {"bodies": NB, "frames": F, "lags": LAGS,
                       "lab_frame_ms": round(t_lab, 3), "msd_lab_ms": round(t_msd3, 3),
                       "body_frame_ms": round(t_body, 3), "msd_body_ms": round(t_msd6, 3),
                       "rotation_msd_ms": round(t_rot, 3), "pore_frame_ms": round(t_pore, 3),
                       "binned_msd_ms": round(t_bin, 3),
                       "msd_lab_gterms_per_s": round(terms * 3 / (t_msd3 * 1e-3) / 1e9, 1)}
    del traj, lab, bod, pf, rad
    torch.cuda.empty_cache()
    # reverse pass on the fixed sphere in uniform flow
    wl5 = W.workload(5)
    wl5["params"]["kT"] = 0.0
    T, K = 200, 20
    a = np.zeros((T, 1, 3))
    a[:, 0, 0] = 1.0 / T
    sim = lbrb.simulation_from_workload(wl5, precision="f32")
    sim.set_graph_steps(100)
    sim.step(200)
    sim.adjoint(T, a, K)                    # warm-up of the reverse pass
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(T)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    sim.adjoint(T, a, K)
    t_adj = time.perf_counter() - t0
    sim.adjoint(T, a, 1)                    # every state kept: no recompute
    t0 = time.perf_counter()
    sim.adjoint(T, a, 1)
    t_all = time.perf_counter() - t0
    sim.close()
    out["adjoint"] = {"window_steps": T, "checkpoint_every": K, "forward_ms": round(t_fwd * 1e3, 3),
                      "adjoint_ms": round(t_adj * 1e3, 3), "ratio": round(t_adj / t_fwd, 2),
                      "all_states_kept_ms": round(t_all * 1e3, 3),
                      "all_states_kept_ratio": round(t_all / t_fwd, 2)}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1"}))
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
    wl = W.workload(args.workload)
    sim = lbrb.simulation_from_workload(wl, precision=args.precision)
    n_beads = sum(b["offsets"].shape[0] for r in wl["replicas"] for b in r["bodies"])
    n_bodies = sum(len(r["bodies"]) for r in wl["replicas"])
    policy = {"auto": lbrb.LB_STEP_AUTO, "serial": lbrb.LB_STEP_SERIAL,
              "overlap": lbrb.LB_STEP_OVERLAP}[args.step_policy]
    m = measure(sim, args.steps, args.warmup, args.timing_steps, args.graph_steps, args.precision,
                policy=policy)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    tag = f"node_step_{args.precision}_{WORKLOAD_TAGS[args.workload]}"
    names = {2: "pore 128x128x256 (radius 40, 1,286,144 fluid nodes), 32 raspberry spheres "
                "R~U[2,6], thermal kT=4e-5",
             3: "256^3 periodic box, 16 raspberry ellipsoids, thermal kT=4e-5",
             4: "512 uneven pore replicas (sides 32-64, pore radius 0.4 side), one ellipsoid "
                "each, thermal kT=4e-5"}
    out = {
        "metric": "MLUPS (D3Q19 LB + raspberry coupling) and % HBM roofline",
        "value": round(m["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(m["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": names[args.workload] + (", FP32 shifted populations"
                                                       if args.precision == "f32"
                                                       else ", FP64 populations"),
                   "fluid_nodes": m["n_fluid"], "all_nodes": m["n_nodes"],
                   "all_node_mlups": round(m["all_node_mlups"], 1), "beads": n_beads,
                   "bodies": n_bodies, "graph_steps": args.graph_steps,
                   "finite_after_run": m["finite"]},
        "roofline": {"bound": "hbm", "achieved": round(m["node_gbs"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(m["node_gbs"] / HBM_PEAK_GBS, 4),
                     "traffic": traffic_from_profiles(tag),
                     "kernel": ("node update of the overlapped step (overlap_free + "
                                "overlap_forced, per step)" if m["overlapped"] else "node_step"),
                     "algorithmic_bytes_per_launch": m["bytes_per_launch"],
                     "mean_launch_us": round(m["node_us"], 3),
                     "couple_mean_launch_us": round(m["couple_us"], 3)},
    }
    if args.workload == 2 and not args.no_compare:
        out["compare"] = compare_runs(args)
    if not args.no_cpu_baseline and args.workload == 2:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
