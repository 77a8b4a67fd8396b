#!/usr/bin/env python3
"""Throughput of the fused lattice-Boltzmann + raspberry-coupling step on one MI355X.

Default workload: a batch of 512 independent replica boxes of uneven size (cubic sides drawn
from {32, 40, 48, 56, 64}; about 66M nodes, 33M of them fluid), each holding a cylindrical
pore of radius 0.4 side along z and one raspberry ellipsoid (prolate, aspect ratio 1-4,
equal-volume radius 0.1 side, about 400 beads), thermal fluid (kT = 4e-5) with independent
counter-based noise per replica, bead friction gamma = 1/6 (the paper's low bead friction in
lattice units), FP32 populations stored shifted by w_i rho0, all replicas in one flat tile
list, HIP-graph replays of 100 steps.  One step = body half kick/drift, bead coupling + force
spreading, body force/torque sums and second half kick, fused collide-and-stream of every
fluid node.  Inputs are synthetic and resident in HBM before timing.

Prints one JSON line.  `value` = fluid-node updates per second / 1e6 (MLUPS) over the timed
steps.  `roofline` is for the dominant kernel, node_step (the update of every fluid node; its
leading workgroups finish the bodies): algorithmic bytes 152 B (FP32) or 304 B (FP64) per
fluid node (19 populations read + written) divided by its mean duration from HIP events
recorded by the dispatch of each launch on the library's stream, in a separate eager window
of the same run; `step_frac` is the same bytes over the whole timed step (coupling, body
finishing, node update and the gaps between launches).  `cpu_baseline` times the FP64 CPU
oracle on 16 sampled replicas of the same batch: a 50-step window on every host thread, and a
shorter window on one thread.

`compare` (unless --no-compare) measures, on the same GPU in the same process:
  batched_fp64    the same 512 replicas in one batch with FP64 populations (precision alone);
  batched_fp32_pore_along_x   the batch with every pore turned along x (the library stores
                  either orientation in rows along the pore axis);
  plain_fp64      16 sampled replicas run one FP64 context at a time (neither batching nor
                  the FP32 storage);
  pore128_f32/64  one 128x128x256 box holding a radius-40 pore with 32 spheres (its population
                  buffers fit in the 256 MB on-package cache, so node_step bandwidth there is
                  partly cache bandwidth);
  box256_f32/64   the 256^3 periodic box with 16 ellipsoids (HBM-resident);
  confined_md     the paper's integration scheme on the pore: 2 MD steps per fluid step, WCA;
  construction, analysis, adjoint   raspberry relaxation, trajectory analysis, reverse pass.
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
METRIC = "MLUPS (D3Q19 LB + raspberry coupling) and % HBM roofline, batched FP32 vs FP64"
NAMES = {2: "pore 128x128x256 (radius 40, 1,286,144 fluid nodes), 32 raspberry spheres R~U[2,6] "
            "(gamma 1/6), thermal kT=4e-5",
         3: "256^3 periodic box, 16 raspberry ellipsoids (gamma 1/6), thermal kT=4e-5",
         4: "batch of 512 uneven pore replicas (cubic sides from {32,40,48,56,64}, pore radius "
            "0.4 side along z), one raspberry ellipsoid each (aspect 1-4, gamma 1/6), thermal "
            "kT=4e-5, independent Philox seeds, one flat tile list"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"])
    ap.add_argument("--workload", type=int, default=4, choices=[2, 3, 4],
                    help="4 = 512 pore replicas in one batch (default), 2 = one pore with 32 "
                         "spheres, 3 = 256^3 box with 16 ellipsoids")
    ap.add_argument("--timing-steps", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target length of each CPU-baseline leg")
    ap.add_argument("--graph-steps", type=int, default=100,
                    help="steps per HIP-graph replay (0 = eager launches, for profilers)")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the untuned node-update launch settings (no lb_autotune)")
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


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def replica_sample(n_replicas, k=16, seed=1):
    import numpy as np
    rng = np.random.default_rng(seed)
    return sorted(rng.choice(n_replicas, min(k, n_replicas), replace=False).tolist())


def cpu_baseline(wl, seconds):
    """The FP64 oracle on a bounded sample of the same batch: 16 sampled replicas, each built
    as its own oracle box.  Leg 1: every host thread, one sizing step per replica, then a
    window of up to 50 steps per replica sized to about `seconds`.  Leg 2: one thread, a
    window sized the same way from leg 1's rate.  Set-up is not timed."""
    sys.path.insert(0, ROOT)
    import numpy as np
    from oracle import pyoracle as po
    from tests.helpers import oracle_from_workload
    reps = wl["replicas"]
    sample = replica_sample(len(reps))
    fluid = [int((reps[r]["mask"] == 0).sum()) if reps[r]["mask"] is not None
             else int(np.prod(reps[r]["shape"])) for r in sample]
    threads = po.num_threads()

    def window(n_steps):
        upd, dt = 0, 0.0
        for r, nf in zip(sample, fluid):
            orc = oracle_from_workload(wl, r)
            t0 = time.perf_counter()
            orc.step(n_steps)
            dt += time.perf_counter() - t0
            upd += nf * n_steps
            del orc
        return upd / dt / 1e6, dt

    rate1, _ = window(1)                                   # sizing
    k_all = int(max(1, min(50, seconds * rate1 * 1e6 / max(1, sum(fluid)))))
    rate_all, t_all = window(k_all)
    po.set_num_threads(1)
    try:
        k_one = int(max(1, min(50, seconds * rate_all / threads * 1e6 / max(1, sum(fluid)))))
        rate_one, t_one = window(k_one)
    finally:
        po.set_num_threads(threads)
    return {"value": round(rate_all, 3), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{len(sample)} sampled replicas of the same batch ({sum(fluid)} fluid "
                      f"nodes), {k_all} steps each on {threads} threads ({t_all:.1f} s), FP64",
            "single_thread": {"value": round(rate_one, 3), "unit": "MLUPS", "cores": 1,
                              "sample": f"the same replicas, {k_one} steps each ({t_one:.1f} s)"},
            "cpu_model": cpu_model()}


def measure(sim, steps, warmup, timing_steps, graph_steps, precision):
    """Timed graph-replayed steps, then an eager window with per-launch HIP events."""
    import torch
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
    # per step: every node-update launch of the step (one per tile group)
    node_s = kt["node_ms"] / timing_steps / 1e3
    couple_s = kt["couple_ms"] / timing_steps / 1e3
    bpn = algorithmic_bytes_per_node(precision)
    achieved = bpn * n_fluid / node_s / 1e9
    step_s = dt / steps
    return {"mlups": n_fluid * steps / dt / 1e6, "all_node_mlups": n_nodes * steps / dt / 1e6,
            "ms_per_step": step_s * 1e3, "n_fluid": n_fluid, "n_nodes": n_nodes,
            "finite": finite, "node_us": node_s * 1e6, "couple_us": couple_s * 1e6,
            "node_gbs": achieved, "step_gbs": bpn * n_fluid / step_s / 1e9,
            "bytes_per_launch": bpn * n_fluid,
            "node_launches_per_step": kt["node_launches"] / timing_steps}


def _short(m, prec):
    return {"mlups": round(m["mlups"], 1), "ms_per_step": round(m["ms_per_step"], 5),
            "node_step_us": round(m["node_us"], 2),
            "node_step_frac": round(m["node_gbs"] / HBM_PEAK_GBS, 4),
            "step_frac": round(m["step_gbs"] / HBM_PEAK_GBS, 4),
            "couple_us": round(m["couple_us"], 2), "finite": m["finite"]}


def compare_runs(args, wl4):
    import numpy as np
    import torch
    from paper_1604_01829_amd import lbrb
    from paper_1604_01829_amd import workloads as W

    out = {}
    # the same batch with the untuned launch settings
    sim = lbrb.simulation_from_workload(wl4, precision="f32")
    m = measure(sim, 400, 100, 50, 100, "f32")
    sim.close()
    del sim
    torch.cuda.empty_cache()
    out["batched_fp32_untuned"] = _short(m, "f32")
    # the same batch with each replica's pore turned along x: the library stores both
    # orientations in rows along the pore axis (lb_row_axis), so the two should agree
    wlx = dict(wl4, replicas=[
        dict(r, mask=np.ascontiguousarray(np.transpose(r["mask"], (2, 1, 0))),
             bodies=[dict(b, pos=np.asarray(b["pos"])[[2, 1, 0]]) for b in r["bodies"]])
        for r in wl4["replicas"]])
    sim = lbrb.simulation_from_workload(wlx, precision="f32")
    sim.autotune()
    m = measure(sim, 400, 100, 50, 100, "f32")
    sim.close()
    del sim
    torch.cuda.empty_cache()
    out["batched_fp32_pore_along_x"] = _short(m, "f32")
    # the same 512 replicas in one batch, FP64 populations: precision alone
    sim = lbrb.simulation_from_workload(wl4, precision="f64")
    sim.autotune()
    m = measure(sim, 200, 50, 50, 100, "f64")
    sim.close()
    del sim
    torch.cuda.empty_cache()
    out["batched_fp64"] = _short(m, "f64")
    # the plain path: a sample of the same replicas, one FP64 context at a time
    upd, tsum = 0, 0.0
    sample = replica_sample(len(wl4["replicas"]))
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
    # one pore with 32 spheres (buffers inside the on-package cache)
    wl2 = W.workload(2)
    for prec, steps in (("f32", 2000), ("f64", 1000)):
        for tuned in (False, True):
            sim = lbrb.simulation_from_workload(wl2, precision=prec)
            tune = sim.autotune() if tuned else None
            m = measure(sim, steps, 200, 100, 100, prec)
            sim.close()
            key = "pore128_" + prec + ("" if tuned else "_untuned")
            out[key] = _short(m, prec)
            if tuned:
                out[key]["tuned"] = tune
                out[key]["traffic"] = traffic_from_profiles(f"node_step_{prec}_pore128x128x256")
    # 256^3 box, 16 ellipsoids: HBM-resident
    wl3 = W.workload(3)
    for prec, tuned in (("f32", False), ("f32", True), ("f64", True)):
        sim = lbrb.simulation_from_workload(wl3, precision=prec)
        tune = sim.autotune() if tuned else None
        m = measure(sim, 400, 100, 100, 100, prec)
        sim.close()
        del sim
        torch.cuda.empty_cache()
        key = "box256_" + prec + ("" if tuned else "_untuned")
        out[key] = _short(m, prec)
        out[key]["node_step_gbs"] = round(m["node_gbs"], 1)
        if tuned:
            out[key]["tuned"] = tune
            out[key]["traffic"] = traffic_from_profiles(f"node_step_{prec}_box256")
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
        res = fn()
        torch.cuda.synchronize()
        return res, (time.perf_counter() - t0) * 1e3

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
    sim.step(T)                             # and of the forward's graphs
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
    # the same sphere released: free, so the reverse pass also runs through the rigid-body
    # integrator (body passes around the bead pass, records rewritten per recomputed step)
    b5 = wl5["replicas"][0]["bodies"][0]
    b5["fixed"] = False
    b5["gamma"] = W.GAMMA_FREE
    b5["omega"] = np.array([0.002, -0.001, 0.0015])
    sim = lbrb.simulation_from_workload(wl5, precision="f32")
    sim.set_graph_steps(100)
    sim.adjoint(T, a, K)                    # warm-up
    sim.step(T)                             # and of the forward's graphs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(T)
    torch.cuda.synchronize()
    t_ffwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    sim.adjoint(T, a, K)
    t_fadj = time.perf_counter() - t0
    sim.close()
    out["adjoint"] = {"window_steps": T, "checkpoint_every": K, "forward_ms": round(t_fwd * 1e3, 3),
                      "adjoint_ms": round(t_adj * 1e3, 3), "ratio": round(t_adj / t_fwd, 2),
                      "all_states_kept_ms": round(t_all * 1e3, 3),
                      "all_states_kept_ratio": round(t_all / t_fwd, 2),
                      "free_body_forward_ms": round(t_ffwd * 1e3, 3),
                      "free_body_adjoint_ms": round(t_fadj * 1e3, 3),
                      "free_body_ratio": round(t_fadj / t_ffwd, 2)}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU: every figure is a one-GPU "
                                   "figure, and --gpus must be 1"}), flush=True)
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
    tune = sim.tuned_settings() if args.no_tune else sim.autotune()
    n_beads = sum(b["offsets"].shape[0] for r in wl["replicas"] for b in r["bodies"])
    n_bodies = sum(len(r["bodies"]) for r in wl["replicas"])
    m = measure(sim, args.steps, args.warmup, args.timing_steps, args.graph_steps, args.precision)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    tag = f"node_step_{args.precision}_{WORKLOAD_TAGS[args.workload]}"
    out = {
        "metric": METRIC,
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
        "config": {"workload": NAMES[args.workload] + (", FP32 shifted populations"
                                                       if args.precision == "f32"
                                                       else ", FP64 populations"),
                   "replicas": len(wl["replicas"]),
                   "fluid_nodes": m["n_fluid"], "all_nodes": m["n_nodes"],
                   "all_node_mlups": round(m["all_node_mlups"], 1), "beads": n_beads,
                   "bodies": n_bodies, "graph_steps": args.graph_steps,
                   "tuned": tune, "finite_after_run": m["finite"]},
        "roofline": {"bound": "hbm", "achieved": round(m["node_gbs"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(m["node_gbs"] / HBM_PEAK_GBS, 4),
                     "traffic": traffic_from_profiles(tag),
                     "kernel": "node_step",
                     "algorithmic_bytes_per_launch": m["bytes_per_launch"],
                     "node_step_us_per_step": round(m["node_us"], 3),
                     "node_launches_per_step": m["node_launches_per_step"],
                     "couple_us_per_step": round(m["couple_us"], 3),
                     "step_achieved": round(m["step_gbs"], 1),
                     "step_frac": round(m["step_gbs"] / HBM_PEAK_GBS, 4)},
    }
    if not args.no_compare and args.workload == 4:
        cmp = compare_runs(args, wl)
        cmp["batched_fp32_over_batched_fp64"] = round(m["mlups"] / cmp["batched_fp64"]["mlups"], 3)
        cmp["batched_fp32_over_plain_fp64"] = round(m["mlups"] / cmp["plain_fp64"]["mlups"], 2)
        cmp["batched_fp64_over_plain_fp64"] = round(cmp["batched_fp64"]["mlups"] /
                                                    cmp["plain_fp64"]["mlups"], 2)
        out["compare"] = cmp
    if not args.no_cpu_baseline and args.workload == 4:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
