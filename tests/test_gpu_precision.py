"""The precision statement of the FP32 shifted-population storage: per observable, the largest
relative error of the GPU's FP32 and FP64 runs against the FP64 oracle (same seeds, identical
noise streams, so the comparison is pathwise), printed as one table line per workload and
precision (PRECISION ...) and held to the parity bounds; and the body-frame mean squared
displacements of the 256^3 precision study (Sec. 2.6-2.7, eqs. (dt_body), (dr_body)).

Relative errors, each the maximum over the checked steps:
  mass      |sum rho - oracle| / oracle                        (FP64 sums on both sides)
  momentum  |sum j - oracle| / sum_x |j(x)|                     (the total itself cancels)
  u_inf     max_x |u - oracle| / max_x |u|
  u_l2      ||u - oracle||_2 / ||u||_2
  pops      max |f_i - oracle| / max |f_i - w_i rho0|           (all 19 populations)
  F_b, T_b  max_b |F_b - oracle| / sum_k |F_k|  (torque: sum_k |r_k - R| |F_k|)
  R         max_b |R - oracle| (lattice units: positions are not relative quantities)
  q         max_b |q - oracle| (unit quaternions)
  J         |J - oracle| / mean_n sum_k |F_k|, J = time-averaged drag along x
"""
import json
import math

import numpy as np
import pytest

from oracle import analysis as OA
from paper_1604_01829_amd import workloads as W
from tests.helpers import compare, gpu_from_workload, oracle_from_workload
from tests.test_gpu_parity import pore_case

pytestmark = pytest.mark.gpu


def _cases():
    w1 = W.workload(1)
    w1t = W.workload(1)
    w1t["params"]["kT"] = 4e-5
    pore = pore_case("f64", 4e-5)
    w3 = W.workload(3, scale=0.25)          # 64^3, 16 thermal ellipsoids
    batch = W.workload(4, scale=4 / 512)    # 4 pore replicas of the batch
    return [("sphere 32^3, deterministic, 500 steps", w1, 0, (1, 10, 100, 500)),
            ("sphere 32^3, thermal, 500 steps", w1t, 0, (1, 10, 100, 500)),
            ("pore 24x22x40, 2 spheres, thermal, 100 steps", pore, 0, (1, 10, 100)),
            ("64^3, 16 ellipsoids, thermal, 50 steps", w3, 0, (1, 10, 50)),
            ("batch replica (pore, ellipsoid), thermal, 50 steps", batch, 0, (1, 10, 50))]


def _errors(wl, r, checks, precision):
    gpu = gpu_from_workload(wl, precision=precision)
    gpu.set_graph_steps(0)
    orc = oracle_from_workload(wl, r)
    nb = orc.n_bodies
    Jg, Jo, gross_sum = np.zeros(nb), np.zeros(nb), 0.0
    out = dict(mass=0.0, momentum=0.0, u_inf=0.0, u_l2=0.0, pops=0.0, F_b=0.0, T_b=0.0, R=0.0,
               q=0.0)
    drift = 0.0   # the oracle's own FP64 rounding drift of unshifted populations, relative
    steps = checks[-1]
    for n in range(1, steps + 1):
        gpu.step(1)
        orc.step(1)
        _, bg, _, _ = gpu.observables(r)
        gross = 0.0
        for b in range(nb):
            Jg[b] += bg[b]["force"][0]
            Jo[b] += orc.body_state(b)["force"][0]
            gross = max(gross, float(np.linalg.norm(orc.bead_forces(b), axis=1).sum()))
        gross_sum += gross
        if n not in checks:
            continue
        e = compare(gpu, orc, r)
        fg, fo = gpu.fields(r), orc.fields()
        fl = fo[..., 0] != 0.0
        du = fg[..., 1:][fl] - fo[..., 1:][fl]
        out["mass"] = max(out["mass"], e["mass"])
        out["momentum"] = max(out["momentum"], e["momentum"] / e["momentum_scale"])
        out["u_inf"] = max(out["u_inf"], e["u_abs"] / e["u_scale"])
        out["u_l2"] = max(out["u_l2"], float(np.linalg.norm(du) / np.linalg.norm(fo[..., 1:][fl])))
        out["pops"] = max(out["pops"], e["pop_abs"] / e["pop_scale"])
        drift = max(drift, n * 2.0 ** -49 * e["pop_max"] / e["pop_scale"])
        if nb:
            out["F_b"] = max(out["F_b"], e["body_force"] / e["scale_force"])
            out["T_b"] = max(out["T_b"], e["body_torque"] / e["scale_torque"])
            out["R"] = max(out["R"], e["body_pos"])
            out["q"] = max(out["q"], e["body_quat"])
    if nb:
        out["J"] = float(np.abs(Jg - Jo).max() / steps / (gross_sum / steps))
    gpu.close()
    return out, drift


@pytest.mark.parametrize("case", range(5))
def test_precision_statement(case):
    name, wl, r, checks = _cases()[case]
    # FP32: the parity bounds; a body that moves with the fluid has a net force far below its
    # gross bead force, and that force's error follows the fluid-velocity error (see the
    # parity tests), hence 1e-4 for F_b, T_b and J.  FP64: 1e-11 per 100 steps (the oracle's
    # own rounding of unshifted populations grows with the steps; for the populations, against
    # their shifted scale, that drift is step * 2^-49 * max|f| as in the parity tests).
    bound32 = dict(mass=1e-6, momentum=1e-5, u_inf=1e-5, u_l2=1e-5, pops=1e-5, F_b=1e-4,
                   T_b=1e-4, R=2e-5, q=1e-6, J=1e-4)
    for precision in ("f64", "f32"):
        e, drift = _errors(wl, r, checks, precision)
        print("PRECISION " + json.dumps({"case": name, "precision": precision,
                                         **{k: float(f"{v:.3g}") for k, v in e.items()}}),
              flush=True)
        for k, v in e.items():
            bound = bound32[k] if precision == "f32" else 1e-11 * max(1, checks[-1] / 100)
            if precision == "f64" and k == "pops":
                bound += drift
            assert v <= bound, (precision, k, v, bound)


def test_ellipsoids_256_body_frame_msds():
    """Over the 5000 steps of the 256^3 workload, poses every 10 steps: the FP32 run's
    body-frame translational and rotational MSDs (the library's lb_traj_body_frame and
    lb_traj_msd) against the FP64 run's, and the library's analysis of the FP64 trajectory
    against oracle/analysis.py on the same trajectory.  Then a short window against the
    oracle itself: 8 steps of the oracle box, poses every step, the body-frame series and
    their MSDs computed by oracle/analysis.py from the oracle's trajectory against the
    library's from its FP32 and FP64 runs."""
    import torch
    from paper_1604_01829_amd import analysis as AN
    wl = W.workload(3)
    T, every, lags = wl["steps"], 10, 100
    traj, msd = {}, {}
    for p in ("f64", "f32"):
        sim = gpu_from_workload(wl, precision=p)
        traj[p] = AN.record(sim, T // every, every)
        bf = AN.body_frame(traj[p])
        msd[p] = AN.msd(bf, lags).cpu().numpy()            # [body, lag, 6]
        sim.close()
        print(f"  {p}: {T} steps recorded", flush=True)
    m64, m32 = msd["f64"], msd["f32"]
    rel_t = float(np.abs(m32[..., :3] - m64[..., :3]).max() / np.abs(m64[..., :3]).max())
    rel_r = float(np.abs(m32[..., 3:] - m64[..., 3:]).max() / np.abs(m64[..., 3:]).max())
    print(f"  body-frame MSD FP32 vs FP64: translation {rel_t:.3g}, rotation {rel_r:.3g} "
          f"(largest translational MSD {np.abs(m64[..., :3]).max():.3g})", flush=True)
    assert rel_t <= 1e-4 and rel_r <= 1e-4
    # the library's analysis against the oracle's on the FP64 trajectory
    tr = traj["f64"].cpu().numpy()
    series = np.concatenate([OA.body_frame_translation(tr), OA.body_frame_rotation(tr)], axis=-1)
    want = OA.msd(series, lags)
    assert np.abs(m64 - want).max() <= 1e-10 * np.abs(want).max()
    del traj
    torch.cuda.empty_cache()
    # a short window against the oracle box itself
    n = 8
    orc = oracle_from_workload(wl)
    nb = orc.n_bodies
    otr = np.zeros((n + 1, nb, 7))
    for b in range(nb):
        s = orc.body_state(b)
        otr[0, b] = np.concatenate([s["pos"], s["quat"]])
    for k in range(1, n + 1):
        orc.step(1)
        for b in range(nb):
            s = orc.body_state(b)
            otr[k, b] = np.concatenate([s["pos"], s["quat"]])
        print(f"  oracle step {k}", flush=True)
    oseries = np.concatenate([OA.body_frame_translation(otr), OA.body_frame_rotation(otr)],
                             axis=-1)
    omsd = OA.msd(oseries, 4)
    for p, tol in (("f64", 1e-9), ("f32", 1e-3)):
        sim = gpu_from_workload(wl, precision=p)
        t0 = torch.empty((n + 1, nb, 7), dtype=torch.float64, device="cuda:0")
        from paper_1604_01829_amd import lbrb
        lbrb.library().rb_record_poses(sim.ctx, lbrb._VP(t0[0].data_ptr()))
        AN.record(sim, n, 1, traj=t0[1:])
        g = AN.msd(AN.body_frame(t0.contiguous()), 4).cpu().numpy()
        sim.close()
        err = float(np.abs(g - omsd).max() / np.abs(omsd).max())
        print(f"  short window, {p} vs oracle: body-frame MSD rel {err:.3g}", flush=True)
        assert err <= tol
