"""GPU library vs the FP64 oracle, element by element, through the C-ABI.

Tolerances (derivation in the design notes):
- FP64 populations: the GPU stores f - w rho0 and sums in another order, and spreads bead
  forces as 2^-56 fixed point; errors stay at round-off, ~1e-15 per step relative to the
  field scale, so 1e-12 of the scale is allowed over <= 100 steps.  The oracle stores the
  unshifted populations (|f| <= rho0/3 at rest), so its own rounding is ~2^-53 of |f| per
  operation and accumulates with the steps (measured ~2.7e-16 per step on rho at rho0 = 1,
  the same sign every step): density, mass and populations are also allowed
  step * 2^-49 * max|f| (2^-49 rho0 per step for density), 6x the measured drift.
- FP32 shifted populations: one FP32 rounding of the shifted populations per step (~6e-8
  relative to |f - w rho0| ~ |u|) accumulates over the run; the workload target is 1e-5 of
  the field scale for velocities and 1e-5 relative for density.
- all 19 populations are compared at every checked step, against the population scale
  max |f_i - w_i rho0| (FP32 stores exactly these shifted values), with the velocity
  tolerance; so every moment, the ghost moments included, is checked.
- body velocity: tol * |V| plus tol / 100 times the gross bead force integrated over the run,
  step * sum_k |F_k| / M.  The coupling takes the fluid velocity from the rounded
  populations, so each step's bead forces carry an error of about gamma * 6e-8 |u| per bead
  (FP32), far below 1e-7 of |F_k|, whose thermal part is identical on both sides; V sums
  those errors over the steps.  Angular velocity: tol times the larger of |omega| and the
  integrated gross torque, step * sum_k |r_k - R| |F_k| / I_min (the net omega of a symmetric
  body is itself a cancelling sum: 3.6e-8 for the sphere of workload 1 after 40 steps).
- body position: the position tolerance plus step times the velocity bound (R integrates V).
- body force and torque: tol times the gross bead sums, plus what the measured errors of the
  fluid velocity and of the body's velocities propagate to through the friction,
  gamma sum_k (|du| + |dV| + |r_k - R| |dw|) (and |r_k - R| times that for the torque).  A body
  that moves with the fluid has a net force far below its gross bead force (workload 1
  without noise, 500 steps: 1.1e-3 gross), so this second term is the one that scales there.
"""
import numpy as np
import pytest

from paper_1604_01829_amd import workloads as W
from tests.helpers import compare, gpu_from_workload, oracle_from_workload

pytestmark = pytest.mark.gpu


def _print(tag, e):
    keys = ["rho", "u_abs", "u_scale", "pop_abs", "pop_scale", "mass", "momentum",
            "momentum_scale", "body_pos", "body_quat", "body_vel", "scale_vel", "scale_vel_int",
            "body_omega", "scale_omega", "body_force", "scale_force", "body_torque",
            "scale_torque"]
    print(tag, " ".join(f"{k}={e[k]:.3g}" for k in keys if k in e), flush=True)
    if "mode_abs" in e:
        print("   moment errors", " ".join(f"{v:.2g}" for v in e["mode_abs"]), flush=True)


ORACLE_ROUNDING_PER_STEP = 2.0 ** -49   # of max|f| (of rho0 for density): see above


def _assert_close(e, tol_rel_u, tol_rho, tol_body):
    steps = e.get("step", 0)
    drift = steps * ORACLE_ROUNDING_PER_STEP
    assert e["rc"] == 0
    assert e["solid_zero"]
    assert e["finite"]
    assert e["rho"] <= max(tol_rho, drift), "rho"
    assert e["u_abs"] <= tol_rel_u * max(e["u_scale"], 1e-12)
    if "pop_abs" in e:
        assert e["pop_solid_zero"]
        assert e["pop_abs"] <= (tol_rel_u * max(e["pop_scale"], 1e-12)
                                + drift * e["pop_max"]), "populations"
    assert e["mass"] <= max(tol_rho, drift), "mass"
    assert e["momentum"] <= tol_rel_u * e["momentum_scale"] + 1e-15
    vel_bound = (tol_rel_u * e["scale_vel"] + 1e-2 * tol_rel_u * e["scale_vel_int"] + 1e-15)
    assert e["body_vel"] <= vel_bound, "vel"
    assert e["body_pos"] <= tol_body + steps * vel_bound, "pos"
    assert e["body_quat"] <= tol_body, "quat"
    assert e["body_omega"] <= tol_rel_u * max(e["scale_omega"], 1e-14) + 1e-15, "omega"
    for k in ("force", "torque"):
        assert e["body_" + k] <= (tol_rel_u * max(e["scale_" + k], 1e-14)
                                  + e.get("scale_" + k + "_prop", 0.0) + 1e-15), k


def small_sphere_case(precision, kT=0.0, steps=(1, 2, 7, 40, 500)):
    wl = W.workload(1)
    wl["params"]["kT"] = kT
    wl["precision"] = precision
    return wl, steps


@pytest.mark.parametrize("kT", [0.0, 4e-5])
def test_sphere_box_f64(kT):
    wl, steps = small_sphere_case("f64", kT)
    gpu = gpu_from_workload(wl)
    gpu.set_graph_steps(0)
    orc = oracle_from_workload(wl)
    done = 0
    for s in steps:
        gpu.step(s - done)
        orc.step(s - done)
        done = s
        e = compare(gpu, orc)
        _print(f"f64 kT={kT} step {s}", e)
        _assert_close(e, 1e-11, 1e-13, 1e-12)
    fb_g = gpu.bead_forces(0, 0)
    fb_o = orc.bead_forces(0)
    assert np.abs(fb_g - fb_o).max() <= 1e-11 * np.abs(fb_o).max() + 1e-17


@pytest.mark.parametrize("kT", [0.0, 4e-5])
def test_sphere_box_f32(kT):
    wl, steps = small_sphere_case("f32", kT)
    gpu = gpu_from_workload(wl)
    gpu.set_graph_steps(0)
    orc = oracle_from_workload(wl)
    done = 0
    for s in steps:
        gpu.step(s - done)
        orc.step(s - done)
        done = s
        e = compare(gpu, orc)
        _print(f"f32 kT={kT} step {s}", e)
        _assert_close(e, 1e-5, 1e-6, 1e-6)


def pore_case(precision, kT):
    rng = np.random.default_rng(77)
    shape = (24, 22, 40)
    mask = W.pore_mask(*shape, 9.0)
    spheres = W.place_spheres_in_pore(rng, 2, 2.0, 3.0, shape, 9.0)
    bodies = []
    for c, R in spheres:
        offs = W.sphere_beads(R, W.sphere_bead_count(R))
        m, I = W.solid_body_mass_inertia(1.0, R, R, R)
        bodies.append(W.body_record(offs, m, I, c, quat=W.random_quaternion(rng),
                                    vel=rng.normal(0, 1e-3, 3), omega=rng.normal(0, 1e-3, 3),
                                    gamma=W.GAMMA_FREE))
    return dict(name="pore", precision=precision, steps=30,
                params=W.default_params(kT=kT, g_ext=(0.0, 0.0, 2e-6), tau_shear=0.8,
                                        tau_bulk=1.1, tau_odd=0.9, tau_even=1.2),
                replicas=[dict(shape=shape, seed=12345, mask=mask, bodies=bodies)])


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("kT", [0.0, 4e-5])
def test_pore_with_spheres(precision, kT):
    wl = pore_case(precision, kT)
    gpu = gpu_from_workload(wl)
    assert gpu.row_axis(0) == 2   # stored in rows along the pore axis
    gpu.set_graph_steps(0)
    orc = oracle_from_workload(wl)
    done = 0
    for s in (1, 3, 30):
        gpu.step(s - done)
        orc.step(s - done)
        done = s
        e = compare(gpu, orc)
        _print(f"pore {precision} kT={kT} step {s}", e)
        if precision == "f64":
            _assert_close(e, 1e-11, 1e-13, 1e-12)
        else:
            _assert_close(e, 1e-5, 1e-6, 1e-6)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_pore_along_x_stored_in_x_rows(precision):
    """The same pore and spheres turned so that the pore runs along x: its rows are stored
    along x (no exchange of axes), against the oracle."""
    wl = pore_case(precision, 4e-5)
    r = wl["replicas"][0]
    r["mask"] = np.ascontiguousarray(np.transpose(r["mask"], (2, 1, 0)))
    r["shape"] = tuple(r["shape"][::-1])
    r["bodies"] = [dict(b, pos=np.asarray(b["pos"])[[2, 1, 0]]) for b in r["bodies"]]
    gpu = gpu_from_workload(wl)
    assert gpu.row_axis(0) == 0
    gpu.set_graph_steps(0)
    orc = oracle_from_workload(wl)
    done = 0
    for s in (1, 3, 30):
        gpu.step(s - done)
        orc.step(s - done)
        done = s
        e = compare(gpu, orc)
        _print(f"pore along x {precision} step {s}", e)
        if precision == "f64":
            _assert_close(e, 1e-11, 1e-13, 1e-12)
        else:
            _assert_close(e, 1e-5, 1e-6, 1e-6)
    gpu.close()
