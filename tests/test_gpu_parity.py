"""GPU library vs the FP64 oracle, element by element, through the C-ABI.

Tolerances (derivation in the design notes):
- FP64 populations: the GPU stores f - w rho0 and sums in another order, and spreads bead
  forces as 2^-56 fixed point; errors stay at round-off, ~1e-15 per step relative to the
  field scale, so 1e-12 of the scale is allowed over <= 100 steps.
- FP32 shifted populations: one FP32 rounding of the shifted populations per step (~6e-8
  relative to |f - w rho0| ~ |u|) accumulates over the run; the workload target is 1e-5 of
  the field scale for velocities and 1e-5 relative for density.
"""
import numpy as np
import pytest

from paper_1604_01829_amd import workloads as W
from tests.helpers import compare, gpu_from_workload, oracle_from_workload

pytestmark = pytest.mark.gpu


def _print(tag, e):
    keys = ["rho", "u_abs", "u_scale", "mass", "momentum", "momentum_scale", "body_pos",
            "body_quat", "body_vel",
            "body_force", "scale_force", "body_torque", "scale_torque"]
    print(tag, " ".join(f"{k}={e[k]:.3g}" for k in keys if k in e), flush=True)


def _assert_close(e, tol_rel_u, tol_rho, tol_body):
    assert e["rc"] == 0
    assert e["solid_zero"]
    assert e["finite"]
    assert e["rho"] <= tol_rho
    assert e["u_abs"] <= tol_rel_u * max(e["u_scale"], 1e-12)
    assert e["mass"] <= tol_rho
    assert e["momentum"] <= tol_rel_u * e["momentum_scale"] + 1e-15
    for k in ("pos", "quat"):
        assert e["body_" + k] <= tol_body
    for k in ("vel", "omega", "force", "torque"):
        assert e["body_" + k] <= tol_rel_u * max(e["scale_" + k], 1e-14) + 1e-15


def small_sphere_case(precision, kT=0.0, steps=(1, 2, 7, 40)):
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
