"""MD sub-stepping and WCA excluded volume on the GPU, against the oracle.

- parity: a pore with a ring lattice of wall sites, two spheres whose inner layers touch each
  other and one touching the pore beads, 2 and 3 MD steps per fluid step, thermal and
  deterministic, FP64 and FP32, element by element against the oracle (tolerances of the other
  parity tests); batched replicas with different site sets; graph replay == eager, bit for
  bit;
- errors: excluded volume or wall sites after the first step, capacities, bad ids, boxes too
  small for the interaction range, the reverse pass with sub-steps;
- full size: a sphere thrown at the wall of workload 2's pore bounces off the pore beads
  (their WCA repulsion, eps = kT), and passes the wall when the repulsion is off.
"""
import math

import numpy as np
import pytest

from paper_1604_01829_amd import lbrb
from paper_1604_01829_amd import workloads as W
from tests.helpers import compare, gpu_from_workload, oracle_from_workload
from tests.test_gpu_parity import _assert_close, _print

pytestmark = pytest.mark.gpu


def md_case(precision, kT, substeps=2, eps=2e-3, seed=31, site_radius=1.5, shift=0.0):
    """28 x 28 x 20 box with a radius-8 pore along z, a ring lattice of wall sites (radius
    site_radius, spacing 1.5, one site radius outside the wall), and three R = 2.5 spheres with
    inner layers (radius 0.5, 0.5 inside): two in contact with each other, one against the
    pore beads."""
    nx, ny, nz = 28, 28, 20
    pore_r = 8.0
    mask = W.pore_mask(nx, ny, nz, pore_r)
    sites = W.pore_wall_sites(nx, ny, nz, pore_r, site_radius=site_radius, spacing=1.5)
    R = 2.5
    shell = W.sphere_beads(R, W.sphere_bead_count(R))
    inner = W.inner_layer_sphere(R)
    m, I = W.solid_body_mass_inertia(1.0, R, R, R)
    c = np.array([nx / 2.0, ny / 2.0, 0.0])
    pos = [c + (-1.2 + shift, -2.6, 5.0), c + (-1.0, 2.35, 5.3), c + (5.6, 0.3, 14.0)]
    rng = np.random.default_rng(seed)
    bodies = []
    for p in pos:
        b = W.body_record(shell, m, I, p, quat=W.random_quaternion(rng),
                          vel=rng.normal(0, 1e-3, 3), omega=rng.normal(0, 1e-3, 3),
                          gamma=W.GAMMA_FREE)
        b["ev"] = (inner, W.INNER_LAYER_RADIUS)
        bodies.append(b)
    return dict(name="md", precision=precision, steps=30,
                params=W.default_params(kT=kT, g_ext=(0.0, 0.0, 2e-6), tau_shear=0.8,
                                        tau_bulk=1.1, tau_odd=0.9, tau_even=1.2,
                                        md_substeps=substeps, wca_epsilon=eps),
                replicas=[dict(shape=(nx, ny, nz), seed=seed, mask=mask, bodies=bodies,
                               wall_sites=(sites, site_radius))])


def _tol(precision):
    return (1e-11, 1e-13, 1e-12) if precision == "f64" else (1e-5, 1e-6, 1e-6)


def test_case_interacts():
    """The parity scene has body-body and body-site contacts from the first step."""
    wl = md_case("f64", 0.0)
    orc = oracle_from_workload(wl)
    F = orc.wca_forces()
    assert np.all(np.linalg.norm(F[:, :3], axis=1) > 0), F


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("kT,substeps", [(0.0, 2), (4e-5, 2), (4e-5, 3)])
def test_substeps_and_wca_parity(precision, kT, substeps):
    wl = md_case(precision, kT, substeps)
    gpu = gpu_from_workload(wl)
    gpu.set_graph_steps(0)
    orc = oracle_from_workload(wl)
    done = 0
    for s in (1, 2, 7, 30):
        gpu.step(s - done)
        orc.step(s - done)
        done = s
        e = compare(gpu, orc)
        _print(f"md {precision} kT={kT} m={substeps} step {s}", e)
        _assert_close(e, *_tol(precision))
    tol = 1e-11 if precision == "f64" else 1e-5
    for b in range(3):
        fb_g, fb_o = gpu.bead_forces(0, b), orc.bead_forces(b)
        assert np.abs(fb_g - fb_o).max() <= tol * np.abs(fb_o).max() + 1e-17


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_tight_pore_contacts_all_around(precision):
    """A sphere on the axis of a pore barely wider than itself: inner sites all around it are
    in range of pore beads at many angles and heights (every path of the site grids)."""
    nx, ny, nz = 24, 24, 18
    mask = W.pore_mask(nx, ny, nz, 2.8)
    sites = W.pore_wall_sites(nx, ny, nz, 2.8, site_radius=1.5, spacing=1.2)
    R = 2.5
    shell = W.sphere_beads(R, W.sphere_bead_count(R))
    m, I = W.solid_body_mass_inertia(1.0, R, R, R)
    b = W.body_record(shell, m, I, (12.1, 11.8, 7.3), quat=(0.8, 0.2, 0.5, -0.1),
                      vel=(2e-3, -1e-3, 1e-3), gamma=W.GAMMA_FREE)
    b["ev"] = (W.inner_layer_sphere(R), W.INNER_LAYER_RADIUS)
    wl = dict(name="tight", precision=precision, steps=20,
              params=W.default_params(kT=4e-5, md_substeps=2, wca_epsilon=2e-3),
              replicas=[dict(shape=(nx, ny, nz), seed=5, mask=mask, bodies=[b],
                             wall_sites=(sites, 1.5))])
    orc = oracle_from_workload(wl)
    F = orc.wca_forces()[0]
    assert np.linalg.norm(F[:3]) > 0
    gpu = gpu_from_workload(wl)
    gpu.set_graph_steps(0)
    done = 0
    for st in (1, 5, 20):
        gpu.step(st - done)
        orc.step(st - done)
        done = st
        e = compare(gpu, orc)
        _print(f"tight {precision} step {st}", e)
        _assert_close(e, *_tol(precision))


def test_batched_replicas_with_different_sites():
    a = md_case("f64", 4e-5, seed=31)
    b = md_case("f64", 4e-5, seed=32, site_radius=1.2, shift=0.15)
    c = md_case("f64", 4e-5, seed=33)
    c["replicas"][0]["wall_sites"] = None
    for bd in c["replicas"][0]["bodies"]:
        bd["ev"] = None
    wl = dict(a)
    wl["replicas"] = a["replicas"] + b["replicas"] + c["replicas"]
    gpu = gpu_from_workload(wl)
    gpu.set_graph_steps(4)
    gpu.step(9)
    for r in range(3):
        orc = oracle_from_workload(wl, r)
        orc.step(9)
        e = compare(gpu, orc, r)
        _print(f"md batched replica {r}", e)
        _assert_close(e, *_tol("f64"))


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_graph_replay_is_eager_bitwise(precision):
    runs = []
    for graph in (0, 10):
        gpu = gpu_from_workload(md_case(precision, 4e-5, 2))
        gpu.set_graph_steps(graph)
        gpu.step(25)
        _, bodies, f, rc = gpu.observables(0, fields=True)
        runs.append((f, [b["pos"] for b in bodies], [b["force"] for b in bodies]))
        gpu.close()
    assert np.array_equal(runs[0][0], runs[1][0])
    for k in (1, 2):
        assert all(np.array_equal(x, y) for x, y in zip(runs[0][k], runs[1][k]))


def test_md_errors():
    wl = md_case("f64", 0.0)
    rep = wl["replicas"][0]
    inner = rep["bodies"][0]["ev"][0]
    base = {k: v for k, v in wl["params"].items()}

    def sim_with(fixed=False, **kw):
        p = lbrb.make_params("f64", max_bodies=3, max_beads=300, **{**base, **kw})
        s = lbrb.Simulation(p, lbrb.make_replicas([(rep["shape"], rep["seed"])]))
        s.set_mask(0, rep["mask"])
        b = rep["bodies"][0]
        s.add_body(0, b["offsets"], b["mass"], b["inertia"], b["pos"], gamma=b["gamma"],
                   fixed=fixed)
        return s

    def code(fn, *a):
        with pytest.raises(lbrb.LBError) as ei:
            fn(*a)
        return ei.value.code

    s = sim_with(max_ev_sites=len(inner) - 1, max_wall_sites=10)
    assert code(s.set_excluded_volume, 0, 0, inner, 0.5) == lbrb.LB_ERR_CAPACITY
    assert code(s.add_wall_sites, 0, rep["wall_sites"][0], 1.5) == lbrb.LB_ERR_CAPACITY
    assert code(s.set_excluded_volume, 0, 1, inner[:3], 0.5) == lbrb.LB_ERR_ARG
    assert code(s.set_excluded_volume, 0, 0, inner[:3], -1.0) == lbrb.LB_ERR_ARG
    assert code(s.add_wall_sites, 0, [[1.0, 2.0, math.inf]], 1.5) == lbrb.LB_ERR_ARG
    s.set_excluded_volume(0, 0, inner[:3], 0.5)
    s.add_wall_sites(0, rep["wall_sites"][0][:10], 1.5)
    s.step(1)
    assert code(s.set_excluded_volume, 0, 0, inner[:3], 0.5) == lbrb.LB_ERR_STATE
    assert code(s.add_wall_sites, 0, rep["wall_sites"][0][:1], 1.5) == lbrb.LB_ERR_STATE
    s.close()
    # a box side shorter than twice the interaction range: the first step refuses
    s = sim_with(max_ev_sites=len(inner), max_wall_sites=10)
    s.set_excluded_volume(0, 0, inner, 0.5)
    s.add_wall_sites(0, rep["wall_sites"][0][:10], 12.0)
    assert code(s.step, 1) == lbrb.LB_ERR_ARG
    s.close()
    # the reverse pass runs with several MD steps per fluid step and with excluded volume
    # (its values are checked against the oracle's reverse pass in test_gpu_adjoint)
    for kw in (dict(md_substeps=2), dict(md_substeps=1, max_ev_sites=len(inner))):
        s = sim_with(fixed=True, kT=0.0, **kw)
        if "max_ev_sites" in kw:
            s.set_excluded_volume(0, 0, inner, 0.5)
        J, dg, do = s.adjoint(2, np.ones((2, 1, 3)), 1)
        assert np.isfinite(J) and np.all(np.isfinite(dg)) and np.all(np.isfinite(do))
        s.close()


def _throw_at_wall(eps, steps=3000):
    """Workload 2's pore (radius 40, 128 x 128 x 256) with its pore beads (eps = kT of the
    workload); one R = 4 sphere whose shell is 3 lattice units off the wall, moving outwards
    at 0.002 (kinetic energy ~13 kT), without fluid coupling or noise, 2 MD steps per fluid
    step.  Returns the radial position of the centre every 50 steps."""
    wl = W.confined_md_workload(substeps=2, eps=eps)
    rep = wl["replicas"][0]
    R = 4.0
    shell = W.sphere_beads(R, W.sphere_bead_count(R))
    m, I = W.solid_body_mass_inertia(1.0, R, R, R)
    b = W.body_record(shell, m, I, (64.0 + 33.0, 64.0, 100.0), vel=(0.002, 0.0, 0.0),
                      gamma=0.0)
    b["ev"] = (W.inner_layer_sphere(R), W.INNER_LAYER_RADIUS)
    rep["bodies"] = [b]
    wl["params"]["kT"] = 0.0
    gpu = gpu_from_workload(wl)
    r = []
    for _ in range(steps // 50):
        gpu.step(50)
        _, bodies, _, rc = gpu.observables(0)
        assert rc == 0
        p = bodies[0]["pos"]
        r.append(math.hypot(p[0] - 64.0, p[1] - 64.0))
    gpu.close()
    return np.array(r)


def test_sphere_bounces_off_the_pore_beads():
    r_on = _throw_at_wall(4e-5)
    r_off = _throw_at_wall(0.0)
    print(f"radial position of the centre: with WCA max {r_on.max():.3f} end {r_on[-1]:.3f}; "
          f"without max {r_off.max():.3f}", flush=True)
    ring = 40.0 + W.PORE_SITE_RADIUS
    sigma = W.PORE_SITE_RADIUS + W.INNER_LAYER_RADIUS
    # the inner layer (radius R - 0.5 = 3.5) stops before it reaches 0.8 sigma of the beads
    assert r_on.max() + 3.5 < ring - 0.8 * sigma
    assert r_on[-1] < r_on.max() - 1.0                 # it came back
    assert r_off.max() > r_on.max() + 1.0              # without the repulsion it goes on


def test_many_contributions_per_node_fp64_spread_stays_exact():
    """The FP64 spread keeps each contribution's remainder below 2^-56 in a second fixed-point
    word; 200 beads at one point of a fixed body with 64 MD steps per fluid step put 12,800
    contributions on each stencil node in one fluid step.  The remainders must sum without
    wrapping (a wrapped word shifts the node force by 2^-48, far above the FP64 tolerance)."""
    shape = (12, 12, 12)
    offs = np.zeros((200, 3))
    wl = dict(name="pile", precision="f64", steps=3,
              params=W.default_params(kT=0.0, u0=(0.01, -0.004, 0.002), md_substeps=64),
              replicas=[dict(shape=shape, seed=99, mask=None,
                             bodies=[W.body_record(offs, 1.0, (1.0, 1.0, 1.0),
                                                   np.array([5.37, 6.21, 4.83]),
                                                   gamma=1e-4, fixed=True)])])
    gpu = gpu_from_workload(wl)
    gpu.set_graph_steps(0)
    orc = oracle_from_workload(wl)
    for s in range(1, 4):
        gpu.step(1)
        orc.step(1)
        e = compare(gpu, orc)
        _print(f"200-bead pile, 64 MD steps, step {s}", e)
        _assert_close(e, *_tol("f64"))
    gpu.close()
