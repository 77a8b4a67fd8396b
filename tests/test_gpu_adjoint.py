"""GPU reverse pass (lb_rb_adjoint) against the FP64 oracle's adjoint and finite differences.

- small periodic and pore boxes with two fixed bodies, FP64 and FP32, against the oracle's
  reverse-mode derivative (itself pinned against central differences of the oracle's forward
  run), with a window that does not divide into whole checkpoint segments;
- a batch of a periodic and a pore replica against each replica's own oracle adjoint;
- the checkpoint interval does not change the result; the call leaves the state that the same
  number of forward steps leaves;
- the fixed R = 4 sphere in uniform flow on 64^3 over 200 steps, checkpoints every 20 steps:
  FP64 gradients against central differences of FP64 forward runs of the library, FP32
  gradients against the FP64 ones;
- the same sphere over the first 40 steps (a window whose 41 states of 40 MB the oracle
  holds), FP64 and FP32 against the oracle's FP64 reverse pass;
- a free body (moving and spinning, so the reverse pass runs through the rigid-body
  integrator) next to a fixed one, periodic and in pores, FP64 and FP32, against the oracle's
  reverse pass; the context afterwards continues exactly as one that only stepped forward;
- the torch.autograd.Function wrapper; error codes.
"""
import numpy as np
import pytest

from oracle import pyoracle as po
from paper_1604_01829_amd import workloads as W

pytestmark = pytest.mark.gpu

TAUS = dict(tau_shear=0.9, tau_bulk=1.2, tau_odd=1.05, tau_even=0.8)


def _case(masked):
    rng = np.random.default_rng(15 if masked else 16)
    if masked == "long":
        # a longer pore: stored in rows along z (its axis)
        shape = (14, 14, 24)
        mask = W.pore_mask(*shape, 6.0)
        gext, u0 = (0.0, 0.0, 1e-4), (0.0, 0.0, 0.0)
        centres = [np.array([7.1, 6.8, 11.9]), np.array([4.3, 9.6, 20.2])]
    elif masked:
        shape = (14, 14, 10)
        mask = W.pore_mask(*shape, 6.0)
        gext, u0 = (0.0, 0.0, 1e-4), (0.0, 0.0, 0.0)
        centres = [np.array([7.1, 6.8, 4.9]), np.array([4.3, 9.6, 1.2])]
    else:
        shape = (12, 11, 10)
        mask = None
        gext, u0 = (2e-5, 0.0, -1e-5), (0.01, 0.003, -0.002)
        centres = [np.array([5.7, 5.2, 4.6]), np.array([1.3, 9.4, 8.8])]
    bodies = [(W.sphere_beads(2.0, 24), centres[0], W.random_quaternion(rng), W.GAMMA_FIXED),
              (W.sphere_beads(1.0, 6), centres[1], W.random_quaternion(rng), 0.5 * W.GAMMA_FIXED)]
    return shape, mask, dict(u0=u0, g_ext=gext, **TAUS), bodies


def _gpu(shape, mask, pp, bodies, precision):
    from paper_1604_01829_amd import lbrb
    nb = sum(len(b[0]) for b in bodies)
    pp = dict(pp)
    params = lbrb.make_params(precision=precision, kT=pp.pop("kT", 0.0), max_bodies=len(bodies),
                              max_beads=nb, **pp)
    sim = lbrb.Simulation(params, lbrb.make_replicas([(shape, 7)]))
    if mask is not None:
        sim.set_mask(0, mask)
    for offs, c, q, g in bodies:
        sim.add_body(0, offs, 1.0, (1, 1, 1), c, quat=q, gamma=g, fixed=True)
    return sim


def _oracle(shape, mask, pp, bodies):
    sim = po.OracleSim(shape, po.make_params(**pp))
    if mask is not None:
        sim.set_mask(mask)
    for offs, c, q, g in bodies:
        sim.add_body(offs, 1.0, (1, 1, 1), c, quat=q, gamma=g, fixed=True)
    return sim


def _weights(steps, n_bodies, seed=9):
    rng = np.random.default_rng(seed)
    a = np.zeros((steps, n_bodies, 3))
    a[:, 0, 0] = 1.0 / steps                    # time-averaged drag of body 0 along x
    return a + 0.02 * rng.standard_normal(a.shape)


def _forward_J(sim, steps, a):
    """J from forward steps of the library: sum_n sum_b a(n,b) . F_b(n)."""
    J = 0.0
    for n in range(steps):
        sim.step(1)
        _, bs, _, _ = sim.observables(0)
        J += sum(float(a[n, b] @ bs[b]["force"]) for b in range(len(bs)))
    return J


@pytest.mark.parametrize("masked", [False, True, "long"], ids=["periodic", "pore", "long pore"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_adjoint_matches_oracle(masked, precision):
    shape, mask, pp, bodies = _case(masked)
    T, K = 13, 5                                 # segments of 5, 5 and 3 steps
    a = _weights(T, len(bodies))
    print(f"adjoint vs oracle: {masked} {precision} T={T} K={K}", flush=True)
    Jo, dgo, doo = _oracle(shape, mask, pp, bodies).adjoint(T, a)
    sim = _gpu(shape, mask, pp, bodies, precision)
    assert sim.row_axis(0) == (2 if masked == "long" else 0)
    Jg, dgg, dog = sim.adjoint(T, a, checkpoint_every=K)
    sim.close()
    if precision == "f64":
        tJ, tg, to = 1e-12, 1e-10, 1e-10
    else:
        tJ, tg, to = 2e-6, 5e-6, 5e-6
    print(f"  J rel {abs(Jg - Jo) / abs(Jo):.2e}  dgamma rel "
          f"{np.abs(dgg - dgo).max() / np.abs(dgo).max():.2e}  doffsets rel "
          f"{np.abs(dog - doo).max() / np.abs(doo).max():.2e}", flush=True)
    assert abs(Jg - Jo) <= tJ * abs(Jo), (Jg, Jo)
    assert np.abs(dgg - dgo).max() <= tg * np.abs(dgo).max(), (dgg, dgo)
    assert np.abs(dog - doo).max() <= to * np.abs(doo).max(), np.abs(dog - doo).max()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_batch_of_a_periodic_and_a_pore_replica(precision):
    """Replicas are independent, so the reverse pass over one context holding a periodic and a
    pore replica (dense and masked tile groups, one bead launch over both) returns the sum of
    the two objectives and each replica's own gradients, in global body and bead order."""
    from paper_1604_01829_amd import lbrb
    sp, _, _, bp = _case(False)
    sm, mask, pp, bm = _case(True)
    T, K = 11, 4                                 # segments of 4, 4 and 3 steps
    a = _weights(T, len(bp) + len(bm), seed=21)
    print(f"batch adjoint vs oracle: {precision} T={T} K={K}", flush=True)
    nb = sum(len(b[0]) for b in bp + bm)
    params = lbrb.make_params(precision=precision, kT=0.0, max_bodies=len(bp) + len(bm),
                              max_beads=nb, **pp)
    sim = lbrb.Simulation(params, lbrb.make_replicas([(sp, 7), (sm, 8)]))
    sim.set_mask(1, mask)
    for r, bodies in ((0, bp), (1, bm)):
        for offs, c, q, g in bodies:
            sim.add_body(r, offs, 1.0, (1, 1, 1), c, quat=q, gamma=g, fixed=True)
    Jg, dgg, dog = sim.adjoint(T, a, checkpoint_every=K)
    sim.close()
    Jp, dgp, dop = _oracle(sp, None, pp, bp).adjoint(T, a[:, :len(bp)])
    Jm, dgm, dom = _oracle(sm, mask, pp, bm).adjoint(T, a[:, len(bp):])
    Jo = Jp + Jm
    dgo = np.concatenate([dgp, dgm])
    doo = np.concatenate([dop, dom])
    tJ, tg, to = (1e-12, 1e-10, 1e-10) if precision == "f64" else (2e-6, 5e-6, 5e-6)
    print(f"  J rel {abs(Jg - Jo) / abs(Jo):.2e}  dgamma rel "
          f"{np.abs(dgg - dgo).max() / np.abs(dgo).max():.2e}  doffsets rel "
          f"{np.abs(dog - doo).max() / np.abs(doo).max():.2e}", flush=True)
    assert abs(Jg - Jo) <= tJ * abs(Jo), (Jg, Jo)
    for got, want in ((dgg[:len(bp)], dgp), (dgg[len(bp):], dgm)):
        assert np.abs(got - want).max() <= tg * np.abs(want).max(), (got, want)
    npb = sum(len(b[0]) for b in bp)
    for got, want in ((dog[:npb], dop), (dog[npb:], dom)):
        assert np.abs(got - want).max() <= to * np.abs(want).max(), np.abs(got - want).max()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_batch_with_free_bodies_wca_noise_and_md_steps(precision):
    """One context, two replicas, every feature of the body passes at once: thermal noise, two
    MD steps per fluid step, WCA (replica 0: two free bodies pressing on each other and on
    pore beads; replica 1: a pore with a free and a fixed body); the objective and gradients
    against each replica's own oracle reverse pass, in global body and bead order."""
    from paper_1604_01829_amd import lbrb
    from tests.test_oracle_adjoint import _wca_case
    s0, p0, b0, walls = _wca_case()
    s1, mask, _, b1 = _free_case(True)
    kT, md, T, K = 4e-5, 2, 9, 4
    common = dict(u0=tuple(p0.u0), tau_shear=p0.tau_shear, tau_bulk=p0.tau_bulk,
                  tau_odd=p0.tau_odd, tau_even=p0.tau_even, g_ext=tuple(p0.g_ext))
    a = _weights(T, 4, seed=41)
    print(f"batch with free bodies, WCA, noise, {md} MD steps: {precision}", flush=True)
    # oracles, seeded as their replicas
    o0 = po.OracleSim(s0, po.make_params(kT=kT, md_substeps=md, wca_epsilon=p0.wca_epsilon,
                                         seed=7, **common))
    for j, b in enumerate(b0):
        o0.add_body(b["offs"], b["mass"], b["inertia"], b["centre"], vel=b["vel"],
                    omega=b["omega"], gamma=b["gamma"])
        o0.set_excluded_volume(j, *b["ev"])
    o0.add_wall_sites(walls, 0.5)
    o1 = po.OracleSim(s1, po.make_params(kT=kT, md_substeps=md, wca_epsilon=p0.wca_epsilon,
                                         seed=8, **common))
    o1.set_mask(mask)
    offs, c, q, g = b1[0]
    o1.add_body(offs, FREE["mass"], FREE["inertia"], c, quat=q, vel=FREE["vel"],
                omega=FREE["omega"], gamma=g)
    offs, c, q, g = b1[1]
    o1.add_body(offs, 1.0, (1, 1, 1), c, quat=q, gamma=g, fixed=True)
    J0, dg0, do0 = o0.adjoint(T, a[:, :2])
    J1, dg1, do1 = o1.adjoint(T, a[:, 2:])
    # the library, both replicas in one context
    nb = sum(len(b["offs"]) for b in b0) + sum(len(b[0]) for b in b1)
    params = lbrb.make_params(precision=precision, kT=kT, max_bodies=4, max_beads=nb,
                              md_substeps=md, wca_epsilon=p0.wca_epsilon, max_ev_sites=16,
                              max_wall_sites=len(walls), **common)
    sim = lbrb.Simulation(params, lbrb.make_replicas([(s0, 7), (s1, 8)]))
    sim.set_mask(1, mask)
    for b in b0:
        bid = sim.add_body(0, b["offs"], b["mass"], b["inertia"], b["centre"], vel=b["vel"],
                           omega=b["omega"], gamma=b["gamma"])
        sim.set_excluded_volume(0, bid, *b["ev"])
    sim.add_wall_sites(0, walls, 0.5)
    offs, c, q, g = b1[0]
    sim.add_body(1, offs, FREE["mass"], FREE["inertia"], c, quat=q, vel=FREE["vel"],
                 omega=FREE["omega"], gamma=g)
    offs, c, q, g = b1[1]
    sim.add_body(1, offs, 1.0, (1, 1, 1), c, quat=q, gamma=g, fixed=True)
    Jg, dgg, dog = sim.adjoint(T, a, checkpoint_every=K)
    sim.close()
    Jo = J0 + J1
    tJ, tg = (1e-12, 1e-10) if precision == "f64" else (2e-6, 5e-6)
    print(f"  J rel {abs(Jg - Jo) / abs(Jo):.2e}", flush=True)
    assert abs(Jg - Jo) <= tJ * abs(Jo), (Jg, Jo)
    for got, want in ((dgg[:2], dg0), (dgg[2:], dg1)):
        assert np.abs(got - want).max() <= tg * np.abs(want).max(), (got, want)
    n0 = sum(len(b["offs"]) for b in b0)
    for got, want in ((dog[:n0], do0), (dog[n0:], do1)):
        err = np.abs(got - want).max() / np.abs(want).max()
        print(f"  doffsets rel {err:.2e}", flush=True)
        assert err <= tg, err


def test_checkpoint_interval_does_not_change_the_gradient():
    shape, mask, pp, bodies = _case(True)
    T = 12
    a = _weights(T, len(bodies))
    res = []
    for K in (1, 4, 7, 12, 40):
        sim = _gpu(shape, mask, pp, bodies, "f64")
        res.append(sim.adjoint(T, a, checkpoint_every=K))
        sim.close()
    J0, dg0, do0 = res[0]
    for J, dg, do in res[1:]:
        assert abs(J - J0) <= 1e-14 * abs(J0)
        assert np.abs(dg - dg0).max() <= 1e-13 * np.abs(dg0).max()
        assert np.abs(do - do0).max() <= 1e-13 * np.abs(do0).max()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_adjoint_leaves_the_forward_state(precision):
    shape, mask, pp, bodies = _case(False)
    T = 9
    a = _weights(T, len(bodies))
    s1 = _gpu(shape, mask, pp, bodies, precision)
    J, _, _ = s1.adjoint(T, a, checkpoint_every=4)
    s2 = _gpu(shape, mask, pp, bodies, precision)
    J2 = _forward_J(s2, T, a)
    assert abs(J - J2) <= (1e-13 if precision == "f64" else 1e-6) * abs(J2)
    assert np.array_equal(s1.populations(), s2.populations())
    _, b1, _, _ = s1.observables(0)
    _, b2, _, _ = s2.observables(0)
    for x, y in zip(b1, b2):
        assert np.array_equal(x["force"], y["force"]) and np.array_equal(x["torque"], y["torque"])
    for b in range(len(bodies)):
        assert np.array_equal(s1.bead_forces(0, b), s2.bead_forces(0, b))
    s1.step(3)
    s2.step(3)
    assert np.array_equal(s1.populations(), s2.populations())


FREE = dict(mass=40.0, inertia=(40.0, 45.0, 50.0), vel=(0.004, -0.002, 0.003),
            omega=(0.01, -0.015, 0.02))


def _free_case(masked):
    """Body 0 of _case made free (moving and spinning at the start, anisotropic inertia),
    body 1 fixed.  The start is shifted so that no bead of the free body passes within 8e-4 of
    a cell face during the window (so neither side crosses a kink of the weights)."""
    shape, mask, pp, bodies = _case(masked)
    offs, c, q, _ = bodies[0]
    return shape, mask, pp, [(offs, c + 0.047, q, W.GAMMA_FREE), bodies[1]]


def _gpu_free(shape, mask, pp, bodies, precision, md=1):
    from paper_1604_01829_amd import lbrb
    nb = sum(len(b[0]) for b in bodies)
    pp = dict(pp)
    params = lbrb.make_params(precision=precision, kT=pp.pop("kT", 0.0), max_bodies=len(bodies),
                              max_beads=nb, md_substeps=md, **pp)
    sim = lbrb.Simulation(params, lbrb.make_replicas([(shape, 7)]))
    if mask is not None:
        sim.set_mask(0, mask)
    offs, c, q, g = bodies[0]
    sim.add_body(0, offs, FREE["mass"], FREE["inertia"], c, quat=q, vel=FREE["vel"],
                 omega=FREE["omega"], gamma=g)
    offs, c, q, g = bodies[1]
    sim.add_body(0, offs, 1.0, (1, 1, 1), c, quat=q, gamma=g, fixed=True)
    return sim


def _oracle_free(shape, mask, pp, bodies, md=1):
    sim = po.OracleSim(shape, po.make_params(md_substeps=md, **pp))
    if mask is not None:
        sim.set_mask(mask)
    offs, c, q, g = bodies[0]
    sim.add_body(offs, FREE["mass"], FREE["inertia"], c, quat=q, vel=FREE["vel"],
                 omega=FREE["omega"], gamma=g)
    offs, c, q, g = bodies[1]
    sim.add_body(offs, 1.0, (1, 1, 1), c, quat=q, gamma=g, fixed=True)
    return sim


@pytest.mark.parametrize("masked,md", [(False, 1), (True, 1), ("long", 1), (False, 2), (True, 3)],
                         ids=["periodic", "pore", "long pore", "periodic-2md", "pore-3md"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_free_body_adjoint_matches_oracle(masked, md, precision):
    """The reverse pass through the rigid-body integrator (a free body next to a fixed one)
    against the oracle's, itself pinned by central differences of the oracle's forward run;
    segments of 5, 5 and 3 steps, so that replays rewrite the moving bead records; one MD step
    per fluid step, and two or three (the paper's scheme: the MD steps of a fluid step on the
    frozen fluid, recomputed with the body tables between them)."""
    shape, mask, pp, bodies = _free_case(masked)
    T, K = 13, 5
    a = _weights(T, len(bodies), seed=23)
    print(f"free-body adjoint vs oracle: {masked} md={md} {precision} T={T} K={K}", flush=True)
    Jo, dgo, doo = _oracle_free(shape, mask, pp, bodies, md).adjoint(T, a)
    sim = _gpu_free(shape, mask, pp, bodies, precision, md)
    Jg, dgg, dog = sim.adjoint(T, a, checkpoint_every=K)
    sim.close()
    print(f"  J rel {abs(Jg - Jo) / abs(Jo):.2e}  dgamma rel "
          f"{np.abs(dgg - dgo).max() / np.abs(dgo).max():.2e}  doffsets rel "
          f"{np.abs(dog - doo).max() / np.abs(doo).max():.2e}", flush=True)
    if precision == "f64":
        tJ, tg, to = 1e-12, 1e-10, 1e-10
    else:
        tJ, tg, to = 2e-6, 5e-6, 5e-6
    assert abs(Jg - Jo) <= tJ * abs(Jo), (Jg, Jo)
    assert np.abs(dgg - dgo).max() <= tg * np.abs(dgo).max(), (dgg, dgo)
    assert np.abs(dog - doo).max() <= to * np.abs(doo).max(), np.abs(dog - doo).max()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_fixed_bodies_with_two_md_steps_match_oracle(precision):
    """Two fixed bodies, two MD steps per fluid step: the couplings of both MD steps spread
    half their force each, and only the last one's force enters the objective."""
    shape, mask, pp, bodies = _case(True)
    T, K = 9, 4
    a = _weights(T, len(bodies))
    osim = po.OracleSim(shape, po.make_params(md_substeps=2, **pp))
    osim.set_mask(mask)
    for offs, c, q, g in bodies:
        osim.add_body(offs, 1.0, (1, 1, 1), c, quat=q, gamma=g, fixed=True)
    Jo, dgo, doo = osim.adjoint(T, a)
    from paper_1604_01829_amd import lbrb
    nb = sum(len(b[0]) for b in bodies)
    params = lbrb.make_params(precision=precision, kT=0.0, max_bodies=len(bodies), max_beads=nb,
                              md_substeps=2, **pp)
    sim = lbrb.Simulation(params, lbrb.make_replicas([(shape, 7)]))
    sim.set_mask(0, mask)
    for offs, c, q, g in bodies:
        sim.add_body(0, offs, 1.0, (1, 1, 1), c, quat=q, gamma=g, fixed=True)
    Jg, dgg, dog = sim.adjoint(T, a, checkpoint_every=K)
    sim.close()
    print(f"  J rel {abs(Jg - Jo) / abs(Jo):.2e}  dgamma rel "
          f"{np.abs(dgg - dgo).max() / np.abs(dgo).max():.2e}  doffsets rel "
          f"{np.abs(dog - doo).max() / np.abs(doo).max():.2e}", flush=True)
    tJ, tg = (1e-12, 1e-10) if precision == "f64" else (2e-6, 5e-6)
    assert abs(Jg - Jo) <= tJ * abs(Jo), (Jg, Jo)
    assert np.abs(dgg - dgo).max() <= tg * np.abs(dgo).max(), (dgg, dgo)
    assert np.abs(dog - doo).max() <= tg * np.abs(doo).max(), np.abs(dog - doo).max()


@pytest.mark.parametrize("md", [1, 2])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_excluded_volume_adjoint_matches_oracle(md, precision):
    """Two free bodies whose excluded-volume sites press on each other and on a plane of pore
    beads (the oracle's finite-difference case): the reverse pass through the WCA pair forces
    (cell lists for the pore beads, the replica's bodies for the pairs between bodies)
    against the oracle's."""
    from tests.test_oracle_adjoint import _wca_case, _run_wca
    from paper_1604_01829_amd import lbrb
    shape, params, bodies, walls = _wca_case()
    params.md_substeps = md
    T, K = 12, 5
    a = _weights(T, 2, seed=29)
    print(f"excluded-volume adjoint vs oracle: md={md} {precision}", flush=True)
    Jo, dgo, doo = _run_wca(shape, params, bodies, walls, T, a, adjoint=True)
    nb = sum(len(b["offs"]) for b in bodies)
    gp = lbrb.make_params(precision=precision, kT=0.0, max_bodies=2, max_beads=nb, md_substeps=md,
                          u0=tuple(params.u0), tau_shear=params.tau_shear,
                          tau_bulk=params.tau_bulk, tau_odd=params.tau_odd,
                          tau_even=params.tau_even, g_ext=tuple(params.g_ext),
                          wca_epsilon=params.wca_epsilon, max_ev_sites=16,
                          max_wall_sites=len(walls))
    sim = lbrb.Simulation(gp, lbrb.make_replicas([(shape, 7)]))
    for j, b in enumerate(bodies):
        bid = sim.add_body(0, b["offs"], b["mass"], b["inertia"], b["centre"], vel=b["vel"],
                           omega=b["omega"], gamma=b["gamma"])
        sim.set_excluded_volume(0, bid, *b["ev"])
    sim.add_wall_sites(0, walls, 0.5)
    Jg, dgg, dog = sim.adjoint(T, a, checkpoint_every=K)
    sim.close()
    print(f"  J rel {abs(Jg - Jo) / abs(Jo):.2e}  dgamma rel "
          f"{np.abs(dgg - dgo).max() / np.abs(dgo).max():.2e}  doffsets rel "
          f"{np.abs(dog - doo).max() / np.abs(doo).max():.2e}", flush=True)
    tJ, tg = (1e-12, 1e-10) if precision == "f64" else (2e-6, 5e-6)
    assert abs(Jg - Jo) <= tJ * abs(Jo), (Jg, Jo)
    assert np.abs(dgg - dgo).max() <= tg * np.abs(dgo).max(), (dgg, dgo)
    assert np.abs(dog - doo).max() <= tg * np.abs(doo).max(), np.abs(dog - doo).max()


@pytest.mark.parametrize("free,md", [(False, 1), (True, 1), (True, 2)],
                         ids=["fixed", "free", "free-2md"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_thermal_adjoint_matches_oracle(free, md, precision):
    """Thermal fluid and bead noise (kT = 4e-5, the oracle seeded as the replica): the pathwise
    reverse pass (every recomputed step draws the forward run's counter-based noise; the bead
    noise amplitude is differentiated in gamma) against the oracle's; fixed bodies take the
    fused schedule, a free body the body passes."""
    T, K = 11, 4
    if free:
        shape, mask, pp, bodies = _free_case(False)
    else:
        shape, mask, pp, bodies = _case(False)
    pp = dict(pp, kT=4e-5)
    a = _weights(T, len(bodies), seed=31)
    print(f"thermal adjoint vs oracle: free={free} md={md} {precision}", flush=True)
    if free:
        orc = po.OracleSim(shape, po.make_params(md_substeps=md, seed=7, **pp))
        offs, c, q, g = bodies[0]
        orc.add_body(offs, FREE["mass"], FREE["inertia"], c, quat=q, vel=FREE["vel"],
                     omega=FREE["omega"], gamma=g)
        offs, c, q, g = bodies[1]
        orc.add_body(offs, 1.0, (1, 1, 1), c, quat=q, gamma=g, fixed=True)
        sim = _gpu_free(shape, mask, pp, bodies, precision, md)
    else:
        orc = po.OracleSim(shape, po.make_params(seed=7, **pp))
        for offs, c, q, g in bodies:
            orc.add_body(offs, 1.0, (1, 1, 1), c, quat=q, gamma=g, fixed=True)
        sim = _gpu(shape, mask, pp, bodies, precision)
    Jo, dgo, doo = orc.adjoint(T, a)
    Jg, dgg, dog = sim.adjoint(T, a, checkpoint_every=K)
    sim.close()
    print(f"  J rel {abs(Jg - Jo) / abs(Jo):.2e}  dgamma rel "
          f"{np.abs(dgg - dgo).max() / np.abs(dgo).max():.2e}  doffsets rel "
          f"{np.abs(dog - doo).max() / np.abs(doo).max():.2e}", flush=True)
    tJ, tg = (1e-12, 1e-10) if precision == "f64" else (2e-6, 5e-6)
    assert abs(Jg - Jo) <= tJ * abs(Jo), (Jg, Jo)
    assert np.abs(dgg - dgo).max() <= tg * np.abs(dgo).max(), (dgg, dgo)
    assert np.abs(dog - doo).max() <= tg * np.abs(doo).max(), np.abs(dog - doo).max()


def test_free_body_adjoint_leaves_the_forward_state():
    """After the reverse pass (whose replays rewrite the bead records) the context continues
    exactly as one that only stepped forward."""
    shape, mask, pp, bodies = _free_case(False)
    T = 9
    a = _weights(T, len(bodies))
    s1 = _gpu_free(shape, mask, pp, bodies, "f64")
    s1.adjoint(T, a, checkpoint_every=4)
    s2 = _gpu_free(shape, mask, pp, bodies, "f64")
    s2.step(T)
    for s in (s1, s2):
        s.step(3)
    assert np.array_equal(s1.populations(), s2.populations())
    _, b1, _, _ = s1.observables(0)
    _, b2, _, _ = s2.observables(0)
    for x, y in zip(b1, b2):
        for k in ("pos", "quat", "vel", "omega", "force", "torque"):
            assert np.array_equal(x[k], y[k]), k
    s1.close()
    s2.close()


def _config5(precision):
    from paper_1604_01829_amd import lbrb
    wl = W.workload(5)
    return wl, lambda gamma=None, offsets=None: _config5_sim(wl, precision, gamma, offsets)


def _config5_sim(wl, precision, gamma, offsets):
    import copy
    from paper_1604_01829_amd import lbrb
    w = copy.deepcopy(wl)
    b = w["replicas"][0]["bodies"][0]
    w["params"]["kT"] = 0.0
    if gamma is not None:
        b["gamma"] = gamma
    if offsets is not None:
        b["offsets"] = offsets
    return lbrb.simulation_from_workload(w, precision=precision)


def test_full_size_sphere_window_gradient():
    """64^3, R = 4 fixed sphere (401 beads), u0 = (0.01, 0, 0), 200 steps, checkpoints every
    20 steps: J = time-averaged drag along x."""
    T, K = 200, 20
    wl, make = _config5("f64")
    a = np.zeros((T, 1, 3))
    a[:, 0, 0] = 1.0 / T
    print("full-size adjoint: f64", flush=True)
    sim = make()
    J, dg, do = sim.adjoint(T, a, checkpoint_every=K)
    sim.close()
    assert J > 0.0                              # the flow drags the sphere along +x
    g0 = wl["replicas"][0]["bodies"][0]["gamma"]
    h = 1e-5 * g0
    fd = (_forward_J(make(gamma=g0 + h), T, a) - _forward_J(make(gamma=g0 - h), T, a)) / (2 * h)
    print(f"  J {J:.6e}  dJ/dgamma {dg[0]:.9e}  central difference {fd:.9e}", flush=True)
    assert abs(fd - dg[0]) <= 1e-6 * abs(fd), (fd, dg[0])
    offs = np.asarray(wl["replicas"][0]["bodies"][0]["offsets"], dtype=np.float64)
    k_big = int(np.argmax(np.linalg.norm(do, axis=1)))
    for k in (k_big, 0):
        for ax in range(3):
            op, om = offs.copy(), offs.copy()
            op[k, ax] += 1e-6
            om[k, ax] -= 1e-6
            fd = (_forward_J(make(offsets=op), T, a) - _forward_J(make(offsets=om), T, a)) / 2e-6
            print(f"  bead {k} axis {ax}: adjoint {do[k, ax]:.9e}  central difference {fd:.9e}",
                  flush=True)
            assert abs(fd - do[k, ax]) <= 1e-5 * np.abs(do).max(), (k, ax, fd, do[k, ax])
    print("full-size adjoint: f32", flush=True)
    _, make32 = _config5("f32")
    sim = make32()
    J32, dg32, do32 = sim.adjoint(T, a, checkpoint_every=K)
    sim.close()
    print(f"  FP32 vs FP64: J rel {abs(J32 - J) / abs(J):.2e}  dgamma rel "
          f"{abs(dg32[0] - dg[0]) / abs(dg[0]):.2e}  doffsets rel "
          f"{np.abs(do32 - do).max() / np.abs(do).max():.2e}", flush=True)
    assert abs(J32 - J) <= 1e-5 * abs(J)
    assert abs(dg32[0] - dg[0]) <= 1e-5 * abs(dg[0])
    assert np.abs(do32 - do).max() <= 1e-5 * np.abs(do).max()


def _free_sphere_sim(precision, gamma=None, offsets=None, kT=0.0):
    """Workload 5's sphere released: free, spinning slowly at the start, in the same uniform
    flow, at the paper's free-body friction."""
    import copy
    from paper_1604_01829_amd import lbrb
    w = copy.deepcopy(W.workload(5))
    b = w["replicas"][0]["bodies"][0]
    w["params"]["kT"] = kT
    b["fixed"] = False
    b["omega"] = np.array([0.002, -0.001, 0.0015])
    b["gamma"] = W.GAMMA_FREE if gamma is None else gamma
    if offsets is not None:
        b["offsets"] = offsets
    return w, lbrb.simulation_from_workload(w, precision=precision)


def test_full_size_free_sphere_window_gradient():
    """64^3, the R = 4 sphere (401 beads) free in the uniform flow, 100 steps, checkpoints every
    20 steps: the FP64 reverse pass through the rigid-body integrator against central
    differences of FP64 forward runs of the library, and FP32 against FP64."""
    T, K = 100, 20
    a = np.zeros((T, 1, 3))
    a[:, 0, 0] = 1.0 / T
    print("full-size free-sphere adjoint: f64", flush=True)
    w, sim = _free_sphere_sim("f64")
    J, dg, do = sim.adjoint(T, a, checkpoint_every=K)
    _, bs, _, _ = sim.observables(0)
    moved = float(np.linalg.norm(bs[0]["pos"] - w["replicas"][0]["bodies"][0]["pos"]))
    sim.close()
    assert moved > 1e-3, moved                  # the flow carries the sphere along
    g0 = W.GAMMA_FREE
    h = 1e-5 * g0
    fd = (_forward_J(_free_sphere_sim("f64", gamma=g0 + h)[1], T, a)
          - _forward_J(_free_sphere_sim("f64", gamma=g0 - h)[1], T, a)) / (2 * h)
    print(f"  moved {moved:.4f}  J {J:.6e}  dJ/dgamma {dg[0]:.9e}  central difference {fd:.9e}",
          flush=True)
    assert abs(fd - dg[0]) <= 1e-6 * abs(fd), (fd, dg[0])
    # the offsets along the gradient's own direction (every bead moves by at most h): one
    # bead's derivative alone (~1e-7) sits at the rounding noise of J over 100 steps divided
    # by 2h (measured ~4e-11), the directional one lies far above it
    offs = np.asarray(w["replicas"][0]["bodies"][0]["offsets"], dtype=np.float64)
    v = do / np.abs(do).max()
    h = 1e-6
    fd = (_forward_J(_free_sphere_sim("f64", offsets=offs + h * v)[1], T, a)
          - _forward_J(_free_sphere_sim("f64", offsets=offs - h * v)[1], T, a)) / (2 * h)
    D = float(np.sum(do * v))
    print(f"  offsets along the gradient: adjoint {D:.9e}  central difference {fd:.9e}",
          flush=True)
    assert abs(fd - D) <= 1e-4 * abs(D), (fd, D)
    print("full-size free-sphere adjoint: f32", flush=True)
    _, sim = _free_sphere_sim("f32")
    J32, dg32, do32 = sim.adjoint(T, a, checkpoint_every=K)
    sim.close()
    print(f"  FP32 vs FP64: J rel {abs(J32 - J) / abs(J):.2e}  dgamma rel "
          f"{abs(dg32[0] - dg[0]) / abs(dg[0]):.2e}  doffsets rel "
          f"{np.abs(do32 - do).max() / np.abs(do).max():.2e}", flush=True)
    assert abs(J32 - J) <= 1e-5 * abs(J)
    # the free body follows the flow, so its drag hardly depends on gamma (d ln J / d ln gamma
    # is ~4e-3 here): dJ/dgamma is a near-cancellation of terms of size J/gamma, and FP32
    # rounding is relative to those terms
    assert abs(dg32[0] - dg[0]) <= 1e-5 * max(abs(dg[0]), abs(J) / g0)
    assert np.abs(do32 - do).max() <= 1e-5 * np.abs(do).max()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_full_size_sphere_against_the_oracle_adjoint(precision):
    """64^3, R = 4 fixed sphere (401 beads), u0 = (0.01, 0, 0): J = drag along x averaged over
    a 40-step window, checkpoints every 20 steps on the GPU, every state kept by the oracle.
    Tolerances: those of the small boxes (FP64: 1e-12 on J, 1e-10 of the largest gradient;
    FP32: 5e-6), relative."""
    import copy
    T, K = 40, 20
    wl = W.workload(5)
    w = copy.deepcopy(wl)
    w["params"]["kT"] = 0.0
    a = np.zeros((T, 1, 3))
    a[:, 0, 0] = 1.0 / T
    print(f"64^3 sphere, {T}-step window, {precision}: oracle reverse pass", flush=True)
    from tests.helpers import oracle_from_workload
    orc = oracle_from_workload(w)
    Jo, dgo, doo = orc.adjoint(T, a)
    print(f"  oracle J {Jo:.9e} dJ/dgamma {dgo[0]:.9e}", flush=True)
    sim = _config5_sim(wl, precision, None, None)
    J, dg, do = sim.adjoint(T, a, checkpoint_every=K)
    sim.close()
    eJ = abs(J - Jo) / abs(Jo)
    eg = abs(dg[0] - dgo[0]) / abs(dgo[0])
    eo = float(np.abs(do - doo).max() / np.abs(doo).max())
    print(f"  GPU {precision}: J rel {eJ:.2e}  dgamma rel {eg:.2e}  doffsets rel {eo:.2e}",
          flush=True)
    tJ, tg = (1e-12, 1e-10) if precision == "f64" else (5e-6, 5e-6)
    assert eJ <= tJ and eg <= tg and eo <= tg


def test_full_size_thermal_free_sphere_gradient():
    """64^3, the released R = 4 sphere in a thermal fluid (kT = 4e-5), 60 steps, checkpoints
    every 20: the pathwise FP64 gradient in gamma (the bead noise amplitude scales with
    sqrt(gamma)) against central differences of FP64 forward runs of the library, which draw
    the same counter-based noise."""
    T, K = 60, 20
    a = np.zeros((T, 1, 3))
    a[:, 0, 0] = 1.0 / T
    kT = 4e-5
    print("full-size thermal free-sphere adjoint: f64", flush=True)
    _, sim = _free_sphere_sim("f64", kT=kT)
    J, dg, do = sim.adjoint(T, a, checkpoint_every=K)
    sim.close()
    g0 = W.GAMMA_FREE
    h = 1e-5 * g0
    fd = (_forward_J(_free_sphere_sim("f64", gamma=g0 + h, kT=kT)[1], T, a)
          - _forward_J(_free_sphere_sim("f64", gamma=g0 - h, kT=kT)[1], T, a)) / (2 * h)
    print(f"  J {J:.6e}  dJ/dgamma {dg[0]:.9e}  central difference {fd:.9e}", flush=True)
    assert abs(fd - dg[0]) <= 1e-6 * max(abs(fd), abs(J) / g0), (fd, dg[0])


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_full_size_free_sphere_against_the_oracle_adjoint(precision):
    """64^3, the R = 4 sphere (401 beads) free in the uniform flow: J = drag along x averaged
    over a 40-step window, checkpoints every 20 steps on the GPU, every state kept by the
    oracle; the tolerances of the small boxes."""
    T, K = 40, 20
    a = np.zeros((T, 1, 3))
    a[:, 0, 0] = 1.0 / T
    print(f"64^3 free sphere, {T}-step window, {precision}: oracle reverse pass", flush=True)
    from tests.helpers import oracle_from_workload
    w, sim = _free_sphere_sim(precision)
    Jo, dgo, doo = oracle_from_workload(w).adjoint(T, a)
    print(f"  oracle J {Jo:.9e} dJ/dgamma {dgo[0]:.9e}", flush=True)
    J, dg, do = sim.adjoint(T, a, checkpoint_every=K)
    sim.close()
    eJ = abs(J - Jo) / abs(Jo)
    eg = abs(dg[0] - dgo[0]) / abs(dgo[0])
    eo = float(np.abs(do - doo).max() / np.abs(doo).max())
    print(f"  GPU {precision}: J rel {eJ:.2e}  dgamma rel {eg:.2e}  doffsets rel {eo:.2e}",
          flush=True)
    tJ, tg = (1e-12, 1e-10) if precision == "f64" else (5e-6, 5e-6)
    assert eJ <= tJ and eg <= tg and eo <= tg


def _confined_sim(precision, gamma0=None, offsets0=None):
    """The paper's confined scheme at full size (workload 2's pore and 32 free spheres, two MD
    steps per fluid step, WCA inner layers and pore beads at eps = the workload's kT),
    deterministic, with a pressure gradient along the pore."""
    from paper_1604_01829_amd import lbrb
    w = W.confined_md_workload(substeps=2)
    w["params"]["kT"] = 0.0
    w["params"]["g_ext"] = (0.0, 0.0, 2e-6)
    b0 = w["replicas"][0]["bodies"][0]
    if gamma0 is not None:
        b0["gamma"] = gamma0
    if offsets0 is not None:
        b0["offsets"] = offsets0
    return w, lbrb.simulation_from_workload(w, precision=precision)


def test_full_size_confined_pore_gradient():
    """128 x 128 x 256 pore, 32 free spheres, two MD steps per fluid step, WCA between inner
    layers and with 2,958 pore beads: J = drag of sphere 0 along the pore averaged over 30
    steps (checkpoints every 10).  FP64 against central differences of FP64 forward runs of
    the library (its gamma, its offsets along the gradient's direction), FP32 against FP64."""
    import time
    import torch
    T, K = 30, 10
    a = np.zeros((T, 32, 3))
    a[:, 0, 2] = 1.0 / T
    print("confined pore, full size: f64 reverse pass", flush=True)
    w, sim = _confined_sim("f64")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J, dg, do = sim.adjoint(T, a, checkpoint_every=K)
    t_adj = time.perf_counter() - t0
    sim.close()
    g0 = w["replicas"][0]["bodies"][0]["gamma"]
    h = 1e-5 * g0
    fd = (_forward_J(_confined_sim("f64", gamma0=g0 + h)[1], T, a)
          - _forward_J(_confined_sim("f64", gamma0=g0 - h)[1], T, a)) / (2 * h)
    print(f"  J {J:.6e}  dJ/dgamma_0 {dg[0]:.9e}  central difference {fd:.9e}  "
          f"reverse pass {t_adj * 1e3:.1f} ms", flush=True)
    assert abs(fd - dg[0]) <= 1e-6 * max(abs(fd), abs(J) / g0), (fd, dg[0])
    offs = np.asarray(w["replicas"][0]["bodies"][0]["offsets"], dtype=np.float64)
    n0 = len(offs)
    v = do[:n0] / np.abs(do[:n0]).max()
    hh = 1e-6
    fdo = (_forward_J(_confined_sim("f64", offsets0=offs + hh * v)[1], T, a)
           - _forward_J(_confined_sim("f64", offsets0=offs - hh * v)[1], T, a)) / (2 * hh)
    D = float(np.sum(do[:n0] * v))
    print(f"  offsets of sphere 0 along the gradient: adjoint {D:.9e}  central difference "
          f"{fdo:.9e}", flush=True)
    assert abs(fdo - D) <= 1e-4 * abs(D), (fdo, D)
    print("confined pore, full size: f32 reverse pass", flush=True)
    _, sim = _confined_sim("f32")
    J32, dg32, do32 = sim.adjoint(T, a, checkpoint_every=K)
    sim.close()
    print(f"  FP32 vs FP64: J rel {abs(J32 - J) / abs(J):.2e}  dgamma rel "
          f"{np.abs(dg32 - dg).max() / np.abs(dg).max():.2e}  doffsets rel "
          f"{np.abs(do32 - do).max() / np.abs(do).max():.2e}", flush=True)
    assert abs(J32 - J) <= 1e-5 * abs(J)
    assert np.abs(dg32 - dg).max() <= 1e-5 * max(np.abs(dg).max(), abs(J) / g0)
    assert np.abs(do32 - do).max() <= 1e-5 * np.abs(do).max()


def test_autograd_function_returns_the_library_gradient():
    import torch
    from paper_1604_01829_amd import lbrb
    shape, mask, pp, bodies = _case(False)
    T = 8
    a = _weights(T, len(bodies))
    sizes = [len(b[0]) for b in bodies]

    def builder(gamma, offsets):
        parts = np.split(offsets, np.cumsum(sizes)[:-1])
        bb = [(parts[k], bodies[k][1], bodies[k][2], float(gamma[k])) for k in range(len(bodies))]
        return _gpu(shape, mask, pp, bb, "f64")

    gamma = torch.tensor([b[3] for b in bodies], dtype=torch.float64, requires_grad=True)
    offsets = torch.tensor(np.concatenate([b[0] for b in bodies]), dtype=torch.float64,
                           requires_grad=True)
    J = lbrb.window_objective(gamma, offsets, builder, T, a, checkpoint_every=3)
    (2.0 * J).backward()
    sim = _gpu(shape, mask, pp, bodies, "f64")
    J0, dg, do = sim.adjoint(T, a, checkpoint_every=3)
    sim.close()
    assert abs(J.item() - J0) <= 1e-13 * abs(J0)
    assert np.allclose(gamma.grad.numpy(), 2.0 * dg, rtol=1e-12, atol=0)
    assert np.allclose(offsets.grad.numpy(), 2.0 * do, rtol=1e-12, atol=1e-300)
    # and the gradient is that of the forward objective
    h = 1e-6
    with torch.no_grad():
        gp, gm = gamma.detach().clone(), gamma.detach().clone()
        gp[1] += h
        gm[1] -= h
        fd = (lbrb.window_objective(gp, offsets.detach(), builder, T, a)
              - lbrb.window_objective(gm, offsets.detach(), builder, T, a)) / (2 * h)
    assert abs(float(fd) - dg[1]) <= 1e-6 * abs(dg[1]), (float(fd), dg[1])


def test_adjoint_error_codes():
    from paper_1604_01829_amd import lbrb
    shape, mask, pp, bodies = _case(False)
    sim = _gpu(shape, mask, pp, bodies, "f64")
    a = _weights(4, len(bodies))
    with pytest.raises(lbrb.LBError) as e:
        sim.adjoint(0, a[:0])
    assert e.value.code == lbrb.LB_ERR_ARG
    nbytes = lbrb.lb_adjoint_workspace_bytes(sim.ctx, 4, 2)
    assert nbytes > 0 and lbrb.lb_adjoint_workspace_bytes(sim.ctx, 4, 0) == 0
    import torch
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(lbrb.LBError) as e:        # workspace one byte short
        lbrb.lb_rb_adjoint(sim.ctx, 4, 2, ws.data_ptr(), nbytes - 1, a, 2,
                           sum(len(b[0]) for b in bodies))
    assert e.value.code == lbrb.LB_ERR_ARG
    sim.close()


def test_gamma_calibration_recovers_a_known_friction():
    """Newton on gamma with the adjoint slope: the drag window of the 64^3 fixed sphere run
    at gamma = 0.5 is the target; starting from the workload's gamma the iteration must
    return 0.5."""
    from paper_1604_01829_amd import lbrb
    T, K = 100, 20
    wl = W.workload(5)
    a = np.zeros((T, 1, 3))
    a[:, 0, 0] = 1.0 / T

    def builder(g):
        return _config5_sim(wl, "f64", g, None)

    sim = builder(0.5)
    target, _, _ = sim.adjoint(T, a, K)
    sim.close()
    g, J, it = lbrb.calibrate_gamma(builder, T, a, target, wl["replicas"][0]["bodies"][0]["gamma"],
                                    checkpoint_every=K, tol=1e-12)
    print(f"  calibrated gamma {g:.12f} in {it} iterations (J {J:.9e}, target {target:.9e})",
          flush=True)
    assert abs(g - 0.5) < 1e-9 and it <= 8


def test_gamma_calibrated_to_a_hydrodynamic_radius():
    """The workload-5 sphere (R = 4, 401 beads, fixed) in a 64^3 box whose fluid starts at
    u0 = 0.01 and decays: gamma such that the friction over steps 800-1000, measured from the
    drag history with the fluid's momentum bookkeeping, is Hasimoto's friction of a sphere of
    hydrodynamic radius R + 0.2 (Newton with the reverse pass's slope).  Then forward runs with
    that gamma in boxes of 48 and 80 (windows scaled with L^2, the flow's development time):
    the Hasimoto-corrected radius is the target there too, to 2 %: the calibration fixed a
    property of the raspberry, not of the box."""
    from paper_1604_01829_amd import analysis as AN
    from paper_1604_01829_amd import lbrb
    wl5 = W.workload(5)
    body = wl5["replicas"][0]["bodies"][0]
    R, u0, eta, rho0 = 4.0, 0.01, 1.0 / 6.0, 1.0
    window = (800, 1000)
    target = R + 0.2

    def builder(g):
        return _config5_sim(wl5, "f64", g, None)

    g, it, xi = lbrb.calibrate_gamma_to_radius(builder, 64, target, u0, rho0, eta, window,
                                               gamma0=body["gamma"], tol=1e-12)
    print(f"  calibrated gamma {g:.9f} in {it} Newton steps (friction {xi:.6f})", flush=True)
    assert g > 0 and it <= 10
    delta = body["pos"] - 32.0
    radii = {}
    for L in (48, 64, 80):
        a, b = (window if L == 64 else
                (round(window[0] * L * L / 64 ** 2), round(window[1] * L * L / 64 ** 2)))
        params = lbrb.make_params("f64", u0=(u0, 0.0, 0.0), max_bodies=1,
                                  max_beads=len(body["offsets"]))
        sim = lbrb.Simulation(params, lbrb.make_replicas([((L, L, L), 1)]))
        sim.add_body(0, body["offsets"], 1.0, (1, 1, 1), L / 2 + delta, gamma=g, fixed=True)
        sim.set_graph_steps(0)
        drag = []
        for _ in range(b):
            sim.step(1)
            drag.append(sim.observables(0)[1][0]["force"][0])
        sim.close()
        xi_L = AN.decay_friction(drag, u0, rho0, L ** 3, (a, b))
        radii[L] = AN.hasimoto_radius(xi_L, L, eta)
        print(f"  L={L}: window {a}-{b}, friction {xi_L:.6f}, R_h {radii[L]:.6f}", flush=True)
    assert abs(radii[64] - target) <= 1e-8 * target
    for L in (48, 80):
        assert abs(radii[L] - target) <= 0.02 * target
