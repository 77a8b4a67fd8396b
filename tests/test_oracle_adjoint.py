"""Pins of the oracle's reverse-mode derivative against central finite differences.

- the collision's vector-Jacobian product against a central difference of the collision
  itself along a random direction (both population and force inputs);
- the whole-window gradient of J = sum_n a(n) . F_b(n) with respect to the bead friction and
  to individual bead offsets, against central differences of J computed by re-running the
  forward oracle, in a periodic box and in a pore with bounce-back walls.  Beads are chosen
  away from cell faces so that the finite difference does not cross a kink of the
  trilinear weights;
- the same for a free body (moving and spinning, anisotropic inertia) beside a fixed one, so
  that the derivative runs through both half kicks, the drift and the quaternion rotation,
  with one, two and three MD steps per fluid step;
- two free bodies whose excluded-volume sites press on each other and on a plane of pore
  beads (WCA pairs active throughout, none near the cutoff), one and two MD steps.
"""
import numpy as np
import pytest

from oracle import pyoracle as po
from paper_1604_01829_amd import workloads as W


def test_collide_vjp_matches_finite_difference():
    rng = np.random.default_rng(21)
    p = po.make_params(tau_shear=0.8, tau_bulk=1.3, tau_odd=1.1, tau_even=0.7)
    for _ in range(10):
        f = po.equilibrium(1.0 + 0.05 * rng.standard_normal(), 0.03 * rng.standard_normal(3))
        f = f + 1e-3 * rng.standard_normal(19)
        F = 1e-3 * rng.standard_normal(3)
        lam = rng.standard_normal(19)
        df = rng.standard_normal(19)
        dF = rng.standard_normal(3)
        lin, lF = po.collide_vjp(p, f, F, lam)
        h = 1e-6
        fp = po.collide_node(p, f + h * df, F + h * dF)
        fm = po.collide_node(p, f - h * df, F - h * dF)
        fd = lam @ (fp - fm) / (2 * h)
        an = lin @ df + lF @ dF
        assert abs(fd - an) < 1e-8 * (abs(an) + 1.0), (fd, an)


def _case(masked):
    rng = np.random.default_rng(5 if masked else 6)
    if masked:
        shape = (14, 14, 10)
        mask = W.pore_mask(*shape, 6.0)
        centre = np.array([7.1, 6.8, 4.9])
        gext = (0.0, 0.0, 1e-4)
        u0 = (0.0, 0.0, 0.0)
    else:
        shape = (12, 11, 10)
        mask = None
        centre = np.array([5.7, 5.2, 4.6])
        gext = (2e-5, 0.0, -1e-5)
        u0 = (0.01, 0.003, -0.002)
    offs = W.sphere_beads(2.0, 24)
    q = W.random_quaternion(rng)
    params = po.make_params(u0=u0, tau_shear=0.9, tau_bulk=1.2, tau_odd=1.05, tau_even=0.8,
                            g_ext=gext)
    return shape, mask, params, offs, centre, q


def _run(shape, mask, params, offs, centre, q, gamma, steps, weights, adjoint=False):
    sim = po.OracleSim(shape, params)
    if mask is not None:
        sim.set_mask(mask)
    sim.add_body(offs, 1.0, (1, 1, 1), centre, quat=q, gamma=gamma, fixed=True)
    if adjoint:
        return sim.adjoint(steps, weights)
    J = 0.0
    for n in range(steps):
        sim.step(1)
        J += float(weights[n, 0] @ sim.body_state(0)["force"])
    return J


@pytest.mark.parametrize("masked", [False, True])
def test_window_gradient_matches_finite_difference(masked):
    shape, mask, params, offs, centre, q, = _case(masked)
    steps, gamma = 12, W.GAMMA_FIXED
    rng = np.random.default_rng(9)
    weights = np.zeros((steps, 1, 3))
    weights[:, 0, 0] = 1.0 / steps                         # time-averaged drag along x
    weights += 0.02 * rng.standard_normal(weights.shape)   # and a generic functional
    J, dg, do = _run(shape, mask, params, offs, centre, q, gamma, steps, weights, adjoint=True)
    assert abs(J - _run(shape, mask, params, offs, centre, q, gamma, steps, weights)) < 1e-15
    # gamma
    h = 1e-6
    fd = (_run(shape, mask, params, offs, centre, q, gamma + h, steps, weights)
          - _run(shape, mask, params, offs, centre, q, gamma - h, steps, weights)) / (2 * h)
    assert abs(fd - dg[0]) < 1e-6 * abs(fd) + 1e-12, (fd, dg[0])
    # offsets of beads whose cell fractions stay clear of the faces
    from scipy.spatial.transform import Rotation
    Rm = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    pos = centre + offs @ Rm.T
    frac = np.mod(pos - 0.5, 1.0)
    ok = np.all(np.minimum(frac, 1 - frac) > 1e-3, axis=1)
    beads = np.flatnonzero(ok)[:4]
    assert len(beads) >= 3
    h = 1e-6
    for k in beads:
        for a in range(3):
            op, om = offs.copy(), offs.copy()
            op[k, a] += h
            om[k, a] -= h
            fd = (_run(shape, mask, params, op, centre, q, gamma, steps, weights)
                  - _run(shape, mask, params, om, centre, q, gamma, steps, weights)) / (2 * h)
            assert abs(fd - do[k, a]) < 1e-5 * np.abs(do).max() + 1e-13, (k, a, fd, do[k, a])


def _free_case(masked):
    """A free sphere (anisotropic inertia, moving and spinning at the start) and a fixed
    smaller body in the same box."""
    shape, mask, params, offs, centre, q = _case(masked)
    rng = np.random.default_rng(31 if masked else 32)
    # the start is shifted so that no bead of the free body passes within 1e-3 of a cell
    # face during the window
    free = dict(offs=offs, mass=40.0, inertia=(40.0, 45.0, 50.0), centre=centre + 0.047, quat=q,
                vel=(0.004, -0.002, 0.003), omega=(0.01, -0.015, 0.02), gamma=W.GAMMA_FREE)
    fixed_centre = np.array([2.3, 9.1, 8.2]) if not masked else np.array([4.3, 9.6, 1.7])
    fixed = dict(offs=W.sphere_beads(1.0, 6), centre=fixed_centre,
                 quat=W.random_quaternion(rng), gamma=0.5 * W.GAMMA_FIXED)
    return shape, mask, params, free, fixed


def _run_free(shape, mask, params, free, fixed, steps, weights, adjoint=False, poses=None):
    sim = po.OracleSim(shape, params)
    if mask is not None:
        sim.set_mask(mask)
    sim.add_body(free["offs"], free["mass"], free["inertia"], free["centre"], quat=free["quat"],
                 vel=free["vel"], omega=free["omega"], gamma=free["gamma"])
    sim.add_body(fixed["offs"], 1.0, (1, 1, 1), fixed["centre"], quat=fixed["quat"],
                 gamma=fixed["gamma"], fixed=True)
    if adjoint:
        return sim.adjoint(steps, weights)
    J = 0.0
    for n in range(steps):
        sim.step(1)
        for b in range(2):
            st = sim.body_state(b)
            J += float(weights[n, b] @ st["force"])
            if poses is not None and b == 0:
                poses.append((st["pos"].copy(), st["quat"].copy()))
    return J


@pytest.mark.parametrize("masked,md,kT", [(False, 1, 0.0), (True, 1, 0.0), (False, 2, 0.0),
                                           (True, 3, 0.0), (False, 1, 4e-5), (True, 2, 4e-5)],
                         ids=["periodic", "pore", "periodic-2md", "pore-3md", "periodic-thermal",
                              "pore-2md-thermal"])
def test_free_body_window_gradient_matches_finite_difference(masked, md, kT):
    """The reverse pass through the rigid-body integrator (both half kicks, the drift, the
    quaternion rotation and the moving bead positions and velocities) against central
    differences of J re-run by the forward oracle, for a free body next to a fixed one; with
    one MD step per fluid step, and with two and three (the paper's scheme: several MD steps
    on the frozen fluid, each spreading its share of the bead force); deterministic, and
    thermal (the pathwise derivative: every run draws the same counter-based noise, and the
    bead noise amplitude sqrt(2 kT gamma / h) depends on gamma)."""
    from scipy.spatial.transform import Rotation
    shape, mask, params, free, fixed = _free_case(masked)
    params.md_substeps = md
    params.kT = kT
    steps = 12
    rng = np.random.default_rng(19)
    weights = np.zeros((steps, 2, 3))
    weights[:, 0, 0] = 1.0 / steps
    weights += 0.02 * rng.standard_normal(weights.shape)
    J, dg, do = _run_free(shape, mask, params, free, fixed, steps, weights, adjoint=True)
    poses = []
    assert abs(J - _run_free(shape, mask, params, free, fixed, steps, weights, poses=poses)) < 1e-15
    # the free body really moves and turns over the window
    assert np.linalg.norm(poses[-1][0] - free["centre"]) > 0.02
    # no bead of the free body comes within 10 h of a cell face at the end of any fluid step
    # (kinks of the weights)
    gap = 1.0
    for pos, q in poses:
        Rm = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        frac = np.mod(pos + free["offs"] @ Rm.T - 0.5, 1.0)
        gap = min(gap, float(np.minimum(frac, 1 - frac).min()))
    assert gap > 1e-5, gap
    h = 1e-6
    for b, body in ((0, free), (1, fixed)):
        bp, bm = dict(body), dict(body)
        bp["gamma"] += h
        bm["gamma"] -= h
        args = ((bp, fixed) if b == 0 else (free, bp)), ((bm, fixed) if b == 0 else (free, bm))
        fd = (_run_free(shape, mask, params, *args[0], steps, weights)
              - _run_free(shape, mask, params, *args[1], steps, weights)) / (2 * h)
        assert abs(fd - dg[b]) < 1e-6 * abs(fd) + 1e-12, (b, fd, dg[b])
    scale = np.abs(do[:len(free["offs"])]).max()
    for k in (0, 5, 11, 17):
        for a in range(3):
            op, om = dict(free), dict(free)
            op["offs"] = free["offs"].copy()
            om["offs"] = free["offs"].copy()
            op["offs"][k, a] += h
            om["offs"][k, a] -= h
            fd = (_run_free(shape, mask, params, op, fixed, steps, weights)
                  - _run_free(shape, mask, params, om, fixed, steps, weights)) / (2 * h)
            assert abs(fd - do[k, a]) < 1e-5 * scale + 1e-13, (k, a, fd, do[k, a])


def _wca_case():
    """Two free bodies with excluded-volume sites next to each other and to a plane of static
    sites (pore beads), in a periodic box with a weak flow, WCA pairs active throughout."""
    shape = (14, 13, 12)
    params = po.make_params(u0=(0.004, 0.0, 0.001), tau_shear=0.9, tau_bulk=1.2, tau_odd=1.05,
                            tau_even=0.8, g_ext=(1e-5, 0.0, 0.0), wca_epsilon=1e-3)
    axes = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float)
    bodies = [dict(offs=W.sphere_beads(2.0, 24), mass=40.0, inertia=(40.0, 45.0, 50.0),
                   centre=np.array([5.3, 6.1, 3.3]), vel=(0.002, -0.001, 0.0005),
                   omega=(0.004, -0.003, 0.005), gamma=W.GAMMA_FREE, ev=(1.0 * axes, 0.8)),
              dict(offs=W.sphere_beads(1.5, 12), mass=15.0, inertia=(8.0, 9.0, 10.0),
                   centre=np.array([8.8, 6.1, 3.3]), vel=(-0.001, 0.0005, 0.0),
                   omega=(-0.002, 0.004, 0.001), gamma=W.GAMMA_FREE, ev=(0.8 * axes, 0.8))]
    gx, gy = np.meshgrid(np.arange(14) + 0.5, np.arange(13) + 0.5, indexing="ij")
    walls = np.stack([gx.ravel(), gy.ravel(), np.full(gx.size, 1.0)], axis=1)
    return shape, params, bodies, walls


def _run_wca(shape, params, bodies, walls, steps, weights, adjoint=False, pairs=None):
    sim = po.OracleSim(shape, params)
    for j, b in enumerate(bodies):
        sim.add_body(b["offs"], b["mass"], b["inertia"], b["centre"], vel=b["vel"],
                     omega=b["omega"], gamma=b["gamma"])
        sim.set_excluded_volume(j, *b["ev"])
    sim.add_wall_sites(walls, 0.5)
    if adjoint:
        return sim.adjoint(steps, weights)
    J = 0.0
    for n in range(steps):
        sim.step(1)
        st = [sim.body_state(j) for j in range(len(bodies))]
        for j in range(len(bodies)):
            J += float(weights[n, j] @ st[j]["force"])
        if pairs is not None:
            pairs.append(st)
    return J


@pytest.mark.parametrize("md", [1, 2])
def test_excluded_volume_window_gradient_matches_finite_difference(md):
    """The reverse pass through the WCA pair forces (body-body and body-pore-bead pairs, whose
    Jacobian moves both partners' positions and rotations) against central differences of
    the forward oracle; no pair distance comes near the cutoff during the window."""
    from scipy.spatial.transform import Rotation
    shape, params, bodies, walls = _wca_case()
    params.md_substeps = md
    steps = 12
    rng = np.random.default_rng(29)
    weights = np.zeros((steps, 2, 3))
    weights[:, 0, 0] = 1.0 / steps
    weights += 0.02 * rng.standard_normal(weights.shape)
    J, dg, do = _run_wca(shape, params, bodies, walls, steps, weights, adjoint=True)
    states = []
    assert abs(J - _run_wca(shape, params, bodies, walls, steps, weights, pairs=states)) < 1e-15
    # WCA pairs are active, and none within 1e-3 of the cutoff, at the end of every step
    cut = 2.0 ** (1.0 / 6.0)
    active, margin = 0, 1.0
    for st in states:
        sites = []
        for j, b in enumerate(bodies):
            q = st[j]["quat"]
            Rm = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
            sites.append(st[j]["pos"] + b["ev"][0] @ Rm.T)
        for x in sites[0]:
            for y, sig in [(y, 1.6) for y in sites[1]] + [(w, 1.3) for w in walls]:
                d = x - y
                d -= np.array(shape) * np.round(d / np.array(shape))
                r = np.linalg.norm(d)
                margin = min(margin, abs(r - cut * sig))
                active += r < cut * sig
        for y in sites[1]:
            for w in walls:
                d = y - w
                d -= np.array(shape) * np.round(d / np.array(shape))
                r = np.linalg.norm(d)
                margin = min(margin, abs(r - cut * 1.3))
                active += r < cut * 1.3
    assert active >= 2 * steps and margin > 1e-3, (active, margin)
    h = 1e-6
    for b in range(2):
        bp = [dict(x) for x in bodies]
        bm = [dict(x) for x in bodies]
        bp[b]["gamma"] += h
        bm[b]["gamma"] -= h
        fd = (_run_wca(shape, params, bp, walls, steps, weights)
              - _run_wca(shape, params, bm, walls, steps, weights)) / (2 * h)
        # relative to the larger of the two: the small body's derivative (~1e-5 of J's scale)
        # sits near the rounding noise of J divided by 2h
        assert abs(fd - dg[b]) < 1e-6 * np.abs(dg).max() + 1e-12, (b, fd, dg[b])
    scale = np.abs(do).max()
    n0 = len(bodies[0]["offs"])
    for k in (0, 7, 19, n0 + 3, n0 + 8):
        b, kk = (0, k) if k < n0 else (1, k - n0)
        for a in range(3):
            bp = [dict(x) for x in bodies]
            bm = [dict(x) for x in bodies]
            bp[b]["offs"] = bodies[b]["offs"].copy()
            bm[b]["offs"] = bodies[b]["offs"].copy()
            bp[b]["offs"][kk, a] += h
            bm[b]["offs"][kk, a] -= h
            fd = (_run_wca(shape, params, bp, walls, steps, weights)
                  - _run_wca(shape, params, bm, walls, steps, weights)) / (2 * h)
            assert abs(fd - do[k, a]) < 1e-5 * scale + 1e-13, (k, a, fd, do[k, a])
