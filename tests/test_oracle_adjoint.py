"""Pins of the oracle's reverse-mode derivative against central finite differences.

- the collision's vector-Jacobian product against a central difference of the collision
  itself along a random direction (both population and force inputs);
- the whole-window gradient of J = sum_n a(n) . F_b(n) with respect to the bead friction and
  to individual bead offsets, against central differences of J computed by re-running the
  forward oracle, in a periodic box and in a pore with bounce-back walls.  Beads are chosen
  away from cell faces so that the finite difference does not cross a kink of the
  trilinear weights.
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
