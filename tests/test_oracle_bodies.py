"""Pins of the oracle's bead coupling and rigid-body update.

- Trilinear stencil: weights sum to 1, reproduce affine fields exactly (periodic unwrap),
  reduce to a single node at node centres.
- Friction special case: a fixed bead in a uniform flow u0 feels F = gamma u0 at step 0 and
  the fluid loses exactly that momentum.
- Quaternion and torque convention against scipy's Rotation (independent implementation):
  the body-frame torque of a fixed body is R(q)^T (R(q) b x F).
- Free rigid motion (gamma = 0): straight-line drift, exact rotation of an isotropic body
  q(n) = q0 (x) exp(w n / 2), and the torque-free precession of a symmetric top in the body
  frame at rate (I3 - I1) w3 / I1 (to the O(dt^2) accuracy of the splitting).
- The friction as specified, gamma = 20 at rho0 = 1, diverges (recorded decision).
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import pyoracle as po
from paper_1604_01829_amd import workloads as W


def _node_centre(idx, shape):
    nx, ny, nz = shape
    return np.array([idx % nx, (idx // nx) % ny, idx // (nx * ny)], dtype=float) + 0.5


def test_trilinear_affine_and_partition():
    rng = np.random.default_rng(5)
    shape = (7, 5, 9)
    L = np.array(shape, dtype=float)
    for _ in range(200):
        r = rng.uniform(-20, 30, size=3)
        idx, w = po.trilinear(shape, r)
        assert abs(w.sum() - 1.0) < 1e-15
        assert np.all(w >= 0)
        # unwrap the corner centres next to r and check the first moment
        cen = np.array([_node_centre(i, shape) for i in idx])
        cen = cen + L * np.round((r - cen) / L)
        assert np.abs(w @ cen - r).max() < 1e-12
        # an affine field is reproduced exactly
        A = rng.standard_normal((3, 3))
        b = rng.standard_normal(3)
        assert np.abs(w @ (cen @ A.T + b) - (A @ r + b)).max() < 1e-11


def test_trilinear_at_node_centre():
    shape = (4, 4, 4)
    idx, w = po.trilinear(shape, (2.5, 1.5, 3.5))
    assert np.isclose(w.max(), 1.0) and np.isclose(np.sort(w)[-2], 0.0)
    assert idx[np.argmax(w)] == 2 + 4 * (1 + 4 * 3)


def test_friction_in_uniform_flow():
    u0 = np.array([0.01, -0.02, 0.005])
    gamma = 0.7
    shape = (6, 5, 4)
    p = po.make_params(u0=u0)
    sim = po.OracleSim(shape, p)
    r = np.array([2.3, 1.9, 3.1])
    sim.add_body([[0.0, 0.0, 0.0]], 1.0, [1, 1, 1], r, gamma=gamma, fixed=True)
    j0 = sim.totals()["momentum"]
    sim.step(1)
    F = sim.bead_forces(0)[0]
    assert np.abs(F - gamma * u0).max() < 1e-17
    st = sim.body_state(0)
    assert np.abs(st["force"] - gamma * u0).max() < 1e-17
    assert np.abs(st["torque"]).max() < 1e-18
    assert np.abs(sim.totals()["momentum"] - (j0 - F)).max() < 1e-14


def test_torque_and_quaternion_convention():
    rng = np.random.default_rng(8)
    u0 = np.array([0.003, 0.011, -0.007])
    gamma = 0.4
    for _ in range(5):
        q = W.random_quaternion(rng)
        b = rng.uniform(-1.5, 1.5, size=3)
        sim = po.OracleSim((8, 8, 8), po.make_params(u0=u0))
        sim.add_body([b], 1.0, [1, 1, 1], (4.2, 3.7, 4.9), quat=q, gamma=gamma, fixed=True)
        sim.step(1)
        Rm = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        F = gamma * u0
        T_lab = np.cross(Rm @ b, F)
        st = sim.body_state(0)
        assert np.abs(st["torque"] - Rm.T @ T_lab).max() < 1e-15
        assert np.abs(st["quat"] - q / np.linalg.norm(q)).max() < 1e-15


def _free_body_sim(inertia, omega, vel=(0.0, 0.0, 0.0), q0=(1.0, 0.0, 0.0, 0.0)):
    sim = po.OracleSim((8, 8, 8), po.make_params())
    sim.add_body(W.sphere_beads(2.0, 20), 3.0, inertia, (4.0, 4.0, 4.0), quat=q0, vel=vel,
                 omega=omega, gamma=0.0)
    return sim


def test_free_drift_and_isotropic_rotation():
    q0 = np.array([0.8, 0.2, -0.4, 0.4])
    q0 /= np.linalg.norm(q0)
    w = np.array([0.013, -0.021, 0.008])
    v = np.array([0.01, 0.02, -0.03])
    sim = _free_body_sim([2.0, 2.0, 2.0], w, vel=v, q0=q0)
    n = 250
    sim.step(n)
    st = sim.body_state(0)
    assert np.abs(st["pos"] - (np.array([4.0, 4.0, 4.0]) + n * v)).max() < 1e-12
    assert np.abs(st["vel"] - v).max() < 1e-18
    assert np.abs(st["omega"] - w).max() < 1e-18
    want = Rotation.from_quat([q0[1], q0[2], q0[3], q0[0]]) * Rotation.from_rotvec(w * n)
    wq = want.as_quat()
    got = st["quat"]
    sign = np.sign(got[0] * wq[3]) or 1.0
    assert np.abs(got - sign * np.array([wq[3], wq[0], wq[1], wq[2]])).max() < 1e-12


def test_symmetric_top_precession():
    I1, I3 = 2.0, 3.0
    w0 = np.array([0.01, 0.0, 0.02])
    sim = _free_body_sim([I1, I1, I3], w0)
    Omega = (I3 - I1) * w0[2] / I1
    for n in (100, 300):
        sim.step(n - sim.step_count)
        w = sim.body_state(0)["omega"]
        phase = math.atan2(w[1], w[0])
        # Euler's equations: d(w1, w2)/dt = Omega (-w2, w1), a rotation about e3 by +Omega t.
        # Two explicit half kicks per step rotate by 2 atan(Omega/2) and stretch by
        # (1 + Omega^2/4) per step -- exactly, since w3 stays constant for I1 = I2 ...
        d = (phase - 2 * n * math.atan(Omega / 2) + math.pi) % (2 * math.pi) - math.pi
        assert abs(d) < 1e-12
        assert abs(math.hypot(w[0], w[1]) - w0[0] * (1 + Omega ** 2 / 4) ** n) < 1e-15
        assert w[2] == w0[2]
        # ... which is the continuous precession up to O(dt^2) per unit time
        d = (phase - Omega * n + math.pi) % (2 * math.pi) - math.pi
        assert abs(d) < Omega ** 3 * n / 12 * 1.01


def test_gamma_as_specified_diverges():
    """The workloads were specified with gamma = 20; the explicit scheme cannot run it."""
    wl = W.workload(1, gamma=W.GAMMA_AS_SPECIFIED)
    rep = wl["replicas"][0]
    b = rep["bodies"][0]
    p = po.make_params(g_ext=wl["params"]["g_ext"])
    sim = po.OracleSim(rep["shape"], p)
    sim.add_body(b["offsets"], b["mass"], b["inertia"], b["pos"], gamma=b["gamma"])
    sim.step(50)
    t = sim.totals()
    assert (not t["finite"]) or abs(t["mass"] - 32768) > 1.0
    # ... while the paper's low friction used instead stays finite and conserves mass
    wl = W.workload(1)
    b = wl["replicas"][0]["bodies"][0]
    sim = po.OracleSim(rep["shape"], p)
    sim.add_body(b["offsets"], b["mass"], b["inertia"], b["pos"], gamma=b["gamma"])
    sim.step(50)
    t = sim.totals()
    assert t["finite"] and abs(t["mass"] - 32768) < 1e-9
