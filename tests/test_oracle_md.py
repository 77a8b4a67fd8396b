"""Pins of the oracle's MD sub-stepping and WCA excluded volume.

- WCA pair (the textbook repulsive Lennard-Jones, sigma = r_a + r_b): energy eps at r = sigma,
  energy and force both zero at the cut 2^(1/6) sigma (the minimum of the full potential),
  zero beyond, force = -dU/dr, minimum image across the periodic box;
- whole-body WCA forces and torques are minus the gradients of the WCA energy with respect to
  the centre and to a rotation; body-body forces obey Newton's third law (total force and
  angular momentum change zero);
- sub-stepping: free drift and free isotropic rotation stay exact with m MD steps per fluid
  step; the bead noise of MD step k has amplitude sqrt(2 kT gamma m) per component and its
  own Philox counter block k; Sum j + Sum_b (M V + h F/2) grows by N_fluid g_ext per fluid
  step (the fluid receives -h F per MD step); with no fluid coupling, velocity Verlet
  conserves the energy with an error of second order in h.
"""
import math

import numpy as np
import pytest

from oracle import pyoracle as po
from paper_1604_01829_amd import workloads as W

EPS = 0.01


def _box(shape=(20, 20, 20), **kw):
    kw.setdefault("wca_epsilon", EPS)
    return po.OracleSim(shape, po.make_params(**kw))


def _one_site_energy_force(r, ra=0.5, rb=1.75, axis=np.array([0.6, -0.48, 0.64])):
    s = _box()
    p = np.array([10.2, 9.7, 10.1])
    s.add_body([[0.0, 0.0, 0.0]], 1.0, (1, 1, 1), p, gamma=0.0, fixed=True)
    s.set_excluded_volume(0, [[0.0, 0.0, 0.0]], ra)
    n = axis / np.linalg.norm(axis)
    s.add_wall_sites([p + r * n], rb)
    return s.wca_energy(), s.wca_forces()[0, :3], n


def test_wca_pair_properties():
    sigma = 0.5 + 1.75
    rc = 2 ** (1 / 6) * sigma
    U, F, n = _one_site_energy_force(sigma)
    assert abs(U - EPS) < 1e-15
    # the force pushes the site away from the wall site, along the line of centres
    assert np.dot(F, n) < 0 and np.linalg.norm(np.cross(F, n)) < 1e-15 * np.linalg.norm(F)
    # energy and force vanish continuously at the cut (the minimum of the full potential)
    for r in (rc * (1 - 1e-7), rc * (1 + 1e-9), 1.3 * sigma):
        U, F, _ = _one_site_energy_force(r)
        assert 0.0 <= U < 1e-12 * EPS and np.linalg.norm(F) < 1e-5 * EPS
    # repulsive and decreasing inside the cut; force = -dU/dr
    prev = math.inf
    for r in np.linspace(0.85 * sigma, 0.999 * rc, 9):
        U, F, n = _one_site_energy_force(r)
        assert 0 < U < prev
        prev = U
        d = 1e-6 * sigma
        Up, _, _ = _one_site_energy_force(r + d)
        Um, _, _ = _one_site_energy_force(r - d)
        assert abs(-np.dot(F, n) - (-(Up - Um) / (2 * d))) < 1e-7 * np.linalg.norm(F)
    # the pair depends on r / sigma only: doubling both radii and r scales U by 1, F by 1/2
    U1, F1, _ = _one_site_energy_force(0.95 * sigma)
    U2, F2, _ = _one_site_energy_force(2 * 0.95 * sigma, ra=1.0, rb=3.5)
    assert abs(U2 - U1) < 1e-15 and np.allclose(F2, 0.5 * F1, rtol=1e-13, atol=0)


def test_wca_minimum_image():
    s = _box()
    s.add_body([[0.0, 0.0, 0.0]], 1.0, (1, 1, 1), (0.4, 10.0, 19.8), gamma=0.0, fixed=True)
    s.set_excluded_volume(0, [[0.0, 0.0, 0.0]], 0.5)
    s.add_wall_sites([[19.9, 10.3, 0.1]], 0.5)    # (0.5, -0.3, -0.3) away through two faces
    t = _box()
    t.add_body([[0.0, 0.0, 0.0]], 1.0, (1, 1, 1), (10.4, 10.0, 9.8), gamma=0.0, fixed=True)
    t.set_excluded_volume(0, [[0.0, 0.0, 0.0]], 0.5)
    t.add_wall_sites([[9.9, 10.3, 10.1]], 0.5)
    assert s.wca_energy() > 0
    assert abs(s.wca_energy() / t.wca_energy() - 1) < 1e-12
    assert np.allclose(s.wca_forces(), t.wca_forces(), rtol=1e-12, atol=1e-18)


def _pair_scene(pos_a=(8.0, 10.0, 10.0), quat_a=(0.9, 0.2, -0.1, 0.3), dtheta=None,
                dpos=None, walls=True):
    """Two bodies whose inner layers overlap, and a few wall sites near the first."""
    s = _box()
    ev = W.sphere_beads(2.0, 60, centre_bead=False)
    qa = np.array(quat_a, float)
    qa /= np.linalg.norm(qa)
    pa = np.array(pos_a, float)
    if dpos is not None:
        pa = pa + dpos
    if dtheta is not None:     # rotate body a by a small lab-frame angle
        ax, ang = dtheta
        dq = np.array([math.cos(ang / 2), *(math.sin(ang / 2) * np.eye(3)[ax])])
        w1, x1, y1, z1 = dq
        w2, x2, y2, z2 = qa
        qa = np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                       w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])
    s.add_body([[0.0, 0.0, 0.0]], 30.0, (50, 50, 50), pa, quat=qa, gamma=0.0, fixed=True)
    s.add_body([[0.0, 0.0, 0.0]], 30.0, (50, 50, 50), (11.7, 10.6, 10.3),
               quat=(0.7, -0.3, 0.5, 0.1), gamma=0.0, fixed=True)
    s.set_excluded_volume(0, ev, 0.5)
    s.set_excluded_volume(1, ev * 1.1, 0.6)
    if walls:
        s.add_wall_sites([[5.5, 10.2, 10.0], [6.0, 8.4, 11.5], [6.2, 11.0, 8.2]], 0.75)
    return s


def test_wca_forces_and_torques_are_gradients():
    s = _pair_scene()
    F = s.wca_forces()
    assert np.linalg.norm(F[0, :3]) > 1e-3 * EPS       # the scene interacts
    d = 1e-6
    for ax in range(3):
        e = np.eye(3)[ax] * d
        dU = (_pair_scene(dpos=e).wca_energy() - _pair_scene(dpos=-e).wca_energy()) / (2 * d)
        assert abs(F[0, ax] + dU) < 1e-6 * np.linalg.norm(F[0, :3])
        dU = (_pair_scene(dtheta=(ax, d)).wca_energy() -
              _pair_scene(dtheta=(ax, -d)).wca_energy()) / (2 * d)
        assert abs(F[0, 3 + ax] + dU) < 1e-6 * np.linalg.norm(F[0, 3:])


def test_wca_newtons_third_law():
    s = _pair_scene(walls=False)
    F = s.wca_forces()
    scale = np.abs(F).max()
    assert scale > 0
    assert np.abs(F[0, :3] + F[1, :3]).max() < 1e-13 * scale
    # angular momentum: sum of R x F + torque about the centres vanishes
    R = [np.array([8.0, 10.0, 10.0]), np.array([11.7, 10.6, 10.3])]
    L = sum(np.cross(R[b], F[b, :3]) + F[b, 3:] for b in range(2))
    assert np.abs(L).max() < 1e-12 * scale * 12


@pytest.mark.parametrize("m", [2, 3])
def test_substeps_keep_free_motion_exact(m):
    s = po.OracleSim((12, 12, 12), po.make_params(md_substeps=m))
    v = np.array([0.013, -0.007, 0.002])
    w = np.array([0.02, -0.01, 0.015])
    s.add_body([[0.0, 0.0, 0.0]], 2.0, (3.0, 3.0, 3.0), (5.0, 6.0, 7.0), vel=v, omega=w,
               gamma=0.0)
    T = 37
    s.step(T)
    st = s.body_state(0)
    assert np.abs(st["pos"] - (np.array([5.0, 6.0, 7.0]) + v * T)).max() < 1e-12
    ang = np.linalg.norm(w) * T
    q = np.array([math.cos(ang / 2), *(math.sin(ang / 2) * w / np.linalg.norm(w))])
    assert np.abs(st["quat"] - q).max() < 1e-12 and np.abs(st["omega"] - w).max() < 1e-15


@pytest.mark.parametrize("m", [1, 2, 3])
def test_substep_bead_noise_amplitude_and_keying(m):
    kT, gamma, seed = 2e-5, 0.4, 0x5EED1234ABCD
    u0 = np.array([0.003, -0.002, 0.001])
    s = po.OracleSim((8, 8, 8), po.make_params(kT=kT, u0=u0, seed=seed, md_substeps=m))
    offs = np.array([[0.3, 0.1, -0.2], [1.1, -0.4, 0.6], [-0.7, 0.2, 0.9]])
    s.add_body(offs, 1.0, (1, 1, 1), (4.2, 3.9, 4.4), gamma=gamma, fixed=True)
    s.step(1)
    got = s.bead_forces(0)
    amp = math.sqrt(2 * kT * gamma * m) * math.sqrt(12)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for k in range(3):
        # the last MD step of fluid step 0 is k_md = m - 1: counter (0, bead, (1 << 16) | k_md, 0)
        w = po.philox([0, k, (1 << 16) | (m - 1), 0], key)
        halves = [w[0] & 0xFFFF, w[0] >> 16, w[1] & 0xFFFF]
        expect = gamma * u0 + amp * np.array([po.uniform16(h) for h in halves])
        assert np.abs(got[k] - expect).max() < 1e-15
    assert np.abs(s.body_state(0)["force"] - got.sum(0)).max() < 1e-15


def test_substep_momentum_bookkeeping():
    """Thermal fluid, two free bodies pushing each other through their inner layers, two MD
    steps per fluid step: Sum j + Sum_b (M V + h F/2) grows by N_fluid g_ext per step."""
    m = 2
    g = np.array([2e-6, -1e-6, 5e-7])
    s = po.OracleSim((14, 12, 12), po.make_params(kT=3e-5, seed=77, g_ext=g, md_substeps=m,
                                                  wca_epsilon=EPS, tau_shear=0.9))
    ev = W.sphere_beads(2.0, 50, centre_bead=False)
    sh = W.sphere_beads(2.5, 70)
    s.add_body(sh, 60.0, (150, 150, 150), (4.0, 6.0, 6.0), vel=(0.004, 0, 0), gamma=0.3)
    s.add_body(sh, 60.0, (150, 150, 150), (8.8, 6.4, 6.2), vel=(-0.004, 0, 0), gamma=0.3)
    s.set_excluded_volume(0, ev, 0.5)
    s.set_excluded_volume(1, ev, 0.5)
    assert np.linalg.norm(s.wca_forces()[:, :3]) > 0        # the layers overlap from the start

    def books():
        t = s.totals()
        tot = t["momentum"].copy()
        for b in range(2):
            st = s.body_state(b)
            tot += 60.0 * st["vel"] + 0.5 * st["force"] / m
        return tot

    n_fluid = 14 * 12 * 12
    start = books()
    for k in range(1, 9):
        s.step(1)
        assert np.abs(books() - (start + k * n_fluid * g)).max() < 1e-13


def _collision_energy_drift(m, steps=70):
    """Two spheres colliding through their inner layers, no fluid coupling (gamma = 0):
    max |E(t) - E(0)| over the run, E = kinetic + rotational + WCA energy."""
    s = po.OracleSim((24, 14, 14), po.make_params(md_substeps=m, wca_epsilon=EPS))
    ev = W.sphere_beads(2.0, 60, centre_bead=False)
    M, I = 30.0, 45.0
    s.add_body([[0.0, 0.0, 0.0]], M, (I, I, I), (6.0, 7.0, 7.0), vel=(0.03, 0, 0), gamma=0.0)
    s.add_body([[0.0, 0.0, 0.0]], M, (I, I, I), (12.5, 7.9, 7.3), vel=(-0.03, 0, 0), gamma=0.0)
    s.set_excluded_volume(0, ev, 0.5)
    s.set_excluded_volume(1, ev, 0.5)

    def energy():
        e = s.wca_energy()
        for b in range(2):
            st = s.body_state(b)
            e += 0.5 * M * st["vel"] @ st["vel"] + 0.5 * I * st["omega"] @ st["omega"]
        return e

    e0 = energy()
    drift = 0.0
    touched = False
    for _ in range(steps):
        s.step(1)
        drift = max(drift, abs(energy() - e0))
        touched = touched or s.wca_energy() > 0
    assert touched
    # the bodies separated again and spin: the collision was off-centre
    assert s.wca_energy() == 0 and np.linalg.norm(s.body_state(0)["omega"]) > 0
    return drift, e0


def test_substeps_conserve_energy_to_second_order():
    d1, e0 = _collision_energy_drift(1)
    d2, _ = _collision_energy_drift(2)
    d4, _ = _collision_energy_drift(4)
    assert d1 < 0.05 * e0
    assert 3.0 < d1 / d2 < 5.0 and 3.0 < d2 / d4 < 5.0
