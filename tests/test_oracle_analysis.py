"""Pins of the oracle's trajectory analysis (oracle/analysis.py).

- the rotation matrix of a quaternion equals scipy's; the matrix as printed in the paper (sign
  of its (1,3) entry) is not orthogonal, which is why the reading replaces it;
- MSD: ballistic motion gives |v|^2 tau^2 exactly; brute force on a tiny input;
- body frame: a screw motion built from body-frame steps (each turned into the lab frame with
  the orientation at the start of its interval) gives back n v_b exactly; per-interval lengths
  are kept;
- projection angles: a rotation about one body axis by theta per interval gives -theta about
  that axis and zero about the others (the printed formulas' sign); a small general rotation
  gives minus its body-frame rotation vector to first order; for isotropic rotational
  diffusion the lab-frame and body-frame estimates of the paper's formulas agree (the purpose
  of its 3/2 factor), both at 2/3 of the generating D_r;
- lab rotation: a rotation about a fixed lab axis normal to the reference vector by theta per
  interval gives Delta Theta = tau theta;
- pore frame: radial, tangential (circle) and axial motion go to x^p, y^p, z^p with the chord
  of the circle in closed form;
- binned MSD: brute force on a tiny input; fits exact on exact data.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation as Rot

from oracle import analysis as A


def _wxyz(r):
    q = r.as_quat()
    return np.array([q[3], q[0], q[1], q[2]])


def _traj_from(rots, pos):
    F = len(rots)
    t = np.zeros((F, 1, 7))
    t[:, 0, :3] = pos
    t[:, 0, 3:] = [_wxyz(r) for r in rots]
    return t


def test_quaternion_matrix_matches_scipy():
    rng = np.random.default_rng(0)
    for _ in range(20):
        r = Rot.from_quat(rng.normal(size=4))
        assert np.abs(A.quat_matrix(_wxyz(r)) - r.as_matrix()).max() < 1e-15
    # the printed matrix differs in the sign of the y w term of its (1,3) entry
    w, x, y, z = _wxyz(Rot.from_quat(rng.normal(size=4)))
    printed = np.array([[1 - 2 * y * y - 2 * z * z, 2 * x * y - 2 * z * w, 2 * x * z - 2 * y * w],
                        [2 * x * y + 2 * z * w, 1 - 2 * x * x - 2 * z * z, 2 * y * z - 2 * x * w],
                        [2 * x * z - 2 * y * w, 2 * y * z + 2 * x * w, 1 - 2 * x * x - 2 * y * y]])
    assert np.abs(printed @ printed.T - np.eye(3)).max() > 1e-3


def test_msd_ballistic_and_brute_force():
    v = np.array([0.3, -0.1, 0.05])
    s = (np.arange(40)[:, None] * v)[:, None, :]
    m = A.msd(s, 6)
    for tau in range(1, 7):
        assert np.abs(m[0, tau - 1] - (v * tau) ** 2).max() < 1e-14 * (v * tau).dot(v * tau)
    rng = np.random.default_rng(1)
    s = rng.normal(size=(7, 2, 3))
    m = A.msd(s, 4)
    for b in range(2):
        for tau in range(1, 5):
            pairs = [(t, t + tau) for t in range(7 - tau)]
            ref = sum((s[j, b] - s[i, b]) ** 2 for i, j in pairs) / len(pairs)
            assert np.abs(m[b, tau - 1] - ref).max() < 1e-15


def test_body_frame_translation_of_a_screw_motion():
    vb = np.array([0.07, -0.02, 0.03])
    step = Rot.from_rotvec([0.2, -0.1, 0.15])
    rots = [Rot.from_rotvec([0.3, 0.5, -0.2])]
    pos = [np.array([1.0, 2.0, 3.0])]
    for _ in range(30):
        pos.append(pos[-1] + rots[-1].as_matrix() @ vb)     # orientation at the interval start
        rots.append(rots[-1] * step)                         # body-frame increment
    t = _traj_from(rots, np.array(pos))
    xb = A.body_frame_translation(t)
    assert np.abs(xb[:, 0] - np.arange(31)[:, None] * vb).max() < 1e-13
    d = np.diff(t[:, 0, :3], axis=0)
    assert np.abs(np.linalg.norm(np.diff(xb[:, 0], axis=0), axis=1) -
                  np.linalg.norm(d, axis=1)).max() < 1e-15


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_projection_angles_of_a_rotation_about_one_body_axis(axis):
    th = 0.05
    r0 = Rot.from_rotvec([0.4, -0.7, 0.2])
    rots = [r0 * Rot.from_rotvec(np.eye(3)[axis] * th * n) for n in range(12)]
    ang = A.body_frame_rotation(_traj_from(rots, np.zeros((12, 3))))
    expect = np.zeros(3)
    expect[axis] = -th
    assert np.abs(np.diff(ang[:, 0], axis=0) - expect).max() < 1e-14


def test_projection_angles_of_a_small_general_rotation():
    r0 = Rot.from_rotvec([0.4, -0.7, 0.2])
    w = np.array([3e-3, -2e-3, 1e-3])
    ang = A.body_frame_rotation(_traj_from([r0, r0 * Rot.from_rotvec(w)], np.zeros((2, 3))))
    assert np.abs(ang[1, 0] + w).max() < 2 * np.dot(w, w)


def test_lab_and_body_rotation_estimates_agree_for_isotropic_diffusion():
    rng = np.random.default_rng(1)
    F, Dr = 20000, 1e-3
    r = Rot.identity()
    rots = []
    for _ in range(F):
        rots.append(r)
        r = r * Rot.from_rotvec(rng.normal(0, math.sqrt(2 * Dr), 3))
    t = _traj_from(rots, np.zeros((F, 3)))
    lags = np.arange(1, 11)
    dl = A.diffusivity(lags, A.rotation_msd(t, [[1.0, 0, 0]], 10)[0], 6)
    mb = A.msd(A.body_frame_rotation(t), 10)[0]
    db = [A.diffusivity(lags, mb[:, c], 3) for c in range(3)]
    for d in db:
        assert abs(d / dl - 1) < 0.05
    assert abs(dl / (2 * Dr / 3) - 1) < 0.05


def test_lab_rotation_about_a_fixed_axis():
    th = 0.07
    rots = [Rot.from_rotvec([0, 0, th * n]) * Rot.from_rotvec([0.3, 0.2, -0.1]) for n in range(30)]
    t = _traj_from(rots, np.zeros((30, 3)))
    # reference vector whose lab image lies in the plane normal to the lab z axis
    ref = Rot.from_rotvec([0.3, 0.2, -0.1]).inv().apply([1.0, 0.0, 0.0])
    m = A.rotation_msd(t, [ref], 8)[0]
    assert np.abs(m - (np.arange(1, 9) * th) ** 2).max() < 1e-12


def test_pore_frame_radial_tangential_axial():
    c = (20.0, 20.0)
    F = 25
    phi0, r0 = 0.7, 5.0
    # radial
    rr = r0 + 0.1 * np.arange(F)
    pos = np.stack([c[0] + rr * math.cos(phi0), c[1] + rr * math.sin(phi0), np.full(F, 3.0)], 1)
    xp, rad = A.pore_frame(pos[:, None, :], c)
    assert np.abs(xp[:, 0, 0] - 0.1 * np.arange(F)).max() < 1e-13
    assert np.abs(xp[:, 0, 1:]).max() < 1e-13 and np.abs(rad[:, 0] - rr).max() < 1e-13
    # tangential: steps of dphi on a circle: chord (r (cos dphi - 1), r sin dphi) per step
    dphi = 0.03
    ph = phi0 + dphi * np.arange(F)
    pos = np.stack([c[0] + r0 * np.cos(ph), c[1] + r0 * np.sin(ph), np.full(F, 3.0)], 1)
    xp, _ = A.pore_frame(pos[:, None, :], c)
    n = np.arange(F)
    assert np.abs(xp[:, 0, 0] - n * r0 * (math.cos(dphi) - 1)).max() < 1e-12
    assert np.abs(xp[:, 0, 1] - n * r0 * math.sin(dphi)).max() < 1e-12
    # axial
    pos = np.stack([np.full(F, c[0] + 2.0), np.full(F, c[1] - 1.0), 0.2 * n], 1)
    xp, _ = A.pore_frame(pos[:, None, :], c)
    assert np.abs(xp[:, 0, 2] - 0.2 * n).max() < 1e-13 and np.abs(xp[:, 0, :2]).max() < 1e-15


def test_binned_msd_brute_force():
    rng = np.random.default_rng(4)
    s = rng.normal(size=(9, 2, 3))
    r = rng.uniform(0, 3, size=(9, 2))
    edges = [0.0, 1.0, 2.0, 3.0]
    sums, counts = A.binned_msd(s, r, edges, 3)
    for k in range(3):
        for tau in range(1, 4):
            acc, cnt = np.zeros(3), 0
            for b in range(2):
                for t in range(9 - tau):
                    if edges[k] <= r[t, b] < edges[k + 1]:
                        acc += (s[t + tau, b] - s[t, b]) ** 2
                        cnt += 1
            assert cnt == counts[k, tau - 1] and np.abs(sums[k, tau - 1] - acc).max() < 1e-14


def test_fits_are_exact_on_exact_data():
    t = np.arange(1, 26) * 200.0
    assert abs(A.diffusivity(t, 6 * 0.0123 * t + 0.5, 6) - 0.0123) < 1e-15
    L = np.array([27.0, 32, 38, 48, 55, 64, 76, 94])
    d0, c = A.hasimoto_d0(L, 0.02 - 0.3 / L)
    assert abs(d0 - 0.02) < 1e-15 and abs(c - 0.3) < 1e-13
    assert A.einstein_resistance(4e-5, d0) == 4e-5 / d0
