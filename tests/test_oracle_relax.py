"""Pins of the oracle's raspberry construction (oracle/orc_relax.c).

- closest point on an ellipsoid: on a sphere it is R x/|x| (inside and outside); a point on the
  surface is its own closest point; on an ellipsoid the result lies on the surface, x - r_s is
  along the surface normal there, and no point of a dense parametric sampling of the surface
  is closer; the equation as printed (with "+1" inside the squares) has a root whose point is
  not on the surface;
- relaxation: 2, 4 and 6 beads on a sphere end antipodal, as a regular tetrahedron and as a
  regular octahedron; from a jittered start at rest the energy (WCA + restraint) of 100 beads
  on a sphere decreases and they end on the surface with nearly equal nearest-neighbour
  distances.
"""
import math

import numpy as np
import pytest

from oracle import pyoracle as po


@pytest.mark.parametrize("x", [(1.0, 2.0, 2.0), (0.3, -0.2, 0.1), (5.0, -4.0, 2.5)])
def test_closest_point_on_a_sphere(x):
    R = 3.0
    x = np.array(x)
    rs, _ = po.closest_point((R, R, R), x)
    assert np.abs(rs - R * x / np.linalg.norm(x)).max() < 1e-13 * R


def test_closest_point_on_the_surface_is_itself():
    a = np.array([4.0, 2.0, 1.5])
    rng = np.random.default_rng(2)
    for _ in range(10):
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        p = a * u / np.linalg.norm(u)          # (x/a)^2 sum = |u|^2 = 1
        rs, t = po.closest_point(a, p)
        assert np.abs(rs - p).max() < 1e-12 and abs(t) < 1e-10


def test_closest_point_on_an_ellipsoid():
    a = np.array([4.0, 2.0, 1.5])
    rng = np.random.default_rng(3)
    th = np.linspace(0.0, math.pi, 721)
    ph = np.linspace(0.0, 2.0 * math.pi, 1441)
    T, P = np.meshgrid(th, ph, indexing="ij")
    surf = np.stack([a[0] * np.sin(T) * np.cos(P), a[1] * np.sin(T) * np.sin(P),
                     a[2] * np.cos(T)], axis=-1).reshape(-1, 3)
    for _ in range(8):
        x = rng.normal(size=3) * np.array([5.0, 3.0, 2.0])
        rs, t = po.closest_point(a, x)
        assert abs(((rs / a) ** 2).sum() - 1.0) < 1e-12
        n = rs / a ** 2                          # grad S / 2
        d = x - rs
        assert np.linalg.norm(np.cross(d, n)) <= 1e-10 * max(np.linalg.norm(d), 1e-12) * np.linalg.norm(n)
        best = np.linalg.norm(surf - x, axis=1).min()
        assert np.linalg.norm(d) <= best + 1e-12
        assert best - np.linalg.norm(d) < 5e-3       # the sampling comes close to it
    # the equation as printed, sum((x a/(t + a^2) + 1)^2) - 1 = 0, solved the same way, does
    # not give a point on the surface
    x = np.array([5.0, 1.0, 0.5])
    f = lambda t: (((x * a / (t + a * a)) + 1.0) ** 2).sum() - 1.0
    lo, hi = -(a * a).min(), 1e4
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if f(mid) > 0 else (lo, mid)
    rs_printed = x * a * a / (0.5 * (lo + hi) + a * a)
    assert abs(((rs_printed / a) ** 2).sum() - 1.0) > 1e-2


def _relax(n, R, steps, seed=0, **kw):
    rng = np.random.default_rng(seed)
    u = rng.normal(size=(n, 3))
    pos = R * u / np.linalg.norm(u, axis=1, keepdims=True)
    p = po.relax_params(**kw)
    return po.relax_shell((R, R, R), pos, np.zeros_like(pos), p, steps)[0], p


def _pair_dists(x):
    return np.array([np.linalg.norm(x[i] - x[j]) for i in range(len(x)) for j in range(i + 1, len(x))])


FAST = dict(damping=10.0, dt=0.01, k_surface=10.0)


def test_two_beads_end_antipodal():
    x, _ = _relax(2, 0.6, 3000, **FAST)
    c = np.dot(x[0], x[1]) / (np.linalg.norm(x[0]) * np.linalg.norm(x[1]))
    assert abs(c + 1.0) < 1e-8


def test_four_beads_end_as_a_regular_tetrahedron():
    x, _ = _relax(4, 0.8, 6000, seed=1, **FAST)
    d = _pair_dists(x)
    r = np.linalg.norm(x, axis=1)
    assert d.std() < 1e-7 * d.mean() and r.std() < 1e-7 * r.mean()
    assert abs(d.mean() / r.mean() - math.sqrt(8.0 / 3.0)) < 1e-6


def test_six_beads_end_as_a_regular_octahedron():
    x, _ = _relax(6, 0.9, 8000, seed=2, **FAST)
    d = np.sort(_pair_dists(x))
    edges, diags = d[:12], d[12:]
    assert edges.std() < 1e-6 * edges.mean() and diags.std() < 1e-6 * diags.mean()
    assert abs(diags.mean() / edges.mean() - math.sqrt(2.0)) < 1e-6


def test_energy_decreases_and_a_shell_spreads_evenly():
    """From a jittered, non-overlapping start (golden-angle points moved by up to 0.3)."""
    R, n = 4.0, 100
    rng = np.random.default_rng(5)
    i = np.arange(n) + 0.5
    z = 1 - 2 * i / n
    ph = math.pi * (3 - math.sqrt(5)) * i
    pos = R * np.stack([np.sqrt(1 - z * z) * np.cos(ph), np.sqrt(1 - z * z) * np.sin(ph), z], 1)
    pos += rng.uniform(-0.3, 0.3, size=pos.shape)
    p = po.relax_params(**FAST)
    vel = np.zeros_like(pos)

    def spread(x):
        nn = np.array([np.sort(np.linalg.norm(x - x[k], axis=1))[1] for k in range(n)])
        return nn.std() / nn.mean()

    s0 = spread(pos)
    energies = [po.shell_energy((R, R, R), pos, p)]
    for _ in range(20):
        pos, vel = po.relax_shell((R, R, R), pos, vel, p, 200)
        energies.append(po.shell_energy((R, R, R), pos, p))
    assert all(b <= a * (1 + 1e-12) for a, b in zip(energies, energies[1:]))
    assert energies[-1] < 0.5 * energies[0]
    assert np.abs(np.linalg.norm(pos, axis=1) - R).max() < 0.1
    assert spread(pos) < 0.5 * s0 and spread(pos) < 0.05
