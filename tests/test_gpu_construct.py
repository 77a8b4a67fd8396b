"""Raspberry construction on the GPU (rb_relax_shells) against the oracle (orc_relax.c).

- a shell on an ellipsoid from a jittered start, 400 steps: every position against the oracle;
- several shells of different sizes in one call, and 70 tiny shells (two launches of 64 and 6
  workgroups): each against its own oracle run;
- the largest shell (2048 beads), a few steps; a crowded 2048-bead shell whose beads have more
  pair candidates than their list holds (they walk all pairs); a thin oblate shell whose two
  faces are within the list radius of each other;
- the tetrahedron end state of four beads on a small sphere;
- a two-layer filled raspberry (prolate 8,4,4 at one bead per unit area): both shells on their
  surfaces with nearly even spacing, interior points inside the inner shell.
The GPU contracts multiply-adds (FMA) where the oracle rounds twice, so trajectories agree to
rounding amplified by the dynamics; the damping keeps that growth small (1e-9 of the largest
coordinate allowed over 400 steps).  The parity runs use a soft restraint and a long step
(k = 10, dt = 0.01, damping 10) from starts without close pairs.
"""
import math

import numpy as np
import pytest

from oracle import pyoracle as po
from paper_1604_01829_amd import construction as C
from paper_1604_01829_amd import workloads as W

pytestmark = pytest.mark.gpu

FAST = dict(k_surface=10.0, sigma=1.4, epsilon=0.1, damping=10.0, dt=0.01, mass=1.0)


def _oracle(axes, pos, steps, params=FAST):
    p = po.relax_params(**params)
    return po.relax_shell(axes, pos, np.zeros_like(pos), p, steps)[0]


def _gpu(axes, init, steps):
    return C.relax_shells(axes, init, FAST, steps)[0]


def _close(g, o, tol, what):
    scale = float(np.abs(o).max())
    err = float(np.abs(g - o).max())
    print(f"{what}: max err {err:.3g} (scale {scale:.3g})", flush=True)
    assert err <= tol * scale, what


def test_one_shell_matches_the_oracle():
    axes = (3.0, 2.0, 1.5)
    init = C.initial_shell(*axes, 40, seed=3)
    (g,) = _gpu([axes], [init], 400)
    _close(g, _oracle(axes, init, 400), 1e-9, "ellipsoid 40 beads")


def test_several_shells_in_one_call():
    shapes = [((3.0, 2.0, 1.5), 40), ((2.0, 2.0, 2.0), 30), ((5.0, 1.5, 1.5), 60),
              ((1.0, 1.0, 1.0), 3)]
    init = [C.initial_shell(*a, n, seed=k) for k, (a, n) in enumerate(shapes)]
    got = _gpu([a for a, _ in shapes], init, 300)
    for (a, n), g, x0 in zip(shapes, got, init):
        _close(g, _oracle(a, x0, 300), 1e-9, f"shell {a} x {n}")


def test_compressed_shell_at_the_default_parameters():
    """One bead per unit area from a separated start, the construction's own parameters."""
    axes = (4.0, 2.0, 2.0)
    init = C.separated_shell(*axes, C.shell_count(*axes), seed=4)
    (g,), _ = C.relax_shells([axes], [init], n_steps=1000)
    _close(g, _oracle(axes, init, 1000, C.DEFAULT_PARAMS), 1e-9, "compressed shell")


def test_more_shells_than_one_launch():
    rng = np.random.default_rng(8)
    axes = [tuple(rng.uniform(0.6, 1.2, 3)) for _ in range(70)]
    init = [C.initial_shell(*a, 3, seed=k, jitter=0.05) for k, a in enumerate(axes)]
    got = _gpu(axes, init, 200)
    for k in (0, 31, 63, 64, 69):
        _close(got[k], _oracle(axes[k], init[k], 200), 1e-9, f"tiny shell {k}")


def test_largest_shell():
    R = 20.0
    init = C.initial_shell(R, R, R, 2048, seed=2, jitter=0.05)
    (g,) = _gpu([(R, R, R)], [init], 20)
    _close(g, _oracle((R, R, R), init, 20), 1e-12, "2048 beads")


def test_crowded_shell_walks_all_pairs():
    """2048 beads on a radius-7 sphere (0.3 units of area each): a bead has about 30 others
    within the pair list's radius, more than the 24 entries a 2048-bead shell gets, so the
    beads walk all pairs; a weak repulsion keeps the start's overlaps tame."""
    R = 7.0
    prm = dict(FAST, epsilon=1e-6)
    init = C.initial_shell(R, R, R, 2048, seed=5, jitter=0.02)
    (g,), _ = C.relax_shells([(R, R, R)], [init], prm, 30)
    _close(g, _oracle((R, R, R), init, 30, prm), 1e-12, "crowded 2048 beads")


def test_thin_oblate_shell():
    """Beads of both faces of a thin oblate shell are within the list radius of each other
    (up to 30 candidates; a 475-bead shell gets lists of 103)."""
    axes = (0.42, 8.66, 8.66)
    init = C.separated_shell(*axes, C.shell_count(*axes), seed=1)
    (g,), _ = C.relax_shells([axes], [init], n_steps=600)
    _close(g, _oracle(axes, init, 600, C.DEFAULT_PARAMS), 1e-9, "thin oblate shell")


def test_tetrahedron():
    rng = np.random.default_rng(1)
    u = rng.normal(size=(4, 3))
    init = 0.8 * u / np.linalg.norm(u, axis=1, keepdims=True)
    (x,) = _gpu([(0.8, 0.8, 0.8)], [init], 6000)
    d = np.array([np.linalg.norm(x[i] - x[j]) for i in range(4) for j in range(i + 1, 4)])
    r = np.linalg.norm(x, axis=1)
    assert d.std() < 1e-7 * d.mean() and abs(d.mean() / r.mean() - math.sqrt(8 / 3)) < 1e-6


def test_two_layer_filled_raspberry():
    a, b, c = 8.0, 4.0, 4.0
    rb = C.build_raspberry(a, b, c, n_steps=20000, seed=4)
    for name, ax in (("outer", (a, b, c)), ("inner", (a - 0.5, b - 0.5, c - 0.5))):
        x = rb[name]
        assert abs(len(x) - W.ellipsoid_area(*ax)) <= 1.0          # one bead per unit area
        off = [np.linalg.norm(x[k] - po.closest_point(ax, x[k])[0]) for k in range(len(x))]
        nn = np.array([np.sort(np.linalg.norm(x - x[k], axis=1))[1] for k in range(len(x))])
        print(f"{name}: {len(x)} beads, max offset {max(off):.3g}, nn {nn.mean():.3f} "
              f"+- {nn.std():.3f}", flush=True)
        assert max(off) < 0.05 and nn.std() < 0.1 * nn.mean()
    f = rb["fill"]
    assert len(f) > 0 and np.all((f[:, 0] / 7.5) ** 2 + (f[:, 1] / 3.5) ** 2 + (f[:, 2] / 3.5) ** 2 < 1)


def test_the_papers_thirty_shells():
    """The construction benchmark's configuration: the paper's 15 ellipsoids of revolution of
    equal volume (aspect ratios 1/10 to 10), outer and inner shells at one bead per unit area,
    relaxed together in one launch at the default parameters; every shell against its own
    oracle run over 200 steps."""
    phis = [1 / 10, 1 / 5, 1 / 4, 1 / 3, 1 / 2, 2 / 3, 4 / 5, 9 / 10, 10 / 9, 5 / 4, 3 / 2, 2, 4,
            5, 10]
    axes, init = [], []
    for k, phi in enumerate(phis):
        bb = (4.25 ** 3 / phi) ** (1 / 3)
        for d in (0.0, 0.5):
            ax = (phi * bb - d, bb - d, bb - d)
            axes.append(ax)
            init.append(C.separated_shell(*ax, C.shell_count(*ax), seed=k))
    got, _ = C.relax_shells(axes, init, n_steps=200)
    for k, (ax, x0, g) in enumerate(zip(axes, init, got)):
        _close(g, _oracle(ax, x0, 200, C.DEFAULT_PARAMS), 1e-9, f"shell {k} {len(x0)} beads")
