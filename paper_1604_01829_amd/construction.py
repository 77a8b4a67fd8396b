"""Raspberry construction by constrained relaxation on the GPU (Sec. 2.1 of arXiv:1604.01829
and its SI "Details for ellipsoidal raspberry construction").

Beads are spread over an ellipsoid by damped MD (``rb_relax_shells``): WCA repulsion between
the beads of a shell and a harmonic restraint to the closest surface point.  A raspberry has
two overlaid shells, the outer (hydrodynamic) one on the surface (a, b, c) and the inner
(excluded-volume) one on (a - d, b - d, c - d), d = 0.5, and is filled with interior
hydrodynamic coupling points (Sec. 2.1).  The paper relaxes at one bead per unit area with
sigma 1.4, epsilon 0.1, damping 1000 and time step 0.001 for about 1e7 steps.
"""
import ctypes
import math

import numpy as np

from . import lbrb
from . import workloads as W

# The paper's script: damping 1000, sigma 1.4, epsilon 0.1, time step 0.001 (it gives no
# restraint stiffness).  At one bead per unit area the shell is compressed (neighbours near 1.03,
# well inside sigma), so the WCA pressure pushes beads off the surface by about F / (2 k):
# k = 1e4 keeps that near 0.01.  The step must keep dt^2 times the stiffest pair (about 2e5 for
# the closest pairs of a random start) small; lighter damping than the paper's reaches the same
# minimum sooner.
PAPER_PARAMS = dict(k_surface=1e4, sigma=1.4, epsilon=0.1, damping=1000.0, dt=0.001, mass=1.0)
DEFAULT_PARAMS = dict(k_surface=1e4, sigma=1.4, epsilon=0.1, damping=100.0, dt=0.001, mass=1.0)
MAX_BEADS = 2048
STEPS_PER_LAUNCH = 20000


def relax_shells(axes, positions, params=None, n_steps=20000, velocities=None, device="cuda:0"):
    """Relax several shells together on the GPU: axes (n_shells, 3), positions a list of
    (n_i, 3) arrays (body frame).  Returns (list of relaxed positions, list of velocities)."""
    import torch
    prm = lbrb.rb_relax_params(**dict(DEFAULT_PARAMS, **(params or {})))
    axes = np.ascontiguousarray(np.asarray(axes, dtype=np.float64).reshape(-1, 3))
    counts = np.array([len(p) for p in positions], dtype=np.int32)
    pos = torch.as_tensor(np.concatenate([np.asarray(p, np.float64).reshape(-1, 3)
                                          for p in positions]), device=device).contiguous()
    if velocities is None:
        vel = torch.zeros_like(pos)
    else:
        vel = torch.as_tensor(np.concatenate(velocities), device=device).contiguous()
    stream = torch.cuda.current_stream(pos.device).cuda_stream
    L = lbrb.library()
    left = int(n_steps)
    while True:
        k = min(left, STEPS_PER_LAUNCH)
        rc = L.rb_relax_shells(len(counts), axes.ctypes.data_as(lbrb._D),
                               counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), pos.data_ptr(),
                               vel.data_ptr(), prm, k, stream)
        if rc != lbrb.LB_OK:
            raise lbrb.LBError(rc, "rb_relax_shells")
        left -= k
        if left <= 0:
            break
    p, v = pos.cpu().numpy(), vel.cpu().numpy()
    cuts = np.cumsum(counts)[:-1]
    return np.split(p, cuts), np.split(v, cuts)


def initial_shell(a, b, c, n, seed=0, jitter=0.1):
    """n golden-angle points stretched onto the ellipsoid, each moved by up to `jitter` (nearly
    even on a sphere; stretching crowds them on an elongated ellipsoid)."""
    rng = np.random.default_rng(seed)
    pts = W.fibonacci_unit_sphere(n) * np.array([a, b, c], dtype=np.float64)
    return pts + rng.uniform(-jitter, jitter, size=pts.shape)


def separated_shell(a, b, c, n, seed=0, min_frac=0.75, tries=50000):
    """n points on the ellipsoid placed one by one at area-uniform random positions, each kept
    only if it is at least min_frac times the mean spacing sqrt(area / n) from every point
    already placed (random sequential addition): a start without close pairs.  When a pass
    cannot place them all (thin shells: the faces of a flat ellipsoid are close), the next
    pass asks for 10 % less separation."""
    rng = np.random.default_rng(seed)
    ax = np.array([a, b, c], dtype=np.float64)
    spacing = math.sqrt(W.ellipsoid_area(a, b, c) / n)
    amax = max(a * b, b * c, a * c)      # largest area element of the map from the unit sphere
    frac = min_frac
    for _ in range(20):
        dmin = frac * spacing
        pts = np.zeros((n, 3))
        m = 0
        for _ in range(tries):
            u = rng.normal(size=3)
            u /= np.linalg.norm(u)
            dA = math.sqrt((b * c * u[0]) ** 2 + (a * c * u[1]) ** 2 + (a * b * u[2]) ** 2)
            if rng.uniform() * amax > dA:
                continue
            p = ax * u
            if m and np.min(np.linalg.norm(pts[:m] - p, axis=1)) < dmin:
                continue
            pts[m] = p
            m += 1
            if m == n:
                return pts
        frac *= 0.9
    raise RuntimeError("could not place the beads")


def shell_count(a, b, c, density=1.0):
    return max(4, int(round(density * W.ellipsoid_area(a, b, c))))


def fill_points(a, b, c, spacing=1.0):
    """Interior coupling points: a cubic lattice of the given spacing through the centre, kept
    where the point lies inside the ellipsoid shrunk by one spacing."""
    ax = [np.arange(-math.floor(s / spacing), math.floor(s / spacing) + 1) * spacing
          for s in (a, b, c)]
    X, Y, Z = np.meshgrid(*ax, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    sa, sb, sc = a - spacing, b - spacing, c - spacing
    if min(sa, sb, sc) <= 0:
        return np.zeros((1, 3))
    keep = (pts[:, 0] / sa) ** 2 + (pts[:, 1] / sb) ** 2 + (pts[:, 2] / sc) ** 2 < 1.0
    return pts[keep]


def build_raspberry(a, b, c, density=1.0, inner_depth=0.5, fill_spacing=1.0, n_steps=20000,
                    params=None, seed=0):
    """Two relaxed shells and the interior points of a raspberry with semi-axes (a, b, c):
    dict(outer=(n,3) hydrodynamic shell, inner=(m,3) excluded-volume shell at depth
    inner_depth, fill=(k,3) interior coupling points)."""
    ai, bi, ci = a - inner_depth, b - inner_depth, c - inner_depth
    n_out, n_in = shell_count(a, b, c, density), shell_count(ai, bi, ci, density)
    if max(n_out, n_in) > MAX_BEADS:
        raise ValueError("a shell needs more than %d beads" % MAX_BEADS)
    init = [separated_shell(a, b, c, n_out, seed), separated_shell(ai, bi, ci, n_in, seed + 1)]
    (outer, inner), _ = relax_shells([(a, b, c), (ai, bi, ci)], init, params, n_steps)
    return dict(outer=outer, inner=inner, fill=fill_points(ai, bi, ci, fill_spacing))
