"""Seeded synthetic inputs: bead shells, pore masks, body placement, and the five workloads.

This module holds no arithmetic of the method itself (no lattice, collision, coupling or
integrator code).  It only produces inputs -- geometry, masses, seeds, parameters -- and is
the single source of inputs shared by the GPU library's tests/benchmark and the CPU oracle.

The paper's own raspberries come from an MD relaxation of beads on a surface (Sec. 2.1) and
its coordinate files are not available.  The stand-ins here keep the same structure: a shell
of beads spread evenly over a sphere or an ellipsoid of revolution (Sec. 1.2, Fig. "rasp")
plus one centre bead, at one to two beads per unit area, in cubic periodic boxes or in boxes
holding a cylindrical pore along z whose boundary nodes sit outside the wall (Sec. 2.3).
"""
import math

import numpy as np

GOLDEN_ANGLE = math.pi * (3.0 - math.sqrt(5.0))

PLACEMENT_SEED_BASE = 1604018290
PHILOX_SEED_BASE = 0x1604_0182_9000

# Bead friction.  The workloads were specified with gamma = 20 (lattice units, rho0 = 1),
# which the explicit coupling and the explicit rigid-body kick cannot integrate: the oracle
# diverges within 50 steps (free bodies need gamma * beads / mass < 2, fixed bodies diverge
# between gamma = 1.5 and 3.3).  The runs use the paper's own bead frictions instead
# (Sec. 3.1: 50, 200 and 1000 M0/t0), converted with rho = 6.004 M0/sigma^3 and the fluid
# step 0.02 t0 (Sec. 2.3): gamma dt / (rho a^3) = 1/6, 2/3 and 10/3.
GAMMA_AS_SPECIFIED = 20.0
GAMMA_PAPER_LOW = 50.0 * 0.02 / 6.004     # xi_bead = 50 M0/t0
GAMMA_PAPER_MID = 200.0 * 0.02 / 6.004    # xi_bead = 200 M0/t0
GAMMA_FREE = GAMMA_PAPER_LOW
GAMMA_FIXED = GAMMA_PAPER_MID


# ------------------------------------------------------------------ bead shells

def fibonacci_unit_sphere(n):
    """n nearly evenly spread points on the unit sphere (Fibonacci / golden-angle lattice)."""
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = GOLDEN_ANGLE * i
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def sphere_beads(radius, n_surface, centre_bead=True):
    """Shell of n_surface beads on a sphere of the given radius, plus the centre (0,0,0)."""
    pts = fibonacci_unit_sphere(n_surface) * radius
    if centre_bead:
        pts = np.vstack([np.zeros((1, 3)), pts])
    return pts


def sphere_bead_count(radius, per_area=2.2):
    """Surface-bead count of a sphere at a given areal density."""
    return int(round(per_area * 4.0 * math.pi * radius * radius))


def ellipsoid_area(a, b, c, n_theta=256, n_phi=512):
    """Surface area of an ellipsoid with semi-axes a, b, c by midpoint quadrature."""
    th = (np.arange(n_theta) + 0.5) * math.pi / n_theta
    ph = (np.arange(n_phi) + 0.5) * 2.0 * math.pi / n_phi
    T, P = np.meshgrid(th, ph, indexing="ij")
    st, ct, sp, cp = np.sin(T), np.cos(T), np.sin(P), np.cos(P)
    # |dr/dtheta x dr/dphi| for r = (a st cp, b st sp, c ct)
    nx = b * c * st * st * cp
    ny = a * c * st * st * sp
    nz = a * b * st * ct
    dA = np.sqrt(nx * nx + ny * ny + nz * nz)
    return float(dA.sum() * (math.pi / n_theta) * (2.0 * math.pi / n_phi))


def ellipsoid_beads(a, b, c, spacing=1.0, centre_bead=True):
    """Beads on an ellipsoid with semi-axes (a, b, c) along the body axes (x, y, z).

    The count is the hexagonal-packing density for the given spacing, 2/(sqrt(3) s^2) per
    unit area; positions are a Fibonacci lattice of the unit sphere stretched to the axes.
    """
    n = max(4, int(round(ellipsoid_area(a, b, c) * 2.0 / (math.sqrt(3.0) * spacing ** 2))))
    pts = fibonacci_unit_sphere(n) * np.array([a, b, c], dtype=np.float64)
    if centre_bead:
        pts = np.vstack([np.zeros((1, 3)), pts])
    return pts


def solid_body_mass_inertia(rho0, a, b, c):
    """Mass and principal inertia of a uniform solid ellipsoid of the fluid's density."""
    m = rho0 * 4.0 / 3.0 * math.pi * a * b * c
    return m, np.array([m * (b * b + c * c) / 5.0, m * (a * a + c * c) / 5.0,
                        m * (a * a + b * b) / 5.0])


def random_quaternion(rng):
    """Uniformly distributed unit quaternion (w, x, y, z) (Shoemake's method)."""
    u1, u2, u3 = rng.random(3)
    q = np.array([math.sqrt(1 - u1) * math.sin(2 * math.pi * u2),
                  math.sqrt(1 - u1) * math.cos(2 * math.pi * u2),
                  math.sqrt(u1) * math.sin(2 * math.pi * u3),
                  math.sqrt(u1) * math.cos(2 * math.pi * u3)])
    return q


# ------------------------------------------------------------------ masks

def pore_mask(nx, ny, nz, radius):
    """uint8 mask (nz, ny, nx), 1 = boundary node: node centres farther than `radius` from
    the pore axis (the z line through the middle of the x-y cross-section)."""
    x = np.arange(nx) + 0.5 - nx / 2.0
    y = np.arange(ny) + 0.5 - ny / 2.0
    r = np.hypot(x[None, :], y[:, None])
    plane = (r > radius).astype(np.uint8)
    return np.ascontiguousarray(np.broadcast_to(plane[None, :, :], (nz, ny, nx)))


def slab_mask(nx, ny, nz, axis=2):
    """uint8 mask with one boundary layer at each end of `axis` (a plane channel)."""
    m = np.zeros((nz, ny, nx), dtype=np.uint8)
    if axis == 2:
        m[0], m[-1] = 1, 1
    elif axis == 1:
        m[:, 0], m[:, -1] = 1, 1
    else:
        m[:, :, 0], m[:, :, -1] = 1, 1
    return m


# ------------------------------------------------------------------ workload records

def default_params(**kw):
    p = dict(rho0=1.0, u0=(0.0, 0.0, 0.0), tau_shear=1.0, tau_bulk=1.0, tau_odd=1.0,
             tau_even=1.0, kT=0.0, g_ext=(0.0, 0.0, 0.0))
    p.update(kw)
    return p


def body_record(offsets, mass, inertia, pos, quat=(1.0, 0.0, 0.0, 0.0), vel=(0.0, 0.0, 0.0),
                omega=(0.0, 0.0, 0.0), gamma=20.0, fixed=False):
    return dict(offsets=np.ascontiguousarray(np.asarray(offsets, dtype=np.float64)),
                mass=float(mass), inertia=np.asarray(inertia, dtype=np.float64),
                pos=np.asarray(pos, dtype=np.float64), quat=np.asarray(quat, dtype=np.float64),
                vel=np.asarray(vel, dtype=np.float64), omega=np.asarray(omega, dtype=np.float64),
                gamma=float(gamma), fixed=bool(fixed))


def _periodic_dist(a, b, box, periodic):
    d = np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)
    for ax in range(3):
        if periodic[ax]:
            d[ax] -= box[ax] * round(d[ax] / box[ax])
    return float(np.linalg.norm(d))


def place_spheres_in_pore(rng, n, r_lo, r_hi, shape, pore_radius, clearance=2.0,
                          max_tries=100000):
    """Non-overlapping spheres off the pore axis: radius ~ U[r_lo, r_hi], radial distance
    ~ U[0.2, 1] * (pore_radius - R - clearance), angle ~ U[0, 2 pi), z ~ U[0, nz)."""
    nx, ny, nz = shape
    placed = []
    tries = 0
    while len(placed) < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("placement failed")
        R = rng.uniform(r_lo, r_hi)
        d = rng.uniform(0.2, 1.0) * (pore_radius - R - clearance)
        th = rng.uniform(0.0, 2.0 * math.pi)
        c = np.array([nx / 2.0 + d * math.cos(th), ny / 2.0 + d * math.sin(th),
                      rng.uniform(0.0, nz)])
        ok = all(_periodic_dist(c, c2, shape, (False, False, True)) >= R + R2 + clearance
                 for c2, R2 in placed)
        if ok:
            placed.append((c, R))
    return placed


def workload(k, scale=1.0, gamma=None):
    """The five synthetic workloads (k = 1..5) as plain records.

    Returns dict(name, precision ('f64'|'f32'), steps, replicas=[dict(shape, seed, mask or
    None, bodies=[body_record...])], params=dict(...)).  `scale` < 1 shrinks the box sizes
    of k = 2, 3 (for small parity cases); the default is the full size.
    """
    rng = np.random.default_rng(PLACEMENT_SEED_BASE + k)
    seed = PHILOX_SEED_BASE + k
    g_free = GAMMA_FREE if gamma is None else float(gamma)
    g_fixed = GAMMA_FIXED if gamma is None else float(gamma)
    if k == 1:
        shape = (32, 32, 32)
        R = 3.0
        offs = sphere_beads(R, 250)
        m, I = solid_body_mass_inertia(1.0, R, R, R)
        pos = rng.uniform(0.0, 32.0, size=3)
        bodies = [body_record(offs, m, I, pos, gamma=g_free)]
        return dict(name="sphere R=3 in a 32^3 periodic box, FP64, deterministic",
                    precision="f64", steps=500,
                    params=default_params(g_ext=(1e-5, 0.0, 0.0)),
                    replicas=[dict(shape=shape, seed=seed, mask=None, bodies=bodies)])
    if k == 2:
        nx, ny, nz = (int(round(128 * scale)), int(round(128 * scale)), int(round(256 * scale)))
        pore_r = 40.0 * scale
        mask = pore_mask(nx, ny, nz, pore_r)
        n_sph = max(1, int(round(32 * scale ** 3)))
        spheres = place_spheres_in_pore(rng, n_sph, 2.0, 6.0, (nx, ny, nz), pore_r)
        bodies = []
        for c, R in spheres:
            offs = sphere_beads(R, sphere_bead_count(R))
            m, I = solid_body_mass_inertia(1.0, R, R, R)
            bodies.append(body_record(offs, m, I, c, gamma=g_free))
        return dict(name="32 spheres R~U[2,6] in a radius-40 pore, 128x128x256, FP32, thermal",
                    precision="f32", steps=2000, params=default_params(kT=4e-5),
                    replicas=[dict(shape=(nx, ny, nz), seed=seed, mask=mask, bodies=bodies)])
    if k == 3:
        L = int(round(256 * scale))
        shapes = [(4, 2), (8, 2), (8, 4), (2, 4)]
        bodies = []
        placed = []
        for (a, b) in shapes:
            for _ in range(4):
                for _t in range(100000):
                    c = rng.uniform(0.0, L, size=3)
                    rad = max(a, b)
                    if all(_periodic_dist(c, c2, (L, L, L), (True, True, True)) >= rad + r2 + 2
                           for c2, r2 in placed):
                        break
                placed.append((c, max(a, b)))
                offs = ellipsoid_beads(a, b, b, spacing=1.0)
                m, I = solid_body_mass_inertia(1.0, a, b, b)
                bodies.append(body_record(offs, m, I, c, quat=random_quaternion(rng),
                                          gamma=g_free))
        return dict(name="16 ellipsoids in a 256^3 periodic box, thermal",
                    precision="f32", steps=5000, params=default_params(kT=4e-5),
                    replicas=[dict(shape=(L, L, L), seed=seed, mask=None, bodies=bodies)])
    if k == 4:
        n_rep = max(1, int(round(512 * scale)))
        sides = [32, 40, 48, 56, 64]
        reps = []
        for r in range(n_rep):
            L = int(sides[rng.integers(0, len(sides))])
            pore_r = 0.4 * L
            mask = pore_mask(L, L, L, pore_r)
            # equal-volume radius 0.1 L, prolate with aspect ratio ~ U[1, 4]
            phi = rng.uniform(1.0, 4.0)
            req = 0.1 * L
            b = req / phi ** (1.0 / 3.0)
            a = phi * b
            offs = ellipsoid_beads(a, b, b, spacing=1.0)
            m, I = solid_body_mass_inertia(1.0, a, b, b)
            d = rng.uniform(0.0, 0.5) * max(0.0, pore_r - a - 2.0)
            th = rng.uniform(0.0, 2.0 * math.pi)
            c = np.array([L / 2.0 + d * math.cos(th), L / 2.0 + d * math.sin(th),
                          rng.uniform(0.0, L)])
            reps.append(dict(shape=(L, L, L), seed=seed + r, mask=mask,
                             bodies=[body_record(offs, m, I, c, quat=random_quaternion(rng),
                                                 gamma=g_free)]))
        return dict(name="512 pore replicas of sides in {32..64}, one ellipsoid each, FP32, "
                         "thermal", precision="f32", steps=10000,
                    params=default_params(kT=4e-5), replicas=reps)
    if k == 5:
        shape = (64, 64, 64)
        R = 4.0
        offs = sphere_beads(R, 400)
        m, I = solid_body_mass_inertia(1.0, R, R, R)
        # centre near the box middle, shifted so that no bead sits within 2e-3 of a cell face
        for _ in range(10000):
            pos = 32.0 + rng.uniform(-0.5, 0.5, size=3)
            frac = np.mod(offs + pos - 0.5, 1.0)
            if np.all(np.minimum(frac, 1.0 - frac) >= 2e-3):
                break
        bodies = [body_record(offs, m, I, pos, gamma=g_fixed, fixed=True)]
        return dict(name="fixed sphere R=4 in uniform flow, 64^3 periodic, FP32",
                    precision="f32", steps=200,
                    params=default_params(u0=(0.01, 0.0, 0.0)),
                    replicas=[dict(shape=shape, seed=seed, mask=None, bodies=bodies)])
    raise ValueError(k)


# ------------------------------------------------------------------ Stokes-flow resistance

# The paper's Stokes-flow set-up (Sec. 2.3, eq. (stokesflow)) in lattice units: grid
# spacing 1 nm, fluid step 0.02 t0 with t0 = 6.352 ps, simulated kinematic viscosity
# 0.8 sigma^2/t0, boundary velocity 2.20 m/s along z on the +-y faces of a 50 nm box.
STOKES_DT_SECONDS = 0.02 * 6.352e-12
STOKES_U_PAPER = 2.20 * STOKES_DT_SECONDS / 1e-9          # 2.79e-4 lattice units per step
STOKES_TAU_PAPER = 0.5 + 3.0 * (0.8 * 0.02)                # nu = 0.016 -> tau = 0.548
STOKES_BOX_PAPER = 50


def stokes_flow_workload(L=STOKES_BOX_PAPER, radius=5.25, U=STOKES_U_PAPER,
                         tau_shear=STOKES_TAU_PAPER, gamma=GAMMA_FIXED, precision="f64",
                         per_area=2.2, seed=0):
    """A fixed spherical raspberry at the centre of a cubic box whose -y and +y faces are
    boundary nodes of one wall (id 1) moving with (0, 0, U); thermostat off.  The fluid
    starts at the wall velocity, so only the disturbance of the particle has to develop.
    The record has the layout of ``workload`` plus walls={id: velocity}."""
    offs = sphere_beads(radius, sphere_bead_count(radius, per_area))
    m, I = solid_body_mass_inertia(1.0, radius, radius, radius)
    pos = np.array([L / 2.0, L / 2.0, L / 2.0]) + np.array([0.013, -0.021, 0.017])
    mask = slab_mask(L, L, L, axis=1)
    bodies = [body_record(offs, m, I, pos, gamma=gamma, fixed=True)]
    return dict(name=f"Stokes flow past a fixed sphere R={radius} in a {L}^3 channel",
                precision=precision, steps=0,
                params=default_params(u0=(0.0, 0.0, U), tau_shear=tau_shear,
                                      tau_bulk=tau_shear),
                replicas=[dict(shape=(L, L, L), seed=PHILOX_SEED_BASE + 60 + seed, mask=mask,
                               bodies=bodies, walls={1: (0.0, 0.0, U)})])


# ------------------------------------------------------------------ excluded volume

# Sec. 2.1 and 2.3: the colloid's inner (excluded-volume) layer sits 0.5 inside the outer
# hydrodynamic shell with Lennard-Jones radius 0.5; pore beads of radius 6.25 are spaced 5
# apart around the pore; sigma_WCA = r_r + r_p and eps = kT.
INNER_LAYER_DEPTH = 0.5
INNER_LAYER_RADIUS = 0.5
PORE_SITE_RADIUS = 6.25
PORE_SITE_SPACING = 5.0


def inner_layer_sphere(radius, per_area=2.2):
    """Excluded-volume sites of a spherical raspberry: a shell INNER_LAYER_DEPTH inside the
    outer radius at the outer shell's areal density (no centre site)."""
    r = radius - INNER_LAYER_DEPTH
    return sphere_beads(r, max(4, sphere_bead_count(r, per_area)), centre_bead=False)


def pore_wall_sites(nx, ny, nz, pore_radius, site_radius=PORE_SITE_RADIUS,
                    spacing=PORE_SITE_SPACING):
    """Rings of pore beads around the z axis through the middle of the x-y cross-section,
    centres one site radius outside the pore wall, about `spacing` apart along each ring and
    between rings (the ring count divides nz, so the lattice is periodic along z).  The
    rings must fit in the box with room for the interaction range."""
    ring = pore_radius + site_radius
    reach = ring + 2.0 ** (1.0 / 6.0) * (site_radius + INNER_LAYER_RADIUS)
    if 2.0 * reach > min(nx, ny):
        raise ValueError("the pore beads and their range do not fit in the box")
    n_rings = max(1, int(round(nz / spacing)))
    n_ang = max(3, int(round(2.0 * math.pi * ring / spacing)))
    th = 2.0 * math.pi * np.arange(n_ang) / n_ang
    pts = []
    for j in range(n_rings):
        z = (j + 0.5) * nz / n_rings
        pts.append(np.stack([nx / 2.0 + ring * np.cos(th), ny / 2.0 + ring * np.sin(th),
                             np.full(n_ang, z)], axis=1))
    return np.concatenate(pts, axis=0)


def confined_md_workload(scale=1.0, substeps=2, eps=None):
    """Workload 2 with the paper's integration scheme: `substeps` MD steps per fluid step,
    inner excluded-volume layers on every sphere, pore beads around the pore, and WCA
    repulsion of energy eps (default kT) between inner layers and pore beads and between
    the inner layers of different spheres.  Records carry params md_substeps/wca_epsilon,
    per replica wall_sites=(positions, radius) and per body ev=(offsets, radius)."""
    wl = workload(2, scale=scale)
    p = wl["params"]
    p["md_substeps"] = int(substeps)
    p["wca_epsilon"] = p["kT"] if eps is None else float(eps)
    rep = wl["replicas"][0]
    nx, ny, nz = rep["shape"]
    rep["wall_sites"] = (pore_wall_sites(nx, ny, nz, 40.0 * scale), PORE_SITE_RADIUS)
    for b in rep["bodies"]:
        R = float(np.linalg.norm(b["offsets"], axis=1).max())
        b["ev"] = (inner_layer_sphere(R), INNER_LAYER_RADIUS)
    wl["name"] = (f"{wl['name']}; {substeps} MD steps per fluid step, WCA inner layers and "
                  "pore beads")
    return wl


# ------------------------------------------------------------------ trajectories

def synthetic_trajectory(n_frames, n_bodies, seed, step=0.05, rot_step=0.03, centre=None,
                         radius=(2.0, 8.0), z0=0.0):
    """Seeded poses [n_frames, n_bodies, 7] (centre x, y, z; quaternion w, x, y, z) for the
    trajectory analysis: centres take Gaussian steps of standard deviation `step` per axis,
    starting at random radii in `radius` around `centre` (x, y) when given; orientations start
    random and are turned each frame by a rotation about a Gaussian body-frame vector of
    standard deviation `rot_step` per component."""
    from scipy.spatial.transform import Rotation as Rot
    rng = np.random.default_rng(seed)
    traj = np.zeros((n_frames, n_bodies, 7))
    for b in range(n_bodies):
        if centre is None:
            p = rng.uniform(0.0, 20.0, size=3)
        else:
            r, th = rng.uniform(*radius), rng.uniform(0.0, 2.0 * math.pi)
            p = np.array([centre[0] + r * math.cos(th), centre[1] + r * math.sin(th), z0])
        steps = rng.normal(0.0, step, size=(n_frames, 3))
        steps[0] = 0.0
        traj[:, b, :3] = p + np.cumsum(steps, axis=0)
        rot = Rot.from_quat(rng.normal(size=4))
        incs = Rot.from_rotvec(rng.normal(0.0, rot_step, size=(n_frames, 3)))
        for f in range(n_frames):
            q = rot.as_quat()
            traj[f, b, 3:] = (q[3], q[0], q[1], q[2])
            rot = rot * incs[f]
    return traj
