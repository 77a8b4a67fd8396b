"""Whole-box pins of the oracle: streaming, viscosity, walls, forcing, conservation.

- Shear wave: the decay factor per step equals the eigenvalue of the linearised one-step map
  S(k) J, where S(k) is the Fourier phase of pull streaming and J the collision Jacobian
  (taken from the single-node collision, itself pinned against textbook BGK+Guo).  This
  checks streaming direction, periodic wrap and node layout to round-off.  The same decay
  also matches the Navier-Stokes rate nu k^2 with nu = c_s^2 (tau_shear - 1/2).
- Plane Poiseuille flow between halfway bounce-back walls: with the two-relaxation-time
  "magic" product (tau_shear - 1/2)(tau_odd - 1/2) = 3/16 the parabola with walls exactly
  midway between nodes is reproduced to round-off (Ginzburg's TRT result).
- Hagen-Poiseuille flow in the staircase pore: u_z(r) = g (R^2 - r^2) / (4 rho nu).
- Mass is conserved and P = sum j + sum_b (M V_b + F_b/2) grows by N_fluid g_ext per step.
"""
import math

import numpy as np
import pytest

from oracle import pyoracle as po
from paper_1604_01829_amd import workloads as W


def _jacobian(p):
    f0 = po.equilibrium(p.rho0, (0.0, 0.0, 0.0))
    h = 1e-6
    J = np.zeros((19, 19))
    for j in range(19):
        e = np.zeros(19)
        e[j] = h
        J[:, j] = (po.collide_node(p, f0 + e, np.zeros(3)) -
                   po.collide_node(p, f0 - e, np.zeros(3))) / (2 * h)
    return J


@pytest.mark.parametrize("tau,L,axis", [(1.0, 32, 0), (0.7, 24, 1), (1.6, 16, 2)])
def test_shear_wave_decay(tau, L, axis):
    p = po.make_params(tau_shear=tau, tau_bulk=1.1, tau_odd=0.9, tau_even=1.3)
    shape = [1, 1, 1]
    shape[axis] = L
    sim = po.OracleSim(tuple(shape), p)
    A = 1e-4
    comp = (axis + 1) % 3     # transverse velocity component
    k = 2 * math.pi / L
    x = np.arange(L) + 0.5
    f = np.zeros((19, L))
    for n in range(L):
        u = [0.0, 0.0, 0.0]
        u[comp] = A * math.sin(k * x[n])
        f[:, n] = po.equilibrium(1.0, u)
    sim.set_populations(f)
    amps = []
    basis_s = np.sin(k * x)
    for step in range(120):
        fl = sim.fields().reshape(-1, 4)
        amps.append(2.0 / L * float(fl[:, 1 + comp] @ basis_s))
        sim.step(1)
    amps = np.array(amps)
    # spectral prediction: eigenvalue of the one-step map with the slowest transverse decay
    c = po.velocities()
    kv = np.zeros(3)
    kv[axis] = k
    S = np.diag(np.exp(-1j * (c @ kv)))
    lam, vec = np.linalg.eig(S @ _jacobian(p))
    jcomp = np.abs(c[:, comp] @ vec)
    shear = lam[np.argmax(jcomp / np.linalg.norm(vec, axis=0))]
    assert abs(shear.imag) < 1e-12
    ratio = amps[30:60] / amps[29:59]
    assert np.abs(ratio - shear.real).max() < 1e-9
    # Navier-Stokes limit, up to the O(k^2) dispersion of the lattice
    nu = (tau - 0.5) / 3.0
    nu_eff = -math.log(shear.real) / k ** 2
    assert abs(nu_eff / nu - 1.0) < 0.3 * k * k


def test_plane_poiseuille_exact_with_magic_parameter():
    nz = 18
    g = 1e-6
    tau_s = 1.0
    tau_odd = 0.5 + (3.0 / 16.0) / (tau_s - 0.5)
    p = po.make_params(tau_shear=tau_s, tau_bulk=tau_s, tau_odd=tau_odd, tau_even=tau_s,
                       g_ext=(g, 0.0, 0.0))
    sim = po.OracleSim((1, 1, nz), p)
    sim.set_mask(W.slab_mask(1, 1, nz, axis=2))
    sim.step(12000)
    u = sim.fields().reshape(nz, 4)[:, 1]
    nu = (tau_s - 0.5) / 3.0
    z = np.arange(nz) + 0.5
    want = g / (2 * nu) * (z - 1.0) * (nz - 1.0 - z)
    want[0] = want[-1] = 0.0
    assert np.abs(u - want).max() < 1e-10 * want.max()


def test_hagen_poiseuille_in_pore():
    n, R, g = 28, 11.0, 1e-6
    tau = 1.0
    p = po.make_params(tau_shear=tau, tau_bulk=tau, tau_odd=tau, tau_even=tau,
                       g_ext=(0.0, 0.0, g))
    sim = po.OracleSim((n, n, 1), p)
    sim.set_mask(W.pore_mask(n, n, 1, R))
    sim.step(6000)
    fl = sim.fields().reshape(n, n, 4)
    x = np.arange(n) + 0.5 - n / 2
    r2 = x[None, :] ** 2 + x[:, None] ** 2
    fluid = r2 < R * R
    nu = (tau - 0.5) / 3.0
    # fit u = a (Reff^2 - r^2) on the fluid nodes
    M = np.stack([np.ones(fluid.sum()), -r2[fluid]], axis=1)
    coef, *_ = np.linalg.lstsq(M, fl[..., 3][fluid], rcond=None)
    a = coef[1]
    reff = math.sqrt(coef[0] / a)
    assert abs(a / (g / (4 * nu)) - 1.0) < 0.02
    assert abs(reff - R) < 0.5
    assert np.all(fl[..., 3][~fluid] == 0.0)


def test_mass_and_momentum_bookkeeping():
    shape = (16, 12, 14)
    g_ext = np.array([2e-5, -1e-5, 3e-6])
    p = po.make_params(tau_shear=0.9, tau_bulk=1.2, tau_odd=1.1, tau_even=0.8, kT=3e-5,
                       g_ext=g_ext, seed=99)
    sim = po.OracleSim(shape, p)
    offs = W.sphere_beads(2.5, 60)
    m, I = W.solid_body_mass_inertia(1.0, 2.5, 2.5, 2.5)
    sim.add_body(offs, m, I, (15.2, 5.1, 0.7), quat=(0.9, 0.1, -0.3, 0.2),
                 vel=(1e-3, 0.0, -2e-3), omega=(1e-3, 2e-3, 0.0), gamma=W.GAMMA_FREE)
    offs2 = W.ellipsoid_beads(3.0, 1.5, 1.5)
    m2, I2 = W.solid_body_mass_inertia(1.0, 3.0, 1.5, 1.5)
    sim.add_body(offs2, m2, I2, (6.0, 6.0, 7.0), gamma=W.GAMMA_FREE)
    N = shape[0] * shape[1] * shape[2]

    def P():
        f = sim.populations().reshape(19, -1)
        c = po.velocities().astype(float)
        mass = math.fsum(f.reshape(-1))
        j = np.array([math.fsum((c[:, a:a + 1] * f).reshape(-1)) for a in range(3)])
        body = np.zeros(3)
        for b in range(2):
            st = sim.body_state(b)
            mass_b = [m, m2][b]
            body += mass_b * st["vel"] + 0.5 * st["force"]
        return mass, j + body

    m0, P0 = P()
    for n in range(1, 41):
        sim.step(1)
        mass, Pn = P()
        assert abs(mass - m0) < 1e-13 * m0
        assert np.abs(Pn - P0 - n * N * g_ext).max() < 1e-13 * N


@pytest.mark.parametrize("masked", [False, True])
def test_node_by_node_first_step_equals_the_box_step(masked):
    """The node-by-node expectation used for sampled checks of large boxes (neighbour
    collisions with their own noise, streamed or bounced back) equals the oracle's own step of
    the whole box."""
    from paper_1604_01829_amd import workloads as W
    from tests.helpers import first_step_expected
    shape, seed, kT = (12, 12, 9), 77, 4e-5
    mask = W.pore_mask(*shape, 4.5) if masked else None
    pp = dict(u0=(0.01, -0.004, 0.002), tau_shear=0.9, tau_bulk=1.1, tau_odd=1.2,
              tau_even=0.8, g_ext=(1e-5, 0.0, -2e-6))
    prm = po.make_params(kT=kT, seed=seed, **pp)
    sim = po.OracleSim(shape, prm)
    if masked:
        sim.set_mask(mask)
    sim.step(1)
    f = sim.fields()
    nodes = [(x, y, z) for z in range(9) for y in range(12) for x in range(12)
             if mask is None or not mask[z, y, x]]
    want = first_step_expected(shape, mask, prm, seed, kT, nodes)
    for (x, y, z), (rho, u) in zip(nodes, want):
        assert abs(f[z, y, x, 0] - rho) < 1e-14
        assert np.abs(f[z, y, x, 1:] - u).max() < 1e-15
