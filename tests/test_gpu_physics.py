"""Physics of the GPU path against closed forms (slow-flow and equilibrium limits).

- Stokes drag on a fixed raspberry sphere in a periodic box, flow driven by a body force on
  the fluid: at steady state the drag equals the total driving force; the friction
  xi(L) = F / <u> follows Hasimoto's result for a periodic array of spheres (eq. hasimoto,
  read with 6 pi eta; here in its resistance form with the higher-order terms of the same
  series), so the hydrodynamic radius solved from each box size must not depend on L.
- Perrin's translational friction factors of a prolate spheroid (eq. perrin_a): the ratio of
  the frictions along and across the long axis of a raspberry ellipsoid, corrected for the
  periodic images by the isotropic leading term of the same series.
- Equipartition of a free raspberry in a thermal fluid: the fluid's own velocity variance is
  kT per degree of freedom; the body's <V_a^2> = kT/M (1 - M/M_total) with the total momentum
  fixed and <w_a^2> = kT/I_a hold up to the bias of the explicit bead coupling (the sampled
  fluid velocity does not yet contain the bead's own reaction force of the step): a few per
  cent at the bead friction of the workloads, shrinking with the friction and independent of
  the body's mass (so not a bias of the rigid-body integrator).
"""
import math

import numpy as np
import pytest

from paper_1604_01829_amd import workloads as W

pytestmark = pytest.mark.gpu

ETA = 1.0 / 6.0      # rho0 nu with tau_shear = 1


def _steady_drag(L, offs, gamma, axis, quat=(1, 0, 0, 0), u_target=2e-3, xi_guess=9.0):
    """Friction of a fixed body in force-driven flow along `axis` (FP64), at steady state."""
    from paper_1604_01829_amd import lbrb
    g = u_target * xi_guess / L ** 3          # keeps the mean flow near u_target (Re ~ 0.05)
    ge = [0.0, 0.0, 0.0]
    ge[axis] = g
    params = lbrb.make_params("f64", tau_shear=1.0, g_ext=tuple(ge), max_bodies=1,
                              max_beads=len(offs))
    sim = lbrb.Simulation(params, lbrb.make_replicas([((L, L, L), 1)]))
    sim.add_body(0, offs, 1.0, (1, 1, 1), (L / 2 + 0.13, L / 2 - 0.21, L / 2 + 0.07), quat=quat,
                 gamma=gamma, fixed=True)
    gN = g * L ** 3
    F = 0.0
    for _ in range(300):
        sim.step(2000)
        _, bs, _, _ = sim.observables(0)
        F = bs[0]["force"][axis]
        if abs(F - gN) < 1e-5 * gN:
            break
    assert abs(F - gN) < 1e-5 * gN, "no steady state"
    U = float(sim.fields(0)[..., 1 + axis].mean())
    sim.close()
    return F / U


def _hasimoto_radius(xi, L):
    """R with 6 pi eta R / xi = 1 - 2.837 x + 4.19 x^3 - 27.4 x^6, x = R / L (bisection)."""
    lo, hi = 1e-3, L / 3.0
    for _ in range(200):
        R = 0.5 * (lo + hi)
        x = R / L
        if 6 * math.pi * ETA * R / xi > 1 - 2.837 * x + 4.19 * x ** 3 - 27.4 * x ** 6:
            hi = R
        else:
            lo = R
    return 0.5 * (lo + hi)


def _perrin(a, b):
    """Perrin's translational frictions / eta of a prolate spheroid (a > b = c): along the
    long axis and across it."""
    e = math.sqrt(a * a - b * b)
    S = 2.0 / e * math.log((a + e) / b)
    fa = 16 * math.pi * (a * a - b * b) / ((2 * a * a - b * b) * S - 2 * a)
    fb = 32 * math.pi * (a * a - b * b) / ((2 * a * a - 3 * b * b) * S + 2 * a)
    return fa, fb


def test_perrin_reduces_to_stokes_for_a_sphere():
    fa, fb = _perrin(2.0 + 1e-6, 2.0)
    assert abs(fa / (6 * math.pi * 2.0) - 1) < 1e-5 and abs(fb / (6 * math.pi * 2.0) - 1) < 1e-5


def _sphere_radius():
    R = 2.0
    offs = W.sphere_beads(R, W.sphere_bead_count(R))
    return R, offs


def test_hasimoto_box_size_correction():
    R, offs = _sphere_radius()
    rh = {}
    for L in (16, 24, 32, 48):
        xi = _steady_drag(L, offs, W.GAMMA_FIXED, 0)
        rh[L] = _hasimoto_radius(xi, L)
        print(f"  L={L}: xi={xi:.5f} R_h={rh[L]:.5f}", flush=True)
    v = np.array(list(rh.values()))
    # the friction drops by 40 % from L = 16 to 48; the corrected radius stays put
    assert (v.max() - v.min()) / v.mean() < 5e-3
    assert R < v.mean() < R + 0.5      # the raspberry's hydrodynamic radius exceeds its bead radius


def test_perrin_friction_ratio_of_a_raspberry_ellipsoid():
    R, sph = _sphere_radius()
    delta = _hasimoto_radius(_steady_drag(32, sph, W.GAMMA_FIXED, 0), 32) - R
    a, b = 4.0, 2.0
    offs = W.ellipsoid_beads(a, b, b)
    fa, fb = _perrin(a + delta, b + delta)
    ratios = []
    for L in (32, 48):
        xa = _steady_drag(L, offs, W.GAMMA_FIXED, 0)     # long axis along x
        xb = _steady_drag(L, offs, W.GAMMA_FIXED, 1)
        corr = 2.837 / (6 * math.pi * ETA * L)           # isotropic image term of the mobility
        ratios.append((1 / xb + corr) / (1 / xa + corr))
        print(f"  L={L}: xi_par={xa:.5f} xi_perp={xb:.5f} corrected ratio {ratios[-1]:.5f}; "
              f"Perrin {fa / fb:.5f} (shell {delta:.3f})", flush=True)
    assert abs(ratios[0] - ratios[1]) < 5e-3
    for r in ratios:
        assert abs(r / (fa / fb) - 1) < 1.5e-2


def _temperatures(density, gamma, samples, seed, every=10):
    from paper_1604_01829_amd import lbrb
    kT, L, R = 4e-5, 32, 3.0
    offs = W.sphere_beads(R, W.sphere_bead_count(R))
    m, I = W.solid_body_mass_inertia(density, R, R, R)
    params = lbrb.make_params("f32", tau_shear=1.0, kT=kT, max_bodies=1, max_beads=len(offs))
    sim = lbrb.Simulation(params, lbrb.make_replicas([((L, L, L), seed)]))
    sim.add_body(0, offs, m, I, (L / 2, L / 2, L / 2), gamma=gamma)
    sim.set_graph_steps(every)
    sim.step(200 * every)
    V, Om, fluid = [], [], []
    for k in range(samples):
        sim.step(every)
        _, bs, _, _ = sim.observables(0)
        V.append(bs[0]["vel"].copy())
        Om.append(bs[0]["omega"].copy())
        if k % 1000 == 0:
            f = sim.fields(0)
            fluid.append(float((f[..., 0] * (f[..., 1:] ** 2).sum(-1)).mean() / (3 * kT)))
    sim.close()
    V, Om = np.array(V), np.array(Om)
    m_total = m + L ** 3          # rho0 = 1: fluid mass = node count
    tt = float((V ** 2).mean() / (kT / m * (1 - m / m_total)))
    tr = float(((Om ** 2).mean(0) / (kT / np.asarray(I))).mean())
    # statistical error of the mean square from 20 block means
    blk = (V ** 2).sum(1).reshape(20, -1).mean(1)
    err = float(blk.std() / blk.mean() / math.sqrt(20))
    return tt, tr, err, float(np.mean(fluid))


def test_equipartition_of_a_free_raspberry():
    g = W.GAMMA_FREE
    runs = {"M, gamma": _temperatures(1.0, g, 30000, 99),
            "8M, gamma": _temperatures(8.0, g, 30000, 98),
            "M, gamma/4": _temperatures(1.0, g / 4, 30000, 97)}
    for k, (tt, tr, e, tf) in runs.items():
        print(f"  {k}: T_trans/kT={tt:.4f} T_rot/kT={tr:.4f} (+-{e:.4f}), fluid {tf:.4f}",
              flush=True)
        assert abs(tf - 1.0) < 5e-3                  # the fluid is at kT
        assert 0.99 < tt < 1.08 and 0.99 < tr < 1.08
    (t1, r1, e1, _), (t8, r8, e8, _), (tq, rq, eq, _) = runs.values()
    # independent of the body's mass within sampling error
    assert abs(t8 - t1) < 4 * math.hypot(e1, e8) + 5e-3
    # smaller with a smaller bead friction
    assert tq < t1 and rq < r1 and tq < 1.04 and rq < 1.04
