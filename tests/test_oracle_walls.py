"""Pins of the oracle's moving walls (halfway bounce-back with the moving-wall momentum term).

- plane Couette flow between walls moving at -U and +U: with all relaxation rates 1 the linear
  profile through walls located halfway between boundary and fluid nodes is reached exactly;
  with other rates the remaining difference is second order in the Mach number (it scales as
  U^2), the linear moving-wall term itself being exact;
- two walls moving together with (U, 0, U/2) carry the fluid along uniformly (Galilean check);
- wall ids with zero velocity are plain walls; velocities are set before the first step only.
"""
import numpy as np
import pytest

from oracle import pyoracle as po


def _couette(U, taus, steps, shape=(4, 18, 3), ids=(1, 2), u_lo=None, u_hi=None):
    nx, ny, nz = shape
    mask = np.zeros((nz, ny, nx), np.uint8)
    mask[:, 0, :] = ids[0]
    mask[:, ny - 1, :] = ids[1]
    sim = po.OracleSim(shape, po.make_params(**taus))
    sim.set_mask(mask)
    sim.set_wall_velocity(ids[0], (-U, 0, 0) if u_lo is None else u_lo)
    sim.set_wall_velocity(ids[1], (U, 0, 0) if u_hi is None else u_hi)
    sim.step(steps)
    return sim.fields()


def _linear(U, ny):
    y = np.arange(1, ny - 1) + 0.5            # fluid node centres
    return -U + 2.0 * U * (y - 1.0) / (ny - 2)  # walls at y = 1 and y = ny - 1


def test_couette_exact_with_unit_rates():
    U, ny = 0.01, 18
    f = _couette(U, dict(tau_shear=1.0), 6000)
    for z in range(3):
        for x in range(4):
            assert np.abs(f[z, 1:ny - 1, x, 1] - _linear(U, ny)).max() < 1e-10 * U
    assert np.abs(f[:, 1:ny - 1, :, 2:]).max() < 1e-14
    assert np.abs(f[:, 1:ny - 1, :, 0] - 1.0).max() < 1e-11
    assert np.all(f[:, 0, :, :] == 0) and np.all(f[:, ny - 1, :, :] == 0)


def test_couette_error_is_second_order_in_mach_number():
    taus = dict(tau_shear=0.8, tau_bulk=1.1, tau_odd=1.2, tau_even=0.9)
    ny = 18
    err = {}
    for U in (0.01, 0.001):
        f = _couette(U, taus, 6000)
        err[U] = np.abs(f[1, 1:ny - 1, 2, 1] - _linear(U, ny)).max() / U
    assert err[0.001] < 1e-8
    assert 80 < err[0.01] / err[0.001] < 120          # relative error ~ U^2


def test_co_moving_walls_carry_the_fluid_uniformly():
    U = 0.01
    f = _couette(U, dict(tau_shear=0.8, tau_bulk=1.1, tau_odd=1.2, tau_even=0.9), 8000,
                 u_lo=(U, 0, 0.5 * U), u_hi=(U, 0, 0.5 * U))
    assert np.abs(f[:, 1:17, :, 1] - U).max() < 1e-12
    assert np.abs(f[:, 1:17, :, 3] - 0.5 * U).max() < 1e-12
    assert np.abs(f[:, 1:17, :, 2]).max() < 1e-14


def test_resting_wall_ids_are_plain_walls_and_velocities_precede_the_first_step():
    shape = (6, 9, 5)
    rng = np.random.default_rng(3)
    p = po.make_params(tau_shear=0.9, g_ext=(1e-5, 0, 2e-6), kT=1e-4, seed=11)
    mask1 = np.zeros(shape[::-1], np.uint8)
    mask1[:, 0, :] = 1
    mask1[:, 8, :] = 1
    maskk = mask1 * rng.integers(1, 256, size=mask1.shape).astype(np.uint8)
    maskk[mask1 == 0] = 0
    a, b = po.OracleSim(shape, p), po.OracleSim(shape, p)
    a.set_mask(mask1)
    b.set_mask(maskk)
    a.step(20)
    b.step(20)
    assert np.array_equal(a.populations(), b.populations())
    with pytest.raises(RuntimeError):
        b.set_wall_velocity(1, (0.01, 0, 0))
    c = po.OracleSim(shape, p)
    for bad in (0, 256):
        with pytest.raises(RuntimeError):
            c.set_wall_velocity(bad, (0.01, 0, 0))
