"""Pins of the oracle's lattice, mode basis, equilibrium and single-node collision.

Each check compares the oracle with something it does not compute itself: the lattice
symmetry conditions of a second-order isotropic velocity set, the printed norms of the
orthogonal D3Q19 basis (Duenweg-Schiller-Ladd form), the textbook polynomial equilibrium and
the textbook population-space BGK collision with Guo's forcing term, written out here in
population space (the oracle works in mode space).
"""
import itertools

import numpy as np
import pytest

from oracle import pyoracle as po


def test_velocity_set_is_d3q19():
    c = po.velocities()
    got = sorted(tuple(v) for v in c)
    want = sorted(v for v in itertools.product((-1, 0, 1), repeat=3) if sum(a * a for a in v) <= 2)
    assert got == want
    assert tuple(c[0]) == (0, 0, 0)
    opp = po.opposite()
    for i in range(19):
        assert np.all(c[opp[i]] == -c[i])


def test_weights_isotropy():
    c = po.velocities().astype(float)
    w = po.weights()
    assert abs(w.sum() - 1.0) < 1e-15
    # first and third moments vanish, second = c_s^2 delta with c_s^2 = 1/3
    assert np.abs(w @ c).max() < 1e-16
    second = np.einsum("i,ia,ib->ab", w, c, c)
    assert np.abs(second - np.eye(3) / 3.0).max() < 1e-15
    third = np.einsum("i,ia,ib,ic->abc", w, c, c, c)
    assert np.abs(third).max() < 1e-16
    # fourth moment = c_s^4 (d_ab d_cd + d_ac d_bd + d_ad d_bc)
    fourth = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    d = np.eye(3)
    want = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
            + np.einsum("ad,bc->abcd", d, d)) / 9.0
    assert np.abs(fourth - want).max() < 1e-15


def test_basis_orthogonal_with_printed_norms():
    E = po.basis()
    w = po.weights()
    gram = np.einsum("ki,i,li->kl", E, w, E)
    b = po.basis_norms()
    assert np.abs(gram - np.diag(b)).max() < 1e-15
    # norms of the D3Q19 orthogonal basis in the Duenweg-Schiller-Ladd normalisation
    printed = [1, 1 / 3, 1 / 3, 1 / 3, 2 / 3, 4 / 3, 4 / 9, 1 / 9, 1 / 9, 1 / 9,
               2 / 3, 2 / 3, 2 / 3, 2 / 9, 2 / 9, 2 / 9, 2, 4 / 3, 4 / 9]
    assert np.allclose(b, printed, rtol=0, atol=1e-15)
    # complete: the modes determine the populations
    assert np.linalg.matrix_rank(E) == 19


def test_hydrodynamic_modes_are_moments():
    """Modes 0-3 are density and momentum; modes 4-9 span the second moments."""
    E = po.basis()
    c = po.velocities().astype(float)
    assert np.allclose(E[0], 1.0)
    assert np.allclose(E[1:4], c.T)
    second = np.stack([c[:, a] * c[:, b] for a in range(3) for b in range(a, 3)])
    span = np.vstack([E[0], E[4:10]])
    # every second moment c_a c_b is a combination of mode 0 and modes 4-9 ...
    coef, res, *_ = np.linalg.lstsq(span.T, second.T, rcond=None)
    assert np.abs(span.T @ coef - second.T).max() < 1e-13
    # ... and mode 4 is the trace part (isotropic), modes 5-9 the traceless part
    trace = (c ** 2).sum(axis=1)
    assert np.allclose(E[4], trace - 1.0)


def textbook_feq(rho, u):
    c = po.velocities().astype(float)
    w = po.weights()
    cu = c @ np.asarray(u)
    uu = float(np.dot(u, u))
    return w * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu)


@pytest.mark.parametrize("rho,u", [(1.0, (0.0, 0.0, 0.0)), (1.3, (0.05, -0.02, 0.07)),
                                   (0.7, (-0.1, 0.08, 0.0))])
def test_equilibrium_is_textbook_polynomial(rho, u):
    f = po.equilibrium(rho, u)
    assert np.abs(f - textbook_feq(rho, u)).max() < 1e-15
    c = po.velocities().astype(float)
    u = np.asarray(u)
    assert abs(f.sum() - rho) < 1e-14
    assert np.abs(f @ c - rho * u).max() < 1e-15
    Pi = np.einsum("i,ia,ib->ab", f, c, c)
    assert np.abs(Pi - (rho / 3.0 * np.eye(3) + rho * np.outer(u, u))).max() < 1e-14


def textbook_bgk_guo(f, F, tau):
    """Population-space BGK collision with Guo, Zheng & Shi's (2002) forcing term."""
    c = po.velocities().astype(float)
    w = po.weights()
    F = np.asarray(F, dtype=float)
    rho = f.sum()
    u = (f @ c + 0.5 * F) / rho
    feq = textbook_feq(rho, u)
    cu = c @ u
    S = w * (3.0 * ((c - u) @ F) + 9.0 * cu * (c @ F))
    return f - (f - feq) / tau + (1.0 - 0.5 / tau) * S


@pytest.mark.parametrize("tau", [0.6, 1.0, 1.7])
def test_collision_equals_bgk_guo_when_all_rates_equal(tau):
    rng = np.random.default_rng(3)
    p = po.make_params(tau_shear=tau, tau_bulk=tau, tau_odd=tau, tau_even=tau)
    for _ in range(5):
        f = textbook_feq(1.0 + 0.1 * rng.standard_normal(), 0.05 * rng.standard_normal(3))
        f = f + 1e-3 * rng.standard_normal(19)
        F = 1e-3 * rng.standard_normal(3)
        got = po.collide_node(p, f, F)
        want = textbook_bgk_guo(f, F, tau)
        assert np.abs(got - want).max() < 2e-15


def test_collision_conserves_mass_and_adds_force():
    rng = np.random.default_rng(4)
    p = po.make_params(tau_shear=0.8, tau_bulk=1.3, tau_odd=1.1, tau_even=0.9, kT=1e-4)
    c = po.velocities().astype(float)
    f = textbook_feq(1.0, (0.02, 0.01, -0.03)) + 1e-3 * rng.standard_normal(19)
    F = np.array([1e-3, -2e-3, 5e-4])
    un = rng.uniform(-0.5, 0.5, 19)
    out = po.collide_node(p, f, F, un)
    assert abs(out.sum() - f.sum()) < 1e-15
    assert np.abs(out @ c - (f @ c + F)).max() < 1e-16


def test_relaxation_rates_act_on_the_right_subspaces():
    """Jacobian of the collision at rest: eigenvalues 1 (x4), 1-1/tau_bulk on the isotropic
    stress, 1-1/tau_shear (x5) on the traceless stress, and the kinetic rates (x6, x3)."""
    taus = dict(tau_shear=0.8, tau_bulk=1.9, tau_odd=1.3, tau_even=0.6)
    p = po.make_params(**taus)
    f0 = textbook_feq(1.0, (0.0, 0.0, 0.0))
    h = 1e-6
    J = np.zeros((19, 19))
    for j in range(19):
        e = np.zeros(19)
        e[j] = h
        J[:, j] = (po.collide_node(p, f0 + e, np.zeros(3)) -
                   po.collide_node(p, f0 - e, np.zeros(3))) / (2 * h)
    lam, vec = np.linalg.eig(J)
    lam = np.sort(lam.real)
    g = {k: 1.0 - 1.0 / v for k, v in taus.items()}
    want = np.sort([1.0] * 4 + [g["tau_bulk"]] + [g["tau_shear"]] * 5 + [g["tau_odd"]] * 6
                   + [g["tau_even"]] * 3)
    assert np.abs(lam - want).max() < 1e-8
    # the bulk eigenvector carries an isotropic stress, the shear ones a traceless stress
    c = po.velocities().astype(float)
    lam_full, vec = np.linalg.eig(J)
    for ev, v in zip(lam_full.real, vec.T.real):
        Pi = np.einsum("i,ia,ib->ab", v, c, c)
        if abs(ev - g["tau_bulk"]) < 1e-6:
            assert np.abs(Pi - np.trace(Pi) / 3 * np.eye(3)).max() < 1e-8 * np.abs(Pi).max()
        if abs(ev - g["tau_shear"]) < 1e-6:
            assert abs(np.trace(Pi)) < 1e-8 * np.abs(Pi).max()
