"""Trajectory analysis on the GPU against the oracle (oracle/analysis.py).

- seeded synthetic trajectories (random walks of centres around a pore axis, random small
  rotations): the lab-, body- and pore-frame series, the radial coordinate, the MSDs of every
  series, the lab rotational MSD and the radially binned MSD, element by element;
- a long trajectory (200,000 frames) for the chunked sums;
- edge cases: one frame, the largest lag, one body;
- a trajectory recorded from a thermal GPU simulation: the same comparisons, and the lag-1
  identity of the body and lab frames (a rotation keeps lengths).
Tolerances: the GPU sums each body's increments in 256 chunks and the oracle in one sequence,
so the cumulative series agree to rounding of the running sum (1e-12 of its magnitude); MSDs
to 1e-10 relative; the rotational MSD to 1e-8 relative (arccos near 1 amplifies the rounding
of the dot product); bin counts exactly.
"""
import numpy as np
import pytest

from oracle import analysis as OA
from paper_1604_01829_amd import analysis as GA
from paper_1604_01829_amd import lbrb
from paper_1604_01829_amd import workloads as W

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def _host(t):
    return t.cpu().numpy()


def _close(g, o, rel, what):
    scale = max(1.0, float(np.abs(o).max()))
    err = float(np.abs(g - o).max())
    print(f"{what}: max err {err:.3g} (scale {scale:.3g})", flush=True)
    assert err <= rel * scale, what


def _compare_all(traj, centre, n_lags, edges, ref):
    t = _dev(traj)
    # series (oracle frame-major, GPU body-major)
    lab_o = OA.lab_frame(traj).transpose(1, 0, 2)
    body_o = np.concatenate([OA.body_frame_translation(traj), OA.body_frame_rotation(traj)],
                            axis=2).transpose(1, 0, 2)
    pore_o, rad_o = OA.pore_frame(traj, centre)
    pore_o = pore_o.transpose(1, 0, 2)
    lab_g, body_g = GA.lab_frame(t), GA.body_frame(t)
    pore_g, rad_g = GA.pore_frame(t, centre)
    _close(_host(lab_g), lab_o, 1e-12, "lab frame")
    _close(_host(body_g), body_o, 1e-12, "body frame")
    _close(_host(pore_g), pore_o, 1e-12, "pore frame")
    _close(_host(rad_g), rad_o.T, 1e-14, "radial")
    for name, g, o in (("lab", lab_g, lab_o), ("body", body_g, body_o), ("pore", pore_g, pore_o)):
        mg = _host(GA.msd(g, n_lags))
        mo = OA.msd(o.transpose(1, 0, 2), n_lags)
        _close(mg / np.abs(mo).max(), mo / np.abs(mo).max(), 1e-10, f"msd {name}")
    rg = _host(GA.rotation_msd(t, ref, n_lags))
    ro = OA.rotation_msd(traj, ref, n_lags)
    assert np.abs(rg - ro).max() <= 1e-8 * np.abs(ro).max(), "rotation msd"
    sg, cg = GA.binned_msd(pore_g, rad_g, edges, n_lags)
    so, co = OA.binned_msd(pore_o.transpose(1, 0, 2), rad_o, edges, n_lags)
    assert np.array_equal(_host(cg), co), "bin counts"
    _close(_host(sg) / max(1.0, np.abs(so).max()), so / max(1.0, np.abs(so).max()), 1e-10,
           "binned msd")
    return lab_g, body_g


@pytest.mark.parametrize("n_frames,n_bodies", [(3000, 4), (257, 1), (1000, 3)])
def test_synthetic_trajectories(n_frames, n_bodies):
    centre = (32.0, 30.0)
    traj = W.synthetic_trajectory(n_frames, n_bodies, seed=n_frames + n_bodies, centre=centre)
    ref = np.random.default_rng(7).normal(size=(n_bodies, 3))
    _compare_all(traj, centre, min(60, n_frames - 1), [0.0, 3.0, 5.0, 7.0, 100.0], ref)


@pytest.mark.parametrize("n_frames,n_bodies,n_lags", [(1000, 2, 150), (300, 1, 299)])
def test_lags_over_several_blocks(n_frames, n_bodies, n_lags):
    """More lags than one workgroup's block of 64 (and not a multiple of it), up to the
    largest, n_frames - 1."""
    centre = (32.0, 30.0)
    traj = W.synthetic_trajectory(n_frames, n_bodies, seed=5 + n_lags, centre=centre)
    ref = np.random.default_rng(8).normal(size=(n_bodies, 3))
    _compare_all(traj, centre, n_lags, [0.0, 4.0, 100.0], ref)


@pytest.mark.parametrize("edges", [np.linspace(2.0, 9.0, 9),          # 8 bins, the tiled kernel
                                   np.linspace(0.0, 12.0, 13)],       # 12 bins, one workgroup per bin
                         ids=["8_bins", "12_bins"])
def test_binned_msd_bin_counts(edges):
    """Binned MSD with the most bins the tiled kernel takes and with more (the per-bin
    kernel); origins outside every bin (radius below 2) are left out."""
    centre = (32.0, 30.0)
    traj = W.synthetic_trajectory(1500, 3, seed=44, centre=centre)
    t = _dev(traj)
    pore_o, rad_o = OA.pore_frame(traj, centre)
    pore_g, rad_g = GA.pore_frame(t, centre)
    sg, cg = GA.binned_msd(pore_g, rad_g, list(edges), 100)
    so, co = OA.binned_msd(pore_o, rad_o, list(edges), 100)
    assert np.array_equal(_host(cg), co), "bin counts"
    scale = max(1.0, np.abs(so).max())
    _close(_host(sg) / scale, so / scale, 1e-10, "binned msd")


def test_long_trajectory():
    traj = W.synthetic_trajectory(200000, 1, seed=99, step=0.02, rot_step=0.02,
                                  centre=(64.0, 64.0), radius=(10.0, 20.0))
    t = _dev(traj)
    g = _host(GA.body_frame(t))[0]
    o = np.concatenate([OA.body_frame_translation(traj), OA.body_frame_rotation(traj)], axis=2)[:, 0]
    _close(g, o, 1e-12, "body frame, 200000 frames")
    mg = _host(GA.msd(GA.body_frame(t), 25))[0]
    mo = OA.msd(o[:, None, :], 25)[0]
    _close(mg / np.abs(mo).max(), mo / np.abs(mo).max(), 1e-10, "msd, 200000 frames")


def test_edge_cases():
    import torch
    traj = W.synthetic_trajectory(1, 2, seed=3)
    assert np.array_equal(_host(GA.body_frame(_dev(traj))), np.zeros((2, 1, 6)))
    traj = W.synthetic_trajectory(12, 1, seed=4)
    t = _dev(traj)
    m = _host(GA.msd(GA.lab_frame(t), 11))
    mo = OA.msd(OA.lab_frame(traj), 11)
    assert np.abs(m - mo).max() <= 1e-12 * np.abs(mo).max()
    L = lbrb.library()
    out = torch.empty(64, dtype=torch.float64, device="cuda:0")
    s = torch.cuda.current_stream().cuda_stream
    assert L.lb_traj_msd(t.data_ptr(), 12, 1, 3, 12, out.data_ptr(), s) == lbrb.LB_ERR_ARG
    assert L.lb_traj_msd(t.data_ptr(), 12, 1, 7, 3, out.data_ptr(), s) == lbrb.LB_ERR_ARG
    assert L.lb_traj_binned_msd(t.data_ptr(), t.data_ptr(), 12, 1, 4, t.data_ptr(), 1, 3,
                                  out.data_ptr(), out.data_ptr(), s) == lbrb.LB_ERR_ARG


def test_recorded_simulation_trajectory():
    R = 3.0
    offs = W.sphere_beads(R, 250)
    m, I = W.solid_body_mass_inertia(1.0, R, R, R)
    wl = dict(name="rec", precision="f32", steps=0, params=W.default_params(kT=4e-5),
              replicas=[dict(shape=(24, 24, 24), seed=11, mask=None,
                             bodies=[W.body_record(offs, m, I, (12.3, 11.6, 12.1),
                                                   gamma=W.GAMMA_FREE),
                                     W.body_record(W.ellipsoid_beads(4.0, 2.0, 2.0),
                                                   *W.solid_body_mass_inertia(1.0, 4, 2, 2),
                                                   (4.0, 5.0, 3.0), quat=(0.6, 0.2, -0.7, 0.3),
                                                   gamma=W.GAMMA_FREE)])])
    sim = lbrb.simulation_from_workload(wl)
    traj_t = GA.record(sim, 400, 5)
    traj = _host(traj_t)
    assert np.all(np.isfinite(traj))
    ref = np.array([offs[1], [4.0, 0.0, 0.0]])
    lab_g, body_g = _compare_all(traj, (12.0, 12.0), 40, [0.0, 4.0, 8.0, 30.0], ref)
    lab1 = _host(GA.msd(lab_g, 1))[:, 0, :].sum(axis=1)
    body1 = _host(GA.msd(body_g[:, :, :3].contiguous(), 1))[:, 0, :].sum(axis=1)
    assert np.abs(lab1 - body1).max() <= 1e-12 * lab1.max()
